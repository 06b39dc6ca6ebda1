// Internal declarations of the near-sorted path (k_runs.hip): the GPU form
// of the partial insertion sort of Section 5.2; not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdq_internal.h"

namespace pdq {

// Descents logged at most; an input with more goes to the partition passes.
constexpr uint32_t kRunMaxDescents = 8192;
// Keys in short runs ("outliers") at most: they are sorted by one LDS
// base-case workgroup (the 8192-key class exists for every key type).
constexpr uint32_t kRunMaxOutliers = 8192;
// Smallest range the path is tried on: it needs a run longer than the
// outlier limit.
constexpr uint64_t kRunMinKeys = 2ull * kRunMaxOutliers;

constexpr uint32_t kRunUnsorted = 0;  // not near-sorted: partition passes
constexpr uint32_t kRunOutliers = 1;  // one long run + outliers
constexpr uint32_t kRunTwoRuns = 2;   // two long runs
constexpr uint32_t kRunSorted = 3;    // no descent at all

struct RunPlan {
  uint32_t state;     // kRun*
  uint32_t nshort;    // short runs (kRunOutliers)
  uint64_t runs;      // maximal non-decreasing runs
  uint64_t descents;  // descents counted (over kRunMaxDescents: counting stopped early)
  uint64_t outliers;  // keys in short runs
  uint64_t a0, a1;    // the (first) long run [a0, a1)
  uint64_t b0, b1;    // the second long run (kRunTwoRuns)
  uint32_t ascent;    // 1: the scanned part has an ascending adjacent pair
  uint32_t pad_;
};

// A short run [start, start + len) gathered to outlier slot dest.
struct RunSpan {
  uint64_t start;
  uint64_t len;
  uint64_t dest;
};

struct RunBufs {
  uint32_t* count;    // [0] descents counted, [1] an ascending pair was seen
  uint32_t* pos;      // kRunMaxDescents logged positions
  RunPlan* plan;
  RunSpan* shorts;    // kRunMaxDescents + 1 entries
  Item* item;         // the outlier buffer as one base-case item
  void* okeys;        // kRunMaxOutliers keys
  uint32_t* ovals;    // kRunMaxOutliers payloads (pairs only)
  uint64_t* splits;   // merge-path split of every merge tile boundary
};

// Merge tile of k_merge (keys per workgroup tile).
constexpr uint64_t kRunMergeTile = 4096;

// Descent scan with copy to c.keys[1] / c.vals[1], then the plan kernel.
hipError_t launch_run_scan(const Ctx& c, const RunBufs& rb, hipStream_t s);
// Copies the plan's short runs into the outlier buffer.
hipError_t launch_run_gather(const Ctx& c, const RunBufs& rb, uint32_t nshort, hipStream_t s);
// Merges the plan's sorted sequences into the user buffer.
hipError_t launch_run_merge(const Ctx& c, const RunBufs& rb, const RunPlan& p, hipStream_t s);

}  // namespace pdq
