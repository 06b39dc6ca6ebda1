// Internal declarations of the batched segmented sort: one persistent launch
// works through a device queue of segments; not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdq_internal.h"

namespace pdq {

// One queued segment of more than kBaseMax keys: [begin, end) in buffer buf.
struct BItem {
  uint64_t begin;
  uint64_t end;
  uint32_t buf;
  uint32_t budget;
  uint32_t flags;
  uint32_t pad;
};

// Queue words. The ring holds cap items; slot state (one word per slot) is
// 2(j+1) while item j waits in the slot and 2(j+1)+1 once it was taken, so a
// consumer of item j and a producer of item j + cap can tell the
// generations apart.
struct BatchQ {
  uint32_t head;     // next item number to claim
  uint32_t tail;     // next item number to push
  uint32_t pending;  // items pushed and not yet finished
  uint32_t error;    // kErrQueue / kErrSplit bits
  uint32_t cap;
  uint32_t pad[59];
};

constexpr uint32_t kErrQueue = 16u;  // a queue wait did not end (ring too small or a lost item)

// Tunable shape of the persistent kernel: threads per workgroup and rows per
// partition tile (a tile is NT * IT keys).
struct BatchShape {
  uint32_t nt;
  uint32_t it;
};

constexpr int kBatchShapes = 4;
constexpr BatchShape kShapes[kBatchShapes] = {{512, 8}, {512, 16}, {1024, 8}, {1024, 16}};

struct BatchArgs {
  BatchQ* q;
  BItem* items;
  uint32_t* state;
};

hipError_t launch_batch_prepare(const Ctx& c, const BatchArgs& b, uint32_t cap, hipStream_t s);
hipError_t launch_batch(const Ctx& c, const BatchArgs& b, int shape, uint32_t grid, hipStream_t s);
// Largest segment the persistent kernel of this shape sorts in LDS at once.
uint32_t batch_lds_max(const Ctx& c, int shape);
// Workgroups of the persistent kernel that fit on the device at once.
uint32_t batch_grid(const Ctx& c, int shape);

}  // namespace pdq
