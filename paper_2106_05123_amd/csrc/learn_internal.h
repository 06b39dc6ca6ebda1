// Internal declarations of the learned multiway first pass: a small MLP fitted
// to the CDF of a key sample proposes up to 255 splitters; one histogram pass
// and one scatter then split the input into up to 511 bins (range bins and
// equality bins) before the partition passes take over. Not part of the
// public C ABI (include/pdq_learned.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdq {

// ---- model: 1 -> 32 -> 32 -> 1 ReLU MLP, residual output ------------------
constexpr int kH = 32;
constexpr int kNParam = 1153;
constexpr int kOffW1 = 0, kOffB1 = 32, kOffW2 = 64, kOffB2 = 64 + 1024, kOffW3 = 64 + 1024 + 32,
              kOffB3 = 64 + 1024 + 64;
constexpr int kParamStride = 1160;      // padded row of a gradient partial; [kNParam] holds the loss sum
constexpr uint64_t kSaltInit = 0x5EED0000ull;
constexpr uint64_t kSaltBatch = 0xBA7C0000ull;
constexpr int kMaxSplitters = 255;
constexpr int kMaxBins = 2 * kMaxSplitters + 1;  // 511
constexpr int kBinStride = 512;                  // padded histogram row
constexpr uint32_t kTrainThreads = 1024;
constexpr uint32_t kTrainChunk = 64;             // samples a training workgroup handles at a time
constexpr uint32_t kBucketTile = 8192;           // keys per histogram / scatter tile
constexpr uint32_t kBucketThreads = 512;
constexpr uint32_t kScanRows = 256;              // tile rows per scan chunk
constexpr int kLeaves = 64;                      // leaves of the model's second stage
constexpr int kCandidates = 3;                   // splitter candidates: root, x-leaves, y-leaves
constexpr int kInfoWords = 8;                    // words of the fit's info array

struct TrainArgs {
  const float* x;         // features of the sorted sample [m]
  const float* t;         // mid-rank targets [m]
  uint64_t m;
  uint64_t seed;
  uint32_t steps;
  uint32_t batch;         // minibatch size, a multiple of grid
  uint32_t grid;          // cooperating workgroups
  uint32_t residual;
  const float* init;      // start from these parameters (null: seeded initialisation)
  float* params;          // out [kNParam]
  float* losses;          // out [steps]
  float* partials;        // [2][grid][kParamStride] gradient exchange
  uint32_t* sync;         // [0] barrier counter (zero before launch), [1] error flag
};

struct FitBufs {
  uint64_t* raw;      // [m] sampled key images, unsorted (scratch)
  uint64_t* sample;   // [m] sorted key images
  float* x;           // [m]
  float* t;           // [m]
  float* y;           // [m] clamped prediction
  float* runmax;      // [m] running maximum of y
  float* params;      // [kNParam]
  float* losses;      // [steps]
  float* partials;    // [2][grid][kParamStride]
  uint32_t* sync;     // [4]
  uint64_t* info;     // [kInfoWords]: dev_log bits, dev_lin bits, use_log, chosen candidate,
                      // sample judge of each candidate (3), histogram go flag
  uint64_t* splitters;  // [256] the chosen candidate's splitters
  uint32_t* count;    // [1]
  // second stage and candidates
  float* runmax2;     // [2][m] running maxima of the leaf predictions
  float* yx;          // [m] x-leaf predictions
  float* yy;          // [m] y-leaf predictions
  double* leaf;       // [2][kLeaves][2] intercept and slope of every leaf
  uint64_t* cand;     // [kCandidates][256] splitters of each candidate
  uint32_t* cand_count;  // [kCandidates]
  uint64_t* est;      // [kCandidates] sample judge of each candidate
};

struct BucketBufs {
  const uint64_t* splitters;
  const uint32_t* count;   // number of splitters u (device)
  uint32_t* rows;          // [ntiles][kBinStride] per-tile counts, then per-tile offsets
  uint32_t* chunk;         // [nchunks][kBinStride] chunk sums, then chunk offsets
  uint64_t* totals;        // [kBinStride] keys per bin
  uint64_t* begin;         // [kBinStride + 1] first position of each bin
  uint64_t ntiles;
  uint64_t nchunks;
  uint32_t* errors;        // scatter: bit kErrScatter when a position falls outside [0, n)
  uint32_t* order;         // order scan: bit 0 some adjacent pair descends, bit 1 some pair ascends
  const uint64_t* go;      // null, or a word that is 0 when the histogram is not wanted
};

constexpr uint32_t kErrScatter = 8u;

// k_learn.hip
hipError_t launch_sample(uint32_t kt, const void* keys, uint64_t n, uint64_t m, uint64_t seed, uint64_t* out,
                         hipStream_t s);
// m a multiple of 4096; sorts raw in place by chunks, writes the merge to sorted
hipError_t launch_sample_sort(uint64_t* raw, uint64_t m, uint64_t* sorted, hipStream_t s);
hipError_t launch_features(const uint64_t* sorted, uint64_t m, float* x, float* t, uint64_t* info, hipStream_t s);
hipError_t launch_train(const TrainArgs& a, hipStream_t s);
hipError_t launch_infer(const float* params, const float* x, uint64_t m, uint32_t residual, float* y,
                        hipStream_t s);
hipError_t launch_gradient(const float* params, const float* x, const float* t, uint32_t batch, uint32_t residual,
                           float* grad, float* loss, hipStream_t s);
hipError_t launch_extract(const uint64_t* sorted, const float* y, uint64_t m, float* runmax, uint64_t* splitters,
                          uint32_t* count, hipStream_t s);
// The three candidates' extractions side by side (one workgroup each):
// predictions y[c], running maxima runmax[c], splitters `stride` apart.
hipError_t launch_extract_candidates(const uint64_t* sorted, uint64_t m, const float* const* y, float* const* runmax,
                                     uint64_t* splitters, uint32_t stride, uint32_t* count, hipStream_t s);

// Running maximum of y[0..m) (clamped predictions), as the extraction computes it.
hipError_t launch_running_max(const float* y, uint64_t m, float* runmax, hipStream_t s);
// Second stage: leaf fits on the running maximum of y, then both leaf
// predictions of every sample.
hipError_t launch_leaves(const float* x, const float* t, const float* y, const float* runmax, uint64_t m,
                         double* leaf, float* yx, float* yy, hipStream_t s);
// est[c] = largest sample count in a range bin of candidate c (ncand
// candidates, splitters `stride` apart).
hipError_t launch_sample_judge(const uint64_t* sorted, uint64_t m, const uint64_t* splitters, uint32_t stride,
                               const uint32_t* count, uint32_t ncand, uint64_t* est, hipStream_t s);
hipError_t launch_pick(const uint64_t* splitters, uint32_t stride, const uint32_t* count, const uint64_t* est,
                       uint32_t ncand, uint64_t go_limit, uint64_t* out, uint32_t* out_count, uint64_t* info,
                       hipStream_t s);

// k_bucket.hip
// bit 0 of *flags: some adjacent pair of keys[0..n) descends; bit 1: some pair ascends.
hipError_t launch_order_scan(uint32_t kt, const void* keys, uint64_t n, uint32_t* flags, hipStream_t s);
hipError_t launch_bucket_hist(uint32_t kt, const void* keys, uint64_t n, const BucketBufs& b, hipStream_t s);
hipError_t launch_bucket_scan(const BucketBufs& b, hipStream_t s);
hipError_t launch_bucket_scatter(uint32_t kt, bool pairs, const void* keys_in, const uint32_t* vals_in,
                                 void* keys_out, uint32_t* vals_out, uint64_t n, const BucketBufs& b,
                                 hipStream_t s);

inline uint64_t bucket_tiles(uint64_t n) { return (n + kBucketTile - 1) / kBucketTile; }
inline uint64_t bucket_chunks(uint64_t n) { return (bucket_tiles(n) + kScanRows - 1) / kScanRows; }

}  // namespace pdq
