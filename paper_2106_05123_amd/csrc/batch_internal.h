// Internal declarations of the batched segmented sort (captured partition
// passes with device-side counts, wide LDS classes, and a persistent tail
// launch over a device queue); not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdq_internal.h"

namespace pdq {

// One queued segment: [begin, end) in buffer buf.
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

// Shapes of the persistent tail kernel: threads per workgroup and rows per
// partition tile (a tile is NT * IT keys). The tail only finishes the few
// segments the captured passes leave, so one shape serves.
struct TailShape {
  uint32_t nt;
  uint32_t it;
};
constexpr int kTailShapes = 1;
constexpr TailShape kTail[kTailShapes] = {{512, 8}};

// Shape of the batched form: the tile of the captured partition passes,
// the slots per lane of the two widest LDS classes when the shape is given
// explicitly (16: 512 and 1024 threads for 8192 and 16384 keys; 32: 256 and
// 512 threads), and the tail kernel's shape.
struct BatchShape {
  uint32_t tile;
  uint32_t wide_e;
  uint32_t tail;
};
constexpr int kBatchShapes = 4;
constexpr BatchShape kShapes[kBatchShapes] = {{8192, 16, 0}, {16384, 16, 0}, {32768, 16, 0}, {8192, 32, 0}};
// The autotuner tries the partition tiles (shapes 0-2); the 32-slot form of
// the widest classes (shape 3) is one of their per-class variants.
constexpr int kTunedShapes = 3;

// Passes the device-counted form queues at most; deeper recursions finish in
// the persistent tail.
constexpr uint32_t kMaxBatchPasses = 32;

struct BatchArgs {
  BatchQ* q;
  BItem* items;
  uint32_t* state;
};

hipError_t launch_batch_zero(const BatchArgs& b, uint32_t cap, hipStream_t s);
hipError_t launch_batch_from_list(const Ctx& c, const BatchArgs& b, int parity, uint32_t src, hipStream_t s);
hipError_t launch_batch(const Ctx& c, const BatchArgs& b, int tail, uint32_t grid, hipStream_t s);
// ORs the queue's error bits into the counter block (after launch_batch).
hipError_t launch_batch_fold(const Ctx& c, const BatchArgs& b, hipStream_t s);
// Workgroups of the persistent kernel of this tail shape that fit on the
// device at once.
uint32_t batch_grid(const Ctx& c, int tail);

}  // namespace pdq
