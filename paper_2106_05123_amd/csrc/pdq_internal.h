// Internal declarations shared by the HIP kernels and the host driver of the
// partition sort. Nothing here is part of the public C ABI (include/pdq.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pdq {

constexpr uint32_t kBaseMax = 4096;     // segments of at most this many keys go to the LDS base case
constexpr uint32_t kWideBaseMax = 16384;  // the batched form's widest LDS class
constexpr int kBaseClasses = 7;         // base-case size classes: <= 64, 256, 1024, 2048, 4096, 8192, 16384 keys
constexpr uint32_t kWave = 64;          // CDNA wavefront width
constexpr uint32_t kSegLeftmost = 1u;   // segment has no predecessor (Section 3)
constexpr uint32_t kSegFresh = 2u;      // parent partition was bad: use fresh candidates (Section 4.2)
constexpr uint32_t kModeRight = 0u;
constexpr uint32_t kModeLeft = 1u;

// Order bits of a segment (positions in a 64-bit word; Cursor::order_bits
// holds them shifted down by 32):
//   kStDesc  some adjacent pair descends
//   kStAsc   some adjacent pair ascends
// They also sit in the tile status words of the deterministic (look-back)
// partition, whose layout is:
//   [63:62] state (0 empty, 1 aggregate, 2 inclusive prefix)
//   [61:60] kStDesc | kStAsc, ORed over the covered tiles
//   [59:0]  count of keys going left
constexpr uint64_t kStAgg = 1ull << 62;
constexpr uint64_t kStIncl = 2ull << 62;
constexpr uint64_t kStStateMask = 3ull << 62;
constexpr uint64_t kStDesc = 1ull << 61;
constexpr uint64_t kStAsc = 1ull << 60;
constexpr uint64_t kStCountMask = (1ull << 60) - 1;

// The reservation partition hands out its tiles from kTicketQueues counters,
// one per XCD (workgroup b uses queue b mod 8; workgroups are dispatched to
// the 8 XCDs round-robin), each over its own share of the pass's tiles and
// on its own cache line: atomics on one line run one after another, and a
// single counter for all tiles of a pass took longer than the pass itself.
constexpr uint32_t kTicketQueues = 8;
constexpr uint32_t kTicketStride = 32;  // 128 bytes

// One live segment of a partition pass. Positions are absolute indices into
// the key arrays; the segment's keys sit in the pass's source buffer.
struct Seg {
  uint64_t begin;
  uint64_t end;
  uint64_t pivot;      // raw key bits of the pivot (pivot kernel)
  uint64_t pidx;       // absolute position of the pivot element in the source buffer
  uint32_t tile_base;  // first tile ticket of the segment in this pass
  uint32_t ntiles;
  uint32_t budget;     // bad partitions still allowed (Section 4.1)
  uint32_t flags;      // kSegLeftmost | kSegFresh
  uint32_t mode;       // kModeRight / kModeLeft (pivot kernel)
};

// What the partition kernel accumulates for segment i of the pass, kept
// apart from the Seg records: every tile reads its Seg, and atomics on a
// cache line that workgroups also read run several times slower than on a
// line that only atomics touch. Cleared by the tile-map kernel.
struct Cursor {
  uint64_t left;       // keys placed left of the pivot (low 32 bits) and right of it
                       // (high 32 bits), reserved tile by tile; with the look-back, the
                       // left count written by the segment's last tile
  uint32_t order_bits; // kStDesc | kStAsc >> 32 of the whole segment (ORed by its tiles)
  uint32_t pad_;
};

// A range handed to a finishing kernel: base case, heapsort or a plain
// (possibly reversing) copy into the user buffer.
struct Item {
  uint64_t begin;
  uint64_t end;
  uint32_t buf;     // 0 user buffer, 1 scratch buffer
  uint32_t reverse; // copy items: bit 0 = write the range in reverse order; bits 1.. = the chunk
                    // of kCopyChunk keys this item covers (of the swapped pairs, for an
                    // in-place reversal)
};

// Keys per copy item: a large retired range is filed as several items, so
// that many workgroups copy it.
constexpr uint64_t kCopyChunk = 1ull << 16;

// Item counts of one set of item lists: the base-case classes, heapsort,
// copies (in this order, contiguous).
constexpr int kItemHeap = kBaseClasses;
constexpr int kItemCopy = kBaseClasses + 1;
constexpr int kItemCounts = kBaseClasses + 2;

// Device-side counters. Host reads a snapshot after each pass.
struct Counters {
  uint64_t list[2];        // per list parity: (segments << 32) | tiles
  uint64_t elems[2];       // per list parity: keys in the list
  uint64_t maxlen[2];      // per list parity: keys of its largest segment
  uint32_t nbase[kBaseClasses];  // item set 0: nbase[], nheap, ncopy
  uint32_t nheap, ncopy, ticket, pad1_;
  // statistics (accumulated over the call)
  uint64_t partitions_right, partitions_left, bad_partitions;
  uint64_t heap_segments, heap_elements;
  uint64_t base_segments, base_elements;
  uint64_t sorted_segments, sorted_elements, equal_elements;
  uint64_t first_pivot_image;
  uint64_t max_seg;        // largest input segment (initial lists)
  uint64_t visits;         // keys of every partitioned segment, summed over the passes
  int64_t first_left;
  int32_t first_mode;
  uint32_t bad_offsets;    // validation: offsets not monotone / not covering [0, n)
  uint32_t errors;         // kErr* bits: an internal inconsistency was caught and its writes skipped
  uint32_t live_passes;    // partition passes that found at least one live segment
  uint32_t items1[kItemCounts];  // item set 1 (the pipelined pass loop alternates sets)
  uint32_t pad3_;
};
static_assert(offsetof(Counters, nheap) == offsetof(Counters, nbase) + 4 * kItemHeap, "item set 0 layout");
static_assert(offsetof(Counters, ncopy) == offsetof(Counters, nbase) + 4 * kItemCopy, "item set 0 layout");

// Item counts of set `set` inside a counter block (kItemCounts words).
__host__ __device__ inline uint32_t* item_counts(Counters* ctr, int set) {
  return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ctr) +
                                     (set ? offsetof(Counters, items1) : offsetof(Counters, nbase)));
}
__host__ __device__ inline const uint32_t* item_counts(const Counters* ctr, int set) {
  return item_counts(const_cast<Counters*>(ctr), set);
}

constexpr uint32_t kErrCapacity = 1u;  // a list append found its list full (only reachable with bad offsets)
constexpr uint32_t kErrLookback = 2u;  // a tile's reservation did not fit its segment
constexpr uint32_t kErrSplit = 4u;     // a segment's left count did not fit the segment

// Everything a kernel needs to know about one sort call.
struct Ctx {
  void* keys[2];        // [0] user keys, [1] scratch keys
  uint32_t* vals[2];    // payloads (null when sorting keys only)
  uint64_t n;
  Seg* segs[2];         // live-segment lists, indexed by pass parity
  uint32_t* tilemap;    // ticket -> segment index
  Cursor* cur;          // segment index -> its partition cursor (the pass being run)
  uint32_t* tickets;    // reservation partition: kTicketQueues counters, kTicketStride words apart
  uint64_t* status;     // ticket -> look-back status word (deterministic partition only)
  Item* base[kBaseClasses];  // the item set being filled or finished
  Item* heap;
  Item* copy;
  Counters* ctr;
  uint32_t* icnt;       // its counts (item_counts): [class] base cases, [kItemHeap], [kItemCopy]
  const uint64_t* offsets;  // segmented input (null: one segment [0, n))
  uint64_t nseg;
  uint32_t tile;        // keys per partition tile
  uint32_t max_active;  // capacity of each live-segment list
  uint32_t max_tiles;   // capacity of tilemap / status
  uint32_t max_items;   // capacity of each item list
  int32_t force_budget;
  uint32_t key_type;
  uint32_t has_vals;
  uint32_t single;      // 1: one segment [0, n) (records the first partition)
  uint32_t device_counts;  // 1: the pass kernels (and finishing kernels launched with this flag)
                           // take their counts from ctr instead of their arguments
  uint32_t accumulate;  // 1 (batched form): item lists accumulate over the passes and are
                        // finished once at the end; 0: each pass's pivot kernel clears the
                        // counts of the set its bookkeeping fills
  uint64_t seed;        // seeds the candidate positions taken after a bad partition
  uint32_t base_max;    // segments of at most this many keys go to the LDS base case
  uint8_t base_var[kBaseClasses];  // workgroup shape of each base-case class (kBaseThreads)
  uint8_t pad2_;
  uint32_t lookback;    // 1: tiles take their places by a decoupled look-back (deterministic order)
  uint32_t fresh_fixed; // 1: fresh candidates at the fixed quarter offsets instead of hashed positions
  uint32_t heapsort;    // 1: the fallback of segments out of budget is the paper's one-lane heapsort
};

// ---- key traits: canonical unsigned image in registers only ---------------
// ord() maps a key's bits to an unsigned integer with the same order; inv()
// undoes it.
struct KeyU32 {
  using T = uint32_t;
  static __device__ __forceinline__ uint32_t ord(uint32_t x) { return x; }
  static __device__ __forceinline__ uint32_t inv(uint32_t x) { return x; }
};
struct KeyI32 {
  using T = uint32_t;
  static __device__ __forceinline__ uint32_t ord(uint32_t x) { return x ^ 0x80000000u; }
  static __device__ __forceinline__ uint32_t inv(uint32_t x) { return x ^ 0x80000000u; }
};
struct KeyF32 {
  using T = uint32_t;
  // negative: flip all bits; non-negative: set the sign bit
  static __device__ __forceinline__ uint32_t ord(uint32_t x) {
    return x ^ (static_cast<uint32_t>(static_cast<int32_t>(x) >> 31) | 0x80000000u);
  }
  static __device__ __forceinline__ uint32_t inv(uint32_t y) {
    return (y & 0x80000000u) ? (y ^ 0x80000000u) : ~y;
  }
};
struct KeyU64 {
  using T = uint64_t;
  static __device__ __forceinline__ uint64_t ord(uint64_t x) { return x; }
  static __device__ __forceinline__ uint64_t inv(uint64_t x) { return x; }
};
struct KeyI64 {
  using T = uint64_t;
  static __device__ __forceinline__ uint64_t ord(uint64_t x) { return x ^ 0x8000000000000000ull; }
  static __device__ __forceinline__ uint64_t inv(uint64_t x) { return x ^ 0x8000000000000000ull; }
};
struct KeyF64 {
  using T = uint64_t;
  // negative: flip all bits; non-negative: set the sign bit
  static __device__ __forceinline__ uint64_t ord(uint64_t x) {
    return x ^ (static_cast<uint64_t>(static_cast<int64_t>(x) >> 63) | 0x8000000000000000ull);
  }
  static __device__ __forceinline__ uint64_t inv(uint64_t y) {
    return (y & 0x8000000000000000ull) ? (y ^ 0x8000000000000000ull) : ~y;
  }
};

// SplitMix64 output function (Steele, Lea and Flood, 2014): the counter-based
// generator behind every random choice of the library.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---- launch entry points (one translation unit each) ---------------------
// Every launcher dispatches on ctx.key_type / ctx.has_vals.
hipError_t launch_reset(const Ctx& c, hipStream_t s);
hipError_t launch_init(const Ctx& c, hipStream_t s);
hipError_t launch_bucket_init(const Ctx& c, const uint64_t* begin, hipStream_t s);
hipError_t launch_pivot(const Ctx& c, int parity, uint32_t nseg, uint32_t src_buf, hipStream_t s);
hipError_t launch_tilemap(const Ctx& c, int parity, uint32_t ntiles, hipStream_t s);
hipError_t launch_partition(const Ctx& c, int parity, uint32_t ntiles, uint32_t src_buf, hipStream_t s);
hipError_t launch_bookkeep(const Ctx& c, int parity, uint32_t nseg, uint32_t src_buf, uint32_t pass,
                           hipStream_t s);
hipError_t launch_base(const Ctx& c, int cls, uint32_t nitems, hipStream_t s);
hipError_t launch_heap(const Ctx& c, uint32_t nitems, hipStream_t s);
hipError_t launch_copy(const Ctx& c, uint32_t nitems, hipStream_t s);
// 64-bit payloads (PDQ_VALS64): idx[i] = i and copy = vals before the sort,
// vals[i] = copy[idx[i]] after it.
hipError_t launch_vals64_prepare(const uint64_t* vals, uint64_t n, uint32_t* idx, uint64_t* copy, hipStream_t s);
hipError_t launch_vals64_gather(uint64_t* vals, uint64_t n, const uint32_t* idx, const uint64_t* copy,
                                hipStream_t s);

inline uint32_t key_bytes(uint32_t key_type) { return key_type >= 4 ? 8u : 4u; }

// Workgroup shapes of the LDS base case: lanes per workgroup for size class
// k (64, 256, 1024, ..., 16384 slots) and variant v, for 32-bit slots and
// 64-bit keys without payload [0] and for 64-bit keys with a payload [1];
// 0 where the variant does not exist (the launcher then takes variant 0).
// Variant 0 is the default; the batched form's autotuner picks per class.
constexpr int kBaseVariants = 3;
constexpr uint16_t kBaseThreads[2][kBaseClasses][kBaseVariants] = {
    {{64, 0, 0}, {64, 128, 256}, {64, 128, 256}, {128, 256, 64}, {256, 512, 128}, {512, 256, 1024}, {1024, 512, 0}},
    {{64, 0, 0}, {64, 128, 256}, {128, 256, 0}, {256, 512, 0}, {512, 1024, 0}, {1024, 0, 0}, {0, 0, 0}}};

__host__ __device__ inline int base_threads(bool wide_pairs, int cls, int var) {
  const int t = kBaseThreads[wide_pairs ? 1 : 0][cls][var < kBaseVariants ? var : 0];
  return t ? t : kBaseThreads[wide_pairs ? 1 : 0][cls][0];
}

// Size class of a base-case segment of n keys (1 <= n <= kWideBaseMax).
__host__ __device__ inline int base_class(uint64_t n) {
  return n <= 64 ? 0 : n <= 256 ? 1 : n <= 1024 ? 2 : n <= 2048 ? 3 : n <= 4096 ? 4 : n <= 8192 ? 5 : 6;
}

// Number of tile tickets a segment [b, e) takes: its tiles start at b, so
// only the last one is partial.
__host__ __device__ inline uint32_t tiles_of(uint64_t b, uint64_t e, uint32_t tile) {
  return static_cast<uint32_t>((e - b + tile - 1) / tile);
}

}  // namespace pdq
