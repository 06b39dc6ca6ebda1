// Per-pass control kernels of the partition sort: initial segment lists,
// pivot choice, tile map, segment bookkeeping, and the finishing copies and
// the fallback sort of segments out of budget.
#include "bitonic.h"
#include "learn_internal.h"
#include "pdq_internal.h"
#include "pivot.h"
#include "wave_ops.h"

namespace pdq {
namespace {

constexpr int kCtlThreads = 256;

__device__ __forceinline__ uint32_t floor_log2_u64(uint64_t x) { return 63u - __clzll(x); }

template <class K>
__device__ __forceinline__ typename K::T load_key(const Ctx& c, uint32_t buf, uint64_t i) {
  return static_cast<const typename K::T*>(c.keys[buf])[i];
}

// Append a range to an item list of capacity cap (every lane calls; `want`
// selects). A full list skips the write and flags the call.
__device__ __forceinline__ void push_item(const Ctx& c, Item* list, uint32_t* ctr, bool want, uint64_t b,
                                          uint64_t e, uint32_t buf, uint32_t reverse) {
  const uint32_t slot = wave_reserve(ctr, want);
  if (want) {
    if (slot < c.max_items) list[slot] = Item{b, e, buf, reverse};
    else atomicOr(&c.ctr->errors, kErrCapacity);
  }
}

// Append a range to the copy list, as one item per chunk of kCopyChunk keys
// (of swapped pairs, for an in-place reversal). Every lane calls.
__device__ __forceinline__ void push_copy(const Ctx& c, bool want, uint64_t b, uint64_t e, uint32_t buf,
                                          uint32_t reverse) {
  const uint64_t span = want ? ((reverse && buf == 0) ? (e - b) / 2 : e - b) : 0;
  const uint32_t nch = want ? static_cast<uint32_t>(span > kCopyChunk ? (span + kCopyChunk - 1) / kCopyChunk : 1)
                            : 0u;
  const uint32_t first = wave_reserve_n(&c.icnt[kItemCopy], nch);
  for (uint32_t k = 0; k < nch; ++k) {
    const uint32_t slot = first + k;
    if (slot < c.max_items) c.copy[slot] = Item{b, e, buf, reverse | (k << 1)};
    else atomicOr(&c.ctr->errors, kErrCapacity);
  }
}

// Append a base-case segment to the list of its size class.
__device__ __forceinline__ void push_base(const Ctx& c, bool want, uint64_t b, uint64_t e, uint32_t buf) {
  const int cls = want ? base_class(e - b) : -1;
#pragma unroll
  for (int k = 0; k < kBaseClasses; ++k) push_item(c, c.base[k], &c.icnt[k], cls == k, b, e, buf, 0u);
}

// Append a live segment to list `parity` and reserve its tile tickets.
__device__ __forceinline__ void push_seg(const Ctx& c, int parity, bool want, uint64_t b, uint64_t e,
                                         uint32_t budget, uint32_t flags) {
  const uint32_t nt = want ? tiles_of(b, e, c.tile) : 0u;
  const uint64_t r = wave_reserve_packed(reinterpret_cast<unsigned long long*>(&c.ctr->list[parity]), want, nt);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->elems[parity]), want ? (e - b) : 0ull);
  const uint64_t wmax = wave_max_u64(want ? (e - b) : 0ull);
  if (lane_id() == 0 && wmax) atomicMax(reinterpret_cast<unsigned long long*>(&c.ctr->maxlen[parity]), wmax);
  if (want && ((r >> 32) >= c.max_active || static_cast<uint64_t>(static_cast<uint32_t>(r)) + nt > c.max_tiles)) {
    atomicOr(&c.ctr->errors, kErrCapacity);
  } else if (want) {
    Seg s;
    s.begin = b;
    s.end = e;
    s.pivot = 0;
    s.pidx = b;
    s.tile_base = static_cast<uint32_t>(r);
    s.ntiles = nt;
    s.budget = budget;
    s.flags = flags;
    s.mode = kModeRight;
    c.segs[parity][r >> 32] = s;
  }
}

__global__ void k_reset(Ctx c) {
  if (threadIdx.x == 0) {
    Counters z = {};
    z.first_mode = -1;
    *c.ctr = z;
  }
}

// Initial lists: every input segment is leftmost, with budget floor(log2 size)
// (Section 4.1) unless forced. Offsets are clamped into [0, n] so that bad
// offsets can never address outside the arrays; they are flagged instead.
__global__ __launch_bounds__(kCtlThreads) void k_init(Ctx c) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool live = i < c.nseg;
  uint64_t b = 0, e = 0;
  if (live) {
    if (c.offsets) {
      b = c.offsets[i];
      e = c.offsets[i + 1];
      bool bad = e < b || e > c.n || b > c.n || (i == 0 && b != 0) || (i + 1 == c.nseg && e != c.n);
      if (bad) atomicOr(&c.ctr->bad_offsets, 1u);
      if (b > c.n) b = c.n;
      if (e > c.n) e = c.n;
      if (e < b) e = b;
    } else {
      b = 0;
      e = c.n;
    }
  }
  const uint64_t size = e - b;
  uint32_t budget = 0;
  if (size >= 2) budget = c.force_budget >= 0 ? static_cast<uint32_t>(c.force_budget) : floor_log2_u64(size);
  const bool big = size > c.base_max;
  const uint64_t wmax = wave_max_u64(size);
  if (lane_id() == 0 && wmax) atomicMax(reinterpret_cast<unsigned long long*>(&c.ctr->max_seg), wmax);
  push_seg(c, 0, big && budget > 0, b, e, budget, kSegLeftmost);
  const bool to_base = size >= 2 && !big;
  const bool to_heap = big && budget == 0;
  push_base(c, to_base, b, e, 0u);
  push_item(c, c.heap, &c.icnt[kItemHeap], to_heap, b, e, 0u, 0u);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->base_segments), to_base ? 1 : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->base_elements), to_base ? size : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->heap_segments), to_heap ? 1 : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->heap_elements), to_heap ? size : 0);
}

// After the learned multiway scatter the bins are contiguous ranges of the
// scratch buffer, in key order. Range bins (even index) become leftmost
// segments: their keys are strictly greater than every key before them, so
// the predecessor rule would always pick partition_right anyway. Equality
// bins (odd index) hold copies of one key and are copied out unchanged.
__global__ __launch_bounds__(kCtlThreads) void k_bucket_init(Ctx c, const uint64_t* begin) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < static_cast<uint32_t>(kBinStride);
  uint64_t b = 0, e = 0;
  if (in) {
    b = begin[i];
    e = begin[i + 1];
  }
  const uint64_t size = e - b;
  const bool eq = in && (i & 1u) && size > 0;
  const bool range = in && !(i & 1u) && size > 0;
  uint32_t budget = 0;
  if (size >= 2) budget = c.force_budget >= 0 ? static_cast<uint32_t>(c.force_budget) : floor_log2_u64(size);
  const bool big = size > c.base_max;
  push_copy(c, eq, b, e, 1u, 0u);
  push_seg(c, 0, range && big && budget > 0, b, e, budget, kSegLeftmost);
  const bool to_base = range && !big;
  const bool to_heap = range && big && budget == 0;
  push_base(c, to_base, b, e, 1u);
  push_item(c, c.heap, &c.icnt[kItemHeap], to_heap, b, e, 1u, 0u);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->base_segments), to_base ? 1 : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->base_elements), to_base ? size : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->heap_segments), to_heap ? 1 : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->heap_elements), to_heap ? size : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->equal_elements), eq ? size : 0);
}

// Pivot choice for every live segment (choose_pivot, pivot.h). The first
// lane also clears the counters of the list the bookkeeping will fill (and,
// unless the item lists accumulate over the passes, the counts of the item
// set it fills).
template <class K>
__global__ __launch_bounds__(kCtlThreads) void k_pivot(Ctx c, int parity, uint32_t nseg, uint32_t src) {
  using T = typename K::T;
  if (c.device_counts) nseg = static_cast<uint32_t>(c.ctr->list[parity] >> 32);
  if (nseg > c.max_active) nseg = c.max_active;  // an overfull list is flagged, never read past
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.ctr->visits += c.ctr->elems[parity];
    if (nseg) c.ctr->live_passes += 1;
    c.ctr->list[parity ^ 1] = 0;
    c.ctr->elems[parity ^ 1] = 0;
    c.ctr->maxlen[parity ^ 1] = 0;
    if (!c.accumulate)
      for (int k = 0; k < kItemCounts; ++k) c.icnt[k] = 0;
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nseg; i += gridDim.x * blockDim.x) {
    Seg* sp = &c.segs[parity][i];
    const PivotChoice<K> pc = choose_pivot<K>(static_cast<const T*>(c.keys[src]), static_cast<const T*>(c.keys[0]),
                                              sp->begin, sp->end, sp->flags, c.seed, c.fresh_fixed != 0);
    sp->pivot = static_cast<uint64_t>(pc.raw);
    sp->pidx = pc.pidx;
    sp->mode = pc.mode;
  }
}

// Ticket -> segment map for the partition kernel, a cleared cursor per
// segment (and, for the look-back partition, a cleared status word per
// ticket).
__global__ __launch_bounds__(kCtlThreads) void k_tilemap(Ctx c, int parity, uint32_t ntiles) {
  const uint32_t t0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (t0 == 0) c.ctr->ticket = 0;
  if (t0 < kTicketQueues) c.tickets[t0 * kTicketStride] = 0;
  if (c.device_counts) ntiles = static_cast<uint32_t>(c.ctr->list[parity]);
  if (ntiles > c.max_tiles) ntiles = c.max_tiles;
  uint32_t nseg = static_cast<uint32_t>(c.ctr->list[parity] >> 32);
  if (nseg > c.max_active) nseg = c.max_active;
  const Seg* segs = c.segs[parity];
  for (uint32_t t = t0; t < nseg; t += gridDim.x * blockDim.x) c.cur[t] = Cursor{};
  for (uint32_t t = t0; t < ntiles; t += gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
      uint32_t mid = (lo + hi + 1) >> 1;
      if (segs[mid].tile_base <= t) lo = mid;
      else hi = mid - 1;
    }
    c.tilemap[t] = lo;
    if (c.lookback) c.status[t] = 0;
  }
}

// One live segment after its partition (every lane of the wave calls).
template <class K>
__device__ __forceinline__ void bookkeep_one(const Ctx& c, int parity, uint32_t i, uint32_t nseg, uint32_t src,
                                             uint32_t pass) {
  using T = typename K::T;
  const bool live = i < nseg;
  const uint32_t dst = src ^ 1u;
  Seg s = {};
  Cursor cu = {};
  if (live) {
    s = c.segs[parity][i];
    cu = c.cur[i];
  }
  const uint64_t size = s.end - s.begin;
  const bool no_desc = live && !(cu.order_bits & static_cast<uint32_t>(kStDesc >> 32));
  const bool no_asc = live && !(cu.order_bits & static_cast<uint32_t>(kStAsc >> 32));
  const bool asc_sorted = no_desc;           // non-decreasing in the source buffer
  const bool desc_sorted = !no_desc && no_asc; // non-increasing in the source buffer
  bool split = live && !asc_sorted && !desc_sorted;
  // the partition kernel's packed cursor: keys placed left (low half) and
  // right (high half) of the pivot
  const uint64_t L = static_cast<uint32_t>(cu.left);
  if (split && L >= size) {
    atomicOr(&c.ctr->errors, kErrSplit);
    split = false;
  }
  const bool is_left = s.mode == kModeLeft;
  const uint64_t R = size - 1 - L;
  const bool bad = split && !is_left && (L < (size >> 3) || R < (size >> 3));

  if (live && c.single && pass == 0 && i == 0) {
    c.ctr->first_pivot_image = static_cast<uint64_t>(K::ord(static_cast<T>(s.pivot)));
    c.ctr->first_left = static_cast<int64_t>(L);
    c.ctr->first_mode = static_cast<int32_t>(s.mode);
  }
  if (split) {
    const uint64_t p = s.begin + L;
    static_cast<T*>(c.keys[0])[p] = static_cast<T>(s.pivot);
    if (c.has_vals) c.vals[0][p] = c.vals[src][s.pidx];
  }
  // already ordered: copy (reversed when descending) into the user buffer
  const bool ordered = asc_sorted || desc_sorted;
  push_copy(c, ordered && !(src == 0 && asc_sorted), s.begin, s.end, src, desc_sorted ? 1u : 0u);
  // partition_left: the left side equals the pivot and is final
  push_copy(c, split && is_left && L > 0 && dst != 0, s.begin, s.begin + L, dst, 0u);

  const uint32_t cbudget = s.budget - (bad ? 1u : 0u);
  const uint32_t cflag_fresh = bad ? kSegFresh : 0u;
  // two children: left (only for partition_right) and right
  for (int side = 0; side < 2; ++side) {
    const bool has = split && (side == 1 || !is_left);
    const uint64_t cb = side == 0 ? s.begin : s.begin + L + 1;
    const uint64_t ce = side == 0 ? s.begin + L : s.end;
    const uint64_t cs = has ? ce - cb : 0;
    const uint32_t cflags = cflag_fresh | (side == 0 ? (s.flags & kSegLeftmost) : 0u);
    const bool to_base = has && cs >= 1 && cs <= c.base_max && !(cs == 1 && dst == 0);
    const bool to_heap = has && cs > c.base_max && cbudget == 0;
    const bool to_live = has && cs > c.base_max && cbudget > 0;
    push_base(c, to_base, cb, ce, dst);
    push_item(c, c.heap, &c.icnt[kItemHeap], to_heap, cb, ce, dst, 0u);
    push_seg(c, parity ^ 1, to_live, cb, ce, cbudget, cflags);
    wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->base_segments), to_base ? 1 : 0);
    wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->base_elements), to_base ? cs : 0);
    wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->heap_segments), to_heap ? 1 : 0);
    wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->heap_elements), to_heap ? cs : 0);
  }

  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->partitions_right), split && !is_left ? 1 : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->partitions_left), split && is_left ? 1 : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->bad_partitions), bad ? 1 : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->sorted_segments), ordered ? 1 : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->sorted_elements), ordered ? size : 0);
  wave_add(reinterpret_cast<unsigned long long*>(&c.ctr->equal_elements), split && is_left ? L : 0);
}

// After a partition pass: place each pivot at its final position in the user
// buffer, retire segments that were already ordered (Section 5.2) and the
// equal-to-pivot side of partition_left (Section 3), count bad partitions and
// charge the budget (Section 4.1), and file every child as live segment, base
// case or heapsort.
template <class K>
__global__ __launch_bounds__(kCtlThreads) void k_bookkeep(Ctx c, int parity, uint32_t nseg, uint32_t src,
                                                         uint32_t pass) {
  if (c.device_counts) nseg = static_cast<uint32_t>(c.ctr->list[parity] >> 32);
  if (nseg > c.max_active) nseg = c.max_active;
  // the loop bound is uniform over each wave: the wave-wide appends see every lane
  for (uint32_t i0 = blockIdx.x * blockDim.x; i0 < nseg; i0 += gridDim.x * blockDim.x)
    bookkeep_one<K>(c, parity, i0 + threadIdx.x, nseg, src, pass);
}

// Copies into the user buffer: plain, reversed, or reversed in place. The
// blocks of row blockIdx.y share the items blockIdx.x, + gridDim.x, ...
template <class K>
__global__ __launch_bounds__(kCtlThreads) void k_copy(Ctx c, uint32_t nitems) {
  using T = typename K::T;
  uint32_t count = c.device_counts ? c.icnt[kItemCopy] : nitems;
  if (count > c.max_items) count = c.max_items;  // an overfull list is flagged, never read past
  T* out = static_cast<T*>(c.keys[0]);
  uint32_t* outv = c.vals[0];
  const uint64_t stride = static_cast<uint64_t>(gridDim.y) * blockDim.x;
  const uint64_t start = static_cast<uint64_t>(blockIdx.y) * blockDim.x + threadIdx.x;
  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
    const Item it = c.copy[item];
    const uint64_t len = it.end - it.begin;
    const T* in = static_cast<const T*>(c.keys[it.buf]);
    const uint32_t* inv = c.vals[it.buf];
    const bool rev = (it.reverse & 1u) != 0;
    // this item's chunk of the range (of the swapped pairs, in place)
    const uint64_t c0 = static_cast<uint64_t>(it.reverse >> 1) * kCopyChunk;
    const uint64_t span = rev && it.buf == 0 ? len / 2 : len;
    const uint64_t c1 = c0 + kCopyChunk < span ? c0 + kCopyChunk : span;
    if (rev && it.buf == 0) {
      for (uint64_t j = c0 + start; j < c1; j += stride) {
        const uint64_t a = it.begin + j, z = it.end - 1 - j;
        T ka = out[a], kz = out[z];
        out[a] = kz;
        out[z] = ka;
        if (c.has_vals) {
          uint32_t va = outv[a], vz = outv[z];
          outv[a] = vz;
          outv[z] = va;
        }
      }
    } else if (rev) {
      for (uint64_t j = c0 + start; j < c1; j += stride) {
        out[it.begin + j] = in[it.end - 1 - j];
        if (c.has_vals) outv[it.begin + j] = inv[it.end - 1 - j];
      }
    } else {
      for (uint64_t j = c0 + start; j < c1; j += stride) {
        out[it.begin + j] = in[it.begin + j];
        if (c.has_vals) outv[it.begin + j] = inv[it.begin + j];
      }
    }
  }
}

// The paper's fallback (PDQ_HEAPSORT): Williams' heapsort of a[0..len) (and
// payloads v, if any) by one lane, in place in the user buffer.
template <class K>
__device__ void sift_down(typename K::T* a, uint32_t* v, uint64_t root, uint64_t n) {
  for (;;) {
    uint64_t child = 2 * root + 1;
    if (child >= n) return;
    if (child + 1 < n && K::ord(a[child]) < K::ord(a[child + 1])) ++child;
    if (!(K::ord(a[root]) < K::ord(a[child]))) return;
    typename K::T t = a[root];
    a[root] = a[child];
    a[child] = t;
    if (v) {
      uint32_t tv = v[root];
      v[root] = v[child];
      v[child] = tv;
    }
    root = child;
  }
}

template <class K>
__device__ void heapsort_range(typename K::T* a, uint32_t* v, uint64_t len) {
  if (len < 2) return;
  for (uint64_t r = len / 2; r-- > 0;) sift_down<K>(a, v, r, len);
  for (uint64_t end = len - 1; end > 0; --end) {
    typename K::T t = a[0];
    a[0] = a[end];
    a[end] = t;
    if (v) {
      uint32_t tv = v[0];
      v[0] = v[end];
      v[end] = tv;
    }
    sift_down<K>(a, v, 0, end);
  }
}

// Fallback sort of Section 4.1, for a segment that used up its bad-partition
// budget. The paper heapsorts the segment in place: O(n log n) whatever the
// input, but one element at a time. Here one workgroup merge-sorts it, also
// O(n log n) whatever the input, with every lane busy: chunks of kFbChunk
// keys are sorted in LDS (the base case's merge sort, each key paired with
// its index so that its payload follows) into the other buffer, then merge
// passes alternate between the two buffers. In a pass, every lane finds
// where its kFbRun outputs of a merged pair of runs start (a merge-path
// binary search) and merges them one by one, ties from the left run. The
// segment's range of the other buffer is free (its keys left it), and the
// result ends in the user buffer.
constexpr int kFbE = 8;
constexpr int kFbChunk = kFbE * kCtlThreads;
constexpr uint64_t kFbRun = 8;

template <class K, bool PAIRS>
__device__ void fallback_sort(const Ctx& c, const Item& it, unsigned char* sh) {
  using T = typename K::T;
  using S = net::Slot<K, PAIRS>;
  using V = typename S::V;
  const int tid = static_cast<int>(threadIdx.x);
  const uint64_t len = it.end - it.begin;
  uint32_t src = it.buf;
  // sorted chunks, into the other buffer
  {
    const T* kin = static_cast<const T*>(c.keys[src]) + it.begin;
    const uint32_t* vin = PAIRS ? c.vals[src] + it.begin : nullptr;
    T* kout = static_cast<T*>(c.keys[src ^ 1u]) + it.begin;
    uint32_t* vout = PAIRS ? c.vals[src ^ 1u] + it.begin : nullptr;
    for (uint64_t cb = 0; cb < len; cb += kFbChunk) {
      const int clen = static_cast<int>(len - cb < static_cast<uint64_t>(kFbChunk) ? len - cb : kFbChunk);
      V x[kFbE];
#pragma unroll
      for (int r = 0; r < kFbE; ++r) {
        const int j = tid * kFbE + r;
        x[r] = j < clen ? S::make(kin[cb + j], static_cast<uint32_t>(j)) : S::pad();
      }
      net::merge_sort<S, kFbE, kCtlThreads>(x, sh, tid);
#pragma unroll
      for (int r = 0; r < kFbE; ++r) {
        const int j = tid * kFbE + r;
        if (j < clen) {
          kout[cb + j] = S::key(x[r]);
          if constexpr (PAIRS) vout[cb + j] = vin[cb + S::idx(x[r])];
        }
      }
    }
    src ^= 1u;
    __threadfence_block();
    __syncthreads();
  }
  // merge passes
  for (uint64_t w = kFbChunk; w < len; w *= 2) {
    const T* sk = static_cast<const T*>(c.keys[src]) + it.begin;
    const uint32_t* sv = PAIRS ? c.vals[src] + it.begin : nullptr;
    T* dk = static_cast<T*>(c.keys[src ^ 1u]) + it.begin;
    uint32_t* dv = PAIRS ? c.vals[src ^ 1u] + it.begin : nullptr;
    for (uint64_t lo = 0; lo < len; lo += 2 * w) {
      const uint64_t mid = lo + w < len ? lo + w : len;
      const uint64_t hi = lo + 2 * w < len ? lo + 2 * w : len;
      const uint64_t na = mid - lo, nb = hi - mid;
      for (uint64_t o = static_cast<uint64_t>(tid) * kFbRun; o < na + nb;
           o += static_cast<uint64_t>(kCtlThreads) * kFbRun) {
        // i = keys of the left run among the first o outputs: A[i'] is among
        // them exactly when A[i'] <= B[o - i' - 1]
        uint64_t ilo = o > nb ? o - nb : 0, ihi = o < na ? o : na;
        while (ilo < ihi) {
          const uint64_t im = (ilo + ihi) / 2;
          if (!(K::ord(sk[mid + (o - im - 1)]) < K::ord(sk[lo + im]))) ilo = im + 1;
          else ihi = im;
        }
        uint64_t i = ilo, j = o - ilo;
        const uint64_t oend = o + kFbRun < na + nb ? o + kFbRun : na + nb;
        for (uint64_t q = o; q < oend; ++q) {
          const bool take_a = j >= nb || (i < na && !(K::ord(sk[mid + j]) < K::ord(sk[lo + i])));
          const uint64_t from = take_a ? lo + i : mid + j;
          dk[lo + q] = sk[from];
          if constexpr (PAIRS) dv[lo + q] = sv[from];
          if (take_a) ++i;
          else ++j;
        }
      }
    }
    src ^= 1u;
    __threadfence_block();
    __syncthreads();
  }
  if (src != 0) {
    const T* sk = static_cast<const T*>(c.keys[src]) + it.begin;
    T* dk = static_cast<T*>(c.keys[0]) + it.begin;
    for (uint64_t j = static_cast<uint64_t>(tid); j < len; j += kCtlThreads) {
      dk[j] = sk[j];
      if constexpr (PAIRS) c.vals[0][it.begin + j] = c.vals[src][it.begin + j];
    }
  }
  __threadfence_block();
  __syncthreads();
}

// One workgroup per fallback item (Section 4.1).
template <class K, bool PAIRS>
__global__ __launch_bounds__(kCtlThreads) void k_heap(Ctx c, uint32_t nitems) {
  using S = net::Slot<K, PAIRS>;
  __shared__ __align__(16) unsigned char sh[net::lds_plane<kFbChunk, kFbE>() * S::kLdsBytes];
  uint32_t count = c.device_counts ? c.icnt[kItemHeap] : nitems;
  if (count > c.max_items) count = c.max_items;
  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
    const Item it = c.heap[item];
    if (it.end - it.begin < 2) {
      // one key: only its place in the user buffer
      if (threadIdx.x == 0 && it.end > it.begin && it.buf != 0) {
        static_cast<typename K::T*>(c.keys[0])[it.begin] = static_cast<const typename K::T*>(c.keys[it.buf])[it.begin];
        if constexpr (PAIRS) c.vals[0][it.begin] = c.vals[it.buf][it.begin];
      }
      continue;
    }
    if (c.heapsort) {
      // the paper's heapsort: the segment moves to the user buffer, then one
      // lane sorts it there
      const uint64_t len = it.end - it.begin;
      typename K::T* a = static_cast<typename K::T*>(c.keys[0]) + it.begin;
      uint32_t* v = PAIRS ? c.vals[0] + it.begin : nullptr;
      if (it.buf != 0) {
        const typename K::T* in = static_cast<const typename K::T*>(c.keys[it.buf]) + it.begin;
        for (uint64_t j = threadIdx.x; j < len; j += blockDim.x) {
          a[j] = in[j];
          if constexpr (PAIRS) v[j] = c.vals[it.buf][it.begin + j];
        }
        __threadfence_block();
        __syncthreads();
      }
      if (threadIdx.x == 0) heapsort_range<K>(a, v, len);
      __syncthreads();
    } else {
      fallback_sort<K, PAIRS>(c, it, sh);
    }
  }
}

template <template <class> class F, class... Args>
hipError_t dispatch_key(uint32_t kt, Args&&... args) {
  switch (kt) {
    case 1: return F<KeyU32>::run(args...);
    case 2: return F<KeyI32>::run(args...);
    case 3: return F<KeyF32>::run(args...);
    case 4: return F<KeyU64>::run(args...);
    case 5: return F<KeyI64>::run(args...);
    case 6: return F<KeyF64>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

inline uint32_t blocks_for(uint64_t n, uint32_t per) { return static_cast<uint32_t>((n + per - 1) / per); }

// Blocks of a control launch over n entries: one entry per lane, or, with
// device counts (n is then a capacity), at most `cap` blocks that loop.
inline uint32_t ctl_blocks(const Ctx& c, uint64_t n, uint32_t cap) {
  const uint32_t b = blocks_for(n, kCtlThreads);
  return c.device_counts && b > cap ? cap : b;
}
constexpr uint32_t kDevCtlBlocks = 512;

template <class K>
struct PivotL {
  static hipError_t run(const Ctx& c, int parity, uint32_t nseg, uint32_t src, hipStream_t s) {
    const uint32_t g = ctl_blocks(c, nseg, kDevCtlBlocks);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pivot<K>, dim3(g), dim3(kCtlThreads), 0, s, c, parity, nseg, src);
    return hipGetLastError();
  }
};
template <class K>
struct BookL {
  static hipError_t run(const Ctx& c, int parity, uint32_t nseg, uint32_t src, uint32_t pass, hipStream_t s) {
    const uint32_t g = ctl_blocks(c, nseg, kDevCtlBlocks);
    if (g == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bookkeep<K>, dim3(g), dim3(kCtlThreads), 0, s, c, parity, nseg, src, pass);
    return hipGetLastError();
  }
};
template <class K>
struct CopyL {
  static hipError_t run(const Ctx& c, uint32_t nitems, hipStream_t s) {
    const uint32_t g = c.device_counts && nitems > 2048 ? 2048 : nitems;
    if (g == 0) return hipSuccess;
    // a row of 8 workgroups per item: items hold at most kCopyChunk keys
    hipLaunchKernelGGL(k_copy<K>, dim3(g, 8), dim3(kCtlThreads), 0, s, c, nitems);
    return hipGetLastError();
  }
};
template <class K>
struct HeapL {
  static hipError_t run(const Ctx& c, uint32_t nitems, hipStream_t s) {
    const uint32_t g = c.device_counts && nitems > 2048 ? 2048 : nitems;
    if (g == 0) return hipSuccess;
    if (c.has_vals) hipLaunchKernelGGL((k_heap<K, true>), dim3(g), dim3(kCtlThreads), 0, s, c, nitems);
    else hipLaunchKernelGGL((k_heap<K, false>), dim3(g), dim3(kCtlThreads), 0, s, c, nitems);
    return hipGetLastError();
  }
};

}  // namespace

hipError_t launch_reset(const Ctx& c, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_init(const Ctx& c, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(blocks_for(c.nseg, kCtlThreads)), dim3(kCtlThreads), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_bucket_init(const Ctx& c, const uint64_t* begin, hipStream_t s) {
  hipLaunchKernelGGL(k_bucket_init, dim3(blocks_for(kBinStride, kCtlThreads)), dim3(kCtlThreads), 0, s, c, begin);
  return hipGetLastError();
}

hipError_t launch_pivot(const Ctx& c, int parity, uint32_t nseg, uint32_t src, hipStream_t s) {
  return dispatch_key<PivotL>(c.key_type, c, parity, nseg, src, s);
}

hipError_t launch_tilemap(const Ctx& c, int parity, uint32_t ntiles, hipStream_t s) {
  const uint32_t g = ctl_blocks(c, ntiles, 4 * kDevCtlBlocks);
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tilemap, dim3(g), dim3(kCtlThreads), 0, s, c, parity, ntiles);
  return hipGetLastError();
}

hipError_t launch_bookkeep(const Ctx& c, int parity, uint32_t nseg, uint32_t src, uint32_t pass, hipStream_t s) {
  return dispatch_key<BookL>(c.key_type, c, parity, nseg, src, pass, s);
}

hipError_t launch_copy(const Ctx& c, uint32_t nitems, hipStream_t s) {
  return dispatch_key<CopyL>(c.key_type, c, nitems, s);
}

hipError_t launch_heap(const Ctx& c, uint32_t nitems, hipStream_t s) {
  return dispatch_key<HeapL>(c.key_type, c, nitems, s);
}

// 64-bit payloads travel through the sort as 32-bit indices: before it,
// idx[i] = i and a copy of the payloads; after it, each output slot fetches
// its payload through its index.
__global__ __launch_bounds__(256) void k_vals64_prepare(const uint64_t* __restrict__ vals, uint64_t n,
                                                        uint32_t* __restrict__ idx, uint64_t* __restrict__ copy) {
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * 256u) {
    idx[i] = static_cast<uint32_t>(i);
    copy[i] = vals[i];
  }
}

__global__ __launch_bounds__(256) void k_vals64_gather(uint64_t* __restrict__ vals, uint64_t n,
                                                       const uint32_t* __restrict__ idx,
                                                       const uint64_t* __restrict__ copy) {
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * 256u) {
    const uint32_t j = idx[i];
    vals[i] = j < n ? copy[j] : 0ull;  // j < n always; the test keeps a corrupted index in bounds
  }
}

static uint32_t stream_grid(uint64_t n) {
  const uint64_t g = (n + 255) / 256;
  return static_cast<uint32_t>(g < 16384 ? (g ? g : 1) : 16384);
}

hipError_t launch_vals64_prepare(const uint64_t* vals, uint64_t n, uint32_t* idx, uint64_t* copy, hipStream_t s) {
  hipLaunchKernelGGL(k_vals64_prepare, dim3(stream_grid(n)), dim3(256), 0, s, vals, n, idx, copy);
  return hipGetLastError();
}

hipError_t launch_vals64_gather(uint64_t* vals, uint64_t n, const uint32_t* idx, const uint64_t* copy,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_vals64_gather, dim3(stream_grid(n)), dim3(256), 0, s, vals, n, idx, copy);
  return hipGetLastError();
}

}  // namespace pdq
