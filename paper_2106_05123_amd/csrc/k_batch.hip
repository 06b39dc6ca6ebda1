// The persistent tail of the batched segmented sort. The captured partition
// passes leave some segments live (those whose recursion is deeper than the
// passes that were queued); this launch works through them with a device
// queue, so the whole sort ends without the host reading anything back.
//
//   from_list the live segments become queue items
//   batch     persistent workgroups take items in order. An item that fits
//             the workgroup's LDS network (NT * E keys) is sorted there in
//             one read and one write. A larger one is partitioned by the
//             workgroup alone -- the same pivot rule, Dutch-flag modes,
//             bad-partition budget and ordered-run detection as the pass
//             kernels (Sections 3, 4.1, 4.2, 5.2) -- into the other buffer;
//             its children are sorted at once when they fit in LDS (while
//             they are still in this XCD's cache) or queued otherwise.
//             A segment out of budget is filed for the fallback sort
//             (Section 4.1), which runs after the launch.
//
// Inside the persistent launch a segment written by one workgroup may be read
// by a workgroup on another XCD, whose L2 is not coherent with the writer's.
// Every access to segment data that another workgroup may touch in the same
// launch is therefore an agent-scope (coherent) load or store; queue slots
// carry generation tags and are published after the item's words completed.
#include "batch_internal.h"
#include "bitonic.h"
#include "pdq_internal.h"
#include "pivot.h"
#include "wave_ops.h"

namespace pdq {
namespace {

template <class T>
__device__ __forceinline__ T cload(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void cstore(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t floor_log2(uint64_t x) { return 63u - __clzll(x); }

constexpr uint32_t kSpinLimit = 1u << 24;

// ---------------------------------------------------------------- queue

// Push one item (one lane). The slot must first be released by the
// consumer of the item one ring-length earlier.
__device__ bool queue_push(const BatchArgs& bq, const BItem& it) {
  BatchQ* q = bq.q;
  __hip_atomic_fetch_add(&q->pending, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t j = __hip_atomic_fetch_add(&q->tail, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t cap = q->cap;
  const uint32_t slot = j % cap;
  const uint32_t free_state = j < cap ? 0u : 2u * (j - cap + 1u) + 1u;
  uint32_t spins = 0;
  while (cload(&bq.state[slot]) != free_state) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      atomicOr(&q->error, kErrQueue);
      return false;
    }
  }
  BItem* d = &bq.items[slot];
  cstore(&d->begin, it.begin);
  cstore(&d->end, it.end);
  cstore(&d->buf, it.buf);
  cstore(&d->budget, it.budget);
  cstore(&d->flags, it.flags);
  __builtin_amdgcn_s_waitcnt(0);  // the item's words are complete before the slot is published
  cstore(&bq.state[slot], 2u * (j + 1u));
  return true;
}

// Claim the next item (one lane). Returns false when every item has been
// finished (or the queue failed).
__device__ bool queue_pop(const BatchArgs& bq, BItem& it) {
  BatchQ* q = bq.q;
  const uint32_t h = __hip_atomic_fetch_add(&q->head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t cap = q->cap;
  const uint32_t slot = h % cap;
  const uint32_t want = 2u * (h + 1u);
  uint32_t spins = 0;
  for (;;) {
    if (cload(&bq.state[slot]) == want) break;
    if (cload(&q->pending) == 0u || cload(&q->error) != 0u) return false;
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      atomicOr(&q->error, kErrQueue);
      return false;
    }
  }
  const BItem* s = &bq.items[slot];
  it.begin = cload(&s->begin);
  it.end = cload(&s->end);
  it.buf = cload(&s->buf);
  it.budget = cload(&s->budget);
  it.flags = cload(&s->flags);
  cstore(&bq.state[slot], want + 1u);
  return true;
}

// ---------------------------------------------------------------- prepare

__global__ void k_batch_zero(BatchArgs b, uint32_t cap) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < cap) b.state[i] = 0;
  if (i == 0) {
    BatchQ z = {};
    z.cap = cap;
    *b.q = z;
  }
}

// After the persistent launch: the queue's error bits join the counter
// block's, so that one word tells the caller about every device-side error
// of the call (pdq_check reads it).
__global__ void k_batch_fold(Ctx c, BatchArgs b) {
  if (threadIdx.x == 0) {
    const uint32_t e = b.q->error;
    if (e) atomicOr(&c.ctr->errors, e);
  }
}

// The segments still live after the captured partition passes (list
// `parity`, keys in buffer `src`) become the queue's first items, with the
// budget and flags their bookkeeping gave them.
__global__ __launch_bounds__(256) void k_batch_from_list(Ctx c, BatchArgs b, int parity, uint32_t src) {
  uint32_t nlive = static_cast<uint32_t>(c.ctr->list[parity] >> 32);
  if (nlive > c.max_active) nlive = c.max_active;
  for (uint32_t i0 = blockIdx.x * blockDim.x; i0 < nlive; i0 += gridDim.x * blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    const bool live = i < nlive;
    const uint32_t j = wave_reserve(&b.q->tail, live);
    if (live) {
      const Seg sg = c.segs[parity][i];
      if (j < b.q->cap) {
        BItem it;
        it.begin = sg.begin;
        it.end = sg.end;
        it.buf = src;
        it.budget = sg.budget;
        it.flags = sg.flags;
        it.pad = 0;
        b.items[j] = it;
        b.state[j] = 2u * (j + 1u);
      } else {
        atomicOr(&b.q->error, kErrQueue);
      }
    }
    const uint64_t nq = __popcll(__ballot(live));
    if (lane_id() == 0 && nq) atomicAdd(&b.q->pending, static_cast<uint32_t>(nq));
  }
}

// ---------------------------------------------------------------- persistent kernel

// LDS sort of in[0..len) into out[0..len) by NTS threads holding E slots
// each (the base case's merge sort, or its bitonic network below 1024
// slots). With NTS == 64 only wave 0 takes part and nothing waits at a
// workgroup barrier.
template <class K, bool PAIRS, int E, int NTS>
__device__ void lds_sort(const typename K::T* in, const uint32_t* vin, typename K::T* out, uint32_t* vout, int len,
                         unsigned char* sh) {
  using S = net::Slot<K, PAIRS>;
  using V = typename S::V;
  constexpr int P = E * NTS;
  constexpr int PL = net::lds_plane<P, E>();
  const int tid = threadIdx.x;
  auto sync = [&]() {
    if constexpr (NTS > 64) {
      __syncthreads();
    } else {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  };
  if (tid >= NTS) return;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int j = r * NTS + tid;
    V v = S::pad();
    if (j < len) v = S::make(cload(in + j), static_cast<uint32_t>(j));
    S::st(sh, PL, net::lds_pos<E>(j), v);
  }
  sync();
  V x[E];
#pragma unroll
  for (int r = 0; r < E; ++r) x[r] = S::ld(sh, PL, net::lds_pos<E>((tid << net::ilog2(E)) | r));
  sync();
  if constexpr (P >= 1024) net::merge_sort<S, E, NTS>(x, sh, tid);
  else net::bitonic<S, E, NTS>(x, sh, tid);
#pragma unroll
  for (int r = 0; r < E; ++r) S::st(sh, PL, net::lds_pos<E>((tid << net::ilog2(E)) | r), x[r]);
  sync();
  V y[E];
#pragma unroll
  for (int r = 0; r < E; ++r) y[r] = S::ld(sh, PL, net::lds_pos<E>(r * NTS + tid));
  if constexpr (PAIRS) {
    uint32_t pv[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int j = r * NTS + tid;
      pv[r] = j < len ? cload(vin + S::idx(y[r])) : 0u;
    }
    sync();  // every payload is read before any is written (in and out may coincide)
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int j = r * NTS + tid;
      if (j < len) {
        out[j] = S::key(y[r]);
        vout[j] = pv[r];
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int j = r * NTS + tid;
      if (j < len) out[j] = S::key(y[r]);
    }
  }
}

template <class K, bool PAIRS, int NT, int IT>
struct Batch {
  using T = typename K::T;
  using S = net::Slot<K, PAIRS>;
  static constexpr int NW = NT / 64;
  // largest network: NT * EB slots (8 per lane at 1024 lanes, where a lane has 128 VGPRs)
  static constexpr int EB = (NT >= 1024 || (sizeof(T) == 8 && PAIRS)) ? 8 : 16;
  static constexpr int kLdsMax = NT * EB;
  static constexpr int kSortBytes = net::lds_plane<NT * EB, EB>() * S::kLdsBytes;
  static constexpr int kCells = IT * NW;  // (row, wave) cells of a partition tile
  static constexpr int kPartBytes = 2 * kCells * 4 + 32 + 16 + (kCells + 1) * static_cast<int>(sizeof(T)) + 16;
  static constexpr int kShBytes = kSortBytes > kPartBytes ? kSortBytes : kPartBytes;
  static_assert(kCells <= 256, "one scan of at most 256 cells per tile");
};

// Sorts [b, e) of buffer `buf` into the user buffer with the smallest
// network that holds it.
template <class K, bool PAIRS, int NT>
__device__ void sort_segment(const Ctx& c, uint64_t b, uint64_t e, uint32_t buf, unsigned char* sh) {
  using T = typename K::T;
  constexpr int EB = Batch<K, PAIRS, NT, 8>::EB;
  const int len = static_cast<int>(e - b);
  const T* in = static_cast<const T*>(c.keys[buf]) + b;
  T* out = static_cast<T*>(c.keys[0]) + b;
  const uint32_t* vin = PAIRS ? c.vals[buf] + b : nullptr;
  uint32_t* vout = PAIRS ? c.vals[0] + b : nullptr;
  if (len <= 256) lds_sort<K, PAIRS, 4, 64>(in, vin, out, vout, len, sh);
  else if (len <= NT * 4) lds_sort<K, PAIRS, 4, NT>(in, vin, out, vout, len, sh);
  else if (len <= NT * 8) lds_sort<K, PAIRS, 8, NT>(in, vin, out, vout, len, sh);
  else if constexpr (EB == 16) lds_sort<K, PAIRS, 16, NT>(in, vin, out, vout, len, sh);
  __syncthreads();
}

// Copies [b, e) of buffer `buf` into the user buffer, reversed or not (in
// place when buf is the user buffer).
template <class K, bool PAIRS, int NT>
__device__ void copy_out(const Ctx& c, uint64_t b, uint64_t e, uint32_t buf, bool reverse) {
  using T = typename K::T;
  T* out = static_cast<T*>(c.keys[0]);
  const T* in = static_cast<const T*>(c.keys[buf]);
  const uint64_t len = e - b;
  if (reverse && buf == 0) {
    for (uint64_t j = threadIdx.x; j < len / 2; j += NT) {
      const uint64_t x = b + j, z = e - 1 - j;
      const T kx = cload(out + x), kz = cload(out + z);
      out[x] = kz;
      out[z] = kx;
      if constexpr (PAIRS) {
        const uint32_t vx = cload(c.vals[0] + x), vz = cload(c.vals[0] + z);
        c.vals[0][x] = vz;
        c.vals[0][z] = vx;
      }
    }
  } else if (buf != 0 || reverse) {
    for (uint64_t j = threadIdx.x; j < len; j += NT) {
      const uint64_t from = reverse ? e - 1 - j : b + j;
      out[b + j] = cload(in + from);
      if constexpr (PAIRS) c.vals[0][b + j] = cload(c.vals[buf] + from);
    }
  }
  __syncthreads();
}

// One workgroup partitions [b, e) of buffer `src` around the pivot into the
// other buffer: keys going left are packed from b upwards, the others from
// e - 1 downwards, tile by tile (NT * IT keys), ranks from wave ballots and
// one scan over the tile's (row, wave) cells. Also records whether any
// adjacent pair of the segment descends or ascends.
template <class K, bool PAIRS, int NT, int IT>
__device__ void partition_wg(const Ctx& c, uint64_t b, uint64_t e, uint32_t src, typename K::T pivot,
                             uint64_t pidx, uint32_t mode, unsigned char* sh, uint64_t& left, bool& desc,
                             bool& asc) {
  using T = typename K::T;
  using B = Batch<K, PAIRS, NT, IT>;
  constexpr int NW = B::NW;
  constexpr int CELLS = B::kCells;
  uint32_t* s_cl = reinterpret_cast<uint32_t*>(sh);  // [IT][NW] left counts, then offsets
  uint32_t* s_cr = s_cl + CELLS;                      // right counts, then offsets
  uint64_t* s_wsum = reinterpret_cast<uint64_t*>(s_cr + CELLS);  // [4] scan totals per wave of cells
  uint32_t* s_tot = reinterpret_cast<uint32_t*>(s_wsum + 4);     // [0] left, [1] right in the tile
  uint32_t* s_flag = s_tot + 2;
  T* s_carry = reinterpret_cast<T*>(s_tot + 4);                  // last key of the previous tile
  T* s_head = s_carry + 1;                                       // first key of each (row, wave) cell
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const T* in = static_cast<const T*>(c.keys[src]);
  T* out = static_cast<T*>(c.keys[src ^ 1u]);
  const uint32_t* vin = PAIRS ? c.vals[src] : nullptr;
  uint32_t* vout = PAIRS ? c.vals[src ^ 1u] : nullptr;
  const auto p = K::ord(pivot);
  uint64_t L = 0, R = 0;
  bool d = false, a = false;
  if (tid == 0) s_flag[0] = 0;
  for (uint64_t t0 = b; t0 < e; t0 += static_cast<uint64_t>(NT) * IT) {
    T k[IT];
    uint32_t v[IT];
    uint64_t ml[IT], mr[IT];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const uint64_t j = t0 + static_cast<uint64_t>(r) * NT + tid;
      const bool valid = j < e;
      k[r] = valid ? cload(in + j) : T(0);
      if constexpr (PAIRS) v[r] = valid ? cload(vin + j) : 0u;
      const auto o = K::ord(k[r]);
      const bool goes_left = mode == kModeRight ? o < p : o <= p;
      const bool counted = valid && j != pidx;
      ml[r] = __ballot(counted && goes_left);
      mr[r] = __ballot(counted && !goes_left);
      if (lane == 0) {
        s_cl[r * NW + w] = __popcll(ml[r]);
        s_cr[r * NW + w] = __popcll(mr[r]);
        s_head[r * NW + w] = k[r];
      }
    }
    __syncthreads();
    // exclusive scan of the cells in (row, wave) order, both sides at once
    // (right count in the high half); every thread takes part in the wave scans
    uint64_t x = 0;
    if (tid < CELLS) x = (static_cast<uint64_t>(s_cr[tid]) << 32) | s_cl[tid];
    const uint64_t incl = wave_incl_scan_u64(x);
    if (lane == 63 && w < 4) s_wsum[w] = incl;
    __syncthreads();
    if (tid < CELLS) {
      uint64_t before = 0;
      for (int q = 0; q < w; ++q) before += s_wsum[q];
      const uint64_t ex = before + incl - x;
      s_cl[tid] = static_cast<uint32_t>(ex);
      s_cr[tid] = static_cast<uint32_t>(ex >> 32);
      if (tid == CELLS - 1) {
        s_tot[0] = static_cast<uint32_t>(ex + x);
        s_tot[1] = static_cast<uint32_t>((ex + x) >> 32);
      }
    }
    __syncthreads();
    // order of adjacent pairs: the successor of (row r, thread t) is
    // (r, t + 1), the next row's first key, or the next tile's first key
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const uint64_t j = t0 + static_cast<uint64_t>(r) * NT + tid;
      T nx = __shfl_down(k[r], 1, 64);
      if (lane == 63) {
        if (w + 1 < NW) nx = s_head[r * NW + w + 1];
        else if (r + 1 < IT) nx = s_head[(r + 1) * NW];
      }
      const bool tile_last = lane == 63 && w + 1 == NW && r + 1 == IT;
      if (j + 1 < e && !tile_last) {
        const auto o = K::ord(k[r]), on = K::ord(nx);
        d |= on < o;
        a |= on > o;
      }
    }
    if (t0 > b && tid == 0) {
      const auto o = K::ord(s_carry[0]), on = K::ord(k[0]);
      d |= on < o;
      a |= on > o;
    }
    // scatter
    const uint64_t tl = s_tot[0], tr = s_tot[1];
#pragma unroll
    for (int r = 0; r < IT; ++r) {
      const bool gl = (ml[r] >> lane) & 1ull, gr = (mr[r] >> lane) & 1ull;
      if (gl) {
        const uint64_t at = b + L + s_cl[r * NW + w] + lanes_below(ml[r]);
        cstore(out + at, k[r]);
        if constexpr (PAIRS) cstore(vout + at, v[r]);
      } else if (gr) {
        const uint64_t at = e - 1 - (R + s_cr[r * NW + w] + lanes_below(mr[r]));
        cstore(out + at, k[r]);
        if constexpr (PAIRS) cstore(vout + at, v[r]);
      }
    }
    L += tl;
    R += tr;
    __syncthreads();
    if (tid == NT - 1) s_carry[0] = k[IT - 1];  // full tile: the last key is real
  }
  const uint32_t bits = (__ballot(d) ? 1u : 0u) | (__ballot(a) ? 2u : 0u);
  if (lane == 0 && bits) atomicOr(&s_flag[0], bits);
  __syncthreads();
  desc = s_flag[0] & 1u;
  asc = s_flag[0] & 2u;
  left = L;
  __syncthreads();
}

template <class K, bool PAIRS, int NT, int IT>
__global__ __launch_bounds__(NT) void k_batch(Ctx c, BatchArgs bq) {
  using T = typename K::T;
  using B = Batch<K, PAIRS, NT, IT>;
  __shared__ __align__(16) unsigned char sh[B::kShBytes];
  __shared__ BItem s_item;
  __shared__ uint32_t s_ok;
  __shared__ T s_pivot;
  __shared__ uint64_t s_pidx;
  __shared__ uint32_t s_mode;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      BItem it;
      s_ok = queue_pop(bq, it) ? 1u : 0u;
      s_item = it;
    }
    __syncthreads();
    if (!s_ok) break;
    const BItem it = s_item;
    const uint64_t b = it.begin, e = it.end, size = e - b;
    if (size <= static_cast<uint64_t>(B::kLdsMax)) {
      sort_segment<K, PAIRS, NT>(c, b, e, it.buf, sh);
    } else if (it.budget == 0) {
      // out of budget: filed for the fallback sort (Section 4.1), which
      // runs after this launch with a whole workgroup per segment
      if (tid == 0) {
        const uint32_t slot = atomicAdd(&c.icnt[kItemHeap], 1u);
        if (slot < c.max_items) c.heap[slot] = Item{b, e, it.buf, 0u};
        else atomicOr(&c.ctr->errors, kErrCapacity);
        atomicAdd(reinterpret_cast<unsigned long long*>(&c.ctr->heap_segments), 1ull);
        atomicAdd(reinterpret_cast<unsigned long long*>(&c.ctr->heap_elements), static_cast<unsigned long long>(size));
      }
    } else {
      if (tid == 0) {
        // the candidates (written by the partition that made this segment)
        // and the predecessor (an ancestor's pivot, published with a coherent
        // store) may come from another XCD in this launch: coherent loads
        const T* user = static_cast<const T*>(c.keys[0]);
        const PivotChoice<K> pc = choose_pivot<K, true>(static_cast<const T*>(c.keys[it.buf]), user, b, e,
                                                        it.flags, c.seed, c.fresh_fixed != 0);
        s_pivot = pc.raw;
        s_pidx = pc.pidx;
        s_mode = pc.mode;
      }
      __syncthreads();
      const T pivot = s_pivot;
      const uint64_t pidx = s_pidx;
      const uint32_t mode = s_mode;
      uint64_t L = 0;
      bool desc = false, asc = false;
      partition_wg<K, PAIRS, NT, IT>(c, b, e, it.buf, pivot, pidx, mode, sh, L, desc, asc);
      const uint32_t dst = it.buf ^ 1u;
      if (!desc || !asc) {
        // already ordered (Section 5.2): copy out, reversed when descending
        copy_out<K, PAIRS, NT>(c, b, e, it.buf, desc);
        if (tid == 0) {
          atomicAdd(reinterpret_cast<unsigned long long*>(&c.ctr->sorted_segments), 1ull);
          atomicAdd(reinterpret_cast<unsigned long long*>(&c.ctr->sorted_elements), static_cast<unsigned long long>(size));
        }
      } else if (L >= size) {
        if (tid == 0) atomicOr(&bq.q->error, kErrSplit);
      } else {
        const bool is_left = mode == kModeLeft;
        const uint64_t R = size - 1 - L;
        const bool bad = !is_left && (L < (size >> 3) || R < (size >> 3));
        if (tid == 0) {
          T* user = static_cast<T*>(c.keys[0]);
          cstore(user + b + L, pivot);
          if constexpr (PAIRS) cstore(c.vals[0] + b + L, cload(c.vals[it.buf] + pidx));
          atomicAdd(reinterpret_cast<unsigned long long*>(is_left ? &c.ctr->partitions_left : &c.ctr->partitions_right), 1ull);
          if (bad) atomicAdd(reinterpret_cast<unsigned long long*>(&c.ctr->bad_partitions), 1ull);
          if (is_left) atomicAdd(reinterpret_cast<unsigned long long*>(&c.ctr->equal_elements), static_cast<unsigned long long>(L));
        }
        __syncthreads();
        const uint32_t cbudget = it.budget - (bad ? 1u : 0u);
        const uint32_t cfresh = bad ? kSegFresh : 0u;
        for (int side = 0; side < 2; ++side) {
          if (side == 0 && is_left) {
            copy_out<K, PAIRS, NT>(c, b, b + L, dst, false);  // keys equal to the pivot are final
            continue;
          }
          const uint64_t cb = side == 0 ? b : b + L + 1;
          const uint64_t ce = side == 0 ? b + L : e;
          const uint64_t cs = ce - cb;
          if (cs == 0) continue;
          if (cs == 1) {
            if (tid == 0) {
              static_cast<T*>(c.keys[0])[cb] = cload(static_cast<const T*>(c.keys[dst]) + cb);
              if constexpr (PAIRS) c.vals[0][cb] = cload(c.vals[dst] + cb);
            }
            continue;
          }
          if (cs <= static_cast<uint64_t>(B::kLdsMax)) {  // the network needs no budget
            sort_segment<K, PAIRS, NT>(c, cb, ce, dst, sh);
          } else if (tid == 0) {
            BItem ch;
            ch.begin = cb;
            ch.end = ce;
            ch.buf = dst;
            ch.budget = cbudget;
            ch.flags = cfresh | (side == 0 ? (it.flags & kSegLeftmost) : 0u);
            ch.pad = 0;
            queue_push(bq, ch);
          }
        }
      }
    }
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_sub(&bq.q->pending, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <class K, bool PAIRS>
hipError_t run_shape(const Ctx& c, const BatchArgs& b, int shape, uint32_t grid, hipStream_t s) {
  switch (shape) {
    case 0: hipLaunchKernelGGL((k_batch<K, PAIRS, 512, 8>), dim3(grid), dim3(512), 0, s, c, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class K, bool PAIRS>
const void* kernel_of(int shape) {
  switch (shape) {
    case 0: return reinterpret_cast<const void*>(&k_batch<K, PAIRS, 512, 8>);
    default: return nullptr;
  }
}

template <class K>
hipError_t run_kp(const Ctx& c, const BatchArgs& b, int shape, uint32_t grid, hipStream_t s) {
  return c.has_vals ? run_shape<K, true>(c, b, shape, grid, s) : run_shape<K, false>(c, b, shape, grid, s);
}

const void* kernel_for(const Ctx& c, int shape) {
  const bool v = c.has_vals != 0;
  switch (c.key_type) {
    case 1: return v ? kernel_of<KeyU32, true>(shape) : kernel_of<KeyU32, false>(shape);
    case 2: return v ? kernel_of<KeyI32, true>(shape) : kernel_of<KeyI32, false>(shape);
    case 3: return v ? kernel_of<KeyF32, true>(shape) : kernel_of<KeyF32, false>(shape);
    case 4: return v ? kernel_of<KeyU64, true>(shape) : kernel_of<KeyU64, false>(shape);
    case 5: return v ? kernel_of<KeyI64, true>(shape) : kernel_of<KeyI64, false>(shape);
    case 6: return v ? kernel_of<KeyF64, true>(shape) : kernel_of<KeyF64, false>(shape);
    default: return nullptr;
  }
}

}  // namespace

hipError_t launch_batch_zero(const BatchArgs& b, uint32_t cap, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_zero, dim3((cap + 255) / 256), dim3(256), 0, s, b, cap);
  return hipGetLastError();
}

hipError_t launch_batch_fold(const Ctx& c, const BatchArgs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_fold, dim3(1), dim3(64), 0, s, c, b);
  return hipGetLastError();
}

hipError_t launch_batch_from_list(const Ctx& c, const BatchArgs& b, int parity, uint32_t src, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_from_list, dim3(64), dim3(256), 0, s, c, b, parity, src);
  return hipGetLastError();
}

uint32_t batch_grid(const Ctx& c, int tail) {
  const void* f = kernel_for(c, tail);
  int per_cu = 0, dev = 0, cus = 0;
  if (!f || hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, static_cast<int>(kTail[tail].nt), 0) != hipSuccess)
    return 0;
  return static_cast<uint32_t>(per_cu > 0 ? per_cu : 1) * static_cast<uint32_t>(cus);
}

hipError_t launch_batch(const Ctx& c, const BatchArgs& b, int shape, uint32_t grid, hipStream_t s) {
  switch (c.key_type) {
    case 1: return run_kp<KeyU32>(c, b, shape, grid, s);
    case 2: return run_kp<KeyI32>(c, b, shape, grid, s);
    case 3: return run_kp<KeyF32>(c, b, shape, grid, s);
    case 4: return run_kp<KeyU64>(c, b, shape, grid, s);
    case 5: return run_kp<KeyI64>(c, b, shape, grid, s);
    case 6: return run_kp<KeyF64>(c, b, shape, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdq
