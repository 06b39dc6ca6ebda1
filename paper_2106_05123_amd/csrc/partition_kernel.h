// The partition pass: one persistent kernel that partitions every live
// segment of a pass around its pivot, out of place. This header holds the
// kernel and its launchers; k_partition.hip instantiates the reservation
// form, k_partition_lb.hip the look-back form.
//
// The method is the paper's partition step (Section 3, partition_right /
// partition_left) with the branchless block classification of Section 5.3,
// recast for a wave64 GPU:
//   * a tile of TILE keys per workgroup, read with coalesced loads (lane l of
//     row i reads position i*NT + l of a sub-tile), kept in registers from
//     the count to the scatter for tiles up to 32768 keys;
//   * classification with one comparison per key (x < p for partition_right,
//     x <= p for partition_left), the pivot element itself excluded;
//   * per-row wave ballots + mbcnt give each key its rank among the keys of
//     its class, an LDS scan over (row, wave) counts gives tile offsets;
//   * the tile reserves its places with one 64-bit atomic on the segment's
//     packed cursor (in an array of its own that only atomics touch): left
//     keys upward from the segment start, the others downward from its end.
//     The order of the tiles' blocks inside each side is the order their
//     reservations arrived in; the partition does not need any particular
//     order inside a side (the paper's partition is not stable either), and
//     no tile ever waits for another. The deterministic
//     form (LB) instead publishes each tile's count and runs a decoupled
//     look-back over the segment's earlier tiles, so the blocks follow tile
//     order in every run;
//   * keys are written straight from registers: within a (row, wave) the
//     ranks of one class are consecutive, so every store instruction writes
//     at most two contiguous runs (the right side of a tile is written in
//     descending order of its ranks, which no later step depends on);
//   * payloads are loaded before the reservation, so they travel while the
//     tile's counts are scanned;
//   * the tile also records whether its adjacent pairs ever descend or
//     ascend (including the pair across its end) and ORs these bits into
//     the segment, which thus learns whether it was already ordered
//     (Section 5.2); in the reservation form a workgroup sends each bit
//     once per segment;
//   * tiles come from ticket counters (one per XCD in the reservation form,
//     a single one in the look-back form); the reservation form maps
//     tickets through a permutation of the pass's tiles that puts tiles
//     running at the same time into different segments (atomics on one
//     cache line run one after another), the look-back form takes them in
//     order.
#pragma once

#include "pdq_internal.h"
#include "wave_ops.h"

namespace pdq {
namespace {

template <class T>
struct TileDesc {
  uint64_t b, e, pidx, chunk;
  T piv;
  uint32_t si, tis, nts;
  bool left_mode;
};

// The segment records and the tile map do not change while a pass runs, so
// they are read through the constant address space: scalar loads, whose
// wait does not also wait for the vector stores of the previous tile.
template <class X>
using ConstPtr = const __attribute__((address_space(4))) X*;

template <class T, int TILE>
__device__ __forceinline__ TileDesc<T> tile_desc(const Seg* segs, const uint32_t* tilemap, uint32_t t) {
  TileDesc<T> d;
  const ConstPtr<uint32_t> tm = reinterpret_cast<ConstPtr<uint32_t>>(reinterpret_cast<uintptr_t>(tilemap));
  d.si = __builtin_amdgcn_readfirstlane(tm[t]);
  const ConstPtr<Seg> sg = reinterpret_cast<ConstPtr<Seg>>(reinterpret_cast<uintptr_t>(segs)) + d.si;
  d.b = sg->begin;
  d.e = sg->end;
  d.pidx = sg->pidx;
  d.piv = static_cast<T>(sg->pivot);
  d.left_mode = sg->mode == kModeLeft;
  d.tis = t - sg->tile_base;
  d.nts = sg->ntiles;
  d.chunk = d.b + static_cast<uint64_t>(d.tis) * TILE;  // tiles start at the segment's first key
  return d;
}

// Stride of a bijection of [0, n): tile number x is taken as tile
// (x * stride) mod n. The stride lies near 0.618 n and is coprime to n, so
// tiles that run at the same time lie far apart in the pass's tile order,
// i.e. in different segments when a pass has many.
__device__ __forceinline__ uint32_t spread_stride(uint32_t n) {
  if (n <= 2) return 1u;
  uint32_t s = static_cast<uint32_t>((static_cast<uint64_t>(n) * 0x9E3779B9ull) >> 32) | 1u;
  for (; s < n; s += 2) {
    uint32_t a = n, b = s;
    while (b) {
      const uint32_t r = a % b;
      a = b;
      b = r;
    }
    if (a == 1) return s;
  }
  return 1u;
}

// Buffer descriptor over a whole array (no range limit; gfx9 layout).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, 0xFFFFFFFF, 0x00020000);
}

template <class T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    return static_cast<T>(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    typedef int v2i __attribute__((ext_vector_type(2)));
    v2i x = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return static_cast<T>(static_cast<uint32_t>(x.x)) | (static_cast<T>(static_cast<uint32_t>(x.y)) << 32);
  }
}

// Loads one sub-tile: row i, lane tid holds slot i*NT + tid of the SUB
// slots starting at absolute index base. A sub-tile wholly inside the array
// is read unconditionally through a buffer descriptor (the row offset rides
// in the scalar offset, so every row shares one vector offset); slots
// outside the segment are ignored later. Only a sub-tile running past the
// end of the array is read with per-slot predicates.
template <class T, int NT, int IT>
__device__ __forceinline__ void load_sub(uint64_t base, uint64_t n, const T* __restrict__ src, int tid, T (&k)[IT]) {
  constexpr int SUB = NT * IT;
  if (base + SUB <= n) {
    const __amdgpu_buffer_rsrc_t rk = make_rsrc(src + base);
    const uint32_t vo = static_cast<uint32_t>(tid) * sizeof(T);
#pragma unroll
    for (int i = 0; i < IT; ++i) k[i] = buf_load<T>(rk, vo, static_cast<uint32_t>(i * NT * sizeof(T)));
  } else {
    const uint32_t lim = static_cast<uint32_t>(n - base);
    const T* __restrict__ ts = src + base;
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const uint32_t off = static_cast<uint32_t>(i * NT + tid);
      k[i] = off < lim ? ts[off] : T(0);
    }
  }
}

// Geometry of one tile (NSUB sub-tiles of SUB slots) inside its chunk:
// slots [lo, hi) belong to the segment, pl is the pivot's slot (or none),
// the successor of slot s is in the segment iff s + 1 < erel.
struct TileGeom {
  uint32_t lo, hi, pl, erel;
};

template <class T, int TILE>
__device__ __forceinline__ TileGeom tile_geom(const TileDesc<T>& d) {
  TileGeom g;
  const uint64_t tlo = d.chunk > d.b ? d.chunk : d.b;
  const uint64_t thi = d.chunk + TILE < d.e ? d.chunk + TILE : d.e;
  g.lo = static_cast<uint32_t>(tlo - d.chunk);
  g.hi = static_cast<uint32_t>(thi - d.chunk);
  g.pl = (d.pidx >= d.chunk && d.pidx < d.chunk + TILE) ? static_cast<uint32_t>(d.pidx - d.chunk) : 0xFFFFFFFFu;
  const uint64_t erel64 = d.e - d.chunk;
  g.erel = erel64 < static_cast<uint64_t>(TILE + 1) ? static_cast<uint32_t>(erel64) : TILE + 1;
  return g;
}

// Classification of one sub-tile (first slot s0 of the tile): bit i of
// lmask = key of row i goes left (x < p for partition_right, x <= p for
// partition_left), bit i of vmask = key of row i is a real, non-pivot key of
// the segment. FULL: every slot is such a key and every in-group successor
// lies inside the segment. Also reports whether adjacent pairs inside a
// (row, wave) group descend / ascend.
template <class K, int NT, int IT, bool FULL, bool PAIRCHECK>
__device__ __forceinline__ void classify(const typename K::T (&k)[IT], const TileGeom& g, uint32_t s0,
                                         bool left_mode, decltype(K::ord(typename K::T(0))) pv, int tid,
                                         uint32_t& lmask, uint32_t& vmask, bool& has_d, bool& has_a) {
  const int lane = tid & 63;
  lmask = 0;
  vmask = FULL ? ((IT == 32) ? 0xFFFFFFFFu : ((1u << IT) - 1u)) : 0u;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const auto ko = K::ord(k[i]);
    bool l;
    const uint32_t off = s0 + static_cast<uint32_t>(i * NT + tid);
    if constexpr (FULL) {
      l = left_mode ? (ko <= pv) : (ko < pv);
    } else {
      const bool v = off >= g.lo && off < g.hi && off != g.pl;
      l = v && (left_mode ? (ko <= pv) : (ko < pv));
      vmask |= (v ? 1u : 0u) << i;
    }
    lmask |= (l ? 1u : 0u) << i;
    if constexpr (PAIRCHECK) {
      const typename K::T nx = __shfl_down(k[i], 1, 64);  // successor inside the group (lanes 0..62)
      const auto z = K::ord(nx);
      bool pair_ok = lane < 63;
      if constexpr (!FULL) pair_ok = pair_ok && off >= g.lo && off < g.hi && off + 1 < g.erel;
      has_d |= pair_ok && (z < ko);
      has_a |= pair_ok && (z > ko);
    }
  }
}

// The partition kernel. A workgroup takes one tile of NSUB sub-tiles (SUB =
// NT*IT keys each) and makes two passes over it:
//   count:   load each sub-tile, classify, record per (row, wave) group its
//            left count and first / last key; no barrier inside the pass;
//   reserve: one barrier, then wave 0 scans the group counts and reserves the
//            tile's places in the segment with one atomic;
//   scatter: write every key straight from registers to its final place; no
//            barrier inside the pass.
// REG (register-resident tile): every lane keeps its NSUB*IT keys in
// registers from the count pass to the scatter and loads its payloads
// before the reservation, so each key and payload crosses HBM exactly once
// each way. Otherwise (tiles larger than the registers hold) the scatter
// pass loads each sub-tile again and classifies it again.
// WPE: waves per SIMD the register allocation must leave room for. 32-bit
// register-resident tiles fit 4 (128 VGPRs) without spilling, which doubles
// the workgroups a CU holds at once; 64-bit keys would spill, so they keep
// the compiler's choice.
template <class K, bool PAIRS, int NT, int IT, int NSUB, bool REG, bool LB,
          int WPE = (REG && sizeof(typename K::T) == 4) ? 4 : 1>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_partition(Ctx c, int parity, uint32_t src_buf) {
  using T = typename K::T;
  constexpr int NW = NT / 64;
  constexpr int SUB = NT * IT;
  constexpr int TILE = SUB * NSUB;
  constexpr int NG = NSUB * IT * NW;  // (sub-tile, row, wave) groups; group q covers slots [64q, 64q + 64)
  constexpr int GPL = (NG + 63) / 64;  // groups per lane of wave 0
  constexpr int RS = REG ? NSUB : 1;   // sub-tiles held in registers
  static_assert(IT <= 32, "row masks are 32-bit");

  __shared__ uint32_t s_cnt[NG];  // per group left counts, then exclusive prefixes over the tile
  __shared__ T s_first[NG];       // first / last key of each group: pairs across groups
  __shared__ T s_last[NG];
  __shared__ uint32_t s_next;     // the workgroup's next ticket
  __shared__ uint32_t s_bits;
  __shared__ uint64_t s_lpre;
  __shared__ uint32_t s_nl;
  __shared__ T s_tail;            // first key after the tile (when the segment continues)

  const T* __restrict__ src = static_cast<const T*>(c.keys[src_buf]);
  T* __restrict__ dst = static_cast<T*>(c.keys[src_buf ^ 1]);
  const uint32_t* __restrict__ srcv = c.vals[src_buf];
  uint32_t* __restrict__ dstv = c.vals[src_buf ^ 1];
  Seg* segs = c.segs[parity];
  uint32_t ntiles = static_cast<uint32_t>(c.ctr->list[parity]);
  if (ntiles > c.max_tiles) ntiles = c.max_tiles;  // an overfull list is flagged, never read past
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;

  // Tickets come from counters in the order workgroups ask (tiles carry
  // uneven work when segments are small, so a fixed share per workgroup
  // would leave the pass waiting for the unluckiest one). The look-back
  // form takes every tile from one counter, in order, and asks for its next
  // ticket only when it is about to finish the current tile: a ticket held
  // long before its tile starts would make every later tile of the segment
  // wait for it. The reservation form takes tickets [q_lo, q_hi) from its
  // XCD's queue and asks for the next one as soon as a tile's keys load.
  const uint32_t nq = LB ? 1u : (gridDim.x < kTicketQueues ? gridDim.x : kTicketQueues);
  const uint32_t q = blockIdx.x % nq;
  const uint32_t q_lo = static_cast<uint32_t>(static_cast<uint64_t>(ntiles) * q / nq);
  const uint32_t q_hi = static_cast<uint32_t>(static_cast<uint64_t>(ntiles) * (q + 1) / nq);
  uint32_t* const qctr = LB ? &c.ctr->ticket : c.tickets + q * kTicketStride;
  if (tid == 0) {
    s_next = q_lo + atomicAdd(qctr, 1u);
    s_bits = 0;
  }
  lds_barrier();
  uint32_t t = __builtin_amdgcn_readfirstlane(s_next);
  if (t >= q_hi) return;
  // reservation form: ticket x is tile (x * stride) mod ntiles, which
  // spreads the tiles of one segment over the pass, so the atomics on one
  // cursor do not all come at once; the look-back form takes tiles in order
  const uint32_t stride = LB ? 1u : spread_stride(ntiles);
  auto tile_of = [&](uint32_t x) -> uint32_t {
    return LB ? x : static_cast<uint32_t>((static_cast<uint64_t>(x) * stride) % ntiles);
  };
  TileDesc<T> d = tile_desc<T, TILE>(segs, c.tilemap, tile_of(t));
  lds_barrier();  // every wave has read s_next
  // reservation form: the segment whose order bits this workgroup last
  // ORed, and the bits it ORed there (wave 0, lane 0)
  uint32_t or_seg = ~0u, or_bits = 0;
  // the next ticket (thread 0): the reservation form asks for it as soon as
  // the tile's keys are on their way, so the answer is back by the tile's
  // end; the look-back form only at the scatter
  uint32_t nticket = 0;
  auto early_ticket = [&]() {
    if constexpr (!LB)
      if (tid == 0) nticket = q_lo + atomicAdd(qctr, 1u);
  };

  for (;;) {
    const TileGeom g = tile_geom<T, TILE>(d);
    const auto pv = K::ord(d.piv);
    // the first key after the tile (last thread), read with the tile's keys
    // and handed over in LDS before the first barrier
    T tail_key = T(0);
    auto load_tail = [&]() {
      if (tid == NT - 1 && g.erel > static_cast<uint32_t>(TILE)) tail_key = src[d.chunk + TILE];
    };

    // sub-tiles that hold keys of the segment: [j0, j1)
    const int j0 = static_cast<int>(g.lo / SUB);
    const int j1 = static_cast<int>((g.hi + SUB - 1) / SUB);

    T kr[RS][IT];                           // REG: the tile's keys
    uint32_t vr[(REG && PAIRS) ? RS : 1][IT];  // REG: its payloads
    uint32_t lmr[RS], vmr[RS];              // REG: class and validity masks per sub-tile

    // ---- count pass
    {
      for (int j = 0; j < NSUB; ++j)
        if ((j < j0 || j >= j1) && lane < IT) s_cnt[(j * IT + lane) * NW + wv] = 0;
      bool has_d = false, has_a = false;
      // one sub-tile: classify, then per (row, wave) group its left count and edge keys
      auto count_sub = [&](int j, const T (&k)[IT], uint32_t& lmask, uint32_t& vmask) {
        const uint32_t s0 = static_cast<uint32_t>(j * SUB);
        uint32_t* gc = s_cnt + j * IT * NW;
        T* gf = s_first + j * IT * NW;
        T* gl = s_last + j * IT * NW;
        const bool full = s0 >= g.lo && s0 + SUB <= g.hi && s0 + SUB < g.erel && !(g.pl >= s0 && g.pl < s0 + SUB);
        if (full)
          classify<K, NT, IT, true, true>(k, g, s0, d.left_mode, pv, tid, lmask, vmask, has_d, has_a);
        else
          classify<K, NT, IT, false, true>(k, g, s0, d.left_mode, pv, tid, lmask, vmask, has_d, has_a);
#pragma unroll
        for (int i = 0; i < IT; ++i) {
          const uint64_t m = __ballot((lmask >> i) & 1u);
          if (lane == 0) {
            gc[i * NW + wv] = static_cast<uint32_t>(__popcll(m));
            gf[i * NW + wv] = k[i];
          }
          if (lane == 63) gl[i * NW + wv] = k[i];
        }
      };
      if constexpr (REG) {
        // every sub-tile's loads are issued at once
#pragma unroll
        for (int j = 0; j < NSUB; ++j)
          if (j >= j0 && j < j1) load_sub<T, NT, IT>(d.chunk + static_cast<uint32_t>(j * SUB), c.n, src, tid, kr[j]);
        load_tail();
        early_ticket();
#pragma unroll
        for (int j = 0; j < NSUB; ++j)
          if (j >= j0 && j < j1) count_sub(j, kr[j], lmr[j], vmr[j]);
        if constexpr (PAIRS) {
          // payloads travel while the counts are scanned
#pragma unroll
          for (int j = 0; j < NSUB; ++j)
            if (j >= j0 && j < j1)
              load_sub<uint32_t, NT, IT>(d.chunk + static_cast<uint32_t>(j * SUB), c.n, srcv, tid, vr[j]);
        }
      } else {
        // the next sub-tile is loaded while this one is classified
        T k[IT], kn[IT];
        load_sub<T, NT, IT>(d.chunk + static_cast<uint32_t>(j0 * SUB), c.n, src, tid, k);
        load_tail();
        early_ticket();
#pragma unroll 1
        for (int j = j0; j < j1; ++j) {
          if (j + 1 < j1) load_sub<T, NT, IT>(d.chunk + static_cast<uint32_t>((j + 1) * SUB), c.n, src, tid, kn);
          uint32_t lmask, vmask;
          count_sub(j, k, lmask, vmask);
#pragma unroll
          for (int i = 0; i < IT; ++i) k[i] = kn[i];
        }
      }
      const bool wd = __any(has_d), wa = __any(has_a);
      if (lane == 0 && (wd || wa))
        atomicOr(&s_bits, (wd ? static_cast<uint32_t>(kStDesc >> 32) : 0u) |
                              (wa ? static_cast<uint32_t>(kStAsc >> 32) : 0u));
    }
    if (tid == NT - 1) s_tail = tail_key;
    lds_barrier();  // B1: group counts, group edge keys, in-group pair bits, tail key

    // ---- wave 0: edge pairs, scan, reservation ----------------------------------
    if (wv == 0) {
      uint32_t loc[GPL];
      uint32_t sum = 0;
      bool ed = false, ea = false;
      const T tn = s_tail;
#pragma unroll
      for (int kk = 0; kk < GPL; ++kk) {
        const int q = lane * GPL + kk;
        loc[kk] = q < NG ? s_cnt[q] : 0u;
        sum += loc[kk];
        const uint32_t slot = static_cast<uint32_t>(q) * 64u + 63u;  // last slot of group q
        if (q < NG && slot >= g.lo && slot < g.hi && slot + 1 < g.erel) {
          const auto a = K::ord(s_last[q]);
          const auto z = K::ord(q + 1 < NG ? s_first[q + 1] : tn);
          ed |= z < a;
          ea |= z > a;
        }
      }
      const uint64_t incl = wave_incl_scan_u64(sum);
      const uint32_t nl = static_cast<uint32_t>(__shfl(incl, 63, 64));
      const bool wd = __any(ed), wa = __any(ea);
      const uint32_t own_bits = s_bits | (wd ? static_cast<uint32_t>(kStDesc >> 32) : 0u) |
                                (wa ? static_cast<uint32_t>(kStAsc >> 32) : 0u);
      uint32_t run = static_cast<uint32_t>(incl) - sum;
#pragma unroll
      for (int kk = 0; kk < GPL; ++kk) {
        if (lane * GPL + kk < NG) s_cnt[lane * GPL + kk] = run;
        run += loc[kk];
      }
      if constexpr (LB) {
        // deterministic order: publish the tile's aggregate, then a decoupled
        // look-back over the segment's earlier tiles (64 a window) gives the
        // left keys of every tile before this one
        const uint64_t own64 = static_cast<uint64_t>(own_bits) << 32;
        if (lane == 0) store_status(&c.status[t], (d.tis == 0 ? kStIncl : kStAgg) | nl | own64);
        uint64_t ex = 0, exb = 0;
        if (d.tis != 0) {
          uint32_t look = t - 1;
          uint32_t rem = d.tis;  // tiles of this segment before this one
          for (;;) {
            uint64_t w = kStIncl;  // lanes past the segment's first tile read as an empty prefix
            if (static_cast<uint32_t>(lane) < rem) w = load_status(&c.status[look - lane]);
            const uint64_t st = w & kStStateMask;
            const uint64_t im = __ballot(st == kStIncl);
            const uint64_t nm = __ballot(st == 0);
            const int fi = im ? static_cast<int>(__builtin_ctzll(im)) : 64;
            const uint64_t upto = fi >= 63 ? ~0ull : ((2ull << fi) - 1);
            if (nm & upto) {
              __builtin_amdgcn_s_sleep(1);
              continue;
            }
            const bool take = lane <= fi;
            const uint64_t cnt = take ? (w & kStCountMask) : 0ull;
            const uint64_t bb = take ? (w & (kStDesc | kStAsc)) : 0ull;
            if (fi < 64) {
              // suffix sums over lanes k..fi are the inclusive prefixes of the
              // tiles between the one found and this one: publish them too
              uint64_t sc = cnt, sb = bb;
              for (int dd = 1; dd < 64; dd <<= 1) {
                const uint64_t tc = __shfl_down(sc, dd, 64);
                const uint64_t tb = __shfl_down(sb, dd, 64);
                if (lane + dd < 64) {
                  sc += tc;
                  sb |= tb;
                }
              }
              if (lane < fi) store_status(&c.status[look - lane], kStIncl | sc | sb);
              ex += __shfl(sc, 0, 64);
              exb |= __shfl(sb, 0, 64);
              break;
            }
            ex += wave_sum_u64(cnt);
            exb |= wave_or_u64(bb);
            look -= 64;
            rem -= 64;
          }
          if (lane == 0) store_status(&c.status[t], kStIncl | (ex + nl) | exb | own64);
        }
        if (lane == 0) {
          // the same packed form as a reservation: left keys before this tile,
          // right keys before it (every valid key before the tile is one or the
          // other); a count that does not fit is handed on as one the scatter
          // rejects
          const uint64_t tlo = d.chunk + g.lo;
          const uint64_t pre_valid = (tlo - d.b) - (d.pidx < tlo ? 1u : 0u);
          s_lpre = ex <= pre_valid ? (ex | ((pre_valid - ex) << 32)) : 0xFFFFFFFFull;
          s_nl = nl;
          s_bits = 0;  // ready for the next tile (all reads of it are done)
          if (d.tis == d.nts - 1) {
            c.cur[d.si].left = ex + nl;
            c.cur[d.si].order_bits = static_cast<uint32_t>((exb | own64) >> 32);
          }
        }
      } else {
        if (lane == 0) {
          // reserve this tile's places: left keys from the segment start, the
          // others from its end, in one atomic on the segment's packed cursor
          const bool piv_in = g.pl >= g.lo && g.pl < g.hi;
          const uint32_t nvalid = (g.hi - g.lo) - (piv_in ? 1u : 0u);
          const uint64_t add = static_cast<uint64_t>(nl) | (static_cast<uint64_t>(nvalid - nl) << 32);
          const uint64_t old = atomicAdd(reinterpret_cast<unsigned long long*>(&c.cur[d.si].left), add);
          // a bit this workgroup already set in this segment is not sent again
          if (or_seg != d.si) {
            or_seg = d.si;
            or_bits = 0;
          }
          const uint32_t fresh = own_bits & ~or_bits;
          if (fresh) atomicOr(&c.cur[d.si].order_bits, fresh);
          or_bits |= own_bits;
          s_lpre = old;
          s_nl = nl;
          s_bits = 0;  // ready for the next tile (all reads of it are done)
        }
      }
    }
    lds_barrier();  // B2: group prefixes, the tile's places

    if constexpr (LB)
      if (tid == 0) nticket = q_lo + atomicAdd(qctr, 1u);  // returns while the tile is written out

    // ---- scatter pass: write from registers ---------------------------------
    {
      const uint32_t nl = __builtin_amdgcn_readfirstlane(s_nl);
      const uint64_t lpre = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(s_lpre));        // left keys placed before
      const uint64_t gpre = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(s_lpre >> 32));  // right keys placed before
      const bool piv_in = g.pl >= g.lo && g.pl < g.hi;
      const uint32_t nvalid = (g.hi - g.lo) - (piv_in ? 1u : 0u);
      // the reservations of all tiles add up to the segment's size minus the
      // pivot, so every write below stays inside [b, e); a tile whose
      // reservation does not fit (a broken counter) writes nothing and
      // flags the call
      const bool sane = nl <= nvalid && lpre + gpre + nvalid <= (d.e - d.b) - 1u;
      if (!sane && tid == 0) atomicOr(&c.ctr->errors, kErrLookback);
      if (sane) {
        const uint32_t nr = nvalid - nl;
        // left keys of this tile occupy [b + lpre, b + lpre + nl); right keys
        // occupy [e - gpre - nr, e - gpre) in descending order of their rank
        T* __restrict__ dl = dst + (d.b + lpre);
        T* __restrict__ drl = dst + (d.e - gpre - nr);
        uint32_t* __restrict__ dlv = PAIRS ? dstv + (d.b + lpre) : nullptr;
        uint32_t* __restrict__ drlv = PAIRS ? dstv + (d.e - gpre - nr) : nullptr;
        // one sub-tile's writes, given its keys, payloads and masks
        auto scatter_sub = [&](int j, const T (&k)[IT], const uint32_t* v, uint32_t lmask, uint32_t vmask) {
          const uint32_t s0 = static_cast<uint32_t>(j * SUB);
          const bool full = s0 >= g.lo && s0 + SUB <= g.hi && !(g.pl >= s0 && g.pl < s0 + SUB);
          // real keys of the tile before slot s0 + x are x + adj for x in a
          // full sub-tile: adj = s0 - lo - (pivot before s0)
          const uint32_t adj = s0 - g.lo - ((piv_in && g.pl < s0) ? 1u : 0u);
          const uint32_t* gc = s_cnt + j * IT * NW;
#pragma unroll
          for (int i = 0; i < IT; ++i) {
            const bool l = (lmask >> i) & 1u;
            const uint64_t m = __ballot(l);
            const uint32_t rx = gc[i * NW + wv] + lanes_below(m);  // left keys before this one in the tile
            if (full || ((vmask >> i) & 1u)) {
              if (l) {
                dl[rx] = k[i];
                if constexpr (PAIRS) dlv[rx] = v[i];
              } else {
                const uint32_t x = static_cast<uint32_t>(i * NT + tid);
                uint32_t before = x + adj;  // real keys of the tile before this one
                if (!full) before = (s0 + x - g.lo) - ((piv_in && g.pl < s0 + x) ? 1u : 0u);
                const uint32_t q = nr - 1u - (before - rx);
                drl[q] = k[i];
                if constexpr (PAIRS) drlv[q] = v[i];
              }
            }
          }
        };
        if constexpr (REG) {
#pragma unroll
          for (int j = 0; j < NSUB; ++j)
            if (j >= j0 && j < j1) scatter_sub(j, kr[j], (REG && PAIRS) ? vr[j] : nullptr, lmr[j], vmr[j]);
        } else {
          T k[IT], kn[IT];
          uint32_t v[PAIRS ? IT : 1], vn[PAIRS ? IT : 1];
          load_sub<T, NT, IT>(d.chunk + static_cast<uint32_t>(j0 * SUB), c.n, src, tid, k);
          if constexpr (PAIRS) load_sub<uint32_t, NT, IT>(d.chunk + static_cast<uint32_t>(j0 * SUB), c.n, srcv, tid, v);
#pragma unroll 1
          for (int j = j0; j < j1; ++j) {
            const uint32_t s0 = static_cast<uint32_t>(j * SUB);
            if (j + 1 < j1) {
              load_sub<T, NT, IT>(d.chunk + s0 + SUB, c.n, src, tid, kn);
              if constexpr (PAIRS) load_sub<uint32_t, NT, IT>(d.chunk + s0 + SUB, c.n, srcv, tid, vn);
            }
            uint32_t lmask, vmask;
            bool dd_ = false, da_ = false;
            const bool fullc = s0 >= g.lo && s0 + SUB <= g.hi && !(g.pl >= s0 && g.pl < s0 + SUB);
            if (fullc)
              classify<K, NT, IT, true, false>(k, g, s0, d.left_mode, pv, tid, lmask, vmask, dd_, da_);
            else
              classify<K, NT, IT, false, false>(k, g, s0, d.left_mode, pv, tid, lmask, vmask, dd_, da_);
            scatter_sub(j, k, PAIRS ? v : nullptr, lmask, vmask);
#pragma unroll
            for (int i = 0; i < IT; ++i) {
              k[i] = kn[i];
              if constexpr (PAIRS) v[i] = vn[i];
            }
          }
        }
      }
    }
    if (tid == 0) s_next = nticket;
    lds_barrier();  // B3: next ticket; LDS is rewritten by the next tile
    t = __builtin_amdgcn_readfirstlane(s_next);
    if (t >= q_hi) break;
    d = tile_desc<T, TILE>(segs, c.tilemap, tile_of(t));
  }
}

int device_cus() {
  static thread_local int dev_cached = -1;
  static thread_local int cus = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev != dev_cached) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cus = v;
    dev_cached = dev;
  }
  return cus;
}

template <class K, bool PAIRS, int NT, int IT, int NSUB, bool REG, bool LB>
hipError_t launch_lb(const Ctx& c, int parity, uint32_t ntiles, uint32_t src, hipStream_t s) {
  static int per_cu = 0;
  if (per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_partition<K, PAIRS, NT, IT, NSUB, REG, LB>, NT, 0) !=
            hipSuccess ||
        nb <= 0)
      nb = 1;
    per_cu = nb;
  }
  uint64_t grid = static_cast<uint64_t>(per_cu) * device_cus();
  if (grid > ntiles) grid = ntiles;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_partition<K, PAIRS, NT, IT, NSUB, REG, LB>), dim3(static_cast<uint32_t>(grid)), dim3(NT), 0, s,
                     c, parity, src);
  return hipGetLastError();
}



template <class K, bool PAIRS, bool LB>
hipError_t launch_tiles(const Ctx& c, int parity, uint32_t ntiles, uint32_t src, hipStream_t s) {
  switch (c.tile) {
    case 1024: return launch_lb<K, PAIRS, 256, 4, 1, true, LB>(c, parity, ntiles, src, s);
    case 2048: return launch_lb<K, PAIRS, 256, 8, 1, true, LB>(c, parity, ntiles, src, s);
    case 4096: return launch_lb<K, PAIRS, 256, 16, 1, true, LB>(c, parity, ntiles, src, s);
    case 8192: return launch_lb<K, PAIRS, 256, 8, 4, true, LB>(c, parity, ntiles, src, s);
    case 16384: return launch_lb<K, PAIRS, 512, 8, 4, true, LB>(c, parity, ntiles, src, s);
    case 32768: return launch_lb<K, PAIRS, 1024, 8, 4, true, LB>(c, parity, ntiles, src, s);
    case 65536: return launch_lb<K, PAIRS, 256, 16, 16, false, LB>(c, parity, ntiles, src, s);
    default: return hipErrorInvalidValue;
  }
}

template <class K, bool LB>
hipError_t launch_key(const Ctx& c, int parity, uint32_t ntiles, uint32_t src, hipStream_t s) {
  return c.has_vals ? launch_tiles<K, true, LB>(c, parity, ntiles, src, s)
                    : launch_tiles<K, false, LB>(c, parity, ntiles, src, s);
}

// One partition mode (LB: look-back, else reservation) for every key type.
template <bool LB>
hipError_t launch_mode(const Ctx& c, int parity, uint32_t ntiles, uint32_t src_buf, hipStream_t s) {
  switch (c.key_type) {
    case 1: return launch_key<KeyU32, LB>(c, parity, ntiles, src_buf, s);
    case 2: return launch_key<KeyI32, LB>(c, parity, ntiles, src_buf, s);
    case 3: return launch_key<KeyF32, LB>(c, parity, ntiles, src_buf, s);
    case 4: return launch_key<KeyU64, LB>(c, parity, ntiles, src_buf, s);
    case 5: return launch_key<KeyI64, LB>(c, parity, ntiles, src_buf, s);
    case 6: return launch_key<KeyF64, LB>(c, parity, ntiles, src_buf, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace pdq
