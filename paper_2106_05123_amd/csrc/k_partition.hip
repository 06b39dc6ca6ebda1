// The partition pass: one persistent kernel that partitions every live
// segment of a pass around its pivot, out of place.
//
// The method is the paper's partition step (Section 3, partition_right /
// partition_left) with the branchless block classification of Section 5.3,
// recast for a wave64 GPU:
//   * a tile of TILE keys per workgroup, read with coalesced loads (lane l of
//     row i reads position i*NT + l of the tile);
//   * classification with one comparison per key (x < p for partition_right,
//     x <= p for partition_left), the pivot element itself excluded;
//   * per-row wave ballots + mbcnt give each key its rank among the keys of
//     its class, an LDS scan over (row, wave) counts gives tile offsets;
//   * a decoupled look-back over the tiles of the segment (tile tickets come
//     from an atomic counter, so every tile waits only on tiles already
//     running) gives the number of left keys before the tile;
//   * keys are regrouped in LDS so that each class is one contiguous run,
//     then written out coalesced: left keys from the segment start upward,
//     right keys from the segment end downward (the right side is thus
//     reversed, which no later step depends on);
//   * the tile also records whether its adjacent pairs ever descend or
//     ascend; the look-back ORs these bits so that the segment's last tile
//     knows whether the whole segment was already ordered (Section 5.2).
#include "pdq_internal.h"
#include "wave_ops.h"

namespace pdq {
namespace {

template <class K, bool PAIRS, int NT, int IT>
__global__ __launch_bounds__(NT) void k_partition(Ctx c, int parity, uint32_t src_buf) {
  using T = typename K::T;
  constexpr int NW = NT / 64;
  constexpr int TILE = NT * IT;
  constexpr int NCNT = IT * NW;
  constexpr int CPL = (NCNT + 63) / 64;  // count entries per lane of the scanning wave

  __shared__ T s_key[TILE];
  __shared__ uint32_t s_val[PAIRS ? TILE : 1];
  __shared__ uint32_t s_cnt[NCNT];
  __shared__ T s_first[NCNT];
  __shared__ uint32_t s_ticket;
  __shared__ uint32_t s_bits;
  __shared__ uint64_t s_lpre;
  __shared__ uint32_t s_nl;

  const T* __restrict__ src = static_cast<const T*>(c.keys[src_buf]);
  T* __restrict__ dst = static_cast<T*>(c.keys[src_buf ^ 1]);
  const uint32_t* __restrict__ srcv = c.vals[src_buf];
  uint32_t* __restrict__ dstv = c.vals[src_buf ^ 1];
  Seg* segs = c.segs[parity];
  const uint32_t ntiles = static_cast<uint32_t>(c.ctr->list[parity]);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;

  for (;;) {
    if (tid == 0) {
      s_ticket = atomicAdd(&c.ctr->ticket, 1u);
      s_bits = 0;
    }
    __syncthreads();
    const uint32_t t = __builtin_amdgcn_readfirstlane(s_ticket);
    if (t >= ntiles) break;

    const uint32_t si = __builtin_amdgcn_readfirstlane(c.tilemap[t]);
    const uint64_t b = segs[si].begin;
    const uint64_t e = segs[si].end;
    const uint64_t pidx = segs[si].pidx;
    const T piv = static_cast<T>(segs[si].pivot);
    const bool left_mode = segs[si].mode == kModeLeft;
    const uint32_t tis = t - segs[si].tile_base;
    const uint32_t nts = segs[si].ntiles;
    const uint64_t chunk = (b / TILE + tis) * static_cast<uint64_t>(TILE);
    const uint64_t tlo = chunk > b ? chunk : b;
    const uint64_t thi = chunk + TILE < e ? chunk + TILE : e;
    const auto pv = K::ord(piv);
    // tile-relative coordinates: slots [lo, hi) of the chunk belong to the
    // segment; pl is the pivot's slot (or none); the successor of slot s
    // exists in the segment iff s + 1 < erel
    const T* __restrict__ tsrc = src + chunk;
    const uint32_t lo = static_cast<uint32_t>(tlo - chunk);
    const uint32_t hi = static_cast<uint32_t>(thi - chunk);
    const uint32_t pl = (pidx >= chunk && pidx < chunk + TILE) ? static_cast<uint32_t>(pidx - chunk) : 0xFFFFFFFFu;
    const uint32_t erel = static_cast<uint32_t>((e - chunk) < static_cast<uint64_t>(TILE + 1) ? (e - chunk) : TILE + 1);

    // ---- load (coalesced rows) and classify -------------------------------
    T key[IT];
    uint32_t val[PAIRS ? IT : 1];
    uint32_t below[IT];  // left keys of lower lanes in the same (row, wave)
    uint32_t lmask = 0;  // bit i: key of row i goes left
    uint32_t vmask = 0;  // bit i: key of row i is a real, non-pivot key
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const uint32_t off = static_cast<uint32_t>(i * NT + tid);
      const bool in = off >= lo && off < hi;
      key[i] = in ? tsrc[off] : T(0);
      if (PAIRS) val[i] = in ? srcv[chunk + off] : 0u;
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const uint32_t off = static_cast<uint32_t>(i * NT + tid);
      const bool v = off >= lo && off < hi && off != pl;
      const auto ko = K::ord(key[i]);
      const bool l = v && (left_mode ? (ko <= pv) : (ko < pv));
      const uint64_t m = __ballot(l);
      below[i] = lanes_below(m);
      if (lane == 0) {
        s_cnt[i * NW + wv] = static_cast<uint32_t>(__popcll(m));
        s_first[i * NW + wv] = key[i];
      }
      lmask |= (l ? 1u : 0u) << i;
      vmask |= (v ? 1u : 0u) << i;
    }
    __syncthreads();

    // ---- adjacent pairs: does the tile's part of the segment ever descend/ascend?
    {
      bool has_d = false, has_a = false;
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        T nx = __shfl_down(key[i], 1, 64);
        const uint32_t off = static_cast<uint32_t>(i * NT + tid);
        const bool pv_ok = off >= lo && off < hi && off + 1 < erel;
        if (lane == 63) {
          if (wv < NW - 1) nx = s_first[i * NW + wv + 1];
          else if (i < IT - 1) nx = s_first[(i + 1) * NW];
          else if (pv_ok) nx = tsrc[TILE];
        }
        const auto a = K::ord(key[i]);
        const auto z = K::ord(nx);
        has_d |= pv_ok && (z < a);
        has_a |= pv_ok && (z > a);
      }
      const bool wd = __any(has_d);
      const bool wa = __any(has_a);
      if (lane == 0 && (wd || wa)) atomicOr(&s_bits, (wd ? static_cast<uint32_t>(kStDesc >> 32) : 0u) |
                                                          (wa ? static_cast<uint32_t>(kStAsc >> 32) : 0u));
    }

    __syncthreads();  // s_bits complete

    // ---- tile scan over (row, wave) counts, then decoupled look-back --------
    if (wv == 0) {
      uint32_t loc[CPL];
      uint32_t sum = 0;
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        const int idx = lane * CPL + k;
        loc[k] = idx < NCNT ? s_cnt[idx] : 0u;
        sum += loc[k];
      }
      const uint64_t incl = wave_incl_scan_u64(sum);
      const uint32_t nl = static_cast<uint32_t>(__shfl(incl, 63, 64));
      uint32_t run = static_cast<uint32_t>(incl) - sum;
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        const int idx = lane * CPL + k;
        if (idx < NCNT) s_cnt[idx] = run;
        run += loc[k];
      }
      const uint64_t own_bits = static_cast<uint64_t>(s_bits) << 32;
      const uint64_t own = static_cast<uint64_t>(nl) | own_bits;
      uint64_t ex = 0, exb = 0;
      if (tis == 0) {
        if (lane == 0) store_status(&c.status[t], kStIncl | own);
      } else {
        if (lane == 0) store_status(&c.status[t], kStAgg | own);
        uint32_t look = t - 1;
        uint32_t rem = tis;  // tiles of this segment before this one
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
          ex += wave_sum_u64(take ? (w & kStCountMask) : 0ull);
          exb |= wave_or_u64(take ? (w & (kStDesc | kStAsc)) : 0ull);
          if (fi < 64) break;
          look -= 64;
          rem -= 64;
        }
        if (lane == 0) store_status(&c.status[t], kStIncl | (ex + nl) | exb | own_bits);
      }
      if (lane == 0) {
        s_lpre = ex;
        s_nl = nl;
        if (tis == nts - 1) {
          segs[si].left = ex + nl;
          segs[si].order_bits = static_cast<uint32_t>((exb | own_bits) >> 32);
        }
      }
    }
    __syncthreads();

    // ---- regroup in LDS: left run [0, nl), right run [nl, nvalid) -----------
    const uint32_t nl = s_nl;
    const uint64_t lpre = s_lpre;
    const uint64_t pre_valid = (tlo - b) - (pidx < tlo ? 1u : 0u);
    // lpre <= pre_valid bounds every write below inside [b, e); it always
    // holds unless the look-back is broken, in which case the tile writes
    // nothing and flags the call
    const bool sane = lpre <= pre_valid;
    if (!sane && tid == 0) atomicOr(&c.ctr->errors, kErrLookback);
    const uint64_t gpre = sane ? pre_valid - lpre : 0;
    const uint64_t lbase = b + lpre;      // where this tile's first left key goes
    const uint64_t rbase = e - 1 - gpre;  // where this tile's first right key goes (then downward)
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      if (sane && ((vmask >> i) & 1u)) {
        const uint32_t rx = s_cnt[i * NW + wv] + below[i];  // left keys before this one in the tile
        uint32_t slot;
        if ((lmask >> i) & 1u) {
          slot = rx;
        } else {
          const uint32_t off = static_cast<uint32_t>(i * NT + tid);
          const uint32_t before = (off - lo) - ((pl >= lo && pl < off) ? 1u : 0u);
          slot = nl + (before - rx);
        }
        s_key[slot] = key[i];
        if (PAIRS) s_val[slot] = val[i];
      }
    }
    __syncthreads();

    // ---- coalesced write: left keys upward from b, right keys downward from e
    const uint32_t nvalid = (hi - lo) - ((pl >= lo && pl < hi) ? 1u : 0u);
#pragma unroll
    for (int j = 0; j < IT; ++j) {
      const uint32_t slot = static_cast<uint32_t>(j * NT + tid);
      if (sane && slot < nvalid) {
        const uint64_t p = slot < nl ? (lbase + slot) : (rbase - (slot - nl));
        dst[p] = s_key[slot];
        if (PAIRS) dstv[p] = s_val[slot];
      }
    }
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

template <class K, bool PAIRS, int NT, int IT>
hipError_t launch_one(const Ctx& c, int parity, uint32_t ntiles, uint32_t src, hipStream_t s) {
  static int per_cu = 0;
  if (per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_partition<K, PAIRS, NT, IT>, NT, 0) != hipSuccess ||
        nb <= 0)
      nb = 1;
    per_cu = nb;
  }
  uint64_t grid = static_cast<uint64_t>(per_cu) * device_cus();
  if (grid > ntiles) grid = ntiles;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_partition<K, PAIRS, NT, IT>), dim3(static_cast<uint32_t>(grid)), dim3(NT), 0, s, c, parity,
                     src);
  return hipGetLastError();
}

template <class K, bool PAIRS>
hipError_t launch_tiles(const Ctx& c, int parity, uint32_t ntiles, uint32_t src, hipStream_t s) {
  switch (c.tile) {
    case 1024: return launch_one<K, PAIRS, 256, 4>(c, parity, ntiles, src, s);
    case 2048: return launch_one<K, PAIRS, 256, 8>(c, parity, ntiles, src, s);
    case 4096: return launch_one<K, PAIRS, 256, 16>(c, parity, ntiles, src, s);
    default: return hipErrorInvalidValue;
  }
}

template <class K>
hipError_t launch_key(const Ctx& c, int parity, uint32_t ntiles, uint32_t src, hipStream_t s) {
  return c.has_vals ? launch_tiles<K, true>(c, parity, ntiles, src, s)
                    : launch_tiles<K, false>(c, parity, ntiles, src, s);
}

}  // namespace

hipError_t launch_partition(const Ctx& c, int parity, uint32_t ntiles, uint32_t src_buf, hipStream_t s) {
  switch (c.key_type) {
    case 1: return launch_key<KeyU32>(c, parity, ntiles, src_buf, s);
    case 2: return launch_key<KeyI32>(c, parity, ntiles, src_buf, s);
    case 3: return launch_key<KeyF32>(c, parity, ntiles, src_buf, s);
    case 4: return launch_key<KeyU64>(c, parity, ntiles, src_buf, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdq
