// Histogram and scatter of the learned multiway first pass.
//
// A key with image v falls into bin 2b (range bin) or 2b - 1 (equality bin),
// where b is the number of splitters <= v and the equality bin is taken when
// v equals splitter b - 1. Range bins hold the keys strictly between two
// consecutive splitters, so every key of bin i precedes every key of bin
// i + 1; equality bins hold copies of one key and are final.
//
//   hist      per tile of 8192 keys: branchless binary search over the
//             splitters in LDS, LDS bin counters, one row of 512 counts
//             (whether the input is ordered was settled by the order scan
//             before the fit: an ordered input is left to the plain path,
//             which retires it in one pass)
//   scan      chunk sums of 64 rows, one workgroup scanning the chunk sums
//             (bin totals, bin starts), then each chunk rescans its rows into
//             absolute per-tile offsets
//   scatter   per tile: classify again, rank within the bin by an LDS atomic,
//             stage the tile in LDS in bin order, write every bin's run
//             contiguously to its offset
#include "learn_internal.h"
#include "pdq_internal.h"
#include "wave_ops.h"

namespace pdq {
namespace {

constexpr uint32_t kNT = kBucketThreads;
constexpr uint32_t kPer = kBucketTile / kBucketThreads;  // keys per thread
static_assert(kPer * kNT == kBucketTile, "tile must be a multiple of the workgroup");

// The u sorted splitters in LDS, padded to 256 with the largest image, in the
// key's own width (32-bit keys have 32-bit images). Entry i sits at
// i + i / 2^kSkew: the probes of one search level are a power of two apart,
// and the skew spreads them over distinct banks.
template <class S>
struct SplitTable {
  static constexpr uint32_t kSkew = sizeof(S) == 8 ? 4 : 5;
  S v[256 + (256 >> kSkew)];
  __device__ __forceinline__ static uint32_t at(uint32_t i) { return i + (i >> kSkew); }
  __device__ __forceinline__ S get(uint32_t i) const { return v[at(i)]; }
};

template <class S>
__device__ __forceinline__ void load_splitters(SplitTable<S>& t, const BucketBufs& b, uint32_t& u) {
  u = *b.count;
  for (uint32_t i = threadIdx.x; i < 256; i += kNT) t.v[SplitTable<S>::at(i)] = i < u ? static_cast<S>(b.splitters[i]) : S(~S(0));
}

// Bins of N key images: branchless binary search for the number b of
// splitters <= img (padding is clamped away), then the equality test. The
// search runs level by level over all N keys, so a level's N table probes
// are in flight together instead of one key's eight probes back to back.
template <class S, uint32_t N>
__device__ __forceinline__ void bins_of(const SplitTable<S>& t, uint32_t u, const S (&img)[N], uint32_t (&bin)[N]) {
  uint32_t pos[N];
#pragma unroll
  for (uint32_t k = 0; k < N; ++k) pos[k] = 0;
#pragma unroll
  for (uint32_t step = 128; step >= 1; step >>= 1) {
    S probe[N];
#pragma unroll
    for (uint32_t k = 0; k < N; ++k) probe[k] = t.get(pos[k] + step - 1);
#pragma unroll
    for (uint32_t k = 0; k < N; ++k) pos[k] += probe[k] <= img[k] ? step : 0u;
  }
  S below[N];
#pragma unroll
  for (uint32_t k = 0; k < N; ++k) {
    pos[k] = pos[k] < u ? pos[k] : u;
    below[k] = t.get(pos[k] > 0 ? pos[k] - 1 : 0);
  }
#pragma unroll
  for (uint32_t k = 0; k < N; ++k) bin[k] = pos[k] > 0 && below[k] == img[k] ? 2 * pos[k] - 1 : 2 * pos[k];
}

// Exclusive scan of s[0..512) in place by the 512 threads; returns the total.
__device__ uint32_t block_exclusive_scan_512(uint32_t* s, uint32_t* s_wsum) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t v = s[tid];
  uint32_t incl = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d, 64);
    if (lane >= static_cast<uint32_t>(d)) incl += t;
  }
  if (lane == 63) s_wsum[w] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (uint32_t k = 0; k < kNT / 64; ++k) {
    if (k < w) before += s_wsum[k];
    total += s_wsum[k];
  }
  __syncthreads();
  s[tid] = before + incl - v;
  __syncthreads();
  return total;
}

template <class K>
__global__ __launch_bounds__(kNT) void k_hist(const typename K::T* __restrict__ keys, uint64_t n, BucketBufs b) {
  if (b.go && *b.go == 0) return;  // the fit's sample judge already failed: nothing to count
  using S = typename K::T;
  __shared__ SplitTable<S> s_sp;
  __shared__ uint32_t s_cnt[kBinStride];
  // the tile's keys are on their way while the splitter table is set up;
  // every lane loads (positions past the end read the last key and are not
  // counted), so the loads are in flight together
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kBucketTile;
  typename K::T v[kPer];
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint64_t i = base + k * kNT + threadIdx.x;
    v[k] = keys[i < n ? i : n - 1];
  }
  uint32_t u;
  load_splitters(s_sp, b, u);
  for (uint32_t i = threadIdx.x; i < kBinStride; i += kNT) s_cnt[i] = 0;
  lds_barrier();
  S img[kPer];
  uint32_t bin[kPer];
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) img[k] = K::ord(v[k]);
  bins_of(s_sp, u, img, bin);
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint64_t i = base + k * kNT + threadIdx.x;
    if (i < n) atomicAdd(&s_cnt[bin[k]], 1u);
  }
  __syncthreads();
  uint32_t* row = b.rows + static_cast<uint64_t>(blockIdx.x) * kBinStride;
  for (uint32_t i = threadIdx.x; i < kBinStride; i += kNT) row[i] = s_cnt[i];
}

// Sum of each bin over the rows of one chunk.
__global__ __launch_bounds__(kBinStride) void k_chunk_sum(BucketBufs b) {
  if (b.go && *b.go == 0) return;  // the fit's sample judge already failed: nothing to count
  const uint64_t r0 = static_cast<uint64_t>(blockIdx.x) * kScanRows;
  const uint64_t r1 = r0 + kScanRows < b.ntiles ? r0 + kScanRows : b.ntiles;
  uint32_t sum = 0;
#pragma unroll 16
  for (uint64_t r = r0; r < r1; ++r) sum += b.rows[r * kBinStride + threadIdx.x];
  b.chunk[static_cast<uint64_t>(blockIdx.x) * kBinStride + threadIdx.x] = sum;
}

// One workgroup: chunk sums -> per-chunk exclusive offsets within each bin,
// bin totals, and the start of every bin (exclusive scan over bins).
__global__ __launch_bounds__(kBinStride) void k_chunk_scan(BucketBufs b) {
  if (b.go && *b.go == 0) return;  // the fit's sample judge already failed: nothing to count
  __shared__ uint32_t s_tot[kBinStride];
  __shared__ uint32_t s_wsum[kBinStride / 64];
  const uint32_t tid = threadIdx.x;
  uint64_t run = 0;
  // sixteen independent loads in flight, then their running sums
  for (uint64_t c0 = 0; c0 < b.nchunks; c0 += 16) {
    uint32_t v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = c0 + q < b.nchunks ? b.chunk[(c0 + q) * kBinStride + tid] : 0u;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (c0 + q < b.nchunks) b.chunk[(c0 + q) * kBinStride + tid] = static_cast<uint32_t>(run);
      run += v[q];
    }
  }
  b.totals[tid] = run;
  s_tot[tid] = static_cast<uint32_t>(run);
  __syncthreads();
  const uint32_t total = block_exclusive_scan_512(s_tot, s_wsum);
  b.begin[tid] = s_tot[tid];
  if (tid == 0) b.begin[kBinStride] = total;
}

// Rows of one chunk -> absolute start of each (tile, bin) run.
__global__ __launch_bounds__(kBinStride) void k_tile_rescan(BucketBufs b) {
  if (b.go && *b.go == 0) return;  // the fit's sample judge already failed: nothing to count
  const uint64_t r0 = static_cast<uint64_t>(blockIdx.x) * kScanRows;
  const uint64_t r1 = r0 + kScanRows < b.ntiles ? r0 + kScanRows : b.ntiles;
  uint32_t run = static_cast<uint32_t>(b.begin[threadIdx.x]) + b.chunk[static_cast<uint64_t>(blockIdx.x) * kBinStride + threadIdx.x];
  for (uint64_t r0b = r0; r0b < r1; r0b += 16) {
    uint32_t v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = r0b + q < r1 ? b.rows[(r0b + q) * kBinStride + threadIdx.x] : 0u;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (r0b + q < r1) b.rows[(r0b + q) * kBinStride + threadIdx.x] = run;
      run += v[q];
    }
  }
}

// Tile of workgroup b among g. Workgroups are handed to the 8 XCDs in turn
// (b on XCD b % 8), each with its own L2; this gives every XCD one
// contiguous range of tiles, so the short runs that neighbouring tiles write
// into the same bin meet in one L2 and leave it as whole cache lines.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t g) {
  constexpr uint32_t kXcd = 8;
  const uint32_t x = b % kXcd, q = g / kXcd, r = g % kXcd;
  return x * q + (x < r ? x : r) + b / kXcd;
}

template <class K, bool PAIRS>
__global__ __launch_bounds__(kNT) void k_scatter(const typename K::T* __restrict__ kin,
                                                 const uint32_t* __restrict__ vin, typename K::T* __restrict__ kout,
                                                 uint32_t* __restrict__ vout, uint64_t n, BucketBufs b) {
  using T = typename K::T;
  __shared__ SplitTable<T> s_sp;
  __shared__ uint32_t s_loc[kBinStride];   // ranks, then local run starts
  __shared__ uint32_t s_goff[kBinStride];  // global run starts of this tile
  __shared__ uint32_t s_wsum[kNT / 64];
  __shared__ T s_key[kBucketTile];
  __shared__ uint16_t s_bin[kBucketTile];
  __shared__ uint32_t s_val[PAIRS ? kBucketTile : 1];
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint64_t base = static_cast<uint64_t>(tile) * kBucketTile;
  const uint32_t cnt = static_cast<uint32_t>(n - base < kBucketTile ? n - base : kBucketTile);
  // the tile's keys are on their way while the tables are set up
  T v[kPer];
  uint32_t pv[PAIRS ? kPer : 1];
  uint32_t bin[kPer], rank[kPer];
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t i = k * kNT + threadIdx.x;
    v[k] = i < cnt ? kin[base + i] : T(0);
    if constexpr (PAIRS) pv[k] = i < cnt ? vin[base + i] : 0u;
  }
  uint32_t u;
  load_splitters(s_sp, b, u);
  const uint32_t* row = b.rows + static_cast<uint64_t>(tile) * kBinStride;
  for (uint32_t i = threadIdx.x; i < kBinStride; i += kNT) {
    s_loc[i] = 0;
    s_goff[i] = row[i];
  }
  lds_barrier();
  {
    T img[kPer];
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) img[k] = K::ord(v[k]);
    bins_of(s_sp, u, img, bin);
  }
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t i = k * kNT + threadIdx.x;
    rank[k] = i < cnt ? atomicAdd(&s_loc[bin[k]], 1u) : 0u;
  }
  __syncthreads();
  block_exclusive_scan_512(s_loc, s_wsum);
#pragma unroll
  for (uint32_t k = 0; k < kPer; ++k) {
    const uint32_t i = k * kNT + threadIdx.x;
    if (i < cnt) {
      const uint32_t at = s_loc[bin[k]] + rank[k];
      s_key[at] = v[k];
      s_bin[at] = static_cast<uint16_t>(bin[k]);
      if constexpr (PAIRS) s_val[at] = pv[k];
    }
  }
  __syncthreads();
  // a full tile takes every slot in a loop the compiler unrolls: the bin
  // and run-start lookups of all the lane's keys are in flight together
  // before the first store
  if (cnt == kBucketTile) {
    uint32_t pos[kPer];  // the row offsets are 32-bit: positions below 2^32
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
      const uint32_t i = k * kNT + threadIdx.x;
      const uint32_t bi = s_bin[i];
      pos[k] = s_goff[bi] + (i - s_loc[bi]);
    }
#pragma unroll
    for (uint32_t k = 0; k < kPer; ++k) {
      const uint32_t i = k * kNT + threadIdx.x;
      if (pos[k] >= n) {  // histogram and scatter disagree: never write outside the output
        atomicOr(b.errors, kErrScatter);
        continue;
      }
      kout[pos[k]] = s_key[i];
      if constexpr (PAIRS) vout[pos[k]] = s_val[i];
    }
    return;
  }
  for (uint32_t i = threadIdx.x; i < cnt; i += kNT) {
    const uint32_t bi = s_bin[i];
    const uint64_t pos = static_cast<uint64_t>(s_goff[bi]) + (i - s_loc[bi]);
    if (pos >= n) {  // histogram and scatter disagree: never write outside the output
      atomicOr(b.errors, kErrScatter);
      continue;
    }
    kout[pos] = s_key[i];
    if constexpr (PAIRS) vout[pos] = s_val[i];
  }
}

// Whether keys[0..n) are ordered, before anything else is spent on them:
// bit 0 of *flags = some adjacent pair descends, bit 1 = some pair ascends.
// Rows of 256 keys are read coalesced, each key with its successor. A
// workgroup ORs its waves' bits in LDS and sends only news to the shared
// word (same-address atomics are slow), and stops as soon as both bits are
// known, so an unordered input costs a few chunks and an ordered one a
// single read.
template <class K>
__global__ __launch_bounds__(256) void k_order_scan(const typename K::T* __restrict__ keys, uint64_t n,
                                                    uint32_t* flags) {
  constexpr uint32_t kRowsPer = 64;  // 16384 keys between two looks at the shared word
  constexpr uint64_t kChunk = 256ull * kRowsPer;
  __shared__ uint32_t s_flags, s_bits;
  if (n < 2) return;  // no adjacent pair (and the loads below read positions n - 2, n - 1)
  const uint64_t nchunks = (n + kChunk - 1) / kChunk;
  for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    if (threadIdx.x == 0) {
      s_flags = __hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_bits = 0;
    }
    __syncthreads();
    const uint32_t f = s_flags;
    if (f == 3u) return;  // the same value for the whole workgroup
    bool d = false, a = false;
    // every lane loads (positions past the last pair read the last pair and
    // count for nothing): 16 rows of loads are issued before any is used
    constexpr uint32_t kGroup = 16;
    for (uint32_t r0 = 0; r0 < kRowsPer; r0 += kGroup) {
      typename K::T xs[kGroup], ys[kGroup];
      bool pair[kGroup];
#pragma unroll
      for (uint32_t q = 0; q < kGroup; ++q) {
        const uint64_t i = ch * kChunk + static_cast<uint64_t>(r0 + q) * 256u + threadIdx.x;
        pair[q] = i + 1 < n;
        const uint64_t ic = pair[q] ? i : n - 2;
        xs[q] = keys[ic];
        ys[q] = keys[ic + 1];
      }
#pragma unroll
      for (uint32_t q = 0; q < kGroup; ++q) {
        const auto x = K::ord(xs[q]), y = K::ord(ys[q]);
        d |= pair[q] && y < x;
        a |= pair[q] && y > x;
      }
    }
    const uint32_t bits = (__any(d) ? 1u : 0u) | (__any(a) ? 2u : 0u);
    if (lane_id() == 0 && bits) atomicOr(&s_bits, bits);
    __syncthreads();
    if (threadIdx.x == 0 && (s_bits & ~f)) atomicOr(flags, s_bits);
  }
}

template <class K>
struct OrderL {
  static hipError_t run(const void* keys, uint64_t n, uint32_t* flags, hipStream_t s) {
    const uint64_t nchunks = (n + 16383) / 16384;
    const uint32_t grid = static_cast<uint32_t>(nchunks < 4096 ? nchunks : 4096);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_order_scan<K>, dim3(grid), dim3(256), 0, s, static_cast<const typename K::T*>(keys), n,
                       flags);
    return hipGetLastError();
  }
};

template <class K>
struct HistL {
  static hipError_t run(const void* keys, uint64_t n, const BucketBufs& b, hipStream_t s) {
    hipLaunchKernelGGL(k_hist<K>, dim3(static_cast<uint32_t>(b.ntiles)), dim3(kNT), 0, s,
                       static_cast<const typename K::T*>(keys), n, b);
    return hipGetLastError();
  }
};

template <class K>
struct ScatterL {
  static hipError_t run(bool pairs, const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, uint64_t n,
                        const BucketBufs& b, hipStream_t s) {
    using T = typename K::T;
    if (pairs)
      hipLaunchKernelGGL((k_scatter<K, true>), dim3(static_cast<uint32_t>(b.ntiles)), dim3(kNT), 0, s,
                         static_cast<const T*>(kin), vin, static_cast<T*>(kout), vout, n, b);
    else
      hipLaunchKernelGGL((k_scatter<K, false>), dim3(static_cast<uint32_t>(b.ntiles)), dim3(kNT), 0, s,
                         static_cast<const T*>(kin), vin, static_cast<T*>(kout), vout, n, b);
    return hipGetLastError();
  }
};

}  // namespace

__global__ void k_zero_word(uint32_t* p) { *p = 0; }

hipError_t launch_bucket_hist(uint32_t kt, const void* keys, uint64_t n, const BucketBufs& b, hipStream_t s) {
  switch (kt) {
    case 1: return HistL<KeyU32>::run(keys, n, b, s);
    case 2: return HistL<KeyI32>::run(keys, n, b, s);
    case 3: return HistL<KeyF32>::run(keys, n, b, s);
    case 4: return HistL<KeyU64>::run(keys, n, b, s);
    case 5: return HistL<KeyI64>::run(keys, n, b, s);
    case 6: return HistL<KeyF64>::run(keys, n, b, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_order_scan(uint32_t kt, const void* keys, uint64_t n, uint32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_word, dim3(1), dim3(1), 0, s, flags);
  switch (kt) {
    case 1: return OrderL<KeyU32>::run(keys, n, flags, s);
    case 2: return OrderL<KeyI32>::run(keys, n, flags, s);
    case 3: return OrderL<KeyF32>::run(keys, n, flags, s);
    case 4: return OrderL<KeyU64>::run(keys, n, flags, s);
    case 5: return OrderL<KeyI64>::run(keys, n, flags, s);
    case 6: return OrderL<KeyF64>::run(keys, n, flags, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_bucket_scan(const BucketBufs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_chunk_sum, dim3(static_cast<uint32_t>(b.nchunks)), dim3(kBinStride), 0, s, b);
  hipLaunchKernelGGL(k_chunk_scan, dim3(1), dim3(kBinStride), 0, s, b);
  hipLaunchKernelGGL(k_tile_rescan, dim3(static_cast<uint32_t>(b.nchunks)), dim3(kBinStride), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_bucket_scatter(uint32_t kt, bool pairs, const void* keys_in, const uint32_t* vals_in,
                                 void* keys_out, uint32_t* vals_out, uint64_t n, const BucketBufs& b,
                                 hipStream_t s) {
  switch (kt) {
    case 1: return ScatterL<KeyU32>::run(pairs, keys_in, vals_in, keys_out, vals_out, n, b, s);
    case 2: return ScatterL<KeyI32>::run(pairs, keys_in, vals_in, keys_out, vals_out, n, b, s);
    case 3: return ScatterL<KeyF32>::run(pairs, keys_in, vals_in, keys_out, vals_out, n, b, s);
    case 4: return ScatterL<KeyU64>::run(pairs, keys_in, vals_in, keys_out, vals_out, n, b, s);
    case 5: return ScatterL<KeyI64>::run(pairs, keys_in, vals_in, keys_out, vals_out, n, b, s);
    case 6: return ScatterL<KeyF64>::run(pairs, keys_in, vals_in, keys_out, vals_out, n, b, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdq
