// Near-sorted inputs: the GPU form of the partial insertion sort of Section
// 5.2. The sequential algorithm, after a partition that swapped nothing,
// lets insertion sort repair a handful of misplaced elements and gives up
// after a few moves; that makes inputs such as "ascending with an element
// appended" linear. Here the whole range is looked at once, before any
// partition pass:
//
//   scan    one coalesced read that counts descents (adjacent pairs with
//           a[i+1] < a[i]) and logs their positions while they number at
//           most kRunMaxDescents, copying the keys (and payloads) to the
//           scratch buffer as it goes; once the count is over the limit the
//           remaining workgroups stop without reading
//   plan    one workgroup sorts the logged positions, cuts the range into
//           maximal non-decreasing runs and decides:
//             - no descent: the range is already sorted;
//             - one long run (more than kRunMaxOutliers keys) and short runs
//               of at most kRunMaxOutliers keys in total ("outliers"):
//               gather and sort the outliers, merge them into the run;
//             - two long runs and nothing else: merge the two runs;
//             - anything else: the partition passes sort the range.
//   gather  the short runs are copied into a small outlier buffer, which
//           the LDS base case then sorts in place
//   merge   merge-path merge of the two sorted sequences (from the scratch
//           copy and the outlier buffer) back into the user buffer
//
// Traffic of a near-sorted input: the scan reads and writes every key once,
// the merge reads and writes every key once.
#include "pdq_internal.h"
#include "runs_internal.h"
#include "wave_ops.h"

namespace pdq {
namespace {

constexpr int kScanNT = 256;
constexpr int kScanRows = 16;
constexpr uint64_t kScanChunk = static_cast<uint64_t>(kScanNT) * kScanRows;

// Counts the descents of keys[0..n) and logs their positions (the index i
// of the pair (i, i+1)) while the count stays within `cap`; copies every
// chunk whose descents were logged to the scratch buffers.
template <class K, bool PAIRS>
__global__ __launch_bounds__(kScanNT) void k_run_scan(const typename K::T* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals, uint64_t n,
                                                      typename K::T* __restrict__ kcopy, uint32_t* __restrict__ vcopy,
                                                      RunBufs rb) {
  using T = typename K::T;
  __shared__ uint32_t s_count, s_local, s_base, s_go;
  const int tid = threadIdx.x;
  const uint64_t nchunks = (n + kScanChunk - 1) / kScanChunk;
  for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    if (tid == 0) {
      s_count = __hip_atomic_load(rb.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_local = 0;
    }
    __syncthreads();
    if (s_count > kRunMaxDescents) return;  // the same value for the whole workgroup
    T k[kScanRows];
    bool d[kScanRows];
    uint32_t mine = 0;
#pragma unroll
    for (int r = 0; r < kScanRows; ++r) {
      const uint64_t i = ch * kScanChunk + static_cast<uint64_t>(r) * kScanNT + tid;
      k[r] = i < n ? keys[i] : T(0);
    }
    // the successor of a key is the next lane's key; the last lane of a wave
    // loads it (it belongs to the next wave or the next row)
    const bool last_lane = lane_id() == 63;
    bool asc = false;
#pragma unroll
    for (int r = 0; r < kScanRows; ++r) {
      const uint64_t i = ch * kScanChunk + static_cast<uint64_t>(r) * kScanNT + tid;
      T nxt = __shfl_down(k[r], 1, 64);
      if (last_lane) nxt = i + 1 < n ? keys[i + 1] : T(0);
      d[r] = i + 1 < n && K::ord(nxt) < K::ord(k[r]);
      asc = asc || (i + 1 < n && K::ord(k[r]) < K::ord(nxt));
      mine += d[r] ? 1u : 0u;
    }
    // some adjacent pair ascends (the learned pass needs both directions);
    // a look first spares the shared word a store from every wave
    if (__ballot(asc) != 0 && lane_id() == 0 &&
        __hip_atomic_load(&rb.count[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
      rb.count[1] = 1u;
    const uint64_t wsum = wave_sum_u64(mine);
    if (lane_id() == 0 && wsum) atomicAdd(&s_local, static_cast<uint32_t>(wsum));
    __syncthreads();
    if (tid == 0) {
      const uint32_t total = s_local;
      // once the count is past the limit the input goes to the partition
      // passes and the exact count no longer matters: a look at the word
      // spares it the read-modify-write of every later workgroup (one
      // address, thousands of workgroups)
      uint32_t old = 0;
      if (total) {
        old = __hip_atomic_load(rb.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old <= kRunMaxDescents) old = atomicAdd(rb.count, total);
      }
      s_base = old;
      s_go = (total == 0 || old + total <= kRunMaxDescents) ? 1u : 0u;
      s_local = 0;
    }
    __syncthreads();
    if (!s_go) return;
#pragma unroll
    for (int r = 0; r < kScanRows; ++r) {
      const uint64_t i = ch * kScanChunk + static_cast<uint64_t>(r) * kScanNT + tid;
      if (d[r]) rb.pos[s_base + atomicAdd(&s_local, 1u)] = static_cast<uint32_t>(i);
      if (i < n) {
        kcopy[i] = k[r];
        if constexpr (PAIRS) vcopy[i] = vals[i];
      }
    }
    __syncthreads();
  }
}

constexpr int kPlanNT = 1024;
constexpr int kPlanSlots = kRunMaxDescents;  // a power of two

// Block-wide exclusive scan of one value per thread (kPlanNT threads).
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t* sh_waves, uint64_t* total) {
  const uint64_t incl = wave_incl_scan_u64(v);
  const int w = threadIdx.x / 64;
  if (lane_id() == 63) sh_waves[w] = incl;
  __syncthreads();
  uint64_t before = 0, all = 0;
  for (int j = 0; j < kPlanNT / 64; ++j) {
    if (j < w) before += sh_waves[j];
    all += sh_waves[j];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// Cuts [0, n) into maximal non-decreasing runs at the logged descents and
// writes the plan (and the short runs' gather list).
__global__ __launch_bounds__(kPlanNT) void k_run_plan(uint64_t n, RunBufs rb) {
  __shared__ uint32_t s_pos[kPlanSlots];
  __shared__ uint64_t s_waves[kPlanNT / 64];
  __shared__ uint64_t s_long[3][2];
  __shared__ uint32_t s_nlong;
  const int tid = threadIdx.x;
  const uint32_t count = __hip_atomic_load(rb.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  RunPlan plan = {};
  plan.descents = count;
  plan.ascent = rb.count[1];
  if (count > kRunMaxDescents) {
    if (tid == 0) *rb.plan = plan;  // state 0: the partition passes sort it
    return;
  }
  if (count == 0) {
    plan.state = kRunSorted;
    if (tid == 0) *rb.plan = plan;
    return;
  }
  // positions in ascending order (bitonic over the padded table)
  for (int i = tid; i < kPlanSlots; i += kPlanNT) s_pos[i] = i < static_cast<int>(count) ? rb.pos[i] : 0xFFFFFFFFu;
  if (tid == 0) s_nlong = 0;
  __syncthreads();
  for (int k = 2; k <= kPlanSlots; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < kPlanSlots; i += kPlanNT) {
        const int p = i ^ j;
        if (p > i) {
          const uint32_t a = s_pos[i], b = s_pos[p];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            s_pos[i] = b;
            s_pos[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // run r = [start_r, end_r), r = 0 .. count; each thread takes the runs
  // r = tid * per .. tid * per + per - 1 (consecutive, so the scan over the
  // short lengths keeps run order)
  const uint32_t nruns = count + 1;
  const uint32_t per = (nruns + kPlanNT - 1) / kPlanNT;
  uint64_t short_len = 0, short_cnt = 0;
  for (uint32_t q = 0; q < per; ++q) {
    const uint32_t r = tid * per + q;
    if (r >= nruns) break;
    const uint64_t st = r == 0 ? 0 : static_cast<uint64_t>(s_pos[r - 1]) + 1;
    const uint64_t en = r == count ? n : static_cast<uint64_t>(s_pos[r]) + 1;
    if (en - st > kRunMaxOutliers) {
      const uint32_t j = atomicAdd(&s_nlong, 1u);
      if (j < 3) {
        s_long[j][0] = st;
        s_long[j][1] = en;
      }
    } else {
      short_len += en - st;
      short_cnt += 1;
    }
  }
  uint64_t total_len = 0, total_cnt = 0;
  const uint64_t dest = block_excl_scan(short_len, s_waves, &total_len);
  const uint64_t slot = block_excl_scan(short_cnt, s_waves, &total_cnt);
  const uint32_t nlong = s_nlong;
  uint32_t state = kRunUnsorted;
  if (nlong == 1 && total_len <= kRunMaxOutliers) state = kRunOutliers;
  if (nlong == 2 && total_len == 0) state = kRunTwoRuns;
  if (state == kRunOutliers) {
    uint64_t d = dest, sl = slot;
    for (uint32_t q = 0; q < per; ++q) {
      const uint32_t r = tid * per + q;
      if (r >= nruns) break;
      const uint64_t st = r == 0 ? 0 : static_cast<uint64_t>(s_pos[r - 1]) + 1;
      const uint64_t en = r == count ? n : static_cast<uint64_t>(s_pos[r]) + 1;
      if (en - st <= kRunMaxOutliers) {
        rb.shorts[sl] = RunSpan{st, en - st, d};
        d += en - st;
        ++sl;
      }
    }
  }
  if (tid == 0) {
    plan.state = state;
    plan.runs = nruns;
    plan.nshort = static_cast<uint32_t>(total_cnt);
    plan.outliers = total_len;
    if (nlong >= 1) {
      plan.a0 = s_long[0][0];
      plan.a1 = s_long[0][1];
    }
    if (nlong >= 2) {
      // the two long runs in position order
      const bool swap = s_long[1][0] < s_long[0][0];
      plan.a0 = s_long[swap ? 1 : 0][0];
      plan.a1 = s_long[swap ? 1 : 0][1];
      plan.b0 = s_long[swap ? 0 : 1][0];
      plan.b1 = s_long[swap ? 0 : 1][1];
    }
    if (state == kRunOutliers) {
      // the base case sorts the outlier buffer in place as one item
      rb.item->begin = 0;
      rb.item->end = total_len;
      rb.item->buf = 0;
      rb.item->reverse = 0;
    }
    *rb.plan = plan;
  }
}

// One workgroup per short run: copies it into the outlier buffer.
template <class T, bool PAIRS>
__global__ __launch_bounds__(256) void k_run_gather(const T* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                    RunBufs rb, T* __restrict__ okeys, uint32_t* __restrict__ ovals) {
  const uint32_t nshort = rb.plan->nshort;
  for (uint32_t r = blockIdx.x; r < nshort; r += gridDim.x) {
    const RunSpan sp = rb.shorts[r];
    for (uint64_t j = threadIdx.x; j < sp.len; j += blockDim.x) {
      okeys[sp.dest + j] = keys[sp.start + j];
      if constexpr (PAIRS) ovals[sp.dest + j] = vals[sp.start + j];
    }
  }
}

constexpr int kMergeNT = 256;
constexpr uint64_t kMergeTile = kRunMergeTile;

// Number of elements of A among the first d outputs of the merge of A and B
// (equal keys: A's first).
template <class K>
__device__ uint64_t merge_split(const typename K::T* a, uint64_t la, const typename K::T* b, uint64_t lb,
                                uint64_t d) {
  uint64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (!(K::ord(b[d - 1 - mid]) < K::ord(a[mid]))) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The merge-path split of every tile boundary d = t * kMergeTile (and of
// the end), one lane each: the searches of neighbouring boundaries share
// their first probes in the cache.
template <class K>
__global__ __launch_bounds__(256) void k_merge_splits(const typename K::T* __restrict__ a, uint64_t la,
                                                      const typename K::T* __restrict__ b, uint64_t lb,
                                                      uint64_t* __restrict__ splits) {
  const uint64_t total = la + lb;
  const uint64_t ntiles = (total + kMergeTile - 1) / kMergeTile;
  const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  const uint64_t d = t * kMergeTile < total ? t * kMergeTile : total;
  splits[t] = merge_split<K>(a, la, b, lb, d);
}

// Merge-path merge of sorted A[0..la) and B[0..lb) into out[0..la+lb), one
// output tile of kMergeTile keys per workgroup: the tile's share of A and B
// comes from the split table, both pieces are staged in LDS, and every key
// finds its place in the tile by a binary search in the other piece (A's
// keys before B's equal keys).
template <class K, bool PAIRS>
__global__ __launch_bounds__(kMergeNT) void k_merge(const typename K::T* __restrict__ a,
                                                    const uint32_t* __restrict__ av, uint64_t la,
                                                    const typename K::T* __restrict__ b,
                                                    const uint32_t* __restrict__ bv, uint64_t lb,
                                                    const uint64_t* __restrict__ splits,
                                                    typename K::T* __restrict__ out, uint32_t* __restrict__ ov) {
  using T = typename K::T;
  __shared__ T s_in[kMergeTile];
  __shared__ T s_out[kMergeTile];
  __shared__ uint32_t s_vin[PAIRS ? kMergeTile : 1];
  __shared__ uint32_t s_vout[PAIRS ? kMergeTile : 1];
  const int tid = threadIdx.x;
  const uint64_t total = la + lb;
  const uint64_t ntiles = (total + kMergeTile - 1) / kMergeTile;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t d0 = t * kMergeTile;
    const uint64_t d1 = d0 + kMergeTile < total ? d0 + kMergeTile : total;
    const uint64_t a0 = splits[t], a1 = splits[t + 1];
    const uint64_t b0 = d0 - a0, b1 = d1 - a1;
    const int na = static_cast<int>(a1 - a0), nb = static_cast<int>(b1 - b0);
    // A's piece at s_in[0, na), B's at s_in[na, na + nb)
    for (int j = tid; j < na + nb; j += kMergeNT) {
      s_in[j] = j < na ? a[a0 + j] : b[b0 + (j - na)];
      if constexpr (PAIRS) s_vin[j] = j < na ? av[a0 + j] : bv[b0 + (j - na)];
    }
    __syncthreads();
    for (int j = tid; j < na + nb; j += kMergeNT) {
      const bool from_a = j < na;
      const auto x = K::ord(s_in[j]);
      // A's key: count B's keys below it; B's key: count A's keys not above it
      int lo = from_a ? na : 0, hi = from_a ? na + nb : na;
      const int base = lo;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const auto y = K::ord(s_in[mid]);
        if (from_a ? (y < x) : !(x < y)) lo = mid + 1;
        else hi = mid;
      }
      const int pos = (from_a ? j : j - na) + (lo - base);
      s_out[pos] = s_in[j];
      if constexpr (PAIRS) s_vout[pos] = s_vin[j];
    }
    __syncthreads();
    for (int j = tid; j < na + nb; j += kMergeNT) {
      out[d0 + j] = s_out[j];
      if constexpr (PAIRS) ov[d0 + j] = s_vout[j];
    }
    __syncthreads();
  }
}

__global__ void k_run_reset(RunBufs rb) {
  if (threadIdx.x == 0) {
    rb.count[0] = 0;
    rb.count[1] = 0;
  }
}

template <class K>
struct RunsL {
  using T = typename K::T;
  static hipError_t scan(const Ctx& c, const RunBufs& rb, hipStream_t s) {
    hipLaunchKernelGGL(k_run_reset, dim3(1), dim3(64), 0, s, rb);
    const uint64_t nchunks = (c.n + kScanChunk - 1) / kScanChunk;
    const uint32_t grid = static_cast<uint32_t>(nchunks < 2048 ? nchunks : 2048);
    const T* k = static_cast<const T*>(c.keys[0]);
    T* kc = static_cast<T*>(c.keys[1]);
    if (c.has_vals)
      hipLaunchKernelGGL((k_run_scan<K, true>), dim3(grid), dim3(kScanNT), 0, s, k, c.vals[0], c.n, kc, c.vals[1], rb);
    else
      hipLaunchKernelGGL((k_run_scan<K, false>), dim3(grid), dim3(kScanNT), 0, s, k, c.vals[0], c.n, kc, c.vals[1],
                         rb);
    hipLaunchKernelGGL(k_run_plan, dim3(1), dim3(kPlanNT), 0, s, c.n, rb);
    return hipGetLastError();
  }
  static hipError_t gather(const Ctx& c, const RunBufs& rb, uint32_t nshort, hipStream_t s) {
    const uint32_t grid = nshort < 1024 ? nshort : 1024;
    if (grid == 0) return hipSuccess;
    const T* k = static_cast<const T*>(c.keys[0]);
    T* ok = static_cast<T*>(rb.okeys);
    if (c.has_vals)
      hipLaunchKernelGGL((k_run_gather<T, true>), dim3(grid), dim3(256), 0, s, k, c.vals[0], rb, ok, rb.ovals);
    else
      hipLaunchKernelGGL((k_run_gather<T, false>), dim3(grid), dim3(256), 0, s, k, c.vals[0], rb, ok, rb.ovals);
    return hipGetLastError();
  }
  static hipError_t merge(const Ctx& c, const RunBufs& rb, const T* a, const uint32_t* av, uint64_t la,
                          const T* b, const uint32_t* bv, uint64_t lb, hipStream_t s) {
    const uint64_t ntiles = (la + lb + kMergeTile - 1) / kMergeTile;
    const uint32_t grid = static_cast<uint32_t>(ntiles < 8192 ? ntiles : 8192);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_splits<K>, dim3(static_cast<uint32_t>((ntiles + 1 + 255) / 256)), dim3(256), 0, s,
                       a, la, b, lb, rb.splits);
    T* out = static_cast<T*>(c.keys[0]);
    if (c.has_vals)
      hipLaunchKernelGGL((k_merge<K, true>), dim3(grid), dim3(kMergeNT), 0, s, a, av, la, b, bv, lb, rb.splits,
                         out, c.vals[0]);
    else
      hipLaunchKernelGGL((k_merge<K, false>), dim3(grid), dim3(kMergeNT), 0, s, a, av, la, b, bv, lb, rb.splits,
                         out, c.vals[0]);
    return hipGetLastError();
  }
  // plan state kRunOutliers: the long run (scratch copy) with the sorted
  // outliers; kRunTwoRuns: the two long runs of the scratch copy
  static hipError_t finish(const Ctx& c, const RunBufs& rb, const RunPlan& p, hipStream_t s) {
    const T* sk = static_cast<const T*>(c.keys[1]);
    const uint32_t* sv = c.vals[1];
    if (p.state == kRunOutliers)
      return merge(c, rb, sk + p.a0, sv ? sv + p.a0 : nullptr, p.a1 - p.a0, static_cast<const T*>(rb.okeys),
                   rb.ovals, p.outliers, s);
    return merge(c, rb, sk + p.a0, sv ? sv + p.a0 : nullptr, p.a1 - p.a0, sk + p.b0, sv ? sv + p.b0 : nullptr,
                 p.b1 - p.b0, s);
  }
};

template <template <class> class F, class... A>
hipError_t dispatch(uint32_t kt, A&&... args) {
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

template <class K>
struct ScanF {
  static hipError_t run(const Ctx& c, const RunBufs& rb, hipStream_t s) { return RunsL<K>::scan(c, rb, s); }
};
template <class K>
struct GatherF {
  static hipError_t run(const Ctx& c, const RunBufs& rb, uint32_t nshort, hipStream_t s) {
    return RunsL<K>::gather(c, rb, nshort, s);
  }
};
template <class K>
struct FinishF {
  static hipError_t run(const Ctx& c, const RunBufs& rb, const RunPlan& p, hipStream_t s) {
    return RunsL<K>::finish(c, rb, p, s);
  }
};

}  // namespace

hipError_t launch_run_scan(const Ctx& c, const RunBufs& rb, hipStream_t s) {
  return dispatch<ScanF>(c.key_type, c, rb, s);
}

hipError_t launch_run_gather(const Ctx& c, const RunBufs& rb, uint32_t nshort, hipStream_t s) {
  return dispatch<GatherF>(c.key_type, c, rb, nshort, s);
}

hipError_t launch_run_merge(const Ctx& c, const RunBufs& rb, const RunPlan& p, hipStream_t s) {
  return dispatch<FinishF>(c.key_type, c, rb, p, s);
}

}  // namespace pdq
