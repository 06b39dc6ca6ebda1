// Kernels of the learned multiway first pass, up to the splitters:
//   sample    m keys at positions SplitMix64(seed ^ j) mod n, as key images,
//             sorted by LDS bitonic chunks and a rank merge
//   features  piecewise-linear log2 or linear scaling of the sorted sample onto
//             [0, 1] (whichever is closer to uniform), and mid-rank targets
//   train     the fused trainer: S Adam steps of the 1 -> 32 -> 32 -> 1 ReLU
//             MLP (residual output), forward, backward and update in one
//             cooperative launch; every workgroup holds all 1153 parameters
//             in LDS and the workgroups exchange gradient partials once a
//             step through a grid barrier
//   infer     float32 prediction, every dot product a chain of fused
//             multiply-adds in index order, clamped to [0, 1]
//   extract   for k = 1..255: the sample key at the k-th sample quantile when
//             it fills at least m/256 sample slots (a heavy key), else the
//             first sample key whose running maximum of the prediction
//             reaches k/256; sorted, duplicates removed
// The arithmetic that decides an integer (features, inference, extraction)
// uses only correctly rounded operations in a fixed order; training is
// float32 with a deterministic reduction order.
#include "learn_internal.h"
#include "pdq_internal.h"
#include "wave_ops.h"

namespace pdq {
namespace {

// ---------------------------------------------------------------- sample

template <class K>
__global__ __launch_bounds__(256) void k_sample(const typename K::T* __restrict__ keys, uint64_t n, uint64_t m,
                                                uint64_t seed, uint64_t* __restrict__ out) {
  const uint64_t j = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x;
  if (j >= m) return;
  const uint64_t pos = mix64(seed ^ j) % n;
  out[j] = static_cast<uint64_t>(K::ord(keys[pos]));
}

// ---------------------------------------------------------------- sample sort
// The sample (m = 16 chunks of 4096 images) is sorted in two launches: each
// chunk by a bitonic network in LDS, then every key goes to its rank in the
// merged order, found by binary search in the other chunks (ties ordered by
// chunk, so the ranks form a permutation).

constexpr uint32_t kChunk = 4096;
constexpr uint32_t kChunkThreads = 1024;

__global__ __launch_bounds__(kChunkThreads) void k_chunk_bitonic(uint64_t* __restrict__ a) {
  __shared__ uint64_t s[kChunk];
  uint64_t* g = a + static_cast<uint64_t>(blockIdx.x) * kChunk;
  for (uint32_t i = threadIdx.x; i < kChunk; i += kChunkThreads) s[i] = g[i];
  for (uint32_t k = 2; k <= kChunk; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      __syncthreads();
      for (uint32_t p = threadIdx.x; p < kChunk / 2; p += kChunkThreads) {
        const uint32_t i = 2 * j * (p / j) + (p % j);
        const uint32_t l = i + j;
        const bool up = (i & k) == 0;
        const uint64_t x = s[i], y = s[l];
        if ((x > y) == up) {
          s[i] = y;
          s[l] = x;
        }
      }
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kChunk; i += kChunkThreads) g[i] = s[i];
}

__global__ __launch_bounds__(256) void k_rank_merge(const uint64_t* __restrict__ in, uint64_t m,
                                                    uint64_t* __restrict__ out) {
  const uint64_t j = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x;
  if (j >= m) return;
  const uint64_t key = in[j];
  const uint64_t r = j / kChunk;
  uint64_t pos = j % kChunk;
  const uint64_t nchunks = m / kChunk;
  for (uint64_t q = 0; q < nchunks; ++q) {
    if (q == r) continue;
    const uint64_t* c = in + q * kChunk;
    uint32_t lo = 0, hi = kChunk;
    while (lo < hi) {  // chunks before r count keys <= key, chunks after count keys < key
      const uint32_t mid = (lo + hi) >> 1;
      const bool left = q < r ? c[mid] <= key : c[mid] < key;
      if (left) lo = mid + 1;
      else hi = mid;
    }
    pos += lo;
  }
  out[pos] = key;
}

// ---------------------------------------------------------------- features

// L(v) = e + (4 f - f^2) / 3 with f = (v - 2^e) / 2^e in [0, 1) and
// e = floor(log2 v); L(0) = -1. The polynomial has p(0) = 0, p(1) = 1 and
// p'(1) = p'(0) / 2, so the slope of L is continuous across every power of
// two. Correctly rounded operations in a fixed order (conversion, exact
// scaling, f * f, 4 f - f * f, / 3, + e); contraction is off here, so no
// multiply is fused into an add (the pragma acts on operators written in
// its scope, not on inlined helpers, so the operators are written out).
__device__ __forceinline__ double pseudo_log2(uint64_t v) {
#pragma clang fp contract(off)
  if (v == 0) return -1.0;
  const int e = 63 - __clzll(static_cast<long long>(v));
  const double f = ldexp(static_cast<double>(v - (1ull << e)), -e);
  const double q = 4.0 * f - f * f;
  return q / 3.0 + static_cast<double>(e);
}

__global__ void k_zero_u64(uint64_t* p, uint32_t count) {
  for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

__global__ void k_zero_u32(uint32_t* p, uint32_t count) {
  for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

// Largest deviation from uniform spacing of both scalings. Non-negative
// doubles order like their bit patterns, so the maximum is an atomicMax.
__global__ __launch_bounds__(256) void k_feat_dev(const uint64_t* __restrict__ s, uint64_t m, uint64_t* info) {
  const uint64_t j = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x;
  const uint64_t lo = s[0], hi = s[m - 1];
  double dl = 0.0, dn = 0.0;
  if (j < m && hi != lo) {
    const double la = pseudo_log2(lo), lb = pseudo_log2(hi);
    const double ref = (static_cast<double>(j) + 0.5) / static_cast<double>(m);
    const double xl = (pseudo_log2(s[j]) - la) / (lb - la);
    const double xn = static_cast<double>(s[j] - lo) / static_cast<double>(hi - lo);
    dl = fabs(xl - ref);
    dn = fabs(xn - ref);
  }
  uint64_t bl = static_cast<uint64_t>(__double_as_longlong(dl));
  uint64_t bn = static_cast<uint64_t>(__double_as_longlong(dn));
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t ol = __shfl_xor(bl, d, 64), on = __shfl_xor(bn, d, 64);
    bl = ol > bl ? ol : bl;
    bn = on > bn ? on : bn;
  }
  if (lane_id() == 0) {
    atomicMax(reinterpret_cast<unsigned long long*>(&info[0]), static_cast<unsigned long long>(bl));
    atomicMax(reinterpret_cast<unsigned long long*>(&info[1]), static_cast<unsigned long long>(bn));
  }
}

// Feature (float32 of the chosen scaling) and mid-rank target of every
// sample key; the target's run of equal keys is found by binary search.
__global__ __launch_bounds__(256) void k_feat_out(const uint64_t* __restrict__ s, uint64_t m, uint64_t* info,
                                                  float* __restrict__ x, float* __restrict__ t) {
  const uint64_t j = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x;
  const uint64_t lo = s[0], hi = s[m - 1];
  const bool flat = hi == lo;
  const bool use_log = flat || info[0] <= info[1];
  if (j == 0) info[2] = use_log ? 1u : 0u;
  if (j >= m) return;
  const uint64_t v = s[j];
  float xv;
  if (flat) {
    xv = 0.5f;
  } else if (use_log) {
    const double la = pseudo_log2(lo), lb = pseudo_log2(hi);
    xv = static_cast<float>((pseudo_log2(v) - la) / (lb - la));
  } else {
    xv = static_cast<float>(static_cast<double>(v - lo) / static_cast<double>(hi - lo));
  }
  x[j] = xv;
  uint64_t a = 0, b = j;
  while (a < b) {
    const uint64_t mid = (a + b) >> 1;
    if (s[mid] < v) a = mid + 1;
    else b = mid;
  }
  const uint64_t first = a;
  a = j;
  b = m;
  while (a < b) {
    const uint64_t mid = (a + b) >> 1;
    if (s[mid] <= v) a = mid + 1;
    else b = mid;
  }
  const uint64_t last = a - 1;
  t[j] = static_cast<float>(static_cast<double>(first + last + 1) / (2.0 * static_cast<double>(m)));
}

// ---------------------------------------------------------------- model

__device__ __forceinline__ float relu(float z) { return z > 0.0f ? z : 0.0f; }

// Seeded initial value of parameter i, exact in double and rounded once to
// float. The first-layer offsets b1 are set afterwards from the knots.
__device__ float init_value(uint64_t seed, int i) {
  const uint64_t h = mix64(seed ^ (kSaltInit + static_cast<uint64_t>(i)));
  const double a = static_cast<double>(h >> 40) * 0x1p-23 - 1.0;  // [-1, 1), 24 bits
  const double lim = static_cast<double>(0x1.bb67aep-2f);         // float(sqrt(6 / 32))
  if (i < kOffB1) return static_cast<float>((a >= 0.0 ? 1.0 : -1.0) * (1.0 + 3.0 * fabs(a)));
  if (i < kOffW2) return 0.0f;
  if (i < kOffB2) return static_cast<float>(a * lim);
  if (i < kOffW3) return 0x1.99999ap-4f;  // float(0.1)
  if (i < kOffB3) return static_cast<float>(a * lim / 8.0);
  return 0.0f;
}

constexpr int kRow = 36;   // row of a [sample][unit] array (float4-aligned)
constexpr int kRowT = 68;  // row of a [unit][sample] array (float4-aligned)
static_assert(kTrainThreads == 1024 && kTrainChunk == 64, "the chunk mapping assumes 1024 threads, 64 samples");

struct TrainSmem {
  float p[kNParam + 7];
  float w2t[kH * kH];             // W2 transposed: [u][v]
  float h1[kTrainChunk * kRow];   // [s][u]
  float h1t[kH * kRowT];          // [u][s]

  float z2t[kH * kRowT];          // [v][s]
  float dz2[kTrainChunk * kRow];  // [s][v]
  float dz2t[kH * kRowT];         // [v][s]
  float dz1t[kH * kRowT];         // [u][s]
  float x[kTrainChunk];
  float t[kTrainChunk];
  float dy[kTrainChunk];
  float red[kTrainThreads / 64];
};

// Per-thread gradient accumulators: thread tid owns dW2 entry tid (v = tid/32,
// u = tid%32); threads 0-511 hold an eighth of the sample sum of a
// (W1[u], b1[u]) or (W3[v], b2[v]) pair; 512-519 an eighth of db3; one lane
// per sample sums the squared residuals.
struct GradAcc {
  float w2;
  float s0, s1;
  float loss;
};

__device__ __forceinline__ void rebuild_w2t(TrainSmem& sm) {
  for (int i = threadIdx.x; i < kH * kH; i += kTrainThreads) sm.w2t[(i & 31) * kH + (i >> 5)] = sm.p[kOffW2 + i];
}

// Orders the LDS accesses of one wave (its lanes exchange values through
// LDS without waiting for the rest of the workgroup).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward and backward of the chunk in sm.x / sm.t (cs valid samples, the
// rest zero); adds its contribution to the gradient of the mean squared
// error over `batch`. Padded samples get dL/dy = 0, so every gradient term
// they would add is zero.
//
// Sixteen lanes handle one sample, two hidden units each; they share a wave,
// so the whole forward and backward pass of a sample needs no workgroup
// barrier. Only the parameter sums over the chunk's samples wait for the
// workgroup.
__device__ void chunk_grad(TrainSmem& sm, uint32_t cs, uint32_t batch, uint32_t residual, GradAcc& g) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int s = tid >> 4, c0 = (tid & 15) * 2;  // one sample, two units
  const float xs = sm.x[s];
  // layer 1
  const float h0 = relu(fmaf(sm.p[kOffW1 + c0], xs, sm.p[kOffB1 + c0]));
  const float h1 = relu(fmaf(sm.p[kOffW1 + c0 + 1], xs, sm.p[kOffB1 + c0 + 1]));
  sm.h1[s * kRow + c0] = h0;
  sm.h1[s * kRow + c0 + 1] = h1;
  sm.h1t[c0 * kRowT + s] = h0;
  sm.h1t[(c0 + 1) * kRowT + s] = h1;
  wave_sync();
  // layer 2
  float a0 = sm.p[kOffB2 + c0], a1 = sm.p[kOffB2 + c0 + 1];
#pragma unroll 8
  for (int u = 0; u < kH; ++u) {
    const float2 w = *reinterpret_cast<const float2*>(&sm.w2t[u * kH + c0]);
    const float h = sm.h1[s * kRow + u];
    a0 = fmaf(w.x, h, a0);
    a1 = fmaf(w.y, h, a1);
  }
  sm.z2t[c0 * kRowT + s] = a0;
  sm.z2t[(c0 + 1) * kRowT + s] = a1;
  // output: the sixteen lanes' parts combined by shuffles; every lane takes
  // the first lane's sum, so all use one value
  float part = fmaf(sm.p[kOffW3 + c0], relu(a0), 0.0f);
  part = fmaf(sm.p[kOffW3 + c0 + 1], relu(a1), part);
  for (int d = 8; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
  part = __shfl(part, lane & ~15, 64);
  float dy = 0.0f;
  if (s < static_cast<int>(cs)) {
    float y = part + sm.p[kOffB3];
    if (residual) y = y + xs;
    const float r = y - sm.t[s];
    if ((tid & 15) == 0) g.loss = fmaf(r, r, g.loss);
    dy = 2.0f * r / static_cast<float>(batch);
  }
  if ((tid & 15) == 0) sm.dy[s] = dy;
  // dL/dz2 = dL/dy * W3, masked by the second layer's ReLU
  const float d0 = a0 > 0.0f ? dy * sm.p[kOffW3 + c0] : 0.0f;
  const float d1 = a1 > 0.0f ? dy * sm.p[kOffW3 + c0 + 1] : 0.0f;
  sm.dz2[s * kRow + c0] = d0;
  sm.dz2[s * kRow + c0 + 1] = d1;
  sm.dz2t[c0 * kRowT + s] = d0;
  sm.dz2t[(c0 + 1) * kRowT + s] = d1;
  wave_sync();
  // dL/dz1 = W2^T dL/dz2, masked by the first layer's ReLU
  {
    float e0 = 0.0f, e1 = 0.0f;
#pragma unroll 8
    for (int v = 0; v < kH; ++v) {
      const float2 w = *reinterpret_cast<const float2*>(&sm.p[kOffW2 + v * kH + c0]);
      const float d = sm.dz2[s * kRow + v];
      e0 = fmaf(w.x, d, e0);
      e1 = fmaf(w.y, d, e1);
    }
    sm.dz1t[c0 * kRowT + s] = h0 > 0.0f ? e0 : 0.0f;
    sm.dz1t[(c0 + 1) * kRowT + s] = h1 > 0.0f ? e1 : 0.0f;
  }
  lds_barrier();  // every sample's columns are in place
  // parameter gradients of the chunk, sums over samples four at a time
  {
    const int v = tid >> 5, u = tid & 31;
#pragma unroll 4
    for (int q = 0; q < static_cast<int>(kTrainChunk); q += 4) {
      const float4 d = *reinterpret_cast<const float4*>(&sm.dz2t[v * kRowT + q]);
      const float4 h = *reinterpret_cast<const float4*>(&sm.h1t[u * kRowT + q]);
      g.w2 = fmaf(d.x, h.x, g.w2);
      g.w2 = fmaf(d.y, h.y, g.w2);
      g.w2 = fmaf(d.z, h.z, g.w2);
      g.w2 = fmaf(d.w, h.w, g.w2);
    }
  }
  if (tid < 512) {
    const int o = tid >> 3, q0 = (tid & 7) * 8;
    const float* ds = o < 32 ? &sm.dz1t[o * kRowT + q0] : &sm.dz2t[(o - 32) * kRowT + q0];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float d = ds[j];
      const float w = o < 32 ? sm.x[q0 + j] : sm.dy[q0 + j];
      const float f = o < 32 ? d : relu(sm.z2t[(o - 32) * kRowT + q0 + j]);
      g.s0 = fmaf(w, f, g.s0);  // W1: dz1 * x ; W3: dy * h2
      g.s1 += d;                // b1: dz1     ; b2: dz2
    }
  } else if (tid < 520) {
    const int q0 = (tid - 512) * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j) g.s0 += sm.dy[q0 + j];
  }
  lds_barrier();
}

__device__ __forceinline__ void store_coherent(float* p, float v) {
  __hip_atomic_store(reinterpret_cast<uint32_t*>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float load_coherent(const float* p) {
  return __uint_as_float(
      __hip_atomic_load(reinterpret_cast<const uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Writes the accumulated gradient (and the loss sum at [kNParam]) to a row;
// `coherent` rows are shared with other workgroups. Every thread calls it.
__device__ void write_grad_row(TrainSmem& sm, float* row, const GradAcc& g, bool coherent) {
  const int tid = threadIdx.x;
  auto put = [&](int i, float v) {
    if (coherent) store_coherent(row + i, v);
    else row[i] = v;
  };
  put(kOffW2 + tid, g.w2);
  float a = g.s0, b = g.s1;
  for (int d = 4; d >= 1; d >>= 1) {
    a += __shfl_xor(a, d, 64);
    b += __shfl_xor(b, d, 64);
  }
  if (tid < 512 && (tid & 7) == 0) {
    const int o = tid >> 3;
    if (o < 32) {
      put(kOffW1 + o, a);
      put(kOffB1 + o, b);
    } else {
      put(kOffW3 + o - 32, a);
      put(kOffB2 + o - 32, b);
    }
  } else if (tid == 512) {
    put(kOffB3, a);
  }
  float l = g.loss;
  for (int d = 32; d >= 1; d >>= 1) l += __shfl_xor(l, d, 64);
  if (lane_id() == 0) sm.red[tid >> 6] = l;
  __syncthreads();
  if (tid == 0) {
    float tot = 0.0f;
    for (int w = 0; w < static_cast<int>(kTrainThreads / 64); ++w) tot += sm.red[w];
    put(kNParam, tot);
  }
}

// The fused trainer. Launched cooperatively: all `grid` workgroups are
// resident, so the per-step grid barrier always completes. Each workgroup
// keeps a full replica of the parameters and the Adam moments of the
// parameters its threads own; all workgroups sum the gradient partials in
// the same order, so the replicas stay identical.
__global__ __launch_bounds__(kTrainThreads) void k_train(TrainArgs a) {
  __shared__ __align__(16) TrainSmem sm;
  const int tid = threadIdx.x;
  const uint32_t wg = blockIdx.x;
  const uint32_t local = a.batch / a.grid;
  for (int i = tid; i < kNParam; i += kTrainThreads) sm.p[i] = a.init ? a.init[i] : init_value(a.seed, i);
  __syncthreads();
  if (!a.init && tid < kH) {
    const uint64_t q = ((2ull * static_cast<uint64_t>(tid) + 1ull) * a.m) / (2ull * kH);
    sm.p[kOffB1 + tid] = static_cast<float>(-(static_cast<double>(sm.p[kOffW1 + tid]) * static_cast<double>(a.x[q])));
  }
  __syncthreads();
  rebuild_w2t(sm);
  constexpr int kOwn = (kNParam + 1 + kTrainThreads - 1) / kTrainThreads;
  float am[kOwn], av[kOwn];
#pragma unroll
  for (int k = 0; k < kOwn; ++k) am[k] = av[k] = 0.0f;
  float b1t = 1.0f, b2t = 1.0f;  // beta1^step, beta2^step
  __syncthreads();

  // this thread's sample of a chunk: the minibatch positions depend only on
  // the seed and the step, so with one chunk per step the next step's
  // sample is fetched while the gradients are exchanged
  auto fetch = [&](uint32_t st, uint32_t c0, uint32_t cs, float& xv, float& tv) {
    xv = 0.0f;
    tv = 0.0f;
    if (tid < static_cast<int>(cs)) {
      const uint64_t gi = static_cast<uint64_t>(st) * a.batch + static_cast<uint64_t>(wg) * local + c0 + tid;
      const uint64_t pos = mix64(a.seed ^ (kSaltBatch + gi)) % a.m;
      xv = a.x[pos];
      tv = a.t[pos];
    }
  };
  const bool one_chunk = local <= kTrainChunk;
  float nx = 0.0f, nt = 0.0f;
  if (one_chunk && tid < static_cast<int>(kTrainChunk)) fetch(1, 0, local, nx, nt);

  bool failed = false;
  for (uint32_t step = 1; step <= a.steps; ++step) {
    GradAcc g = {0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t c0 = 0; c0 < local; c0 += kTrainChunk) {
      const uint32_t cs = local - c0 < kTrainChunk ? local - c0 : kTrainChunk;
      if (tid < static_cast<int>(kTrainChunk)) {
        float xv = nx, tv = nt;
        if (!one_chunk) fetch(step, c0, cs, xv, tv);
        sm.x[tid] = xv;
        sm.t[tid] = tv;
      }
      lds_barrier();
      chunk_grad(sm, cs, a.batch, a.residual, g);
    }
    // Gradient exchange. The partial rows are written and read with
    // agent-scope atomic stores and loads, which are performed at the
    // chip-wide coherence point (no copy of them stays in an XCD's L2), so
    // no cache maintenance is needed (agent-scope release/acquire fences
    // would write back and invalidate whole L2s every step: ~25 us a step).
    // What the exchange needs is the order "every wave's row stores have
    // completed, then lane 0 announces the workgroup". A workgroup barrier
    // alone does not give it (it orders the waves, not the completion of
    // their global stores), so every wave first waits until its own stores
    // are acknowledged (s_waitcnt with all counters at zero: vmcnt counts
    // outstanding stores too). Lane 0's increment is issued after the
    // barrier, hence after every row store completed; a reader issues its
    // row loads only after its spin has seen all `grid` increments of the
    // step, and those loads read the coherence point, so they return the
    // completed rows.
    float* rows = a.partials + static_cast<size_t>(step & 1u) * a.grid * kParamStride;
    write_grad_row(sm, rows + static_cast<size_t>(wg) * kParamStride, g, true);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (one_chunk && step < a.steps && tid < static_cast<int>(kTrainChunk)) fetch(step + 1, 0, local, nx, nt);
    if (tid == 0 && !failed) {
      __hip_atomic_fetch_add(&a.sync[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t target = a.grid * step;
      uint32_t spins = 0;
      while (__hip_atomic_load(&a.sync[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        // a barrier that does not complete (another workgroup gave up, or
        // none arrives within ~0.2 s) ends the training; the host sees the flag
        if (__hip_atomic_load(&a.sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
          failed = true;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1u << 23)) {
          atomicOr(&a.sync[1], 1u);
          failed = true;
          break;
        }
      }
    }
    __syncthreads();
    // sum the partials in workgroup order and take an Adam step
    b1t *= 0.9f;
    b2t *= 0.999f;
    const float bc1 = 1.0f - b1t, bc2 = 1.0f - b2t;
    const float ph = a.steps > 1 ? 3.14159265f * static_cast<float>(step - 1) / static_cast<float>(a.steps - 1) : 0.0f;
    const float lr = 1e-4f + 0.5f * (1e-2f - 1e-4f) * (1.0f + cosf(ph));
#pragma unroll
    for (int k = 0; k < kOwn; ++k) {
      const int i = tid + k * kTrainThreads;
      if (i > kNParam) break;
      float gs = 0.0f;
      uint32_t w = 0;
      for (; w + 8 <= a.grid; w += 8) {  // eight independent loads in flight
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = load_coherent(rows + static_cast<size_t>(w + q) * kParamStride + i);
#pragma unroll
        for (int q = 0; q < 8; ++q) gs += v[q];
      }
      for (; w < a.grid; ++w) gs += load_coherent(rows + static_cast<size_t>(w) * kParamStride + i);
      if (i == kNParam) {
        if (wg == 0) a.losses[step - 1] = gs / static_cast<float>(a.batch);
        continue;
      }
      am[k] = 0.9f * am[k] + 0.1f * gs;
      av[k] = 0.999f * av[k] + 0.001f * gs * gs;
      const float mh = am[k] / bc1, vh = av[k] / bc2;
      sm.p[i] -= lr * mh / (sqrtf(vh) + 1e-8f);
    }
    __syncthreads();
    rebuild_w2t(sm);
    __syncthreads();
  }
  if (wg == 0)
    for (int i = tid; i < kNParam; i += kTrainThreads) a.params[i] = sm.p[i];
}

// Gradient of the mean squared error over x[0..batch), t[0..batch) in one
// workgroup (the trainer's arithmetic without the optimiser).
__global__ __launch_bounds__(kTrainThreads) void k_gradient(const float* __restrict__ params,
                                                            const float* __restrict__ x,
                                                            const float* __restrict__ t, uint32_t batch,
                                                            uint32_t residual, float* grad, float* loss) {
  __shared__ __align__(16) TrainSmem sm;
  __shared__ float s_row[kParamStride];
  const int tid = threadIdx.x;
  for (int i = tid; i < kNParam; i += kTrainThreads) sm.p[i] = params[i];
  __syncthreads();
  rebuild_w2t(sm);
  __syncthreads();
  GradAcc g = {0.0f, 0.0f, 0.0f, 0.0f};
  for (uint32_t c0 = 0; c0 < batch; c0 += kTrainChunk) {
    const uint32_t cs = batch - c0 < kTrainChunk ? batch - c0 : kTrainChunk;
    if (tid < static_cast<int>(kTrainChunk)) {
      sm.x[tid] = tid < static_cast<int>(cs) ? x[c0 + tid] : 0.0f;
      sm.t[tid] = tid < static_cast<int>(cs) ? t[c0 + tid] : 0.0f;
    }
    lds_barrier();
    chunk_grad(sm, cs, batch, residual, g);
  }
  write_grad_row(sm, s_row, g, false);
  __syncthreads();
  for (int i = tid; i < kNParam; i += kTrainThreads) grad[i] = s_row[i];
  if (tid == 0) *loss = s_row[kNParam] / static_cast<float>(batch);
}

// ---------------------------------------------------------------- inference

__global__ __launch_bounds__(256) void k_infer(const float* __restrict__ p, const float* __restrict__ x, uint64_t m,
                                               uint32_t residual, float* __restrict__ y) {
  const uint64_t j = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x;
  if (j >= m) return;
  const float xv = x[j];
  float h1[kH];
#pragma unroll
  for (int u = 0; u < kH; ++u) h1[u] = relu(fmaf(p[kOffW1 + u], xv, p[kOffB1 + u]));
  float out = p[kOffB3];
  for (int v = 0; v < kH; ++v) {
    float acc = p[kOffB2 + v];
#pragma unroll
    for (int u = 0; u < kH; ++u) acc = fmaf(p[kOffW2 + v * kH + u], h1[u], acc);
    out = fmaf(p[kOffW3 + v], relu(acc), out);
  }
  if (residual) out = out + xv;
  y[j] = out < 0.0f ? 0.0f : (out > 1.0f ? 1.0f : out);
}

// ---------------------------------------------------------------- splitters

constexpr uint32_t kExtractThreads = 1024;

// One extraction per workgroup: prediction, its running maximum, the
// splitters and their count.
struct ExtractJob {
  const float* y;
  float* r;
  uint64_t* sp;
  uint32_t* count;
};
struct ExtractJobs {
  ExtractJob job[kCandidates];
};

__global__ __launch_bounds__(kExtractThreads) void k_extract(const uint64_t* __restrict__ s, uint64_t m,
                                                             ExtractJobs jobs) {
  __shared__ float s_max[kExtractThreads];
  __shared__ uint64_t s_cand[kMaxSplitters];
  __shared__ uint32_t s_valid[kMaxSplitters];
  __shared__ uint32_t s_keep[256];
  const ExtractJob J = jobs.job[blockIdx.x];
  const float* __restrict__ y = J.y;
  float* r = J.r;
  uint64_t* __restrict__ sp = J.sp;
  uint32_t* count = J.count;
  const uint32_t tid = threadIdx.x;
  const uint64_t per = (m + kExtractThreads - 1) / kExtractThreads;
  const uint64_t b = tid * per < m ? tid * per : m;
  const uint64_t e = b + per < m ? b + per : m;
  float mx = 0.0f;  // predictions are clamped to [0, 1]
#pragma unroll 16
  for (uint64_t i = b; i < e; ++i) mx = y[i] > mx ? y[i] : mx;
  s_max[tid] = mx;
  __syncthreads();
  for (uint32_t d = 1; d < kExtractThreads; d <<= 1) {
    const float o = tid >= d ? s_max[tid - d] : 0.0f;
    __syncthreads();
    s_max[tid] = o > s_max[tid] ? o : s_max[tid];
    __syncthreads();
  }
  float run = tid > 0 ? s_max[tid - 1] : 0.0f;
  // 16 loads of y, then their 16 running maxima: stores to r (another
  // buffer, which the compiler cannot tell) would otherwise hold back each
  // next load
  for (uint64_t i0 = b; i0 < e; i0 += 16) {
    float v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = y[i0 + q < e ? i0 + q : e - 1];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (i0 + q < e) {
        run = v[q] > run ? v[q] : run;
        r[i0 + q] = run;
      }
    }
  }
  __threadfence_block();
  __syncthreads();
  // candidate k: the heavy key at the k-th sample quantile, else the first
  // crossing of k/256 by the running maximum
  if (tid < kMaxSplitters) {
    const uint64_t q = (static_cast<uint64_t>(tid + 1) * m) / 256u;
    const uint64_t key = s[q];
    // [first, last): the run of key in the sorted sample; the searches are
    // skipped when a neighbour already shows the run is q alone
    uint64_t first = q, last = q + 1;
    if (q > 0 && s[q - 1] == key) {
      uint64_t lo = 0, hi = q;
      while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (s[mid] < key) lo = mid + 1;
        else hi = mid;
      }
      first = lo;
    }
    if (q + 1 < m && s[q + 1] == key) {
      uint64_t lo = q + 1, hi = m;
      while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (s[mid] <= key) lo = mid + 1;
        else hi = mid;
      }
      last = lo;
    }
    const bool heavy = (last - first) * 256u >= m;
    uint64_t idx = q;
    if (!heavy) {
      // first i with r[i] >= thr: the first lane block whose running
      // maximum reaches thr (s_max holds them, in LDS), then inside it
      const float thr = static_cast<float>(tid + 1) / 256.0f;
      uint32_t tlo = 0, thi = kExtractThreads;
      while (tlo < thi) {
        const uint32_t mid = (tlo + thi) >> 1;
        if (s_max[mid] < thr) tlo = mid + 1;
        else thi = mid;
      }
      uint64_t lo = m, hi = m;
      if (tlo < kExtractThreads) {
        lo = static_cast<uint64_t>(tlo) * per < m ? static_cast<uint64_t>(tlo) * per : m;
        hi = lo + per < m ? lo + per : m;
      }
      while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (r[mid] < thr) lo = mid + 1;
        else hi = mid;
      }
      idx = lo;
    }
    s_valid[tid] = idx < m ? 1u : 0u;
    s_cand[tid] = idx < m ? s[idx] : 0ull;
  }
  __syncthreads();
  // sorted distinct candidates: a candidate is kept at its first occurrence,
  // then written at its rank among the kept ones
  uint32_t keep = 0;
  uint64_t mine = 0;
  if (tid < kMaxSplitters && s_valid[tid]) {
    mine = s_cand[tid];
    keep = 1;
    for (uint32_t j = 0; j < tid; ++j)
      if (s_valid[j] && s_cand[j] == mine) keep = 0;
  }
  if (tid < 256) s_keep[tid] = keep;
  __syncthreads();
  if (keep) {
    uint32_t rank = 0;
    for (uint32_t j = 0; j < kMaxSplitters; ++j) rank += (s_keep[j] && s_cand[j] < mine) ? 1u : 0u;
    sp[rank] = mine;
  }
  if (tid == 0) {
    uint32_t u = 0;
    for (uint32_t k = 0; k < kMaxSplitters; ++k) u += s_keep[k];
    *count = u;
  }
}

// ---------------------------------------------------------------- leaves

// Running maximum r of y[0..m) (one workgroup: per-lane block maxima, a scan
// over the lanes, then each lane's block; a maximum is exact in any order).
__global__ __launch_bounds__(kExtractThreads) void k_running_max(const float* __restrict__ y, uint64_t m,
                                                                 float* __restrict__ r) {
  __shared__ float s_max[kExtractThreads];
  const uint32_t tid = threadIdx.x;
  const uint64_t per = (m + kExtractThreads - 1) / kExtractThreads;
  const uint64_t b = tid * per < m ? tid * per : m;
  const uint64_t e = b + per < m ? b + per : m;
  float mx = 0.0f;
#pragma unroll 16
  for (uint64_t i = b; i < e; ++i) mx = y[i] > mx ? y[i] : mx;
  s_max[tid] = mx;
  __syncthreads();
  for (uint32_t d = 1; d < kExtractThreads; d <<= 1) {
    const float o = tid >= d ? s_max[tid - d] : 0.0f;
    __syncthreads();
    s_max[tid] = o > s_max[tid] ? o : s_max[tid];
    __syncthreads();
  }
  float run = tid > 0 ? s_max[tid - 1] : 0.0f;
#pragma unroll 16
  for (uint64_t i = b; i < e; ++i) {
    run = y[i] > run ? y[i] : run;
    r[i] = run;
  }
}

// One lane per (kind, leaf): kind 0 fits t = a + b x, kind 1 t = a + b y
// (y the clamped prediction) over the samples of leaf j, those whose running
// maximum r of y satisfies floor(64 r) == j (the last leaf also takes
// r == 1). Sums run in index order in double: a float times a float is
// exact in double, so only the additions round, as in the oracle.
// Contraction is off: k * sum u^2 - (sum u)^2 fused into one rounding would
// differ from the oracle's two, and this difference of two large sums is
// where the rounding shows.
__global__ __launch_bounds__(2 * kLeaves) void k_leaf_fit(const float* __restrict__ x, const float* __restrict__ t,
                                                          const float* __restrict__ y, const float* __restrict__ r,
                                                          uint64_t m, double* __restrict__ leaf) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x;
  const int kind = lane / kLeaves, j = lane % kLeaves;
  auto first_at_least = [&](float thr) {
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (r[mid] < thr) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  const uint64_t lo = first_at_least(static_cast<float>(j) / static_cast<float>(kLeaves));
  const uint64_t hi = j == kLeaves - 1 ? m : first_at_least(static_cast<float>(j + 1) / static_cast<float>(kLeaves));
  const float* u = kind == 0 ? x : y;
  double sx = 0.0, st = 0.0, sxx = 0.0, sxt = 0.0;
  // sixteen samples' loads in flight at a time; the sums still run in index order
  constexpr int kBatch = 16;
  uint64_t i = lo;
  for (; i + kBatch <= hi; i += kBatch) {
    float ub[kBatch], tb[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      ub[q] = u[i + q];
      tb[q] = t[i + q];
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const double ui = static_cast<double>(ub[q]), ti = static_cast<double>(tb[q]);
      sx = sx + ui;
      st = st + ti;
      sxx = sxx + ui * ui;
      sxt = sxt + ui * ti;
    }
  }
  for (; i < hi; ++i) {
    const double ui = static_cast<double>(u[i]), ti = static_cast<double>(t[i]);
    sx = sx + ui;
    st = st + ti;
    sxx = sxx + ui * ui;
    sxt = sxt + ui * ti;
  }
  const uint64_t cnt = hi > lo ? hi - lo : 0;
  const double k = static_cast<double>(cnt);
  const double den = k * sxx - sx * sx;
  double a, b;
  if (cnt < 2 || !(den > 0.0)) {
    b = 0.0;
    a = cnt ? st / k : 0.0;
  } else {
    b = (k * sxt - sx * st) / den;
    a = (st - b * sx) / k;
  }
  leaf[(kind * kLeaves + j) * 2] = a;
  leaf[(kind * kLeaves + j) * 2 + 1] = b;
}

// Leaf predictions of every sample: (float)(a + b u) of its leaf.
__global__ __launch_bounds__(256) void k_leaf_eval(const float* __restrict__ x, const float* __restrict__ y,
                                                   const float* __restrict__ r, uint64_t m,
                                                   const double* __restrict__ leaf, float* __restrict__ yx,
                                                   float* __restrict__ yy) {
#pragma clang fp contract(off)
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256u + threadIdx.x;
  if (i >= m) return;
  int j = static_cast<int>(r[i] * static_cast<float>(kLeaves));  // exact scaling, then floor (r >= 0)
  j = j < kLeaves - 1 ? j : kLeaves - 1;
  yx[i] = static_cast<float>(leaf[j * 2] + leaf[j * 2 + 1] * static_cast<double>(x[i]));
  yy[i] = static_cast<float>(leaf[(kLeaves + j) * 2] + leaf[(kLeaves + j) * 2 + 1] * static_cast<double>(y[i]));
}

// ---------------------------------------------------------------- judge on the sample

__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t* s, uint64_t m, uint64_t v) {
  uint64_t lo = 0, hi = m;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (s[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ uint64_t upper_bound_u64(const uint64_t* s, uint64_t m, uint64_t v) {
  uint64_t lo = 0, hi = m;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (s[mid] <= v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Workgroup c: the largest number of sorted sample keys in one range bin of
// candidate c's splitters (range bin b holds the keys strictly between
// splitters b - 1 and b).
__global__ __launch_bounds__(256) void k_sample_judge(const uint64_t* __restrict__ s, uint64_t m,
                                                      const uint64_t* __restrict__ sp, uint32_t stride,
                                                      const uint32_t* __restrict__ count, uint64_t* est) {
  __shared__ uint64_t s_max[256];
  const uint32_t c = blockIdx.x, b = threadIdx.x;
  const uint64_t* cs = sp + static_cast<uint64_t>(c) * stride;
  const uint32_t u = count[c];
  uint64_t v = 0;
  if (b <= u) {
    const uint64_t end = b < u ? lower_bound_u64(s, m, cs[b]) : m;
    const uint64_t begin = b > 0 ? upper_bound_u64(s, m, cs[b - 1]) : 0;
    v = end > begin ? end - begin : 0;
  }
  s_max[b] = v;
  __syncthreads();
  for (uint32_t d = 128; d > 0; d >>= 1) {
    if (b < d) s_max[b] = s_max[b + d] > s_max[b] ? s_max[b + d] : s_max[b];
    __syncthreads();
  }
  if (b == 0) est[c] = s_max[0];
}

// The candidate with the smallest sample judge (the first on ties) becomes
// the fit's splitters; info[3] = its index, info[4 + c] = judge of c,
// info[7] = 1 when the winner's judge is at most `go_limit` (the histogram
// runs only then).
__global__ __launch_bounds__(256) void k_pick(const uint64_t* __restrict__ sp, uint32_t stride,
                                              const uint32_t* __restrict__ count, const uint64_t* __restrict__ est,
                                              uint32_t ncand, uint64_t go_limit, uint64_t* out, uint32_t* out_count,
                                              uint64_t* info) {
  uint32_t best = 0;
  for (uint32_t c = 1; c < ncand; ++c)
    if (est[c] < est[best]) best = c;
  const uint32_t u = count[best];
  for (uint32_t i = threadIdx.x; i < u; i += blockDim.x) out[i] = sp[static_cast<uint64_t>(best) * stride + i];
  if (threadIdx.x == 0) {
    *out_count = u;
    info[3] = best;
    for (uint32_t c = 0; c < ncand; ++c) info[4 + c] = est[c];
    info[7] = est[best] <= go_limit ? 1u : 0u;
  }
}

template <class K>
struct SampleL {
  static hipError_t run(const void* keys, uint64_t n, uint64_t m, uint64_t seed, uint64_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sample<K>, dim3(static_cast<uint32_t>((m + 255) / 256)), dim3(256), 0, s,
                       static_cast<const typename K::T*>(keys), n, m, seed, out);
    return hipGetLastError();
  }
};

}  // namespace

hipError_t launch_sample(uint32_t kt, const void* keys, uint64_t n, uint64_t m, uint64_t seed, uint64_t* out,
                         hipStream_t s) {
  switch (kt) {
    case 1: return SampleL<KeyU32>::run(keys, n, m, seed, out, s);
    case 2: return SampleL<KeyI32>::run(keys, n, m, seed, out, s);
    case 3: return SampleL<KeyF32>::run(keys, n, m, seed, out, s);
    case 4: return SampleL<KeyU64>::run(keys, n, m, seed, out, s);
    case 5: return SampleL<KeyI64>::run(keys, n, m, seed, out, s);
    case 6: return SampleL<KeyF64>::run(keys, n, m, seed, out, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sample_sort(uint64_t* raw, uint64_t m, uint64_t* sorted, hipStream_t s) {
  if (m % kChunk) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chunk_bitonic, dim3(static_cast<uint32_t>(m / kChunk)), dim3(kChunkThreads), 0, s, raw);
  hipLaunchKernelGGL(k_rank_merge, dim3(static_cast<uint32_t>((m + 255) / 256)), dim3(256), 0, s, raw, m, sorted);
  return hipGetLastError();
}

hipError_t launch_features(const uint64_t* sorted, uint64_t m, float* x, float* t, uint64_t* info, hipStream_t s) {
  const uint32_t blocks = static_cast<uint32_t>((m + 255) / 256);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, info, 4u);
  hipLaunchKernelGGL(k_feat_dev, dim3(blocks), dim3(256), 0, s, sorted, m, info);
  hipLaunchKernelGGL(k_feat_out, dim3(blocks), dim3(256), 0, s, sorted, m, info, x, t);
  return hipGetLastError();
}

hipError_t launch_train(const TrainArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, a.sync, 4u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  TrainArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_train), dim3(a.grid), dim3(kTrainThreads), args,
                                    0, s);
}

hipError_t launch_gradient(const float* params, const float* x, const float* t, uint32_t batch, uint32_t residual,
                           float* grad, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_gradient, dim3(1), dim3(kTrainThreads), 0, s, params, x, t, batch, residual, grad, loss);
  return hipGetLastError();
}

hipError_t launch_infer(const float* params, const float* x, uint64_t m, uint32_t residual, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_infer, dim3(static_cast<uint32_t>((m + 255) / 256)), dim3(256), 0, s, params, x, m, residual,
                     y);
  return hipGetLastError();
}

hipError_t launch_extract(const uint64_t* sorted, const float* y, uint64_t m, float* runmax, uint64_t* splitters,
                          uint32_t* count, hipStream_t s) {
  ExtractJobs jobs = {};
  jobs.job[0] = ExtractJob{y, runmax, splitters, count};
  hipLaunchKernelGGL(k_extract, dim3(1), dim3(kExtractThreads), 0, s, sorted, m, jobs);
  return hipGetLastError();
}

hipError_t launch_extract_candidates(const uint64_t* sorted, uint64_t m, const float* const* y, float* const* runmax,
                                     uint64_t* splitters, uint32_t stride, uint32_t* count, hipStream_t s) {
  ExtractJobs jobs = {};
  for (int c = 0; c < kCandidates; ++c)
    jobs.job[c] = ExtractJob{y[c], runmax[c], splitters + static_cast<uint64_t>(c) * stride, count + c};
  hipLaunchKernelGGL(k_extract, dim3(kCandidates), dim3(kExtractThreads), 0, s, sorted, m, jobs);
  return hipGetLastError();
}

}  // namespace pdq

namespace pdq {

hipError_t launch_running_max(const float* y, uint64_t m, float* runmax, hipStream_t s) {
  hipLaunchKernelGGL(k_running_max, dim3(1), dim3(kExtractThreads), 0, s, y, m, runmax);
  return hipGetLastError();
}

hipError_t launch_leaves(const float* x, const float* t, const float* y, const float* runmax, uint64_t m,
                         double* leaf, float* yx, float* yy, hipStream_t s) {
  hipLaunchKernelGGL(k_leaf_fit, dim3(1), dim3(2 * kLeaves), 0, s, x, t, y, runmax, m, leaf);
  hipLaunchKernelGGL(k_leaf_eval, dim3(static_cast<uint32_t>((m + 255) / 256)), dim3(256), 0, s, x, y, runmax, m,
                     leaf, yx, yy);
  return hipGetLastError();
}

hipError_t launch_sample_judge(const uint64_t* sorted, uint64_t m, const uint64_t* splitters, uint32_t stride,
                               const uint32_t* count, uint32_t ncand, uint64_t* est, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_judge, dim3(ncand), dim3(256), 0, s, sorted, m, splitters, stride, count, est);
  return hipGetLastError();
}

hipError_t launch_pick(const uint64_t* splitters, uint32_t stride, const uint32_t* count, const uint64_t* est,
                       uint32_t ncand, uint64_t go_limit, uint64_t* out, uint32_t* out_count, uint64_t* info,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_pick, dim3(1), dim3(256), 0, s, splitters, stride, count, est, ncand, go_limit, out, out_count,
                     info);
  return hipGetLastError();
}

}  // namespace pdq
