// LDS-resident base case: every segment of at most 4096 keys is sorted by
// one workgroup in LDS and written to its final place in the user buffer.
//
// The paper sorts small subsequences with insertion sort (Section 5.1) and
// notes that sorting networks lost on its CPU through code size (Section 2);
// on a GPU a workgroup-wide bitonic network is the natural small sort. Each
// key is paired with its index inside the segment, so padding entries
// (index >= size) sort after every real key, including real maximal keys,
// and payloads are fetched by index afterwards.
#include "pdq_internal.h"

namespace pdq {
namespace {

constexpr int kBaseThreads = 256;

__device__ __forceinline__ uint32_t next_pow2(uint32_t x) { return x <= 1 ? 1u : 1u << (32 - __clz(x - 1)); }

// 32-bit keys: (canonical key << 32 | index) sorts as one 64-bit integer.
template <class K, bool PAIRS>
__global__ __launch_bounds__(kBaseThreads) void k_base32(Ctx c) {
  __shared__ uint64_t s[kBaseMax];
  __shared__ uint32_t sv[PAIRS ? kBaseMax : 1];
  const Item it = c.base[blockIdx.x];
  const uint32_t len = static_cast<uint32_t>(it.end - it.begin);
  const uint32_t P = next_pow2(len);
  const uint32_t* in = static_cast<const uint32_t*>(c.keys[it.buf]) + it.begin;
  const uint32_t* inv = PAIRS ? c.vals[it.buf] + it.begin : nullptr;
  for (uint32_t j = threadIdx.x; j < P; j += kBaseThreads) {
    if (j < len) {
      s[j] = (static_cast<uint64_t>(K::ord(in[j])) << 32) | j;
      if (PAIRS) sv[j] = inv[j];
    } else {
      s[j] = ~0ull;
    }
  }
  __syncthreads();
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t t = threadIdx.x; t < P / 2; t += kBaseThreads) {
        const uint32_t lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const uint32_t hi = lo | j;
        const bool up = (lo & k) == 0;
        const uint64_t a = s[lo], b = s[hi];
        if ((a > b) == up) {
          s[lo] = b;
          s[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  uint32_t* out = static_cast<uint32_t*>(c.keys[0]) + it.begin;
  uint32_t* outv = PAIRS ? c.vals[0] + it.begin : nullptr;
  for (uint32_t j = threadIdx.x; j < len; j += kBaseThreads) {
    const uint64_t x = s[j];
    out[j] = K::inv(static_cast<uint32_t>(x >> 32));
    if (PAIRS) outv[j] = sv[static_cast<uint32_t>(x)];
  }
}

// 64-bit keys: keys and indices in two arrays, compared lexicographically.
template <class K, bool PAIRS>
__global__ __launch_bounds__(kBaseThreads) void k_base64(Ctx c) {
  __shared__ uint64_t s[kBaseMax];
  __shared__ uint16_t si[kBaseMax];
  __shared__ uint32_t sv[PAIRS ? kBaseMax : 1];
  const Item it = c.base[blockIdx.x];
  const uint32_t len = static_cast<uint32_t>(it.end - it.begin);
  const uint32_t P = next_pow2(len);
  const uint64_t* in = static_cast<const uint64_t*>(c.keys[it.buf]) + it.begin;
  const uint32_t* inv = PAIRS ? c.vals[it.buf] + it.begin : nullptr;
  for (uint32_t j = threadIdx.x; j < P; j += kBaseThreads) {
    if (j < len) {
      s[j] = K::ord(in[j]);
      si[j] = static_cast<uint16_t>(j);
      if (PAIRS) sv[j] = inv[j];
    } else {
      s[j] = ~0ull;
      si[j] = static_cast<uint16_t>(j);
    }
  }
  __syncthreads();
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t t = threadIdx.x; t < P / 2; t += kBaseThreads) {
        const uint32_t lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const uint32_t hi = lo | j;
        const bool up = (lo & k) == 0;
        const uint64_t a = s[lo], b = s[hi];
        const uint16_t ia = si[lo], ib = si[hi];
        const bool gt = a > b || (a == b && ia > ib);
        if (gt == up) {
          s[lo] = b;
          s[hi] = a;
          si[lo] = ib;
          si[hi] = ia;
        }
      }
      __syncthreads();
    }
  }
  uint64_t* out = static_cast<uint64_t*>(c.keys[0]) + it.begin;
  uint32_t* outv = PAIRS ? c.vals[0] + it.begin : nullptr;
  for (uint32_t j = threadIdx.x; j < len; j += kBaseThreads) {
    out[j] = K::inv(s[j]);
    if (PAIRS) outv[j] = sv[si[j]];
  }
}

template <class K, bool PAIRS>
hipError_t launch_k(const Ctx& c, uint32_t nitems, hipStream_t s) {
  if constexpr (sizeof(typename K::T) == 4)
    hipLaunchKernelGGL((k_base32<K, PAIRS>), dim3(nitems), dim3(kBaseThreads), 0, s, c);
  else
    hipLaunchKernelGGL((k_base64<K, PAIRS>), dim3(nitems), dim3(kBaseThreads), 0, s, c);
  return hipGetLastError();
}

template <class K>
hipError_t launch_kp(const Ctx& c, uint32_t nitems, hipStream_t s) {
  return c.has_vals ? launch_k<K, true>(c, nitems, s) : launch_k<K, false>(c, nitems, s);
}

}  // namespace

hipError_t launch_base(const Ctx& c, uint32_t nitems, hipStream_t s) {
  switch (c.key_type) {
    case 1: return launch_kp<KeyU32>(c, nitems, s);
    case 2: return launch_kp<KeyI32>(c, nitems, s);
    case 3: return launch_kp<KeyF32>(c, nitems, s);
    case 4: return launch_kp<KeyU64>(c, nitems, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdq
