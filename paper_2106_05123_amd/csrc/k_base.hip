// LDS-resident base case: every segment of at most 4096 keys is sorted by
// one workgroup and written to its final place in the user buffer.
//
// The paper sorts small subsequences with insertion sort (Section 5.1) and
// notes that sorting networks lost on its CPU through code size (Section 2);
// on a GPU a bitonic network (bitonic.h) is the natural small sort. A
// segment of P = E * NT slots (padded to a power of two) is held E slots per
// lane in registers; payloads are gathered by index at the end.
#include "bitonic.h"
#include "pdq_internal.h"
#include "wave_ops.h"

namespace pdq {
namespace {

using net::ilog2;
using net::lds_plane;
using net::lds_pos;
using net::Slot;

// One workgroup per base-case segment of at most E * NT keys.
template <class K, bool PAIRS, int E, int NT>
__global__ __launch_bounds__(NT) void k_base(Ctx c, int cls) {
  using T = typename K::T;
  using S = Slot<K, PAIRS>;
  using V = typename S::V;
  constexpr int P = E * NT;
  constexpr int PL = lds_plane<P, E>();
  __shared__ __align__(16) unsigned char sh[PL * S::kLdsBytes];
  if (c.device_counts && blockIdx.x >= c.ctr->nbase[cls]) return;
  const Item it = c.base[cls][blockIdx.x];
  const int len = static_cast<int>(it.end - it.begin);
  const int tid = threadIdx.x;
  const T* in = static_cast<const T*>(c.keys[it.buf]) + it.begin;

  // coalesced load into LDS, then each lane picks up its E consecutive slots
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int j = r * NT + tid;
    S::st(sh, PL, lds_pos<E>(j), j < len ? S::make(in[j], static_cast<uint32_t>(j)) : S::pad());
  }
  __syncthreads();
  V x[E];
#pragma unroll
  for (int r = 0; r < E; ++r) x[r] = S::ld(sh, PL, lds_pos<E>((tid << ilog2(E)) | r));
  __syncthreads();

  if constexpr (E * NT >= 1024) net::merge_sort<S, E, NT>(x, sh, tid);
  else net::bitonic<S, E, NT>(x, sh, tid);

  // back through LDS so that the final writes are coalesced
#pragma unroll
  for (int r = 0; r < E; ++r) S::st(sh, PL, lds_pos<E>((tid << ilog2(E)) | r), x[r]);
  __syncthreads();
  V y[E];
#pragma unroll
  for (int r = 0; r < E; ++r) y[r] = S::ld(sh, PL, lds_pos<E>(r * NT + tid));
  T* out = static_cast<T*>(c.keys[0]) + it.begin;
  if constexpr (PAIRS) {
    // gather every payload before anything is written: the segment may be
    // sorted in place, in the buffer the payloads are read from
    const uint32_t* vin = c.vals[it.buf] + it.begin;
    uint32_t pv[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int j = r * NT + tid;
      pv[r] = j < len ? vin[S::idx(y[r])] : 0u;
    }
    __syncthreads();
    uint32_t* vout = c.vals[0] + it.begin;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int j = r * NT + tid;
      if (j < len) {
        out[j] = S::key(y[r]);
        vout[j] = pv[r];
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int j = r * NT + tid;
      if (j < len) out[j] = S::key(y[r]);
    }
  }
}

template <class K, bool PAIRS>
hipError_t launch_cls(const Ctx& c, int cls, uint32_t nitems, hipStream_t s) {
  switch (cls) {
    case 0: hipLaunchKernelGGL((k_base<K, PAIRS, 1, 64>), dim3(nitems), dim3(64), 0, s, c, cls); break;
    case 1: hipLaunchKernelGGL((k_base<K, PAIRS, 4, 64>), dim3(nitems), dim3(64), 0, s, c, cls); break;
    case 2: hipLaunchKernelGGL((k_base<K, PAIRS, 16, 64>), dim3(nitems), dim3(64), 0, s, c, cls); break;
    case 3: hipLaunchKernelGGL((k_base<K, PAIRS, 16, 128>), dim3(nitems), dim3(128), 0, s, c, cls); break;
    case 4: hipLaunchKernelGGL((k_base<K, PAIRS, 16, 256>), dim3(nitems), dim3(256), 0, s, c, cls); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class K>
hipError_t launch_kp(const Ctx& c, int cls, uint32_t nitems, hipStream_t s) {
  return c.has_vals ? launch_cls<K, true>(c, cls, nitems, s) : launch_cls<K, false>(c, cls, nitems, s);
}

}  // namespace

hipError_t launch_base(const Ctx& c, int cls, uint32_t nitems, hipStream_t s) {
  switch (c.key_type) {
    case 1: return launch_kp<KeyU32>(c, cls, nitems, s);
    case 2: return launch_kp<KeyI32>(c, cls, nitems, s);
    case 3: return launch_kp<KeyF32>(c, cls, nitems, s);
    case 4: return launch_kp<KeyU64>(c, cls, nitems, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdq
