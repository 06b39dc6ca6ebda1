// LDS-resident base case: every segment of at most 4096 keys (16384 in the
// batched form) is sorted by one workgroup and written to its final place in
// the user buffer.
//
// The paper sorts small subsequences with insertion sort (Section 5.1) and
// notes that sorting networks lost on its CPU through code size (Section 2).
// Here a segment of P = E * NT slots (padded to a power of two) is held E
// slots per lane in registers and sorted in one workgroup (bitonic.h): a
// bitonic network below 1024 slots; from 2048 slots an LDS bucket sort when
// the keys spread over their range (a segment between two pivots usually
// does), else, and from 1024 slots, a merge sort. Payloads are gathered by
// index at the end.
#include "bitonic.h"
#include "pdq_internal.h"
#include "wave_ops.h"

namespace pdq {
namespace {

using net::ilog2;
using net::lds_plane;
using net::lds_pos;
using net::Slot;

// Smallest block (E * NT slots) that tries the bucket sort before the merge
// sort: segments that reach the base case lie between two pivots, so their
// keys usually spread over their range and the buckets come out even.
constexpr int kBucketMinSlots = 2048;

// One workgroup per base-case segment of at most E * NT keys; a workgroup
// takes items blockIdx.x, blockIdx.x + gridDim.x, ... of its class list
// (the list length comes from the device counters in the batched form).
template <class K, bool PAIRS, int E, int NT>
__global__ __launch_bounds__(NT) void k_base(Ctx c, int cls, uint32_t nitems) {
  using T = typename K::T;
  using S = Slot<K, PAIRS>;
  using V = typename S::V;
  constexpr int P = E * NT;
  constexpr int PL = lds_plane<P, E>();
  constexpr bool kBucket = S::kBucket && P >= kBucketMinSlots;
  // the bucket sort's finish: sorted lane runs and neighbour merges without
  // a payload, the in-bucket rank count (one compare a member) with one;
  // with 8 slots a lane the network finish would cap buckets at 8 keys,
  // which evenly spread keys overflow too often
  constexpr bool kBucketNet = !PAIRS && E >= 16;
  __shared__ __align__(16) unsigned char sh[PL * S::kLdsBytes];
  __shared__ __align__(8) uint32_t bk[kBucket ? net::bucket_words<P, NT>() : 1];
  // a list longer than its capacity (only invalid offsets make one; it is
  // flagged) is read no further than its capacity
  uint32_t count = c.device_counts ? c.icnt[cls] : nitems;
  if (count > c.max_items) count = c.max_items;
  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
    // an opaque copy of the lane index keeps the per-slot addresses inside
    // the loop instead of holding dozens of them in registers across items
    int tid = static_cast<int>(threadIdx.x);
    asm volatile("" : "+v"(tid));
    const Item it = c.base[cls][item];
    const int len = static_cast<int>(it.end - it.begin);
    if (len < 1) continue;  // never pushed; the loads below read position len - 1
    const T* in = static_cast<const T*>(c.keys[it.buf]) + it.begin;

    // coalesced load straight into registers: x[r] is segment position
    // r * NT + tid (the sorts below take their slots in any arrangement).
    // Every lane loads (positions past the end read the last key and are
    // replaced by padding), so the E loads are in flight together.
    V x[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int j = r * NT + tid;
      const V v = S::make(in[j < len ? j : len - 1], static_cast<uint32_t>(j));
      x[r] = S::sel(j < len, v, S::pad());
    }

    // the sorts leave lane tid holding places [tid * E, tid * E + E) in its
    // registers, which go back through the padded LDS layout; the bucket
    // sort's rank-count finish leaves a plain array in LDS instead
    int res = net::kBkFailed;
    if constexpr (kBucket) res = net::bucket_sort<S, E, NT, kBucketNet>(x, sh, bk, tid, len);
    if (res != net::kBkInLds) {
      if (res == net::kBkFailed) {
        if constexpr (P >= 1024) net::merge_sort<S, E, NT>(x, sh, tid);
        else net::bitonic<S, E, NT>(x, sh, tid);
      }
      // back through LDS so that the final writes are coalesced
#pragma unroll
      for (int r = 0; r < E; ++r) S::st(sh, PL, lds_pos<E>((tid << ilog2(E)) | r), x[r]);
      __syncthreads();
    }
    V y[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int j = r * NT + tid;
      if constexpr (kBucket && !kBucketNet)
        y[r] = res == net::kBkInLds ? reinterpret_cast<const V*>(sh)[j] : S::ld(sh, PL, lds_pos<E>(j));
      else
        y[r] = S::ld(sh, PL, lds_pos<E>(j));
    }
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
    __syncthreads();  // LDS is rewritten by the next item
  }
}

// Workgroups of a device-counted base-case launch, per workgroup the
// occupancy query allows on a CU. Workgroups take the list's items by
// index and depend on nothing else, so a grid larger than what is resident
// only queues; four times the query's answer measured slightly faster than
// once (learned 2^28 sort 10.15 -> 10.06 ms, batched graph 9.64 -> 9.56 ms).
constexpr int kBaseOversub = 4;

// Workgroups of a base-case launch: one per item, or, with device counts,
// as many as the device holds at once (each then loops over the list).
template <class F>
uint32_t base_grid(F* f, int nt, uint32_t nitems, bool device_counts) {
  if (!device_counts) return nitems;
  static thread_local int dev_cached = -1;
  static thread_local int cus = 256;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev != dev_cached) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    dev_cached = dev;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, nt, 0) != hipSuccess || per_cu <= 0) per_cu = 1;
  const uint64_t g = static_cast<uint64_t>(per_cu) * kBaseOversub * cus;
  return static_cast<uint32_t>(g < nitems ? g : nitems);
}

template <class K, bool PAIRS, int E, int NT>
hipError_t launch_shape(const Ctx& c, int cls, uint32_t nitems, hipStream_t s) {
  const uint32_t grid = base_grid(k_base<K, PAIRS, E, NT>, NT, nitems, c.device_counts != 0);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_base<K, PAIRS, E, NT>), dim3(grid), dim3(NT), 0, s, c, cls, nitems);
  return hipGetLastError();
}

template <class K, bool PAIRS, int P, int NT>
hipError_t launch_lanes(const Ctx& c, int cls, uint32_t nitems, hipStream_t s) {
  return launch_shape<K, PAIRS, P / NT, NT>(c, cls, nitems, s);
}

// The class's workgroup shape from its variant (kBaseThreads): every shape
// a class can take is instantiated here.
template <class K, bool PAIRS>
hipError_t launch_cls(const Ctx& c, int cls, uint32_t nitems, hipStream_t s) {
  // 64-bit keys with a payload hold three registers a slot: at most 8 slots
  // per lane keep them out of the register limit that 16 would hit
  constexpr bool kWidePairs = sizeof(typename K::T) == 8 && PAIRS;
  const int nt = base_threads(kWidePairs, cls, c.base_var[cls]);
  switch (cls) {
    case 0: return launch_lanes<K, PAIRS, 64, 64>(c, cls, nitems, s);
    case 1:
      if (nt == 128) return launch_lanes<K, PAIRS, 256, 128>(c, cls, nitems, s);
      if (nt == 256) return launch_lanes<K, PAIRS, 256, 256>(c, cls, nitems, s);
      return launch_lanes<K, PAIRS, 256, 64>(c, cls, nitems, s);
    case 2:
      if (nt == 256) return launch_lanes<K, PAIRS, 1024, 256>(c, cls, nitems, s);
      if constexpr (!kWidePairs)
        if (nt == 64) return launch_lanes<K, PAIRS, 1024, 64>(c, cls, nitems, s);
      return launch_lanes<K, PAIRS, 1024, 128>(c, cls, nitems, s);
    case 3:
      if constexpr (kWidePairs) {
        if (nt == 512) return launch_lanes<K, PAIRS, 2048, 512>(c, cls, nitems, s);
      } else {
        if (nt == 64) return launch_lanes<K, PAIRS, 2048, 64>(c, cls, nitems, s);
        if (nt == 128) return launch_lanes<K, PAIRS, 2048, 128>(c, cls, nitems, s);
      }
      return launch_lanes<K, PAIRS, 2048, 256>(c, cls, nitems, s);
    case 4:
      if constexpr (kWidePairs) {
        if (nt == 1024) return launch_lanes<K, PAIRS, 4096, 1024>(c, cls, nitems, s);
      } else {
        if (nt == 128) return launch_lanes<K, PAIRS, 4096, 128>(c, cls, nitems, s);
        if (nt == 256) return launch_lanes<K, PAIRS, 4096, 256>(c, cls, nitems, s);
      }
      return launch_lanes<K, PAIRS, 4096, 512>(c, cls, nitems, s);
    case 5:
      if constexpr (!kWidePairs) {
        if (nt == 256) return launch_lanes<K, PAIRS, 8192, 256>(c, cls, nitems, s);
        if (nt == 512) return launch_lanes<K, PAIRS, 8192, 512>(c, cls, nitems, s);
      }
      return launch_lanes<K, PAIRS, 8192, 1024>(c, cls, nitems, s);
    case 6:
      // 64-bit keys with a payload need 12 LDS bytes a slot: their widest class is 8192
      if constexpr (kWidePairs) return hipErrorInvalidValue;
      else
        return nt == 512 ? launch_lanes<K, PAIRS, 16384, 512>(c, cls, nitems, s)
                         : launch_lanes<K, PAIRS, 16384, 1024>(c, cls, nitems, s);
    default: return hipErrorInvalidValue;
  }
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
    case 5: return launch_kp<KeyI64>(c, cls, nitems, s);
    case 6: return launch_kp<KeyF64>(c, cls, nitems, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdq
