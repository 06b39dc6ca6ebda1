// Pivot choice of one segment, shared by the pass-based partition sort and
// the persistent tail of the device-counted passes.
#pragma once

#include "pdq_internal.h"

namespace pdq {

template <class K>
struct PivotChoice {
  typename K::T raw;  // pivot key bits
  uint64_t pidx;      // its absolute position in the source buffer
  uint32_t mode;      // kModeRight / kModeLeft
};

// Tukey's ninther, the median of the medians of three triples (Section 2).
// Normally the triples are (first, mid, last), (first+1, mid-1, last-1),
// (first+2, mid+1, last-2). After a bad partition the segment takes fresh
// candidates (Section 4.2). By default they sit at nine positions drawn from
// a counter-based hash of (seed, begin, end) -- the randomised form of the
// rule: an out-of-place partition that keeps order keeps periodic input
// structure intact, so fixed offsets can keep landing on equally bad
// candidates pass after pass. With `fixed` the deterministic form is used
// instead: the first and last candidate of every triple are taken a quarter
// of the segment further in (first -> first + size/4, first+1 -> first+1 +
// size/4, ..., last -> last - size/4, ...), the positions the sequential
// algorithm swaps into place, read here where they are rather than moved
// (the partition does not depend on where the candidates sit).
// Then the predecessor rule of Section 3 selects partition_left
// when the predecessor is not below the pivot; the predecessor is an
// ancestor's pivot and already sits at its final place in the user buffer
// (Lemma 1). Segments have more than 4096 keys, so every offset is in range.
// COHERENT reads the candidates and the predecessor with agent-scope loads:
// the persistent batched kernel reads keys and pivots that another
// workgroup, possibly on another XCD with its own L2, wrote earlier in the
// same launch. The pass kernels read what earlier launches wrote, which a
// kernel boundary makes visible, and use plain loads.
template <bool COHERENT, class T>
__device__ __forceinline__ T pivot_load(const T* p) {
  if constexpr (COHERENT) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}

template <class K, bool COHERENT = false>
__device__ __forceinline__ PivotChoice<K> choose_pivot(const typename K::T* keys, const typename K::T* user,
                                                       uint64_t b, uint64_t e, uint32_t flags, uint64_t seed,
                                                       bool fixed) {
  using T = typename K::T;
  const uint64_t size = e - b;
  const uint64_t m = size / 2;
  uint64_t off[9] = {0, m, size - 1, 1, m - 1, size - 2, 2, m + 1, size - 3};
  if ((flags & kSegFresh) && fixed) {
    const uint64_t q = size / 4;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      off[3 * t] += q;
      off[3 * t + 2] -= q;
    }
  } else if (flags & kSegFresh) {
    const uint64_t h0 = mix64(seed ^ mix64(b ^ mix64(e)));
#pragma unroll
    for (int k = 0; k < 9; ++k) off[k] = mix64(h0 + static_cast<uint64_t>(k)) % size;
  }
  T raw[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) raw[k] = pivot_load<COHERENT>(keys + b + off[k]);
  uint64_t mo[3], mp[3];
  T mr[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const uint64_t o0 = K::ord(raw[3 * t]), o1 = K::ord(raw[3 * t + 1]), o2 = K::ord(raw[3 * t + 2]);
    int sel;
    if (o0 < o1) sel = (o1 < o2) ? 1 : ((o0 < o2) ? 2 : 0);
    else sel = (o0 < o2) ? 0 : ((o1 < o2) ? 2 : 1);
    mo[t] = sel == 0 ? o0 : (sel == 1 ? o1 : o2);
    mp[t] = off[3 * t + sel];
    mr[t] = raw[3 * t + sel];
  }
  int sel;
  if (mo[0] < mo[1]) sel = (mo[1] < mo[2]) ? 1 : ((mo[0] < mo[2]) ? 2 : 0);
  else sel = (mo[0] < mo[2]) ? 0 : ((mo[1] < mo[2]) ? 2 : 1);
  PivotChoice<K> pc;
  pc.raw = mr[sel];
  pc.pidx = b + mp[sel];
  pc.mode = kModeRight;
  if (!(flags & kSegLeftmost)) {
    const T pred = pivot_load<COHERENT>(user + b - 1);
    if (!(static_cast<uint64_t>(K::ord(pred)) < mo[sel])) pc.mode = kModeLeft;
  }
  return pc;
}

}  // namespace pdq
