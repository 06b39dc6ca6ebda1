// Wavefront-level helpers (wave64) used by the pass kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdq {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, 64);
    v = o > v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v |= __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const uint32_t lane = lane_id();
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t t = __shfl_up(v, d, 64);
    if (lane >= static_cast<uint32_t>(d)) v += t;
  }
  return v;
}

// Every lane of the wave must call this (no lane may have exited). Lanes
// with `want` reserve `units` in a packed counter (count << 32 | units).
// Returns, for wanting lanes, (index << 32 | first unit) of their slot.
__device__ __forceinline__ uint64_t wave_reserve_packed(unsigned long long* ctr, bool want,
                                                        uint32_t units) {
  const uint64_t v = want ? ((1ull << 32) | units) : 0ull;
  const uint64_t incl = wave_incl_scan_u64(v);
  const uint64_t total = __shfl(incl, 63, 64);
  uint64_t base = 0;
  if (lane_id() == 63 && total != 0) base = atomicAdd(ctr, static_cast<unsigned long long>(total));
  base = __shfl(base, 63, 64);
  return base + (incl - v);
}

// Every lane must call this. Lane i gets n_i consecutive slots of a 32-bit
// counter (lanes in order); returns the first.
__device__ __forceinline__ uint32_t wave_reserve_n(uint32_t* ctr, uint32_t n) {
  const uint64_t incl = wave_incl_scan_u64(n);
  const uint64_t total = __shfl(incl, 63, 64);
  uint32_t base = 0;
  if (lane_id() == 63 && total != 0) base = atomicAdd(ctr, static_cast<uint32_t>(total));
  base = __shfl(base, 63, 64);
  return base + static_cast<uint32_t>(incl - n);
}

// Every lane must call this. Wanting lanes get consecutive slots of a
// 32-bit counter; returns the slot index.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t* ctr, bool want) {
  const uint64_t m = __ballot(want);
  uint32_t base = 0;
  if (lane_id() == 0 && m != 0) base = atomicAdd(ctr, static_cast<uint32_t>(__popcll(m)));
  base = __shfl(base, 0, 64);
  return base + lanes_below(m);
}

// Every lane must call this. Adds the wave's sum of v to *ctr.
__device__ __forceinline__ void wave_add(unsigned long long* ctr, uint64_t v) {
  const uint64_t s = wave_sum_u64(v);
  if (lane_id() == 0 && s != 0) atomicAdd(ctr, static_cast<unsigned long long>(s));
}

// Workgroup barrier that orders LDS only. __syncthreads() also fences
// global memory, which on this target waits for every outstanding global
// load and store of the wave; the partition kernel keeps loads and stores in
// flight across its barriers, and its barriers only hand LDS data between
// waves.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Agent-scope relaxed loads/stores for the look-back status words: the
// value travels inside the word, so no ordering of other memory is needed,
// only visibility across the chip.
__device__ __forceinline__ uint64_t load_status(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_status(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace pdq
