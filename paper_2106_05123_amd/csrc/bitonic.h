// Bitonic sorting network over E * NT slots held E per lane in registers,
// shared by the base case and the batched segmented sort.
//
// Slot index i = (wave << (e + 6)) | (lane << e) | r, so a compare-exchange
// across index bit b runs
//   b < e        inside one lane's registers,
//   e <= b < e+6 across lanes with a lane-xor shuffle,
//   b >= e+6     across waves through LDS.
// Keys are compared on their canonical images; with a payload each key is
// paired with its index in the segment, so equal keys stay distinguishable
// and padding (index >= size) sorts after every real key.
#pragma once

#include "pdq_internal.h"

namespace pdq {
namespace net {

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// (64-bit image, 32-bit index) pair for 64-bit keys with a payload.
struct KV {
  uint64_t k;
  uint32_t i;
};

// How one sort slot is built, compared, moved across lanes and stored.
template <class K, bool PAIRS, bool WIDE = (sizeof(typename K::T) == 8)>
struct Slot;

// 32-bit keys, no payload: the canonical image itself.
template <class K>
struct Slot<K, false, false> {
  using V = uint32_t;
  static constexpr int kLdsBytes = 4;
  __device__ static V make(uint32_t raw, uint32_t) { return K::ord(raw); }
  __device__ static V pad() { return 0xFFFFFFFFu; }
  __device__ static V sel(bool c, V a, V b) { return c ? a : b; }
  __device__ static bool lt(V a, V b) { return a < b; }
  __device__ static V xch(V a, int m) { return __shfl_xor(a, m, 64); }
  __device__ static uint32_t key(V v) { return K::inv(v); }
  __device__ static uint32_t idx(V) { return 0; }
  __device__ static void st(unsigned char* s, int, int i, V v) { reinterpret_cast<V*>(s)[i] = v; }
  __device__ static V ld(const unsigned char* s, int, int i) { return reinterpret_cast<const V*>(s)[i]; }
};

// 32-bit keys with payload: image in the high half, index in the low half.
template <class K>
struct Slot<K, true, false> {
  using V = uint64_t;
  static constexpr int kLdsBytes = 8;
  __device__ static V make(uint32_t raw, uint32_t i) { return (static_cast<uint64_t>(K::ord(raw)) << 32) | i; }
  __device__ static V pad() { return ~0ull; }
  __device__ static V sel(bool c, V a, V b) { return c ? a : b; }
  __device__ static bool lt(V a, V b) { return a < b; }
  __device__ static V xch(V a, int m) { return __shfl_xor(a, m, 64); }
  __device__ static uint32_t key(V v) { return K::inv(static_cast<uint32_t>(v >> 32)); }
  __device__ static uint32_t idx(V v) { return static_cast<uint32_t>(v); }
  __device__ static void st(unsigned char* s, int, int i, V v) { reinterpret_cast<V*>(s)[i] = v; }
  __device__ static V ld(const unsigned char* s, int, int i) { return reinterpret_cast<const V*>(s)[i]; }
};

// 64-bit keys, no payload: the canonical image itself.
template <class K>
struct Slot<K, false, true> {
  using V = uint64_t;
  static constexpr int kLdsBytes = 8;
  __device__ static V make(uint64_t raw, uint32_t) { return K::ord(raw); }
  __device__ static V pad() { return ~0ull; }
  __device__ static V sel(bool c, V a, V b) { return c ? a : b; }
  __device__ static bool lt(V a, V b) { return a < b; }
  __device__ static V xch(V a, int m) { return __shfl_xor(a, m, 64); }
  __device__ static uint64_t key(V v) { return K::inv(v); }
  __device__ static uint32_t idx(V) { return 0; }
  __device__ static void st(unsigned char* s, int, int i, V v) { reinterpret_cast<V*>(s)[i] = v; }
  __device__ static V ld(const unsigned char* s, int, int i) { return reinterpret_cast<const V*>(s)[i]; }
};

// 64-bit keys with payload: (image, index), stored as two LDS planes.
template <class K>
struct Slot<K, true, true> {
  using V = KV;
  static constexpr int kLdsBytes = 12;
  __device__ static V make(uint64_t raw, uint32_t i) { return KV{K::ord(raw), i}; }
  __device__ static V pad() { return KV{~0ull, 0xFFFFFFFFu}; }
  // field by field: a select of whole structs goes through scratch memory
  __device__ static V sel(bool c, V a, V b) { return KV{c ? a.k : b.k, c ? a.i : b.i}; }
  __device__ static bool lt(V a, V b) { return a.k < b.k || (a.k == b.k && a.i < b.i); }
  __device__ static V xch(V a, int m) { return KV{__shfl_xor(a.k, m, 64), static_cast<uint32_t>(__shfl_xor(a.i, m, 64))}; }
  __device__ static uint64_t key(V v) { return K::inv(v.k); }
  __device__ static uint32_t idx(V v) { return v.i; }
  // a plane of `plane` keys, then a plane of `plane` indices
  __device__ static void st(unsigned char* s, int plane, int i, V v) {
    reinterpret_cast<uint64_t*>(s)[i] = v.k;
    reinterpret_cast<uint32_t*>(s + 8 * plane)[i] = v.i;
  }
  __device__ static V ld(const unsigned char* s, int plane, int i) {
    return KV{reinterpret_cast<const uint64_t*>(s)[i], reinterpret_cast<const uint32_t*>(s + 8 * plane)[i]};
  }
};

// LDS slot of index i: one padding slot every E slots keeps the per-lane
// strided accesses of the register layout off a single bank.
template <int E>
__device__ __forceinline__ int lds_pos(int i) {
  if constexpr (E == 1) return i;
  else return i + (i >> ilog2(E));
}

template <int P, int E>
constexpr int lds_plane() {
  return E == 1 ? P : P + P / E;
}

template <class S, int E, int NT>
__device__ __forceinline__ void bitonic(typename S::V (&x)[E], unsigned char* sh, int tid) {
  using V = typename S::V;
  constexpr int e = ilog2(E);
  constexpr int p = ilog2(E * NT);
  constexpr int PL = lds_plane<E * NT, E>();
  const int lane = tid & 63;
  const int base = tid << e;  // index of x[0]: (wave << (e+6)) | (lane << e)
#pragma unroll
  for (int kb = 1; kb <= p; ++kb) {
#pragma unroll
    for (int b = kb - 1; b >= 0; --b) {
      if (b < e) {
        // partners inside this lane's registers
#pragma unroll
        for (int r = 0; r < E; ++r) {
          if (r & (1 << b)) continue;
          const int r2 = r | (1 << b);
          const bool up = (((base | r) >> kb) & 1) == 0;
          const V a = x[r], c = x[r2];
          const bool sw = S::lt(c, a) == up;  // out of order for this block's direction
          x[r] = S::sel(sw, c, a);
          x[r2] = S::sel(sw, a, c);
        }
      } else if (b < e + 6) {
        // partners in lane ^ m, same register
        const int m = 1 << (b - e);
        const bool lower = (lane & m) == 0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const bool up = (((base | r) >> kb) & 1) == 0;
          const V y = S::xch(x[r], m);
          const bool take_min = lower == up;
          const bool y_less = S::lt(y, x[r]);
          x[r] = S::sel(y_less == take_min, y, x[r]);
        }
      } else {
        // partners in another wave: exchange through LDS
#pragma unroll
        for (int r = 0; r < E; ++r) S::st(sh, PL, lds_pos<E>(base | r), x[r]);
        __syncthreads();
        const bool lower = ((base >> b) & 1) == 0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const bool up = (((base | r) >> kb) & 1) == 0;
          const V y = S::ld(sh, PL, lds_pos<E>((base | r) ^ (1 << b)));
          const bool take_min = lower == up;
          const bool y_less = S::lt(y, x[r]);
          x[r] = S::sel(y_less == take_min, y, x[r]);
        }
        __syncthreads();
      }
    }
  }
}

// Merge sort of P = E * NT slots. On entry lane tid holds slots
// [tid*E, tid*E + E) in any order; on exit the same positions of the sorted
// sequence. Each lane first sorts its E registers (a bitonic network inside
// the lane), then log2(NT) merge levels double the sorted run length: all
// runs go to LDS, and each lane produces its E outputs of the merged pair by
// a merge-path binary search for its starting split followed by E steps of a
// sequential merge, one LDS read per step (ties taken from the left run).
template <class S, int E, int NT>
__device__ __forceinline__ void merge_sort(typename S::V (&x)[E], unsigned char* sh, int tid) {
  using V = typename S::V;
  constexpr int e = ilog2(E);
  constexpr int P = E * NT;
  constexpr int PL = lds_plane<P, E>();
  // runs of E inside each lane
#pragma unroll
  for (int kb = 1; kb <= e; ++kb) {
#pragma unroll
    for (int b = kb - 1; b >= 0; --b) {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        if (r & (1 << b)) continue;
        const int r2 = r | (1 << b);
        const bool up = ((r >> kb) & 1) == 0;
        const V a = x[r], c = x[r2];
        const bool sw = S::lt(c, a) == up;
        x[r] = S::sel(sw, c, a);
        x[r2] = S::sel(sw, a, c);
      }
    }
  }
  const V pad = S::pad();
  for (int run = E; run < P; run <<= 1) {
#pragma unroll
    for (int r = 0; r < E; ++r) S::st(sh, PL, lds_pos<E>(tid * E + r), x[r]);
    __syncthreads();
    const int o = (tid * E) & (2 * run - 1);  // output position inside the merged pair
    const int pa = tid * E - o;               // start of the left run; the right run follows it
    const int pb = pa + run;
    int lo = o > run ? o - run : 0, hi = o < run ? o : run;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      // left[mid] <= right[o - mid - 1]: left[mid] is merged before position o
      if (!S::lt(S::ld(sh, PL, lds_pos<E>(pb + o - mid - 1)), S::ld(sh, PL, lds_pos<E>(pa + mid)))) lo = mid + 1;
      else hi = mid;
    }
    int i = lo, j = o - lo;
    V a = pad, c = pad;
    if (i < run) a = S::ld(sh, PL, lds_pos<E>(pa + i));
    if (j < run) c = S::ld(sh, PL, lds_pos<E>(pb + j));
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const bool take_left = !S::lt(c, a);
      x[r] = S::sel(take_left, a, c);
      if (take_left) ++i;
      else ++j;
      if (r + 1 < E) {
        const bool more = take_left ? i < run : j < run;
        const int at = take_left ? pa + i : pb + j;
        V nv = pad;
        if (more) nv = S::ld(sh, PL, lds_pos<E>(at));
        a = S::sel(take_left, nv, a);
        c = S::sel(take_left, c, nv);
      }
    }
    __syncthreads();
  }
}

}  // namespace net
}  // namespace pdq
