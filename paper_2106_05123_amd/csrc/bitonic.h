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
  using I = uint32_t;
  static constexpr int kLdsBytes = 4;
  __device__ static I img(V v) { return v; }
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
  using I = uint32_t;
  static constexpr int kLdsBytes = 8;
  __device__ static I img(V v) { return static_cast<uint32_t>(v >> 32); }
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
  using I = uint64_t;
  static constexpr int kLdsBytes = 8;
  __device__ static I img(V v) { return v; }
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
  using I = uint64_t;
  static constexpr int kLdsBytes = 12;
  __device__ static I img(V v) { return v.k; }
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

// ---------------------------------------------------------------- radix sort

// LSD radix sort of the block's P = E * NT slots, the alternative to the
// merge sort for segments whose keys span few bits (a segment that reaches
// the base case lies between two pivots, so its keys usually span a small
// part of the key range: about 2^16 for 4096 uniform 32-bit keys out of
// 2^28). Digits are kRadixBits of (image - minimum image); each pass ranks
// the slots stably the way a block radix sort does: every lane counts its
// own keys per digit in a private column of a [digit][lane] counter matrix
// (its rank among its own keys with that digit is the count before it), one
// exclusive scan over the matrix in (digit, lane) order turns the counts
// into first positions, and every slot is written to first position + rank.
// Slots at positions >= len are padding: they take the largest digit in
// every pass and, being last and the sort stable, stay last. Returns false,
// with x untouched, when the real images span more than
// kRadixBits * kRadixMaxPasses bits (the merge sort then runs).
constexpr int kRadixBits = 6;
constexpr int kRadixDigits = 1 << kRadixBits;  // also the counters each lane scans
constexpr int kRadixMaxPasses = 3;

// The counter matrix: kRadixDigits * NT 16-bit counts (P <= 65535), with two
// padding halves after every kRadixDigits entries so that the lanes' scan
// segments start in different banks.
template <int NT>
constexpr int radix_counters() {
  return kRadixDigits * NT + 2 * NT;
}
__device__ __forceinline__ int cnt_pos(int f) { return f + 2 * (f >> 6); }

template <class S, int E, int NT>
__device__ __forceinline__ bool radix_sort(typename S::V (&x)[E], unsigned char* sh, uint16_t* cnt, int tid,
                                           int len) {
  using I = typename S::I;
  constexpr int PL = lds_plane<E * NT, E>();
  constexpr int kWaves = NT / 64;
  static_assert(kRadixDigits == 64, "each lane scans one 64-entry segment of the counter matrix");
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // range of the real images (the counter area holds the wave partials)
  I lo = ~I(0), hi = I(0);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (tid * E + r < len) {
      const I v = S::img(x[r]);
      lo = v < lo ? v : lo;
      hi = v > hi ? v : hi;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    const I olo = __shfl_xor(lo, d, 64), ohi = __shfl_xor(hi, d, 64);
    lo = olo < lo ? olo : lo;
    hi = ohi > hi ? ohi : hi;
  }
  I* part = reinterpret_cast<I*>(cnt);
  if (lane == 0) {
    part[2 * wave] = lo;
    part[2 * wave + 1] = hi;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const I plo = part[2 * w], phi = part[2 * w + 1];
    lo = plo < lo ? plo : lo;
    hi = phi > hi ? phi : hi;
  }
  __syncthreads();
  const I span = hi > lo ? hi - lo : I(0);
  int bits = 0;
  if (span) bits = static_cast<int>(sizeof(I) * 8) - (sizeof(I) == 8 ? __clzll(static_cast<long long>(span))
                                                                     : __clz(static_cast<int>(span)));
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  if (passes > kRadixMaxPasses) return false;  // the same decision in every lane
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    // this lane's column of the counter matrix
#pragma unroll 8
    for (int d = 0; d < kRadixDigits; ++d) cnt[cnt_pos(d * NT + tid)] = 0;
    uint32_t dig[E];
    uint32_t rank[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      dig[r] = tid * E + r < len ? static_cast<uint32_t>((S::img(x[r]) - lo) >> shift) & (kRadixDigits - 1)
                                 : static_cast<uint32_t>(kRadixDigits - 1);
      const int at = cnt_pos(static_cast<int>(dig[r]) * NT + tid);
      rank[r] = cnt[at];
      cnt[at] = static_cast<uint16_t>(rank[r] + 1);
    }
    __syncthreads();
    // exclusive scan in (digit, lane) order: lane t owns entries
    // [64 t, 64 t + 64), i.e. digit 64 t / NT, lanes (64 t) % NT ...
    uint16_t* seg = cnt + cnt_pos(tid * kRadixDigits);
    uint32_t sum = 0;
#pragma unroll 16
    for (int k = 0; k < kRadixDigits; ++k) sum += seg[k];
    uint32_t incl = sum;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t t = __shfl_up(incl, d, 64);
      if (lane >= d) incl += t;
    }
    uint32_t* wsum = reinterpret_cast<uint32_t*>(sh);  // the data planes are free until the scatter
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
      if (w < wave) run += wsum[w];
#pragma unroll 16
    for (int k = 0; k < kRadixDigits; ++k) {
      const uint32_t c = seg[k];
      seg[k] = static_cast<uint16_t>(run);
      run += c;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int at = static_cast<int>(cnt[cnt_pos(static_cast<int>(dig[r]) * NT + tid)] + rank[r]);
      S::st(sh, PL, lds_pos<E>(at), x[r]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) x[r] = S::ld(sh, PL, lds_pos<E>(tid * E + r));
    __syncthreads();
  }
  return true;
}

}  // namespace net
}  // namespace pdq
