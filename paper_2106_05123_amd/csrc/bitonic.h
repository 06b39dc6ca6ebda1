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
  using Key = K;
  using I = uint32_t;  // the key image (bucket sort)
  static constexpr bool kBucket = true;
  static constexpr bool kUnique = false;  // equal keys give equal slots
  __device__ static I img(V v) { return v; }
  static constexpr int kLdsBytes = 4;
  __device__ static V make(uint32_t raw, uint32_t) { return K::ord(raw); }
  __device__ static V pad() { return 0xFFFFFFFFu; }
  __device__ static V sel(bool c, V a, V b) { return c ? a : b; }
  __device__ static bool lt(V a, V b) { return a < b; }
  __device__ static V xch(V a, int m) { return __shfl_xor(a, m, 64); }
  __device__ static V shf(V a, int src) { return __shfl(a, src, 64); }
  __device__ static uint32_t key(V v) { return K::inv(v); }
  __device__ static uint32_t idx(V) { return 0; }
  __device__ static void st(unsigned char* s, int, int i, V v) { reinterpret_cast<V*>(s)[i] = v; }
  __device__ static V ld(const unsigned char* s, int, int i) { return reinterpret_cast<const V*>(s)[i]; }
};

// 32-bit keys with payload: image in the high half, index in the low half.
template <class K>
struct Slot<K, true, false> {
  using V = uint64_t;
  using Key = K;
  using I = uint32_t;
  static constexpr bool kBucket = true;
  static constexpr bool kUnique = true;  // the index makes every slot distinct
  __device__ static I img(V v) { return static_cast<uint32_t>(v >> 32); }
  static constexpr int kLdsBytes = 8;
  __device__ static V make(uint32_t raw, uint32_t i) { return (static_cast<uint64_t>(K::ord(raw)) << 32) | i; }
  __device__ static V pad() { return ~0ull; }
  __device__ static V sel(bool c, V a, V b) { return c ? a : b; }
  __device__ static bool lt(V a, V b) { return a < b; }
  __device__ static V xch(V a, int m) { return __shfl_xor(a, m, 64); }
  __device__ static V shf(V a, int src) { return __shfl(a, src, 64); }
  __device__ static uint32_t key(V v) { return K::inv(static_cast<uint32_t>(v >> 32)); }
  __device__ static uint32_t idx(V v) { return static_cast<uint32_t>(v); }
  __device__ static void st(unsigned char* s, int, int i, V v) { reinterpret_cast<V*>(s)[i] = v; }
  __device__ static V ld(const unsigned char* s, int, int i) { return reinterpret_cast<const V*>(s)[i]; }
};

// 64-bit keys, no payload: the canonical image itself.
template <class K>
struct Slot<K, false, true> {
  using V = uint64_t;
  using Key = K;
  using I = uint64_t;
  static constexpr bool kBucket = true;
  static constexpr bool kUnique = false;
  __device__ static I img(V v) { return v; }
  static constexpr int kLdsBytes = 8;
  __device__ static V make(uint64_t raw, uint32_t) { return K::ord(raw); }
  __device__ static V pad() { return ~0ull; }
  __device__ static V sel(bool c, V a, V b) { return c ? a : b; }
  __device__ static bool lt(V a, V b) { return a < b; }
  __device__ static V xch(V a, int m) { return __shfl_xor(a, m, 64); }
  __device__ static V shf(V a, int src) { return __shfl(a, src, 64); }
  __device__ static uint64_t key(V v) { return K::inv(v); }
  __device__ static uint32_t idx(V) { return 0; }
  __device__ static void st(unsigned char* s, int, int i, V v) { reinterpret_cast<V*>(s)[i] = v; }
  __device__ static V ld(const unsigned char* s, int, int i) { return reinterpret_cast<const V*>(s)[i]; }
};

// 64-bit keys with payload: (image, index), stored as two LDS planes.
template <class K>
struct Slot<K, true, true> {
  using V = KV;
  using Key = K;
  using I = uint64_t;
  static constexpr bool kBucket = false;  // two LDS planes: the bucket sort does not serve it
  static constexpr bool kUnique = true;
  __device__ static I img(V v) { return v.k; }
  static constexpr int kLdsBytes = 12;
  __device__ static V make(uint64_t raw, uint32_t i) { return KV{K::ord(raw), i}; }
  __device__ static V pad() { return KV{~0ull, 0xFFFFFFFFu}; }
  // field by field: a select of whole structs goes through scratch memory
  __device__ static V sel(bool c, V a, V b) { return KV{c ? a.k : b.k, c ? a.i : b.i}; }
  __device__ static bool lt(V a, V b) { return a.k < b.k || (a.k == b.k && a.i < b.i); }
  __device__ static V xch(V a, int m) { return KV{__shfl_xor(a.k, m, 64), static_cast<uint32_t>(__shfl_xor(a.i, m, 64))}; }
  __device__ static V shf(V a, int src) { return KV{__shfl(a.k, src, 64), static_cast<uint32_t>(__shfl(a.i, src, 64))}; }
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

// Ascending bitonic sort of one lane's E registers.
template <class S, int E>
__device__ __forceinline__ void lane_sort(typename S::V (&x)[E]) {
  using V = typename S::V;
  constexpr int e = ilog2(E);
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
}

// Ascending bitonic merge of one lane's E registers holding a bitonic sequence.
template <class S, int E>
__device__ __forceinline__ void lane_merge(typename S::V (&x)[E]) {
  using V = typename S::V;
#pragma unroll
  for (int j = E / 2; j > 0; j >>= 1) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      if (r & j) continue;
      const V a = x[r], c = x[r + j];
      const bool sw = S::lt(c, a);
      x[r] = S::sel(sw, c, a);
      x[r + j] = S::sel(sw, a, c);
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
  constexpr int P = E * NT;
  constexpr int PL = lds_plane<P, E>();
  lane_sort<S, E>(x);  // runs of E inside each lane
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


// ---------------------------------------------------------------- bucket sort

// Floating-point keys: the value behind a canonical image. The bucket sort
// cuts the range of values, not of images, when every key is finite.
template <class K>
struct FloatOf {
  static constexpr bool kFloat = false;
  using F = float;
  template <class I>
  __device__ static F val(I) { return F(0); }
};
template <>
struct FloatOf<KeyF32> {
  static constexpr bool kFloat = true;
  using F = float;
  __device__ static F val(uint32_t img) { return __uint_as_float(KeyF32::inv(img)); }
};
template <>
struct FloatOf<KeyF64> {
  static constexpr bool kFloat = true;
  using F = double;
  __device__ static F val(uint64_t img) { return __longlong_as_double(static_cast<long long>(KeyF64::inv(img))); }
};


// Bucket sort of the real slots of a P = E * NT block, for segments whose
// keys spread over their range (a segment that reaches the base case lies
// between two pivots, or inside one bin of a learned model). The range
// [lo, hi] of the key images is cut into nb = 2^b equal-width buckets, nb
// the power of two with about kBkMean keys a bucket (at most P / kBkMean).
// Floating-point keys cut the range of their values instead when every key
// is finite: images crowd a few exponents (values near zero, or a range
// that spans zero, put most keys in a sliver of the image range), values
// do not. Either way the bucket index never decreases as the key grows.
// Every key takes a rank inside its bucket from an LDS atomic on its
// bucket's 16-bit counter (two to a word), the counters are scanned into
// bucket starts, and each key is stored at its bucket's start plus its
// arrival rank. Buckets are ordered like their keys, so every key now sits
// inside the range of places it takes in the sorted block; only the order
// inside each bucket is left. Two ways finish it:
//  * NET (network finish): each lane sorts the E consecutive places
//    [tid * E, tid * E + E) in its registers, then neighbouring lanes merge
//    their runs twice, lanes (2m, 2m+1) and then (2m+1, 2m+2), each keeping
//    its half of the pair (a half-cleaner and a bitonic merge). A bucket of
//    at most E keys spans at most two lanes, and the merge at its boundary
//    sorts it whole; merges at other boundaries leave it alone. Buckets are
//    capped at min(E, 16) keys, and the result is left in x, lane tid
//    holding places [tid * E, tid * E + E).
//  * rank count: every key counts the members of its bucket that sort
//    before it, which is its place inside the bucket, and is written to its
//    bucket's start plus that place. With a payload every slot is distinct;
//    without one, a key also counts its equals and writes its value over all
//    of their places (they hold the same bits). Buckets are capped at kBkMax
//    keys, and the result is left in LDS as a plain array of len slots.
//
// On entry x[r] holds the slot of segment position r * NT + tid (padding
// from position len on). Keys that cluster (a sample of one key a lane
// crowds one sixty-fourth of the range) or a bucket above the cap (many
// copies of few values) make the call return kBkFailed with x untouched,
// and the caller sorts x another way.
enum BucketResult : int { kBkFailed = 0, kBkInLds = 1, kBkInRegs = 2 };
constexpr int kBkMean = 2;
constexpr int kBkMax = 32;
// positions whose buckets are ranked together (independent LDS reads)
constexpr int kBkGroup = 4;

// coarse ranges of the sample test
constexpr int kBkCoarse = 64;

// LDS words the bucket sort needs besides the block's data plane.
template <int P, int NT>
constexpr int bucket_words() {
  return P / kBkMean / 2 + 1 + kBkCoarse + 4 * (NT / 64) + 2;
}

template <class S, int E, int NT, bool NET>
__device__ __forceinline__ int bucket_sort(typename S::V (&x)[E], unsigned char* sh, uint32_t* bk, int tid,
                                           int len) {
  using V = typename S::V;
  using I = typename S::I;
  constexpr int P = E * NT;
  constexpr int W = NT / 64;
  constexpr int kWords = P / kBkMean / 2;  // packed counters, two buckets a word
  constexpr int kCap = NET ? (E < 16 ? E : 16) : kBkMax;  // largest bucket
  const int lane = tid & 63, wave = tid >> 6;
  uint32_t* cnt = bk;                                          // [kWords + 1]
  uint32_t* coarse = bk + kWords + 1;                          // [kBkCoarse]
  I* red = reinterpret_cast<I*>(bk + kWords + 1 + kBkCoarse);  // [2 W] wave minima and maxima
  uint32_t* sc = bk + kWords + 1 + kBkCoarse + 4 * W;          // [0] largest bucket
  static_assert(E * NT == P && (kBkGroup & (kBkGroup - 1)) == 0 && E % kBkGroup == 0, "bucket sort shape");
  // x[r] is a real key for r < nreal (positions r * NT + tid below len)
  const int nreal = tid < len ? (len - 1 - tid) / NT + 1 : 0;
  // 1. range of the real images
  I lo = ~I(0), hi = I(0);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (r < nreal) {
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
  if (lane == 0) {
    red[2 * wave] = lo;
    red[2 * wave + 1] = hi;
  }
  for (int i = tid; i <= kWords + kBkCoarse; i += NT) cnt[i] = 0;  // counters and coarse ranges
  if (tid == 0) sc[0] = 0;
  __syncthreads();
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const I plo = red[2 * w], phi = red[2 * w + 1];
    lo = plo < lo ? plo : lo;
    hi = phi > hi ? phi : hi;
  }
  const I span = hi > lo ? static_cast<I>(hi - lo) : I(0);
  int nbits = 0;
  while ((kBkMean << nbits) < len && (2 << nbits) <= 2 * kWords) ++nbits;
  int sbits = 0;
  if constexpr (sizeof(I) == 8) sbits = span ? 64 - __clzll(static_cast<long long>(span)) : 0;
  else sbits = span ? 32 - __clz(static_cast<int>(span)) : 0;
  const int shift = sbits > nbits ? sbits - nbits : 0;
  using FO = FloatOf<typename S::Key>;
  using F = typename FO::F;
  bool lin = false;  // buckets over the values
  F f0 = F(0), fscale = F(0);
  if constexpr (FO::kFloat) {
    // the extreme images hold the extreme values; NaNs and infinities sort
    // outermost, so finite ends mean every key is finite
    const F a = FO::val(lo), b = FO::val(hi);
    const F w = b - a;
    if (isfinite(a) && isfinite(b) && isfinite(w) && w > F(0)) {
      lin = true;
      f0 = a;
      fscale = static_cast<F>(1 << nbits) / w;
    }
  }
  const uint32_t dmax = (1u << nbits) - 1u;
  // bucket of an image: monotone in the key (subtraction, scaling by a
  // positive factor and truncation all keep the order), at most dmax
  auto digit = [&](I img) -> uint32_t {
    if constexpr (FO::kFloat) {
      if (lin) {
        const F t = (FO::val(img) - f0) * fscale;
        const uint32_t d = t < static_cast<F>(dmax) ? static_cast<uint32_t>(t) : dmax;
        return d;
      }
    }
    return static_cast<uint32_t>((img - lo) >> shift);
  };
  // sample test: each lane's first key (lanes past the end take no part)
  // goes to one of kBkCoarse ranges of buckets. Keys that
  // spread evenly put a few times NT / kBkCoarse in each; a range holding
  // over an eighth of the sample means clustered keys, whose buckets would
  // overflow after the full count, so the merge sort takes them at once.
  {
    const int cshift = nbits > 6 ? nbits - 6 : 0;
    if (tid < len) atomicAdd(&coarse[digit(S::img(x[0])) >> cshift], 1u);
    __syncthreads();
    uint32_t cm = coarse[lane];
    for (int d = 32; d >= 1; d >>= 1) {
      const uint32_t t = __shfl_xor(cm, d, 64);
      cm = t > cm ? t : cm;
    }
    constexpr uint32_t kThr = NT / 8 > 8 ? NT / 8 : 8;
    if (cm > kThr) return kBkFailed;  // every wave reduces the same LDS words: a uniform exit
  }
  // 2. rank of every real key inside its bucket (bucket index in the high
  //    half of br, arrival rank in the low half; both stay below 2^16)
  uint32_t br[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    br[r] = 0;
    if (r < nreal) {
      const uint32_t d = digit(S::img(x[r]));
      const uint32_t sh16 = (d & 1u) << 4;
      const uint32_t old = atomicAdd(&cnt[d >> 1], 1u << sh16);
      br[r] = (d << 16) | ((old >> sh16) & 0xFFFFu);
    }
  }
  __syncthreads();
  // 3. exclusive scan of the counters into bucket starts (kept packed);
  //    the word after the last holds len, the end of the last bucket
  constexpr int kPer = (kWords + NT - 1) / NT;
  uint32_t cw[kPer];
  uint32_t own = 0, mx = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = tid * kPer + k;
    cw[k] = i < kWords ? cnt[i] : 0u;
    const uint32_t c0 = cw[k] & 0xFFFFu, c1 = cw[k] >> 16;
    own += c0 + c1;
    mx = c0 > mx ? c0 : mx;
    mx = c1 > mx ? c1 : mx;
  }
  uint32_t incl = own;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  for (int d = 32; d >= 1; d >>= 1) {
    const uint32_t t = __shfl_xor(mx, d, 64);
    mx = t > mx ? t : mx;
  }
  // the range words are free again: every lane read them before the
  // counting barrier
  uint32_t* wsum = reinterpret_cast<uint32_t*>(red);
  if (lane == 63) wsum[wave] = incl;
  if (lane == 0) atomicMax(&sc[0], mx);
  __syncthreads();
  if (sc[0] > static_cast<uint32_t>(kCap)) return kBkFailed;  // one LDS word: the same for every lane
  uint32_t run = incl - own;
  for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = tid * kPer + k;
    if (i < kWords) {
      const uint32_t c0 = cw[k] & 0xFFFFu;
      cnt[i] = run | ((run + c0) << 16);
      run += c0 + (cw[k] >> 16);
    }
  }
  if (tid == 0) cnt[kWords] = static_cast<uint32_t>(len);
  __syncthreads();
  // 4. scatter to bucket start + arrival rank
  V* data = reinterpret_cast<V*>(sh);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (r < nreal) {
      const uint32_t d = br[r] >> 16;
      const uint32_t st = (cnt[d >> 1] >> ((d & 1u) << 4)) & 0xFFFFu;
      const int at = static_cast<int>(st + (br[r] & 0xFFFFu));
      if constexpr (NET) data[lds_pos<E>(at)] = x[r];  // lane runs are read back: the padded layout
      else data[at] = x[r];
    }
  }
  if constexpr (NET) {
    __syncthreads();
    // 5. sort the lane's run of E places, then merge with the neighbours
    const V pad = S::pad();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int at = tid * E + r;
      x[r] = at < len ? data[lds_pos<E>(at)] : pad;
    }
    lane_sort<S, E>(x);
    // round 0: partners tid ^ 1, always in one wave: the partner's run comes
    // by shuffles, no LDS and no barrier
    {
      const bool lower = (lane & 1) == 0;
      V b[E];
#pragma unroll
      for (int r = 0; r < E; ++r) b[r] = S::xch(x[E - 1 - r], 1);
      // half-cleaner against the partner's run reversed: the lower lane
      // keeps the E smallest of the pair, the upper lane the E largest,
      // each as a bitonic sequence
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const bool take = lower ? S::lt(b[r], x[r]) : S::lt(x[r], b[r]);
        x[r] = S::sel(take, b[r], x[r]);
      }
      lane_merge<S, E>(x);
    }
    // round 1: partners (2m+1, 2m+2). Inside a wave by shuffles; across a
    // wave boundary (lane 63 with the next wave's lane 0) the two runs go
    // through LDS, in the counters' space (read for the last time by the
    // scatter, before the barrier that preceded this step)
    {
      V* edge = reinterpret_cast<V*>(bk);  // [wave][0: lane 0, 1: lane 63][E]
      if (lane == 0 || lane == 63) {
#pragma unroll
        for (int r = 0; r < E; ++r) edge[(2 * wave + (lane == 63 ? 1 : 0)) * E + r] = x[r];
      }
      __syncthreads();
      const int partner = (tid & 1) ? tid + 1 : tid - 1;
      const int src = (lane & 1) ? lane + 1 : lane - 1;  // lanes 0 and 63 read LDS instead
      V b[E];
#pragma unroll
      for (int r = 0; r < E; ++r) b[r] = S::shf(x[E - 1 - r], src & 63);
      if (lane == 63 && partner < NT) {
#pragma unroll
        for (int r = 0; r < E; ++r) b[r] = edge[(2 * (wave + 1)) * E + (E - 1 - r)];
      }
      if (lane == 0 && partner >= 0) {
#pragma unroll
        for (int r = 0; r < E; ++r) b[r] = edge[(2 * (wave - 1) + 1) * E + (E - 1 - r)];
      }
      if (partner >= 0 && partner < NT) {
        const bool lower = tid < partner;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const bool take = lower ? S::lt(b[r], x[r]) : S::lt(x[r], b[r]);
          x[r] = S::sel(take, b[r], x[r]);
        }
        lane_merge<S, E>(x);
      }
    }
    return kBkInRegs;
  }
  // padding after the last key (len + kBkMax <= P + P / E: inside the
  // block's LDS plane), so that reads past a bucket's end find keys of later
  // buckets or padding, neither of which sorts before a key of the bucket
  if (tid < kBkMax) data[len + tid] = S::pad();
  __syncthreads();
  // 5. every key counts the slots of its bucket that sort before it, and
  //    without a payload also its equals; kBkGroup keys at a time for
  //    independent LDS reads. Reads run to the longest of the lane's buckets
  //    (start + k < len + kBkMax); past a key's own bucket they find greater
  //    keys or padding, so nothing is masked. (A key equal to the padding is
  //    in the last bucket: the padding it counts as equal only stretches its
  //    writes past position len, which is never read.) br[r] becomes the
  //    key's first place.
  uint32_t eq[E];
#pragma unroll
  for (int g = 0; g < E; g += kBkGroup) {
    int s[kBkGroup];
    uint32_t lt[kBkGroup], ne[kBkGroup];
    int nmax = 0;
#pragma unroll
    for (int q = 0; q < kBkGroup; ++q) {
      const int r = g + q;
      s[q] = 0;
      lt[q] = 0;
      ne[q] = 0;
      if (r < nreal) {
        const uint32_t d = br[r] >> 16;
        const uint32_t a = (cnt[d >> 1] >> ((d & 1u) << 4)) & 0xFFFFu;
        const uint32_t e = (cnt[(d + 1) >> 1] >> (((d + 1) & 1u) << 4)) & 0xFFFFu;
        s[q] = static_cast<int>(a);
        const int n = static_cast<int>(e - a);
        nmax = n > nmax ? n : nmax;
      }
    }
    for (int k = 0; k < nmax; ++k) {
#pragma unroll
      for (int q = 0; q < kBkGroup; ++q) {
        const V v = data[s[q] + k];
        lt[q] += S::lt(v, x[g + q]) ? 1u : 0u;
        if constexpr (!S::kUnique) ne[q] += v == x[g + q] ? 1u : 0u;
      }
    }
#pragma unroll
    for (int q = 0; q < kBkGroup; ++q) {
      br[g + q] = static_cast<uint32_t>(s[q]) + lt[q];
      eq[g + q] = ne[q];
    }
  }
  __syncthreads();
  // 6. every key to its place (without a payload, over its equals' places)
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (r < nreal) {
      if constexpr (S::kUnique) {
        data[br[r]] = x[r];
      } else {
        for (uint32_t t = 0; t < eq[r]; ++t) data[br[r] + t] = x[r];
      }
    }
  }
  __syncthreads();
  return kBkInLds;
}

}  // namespace net
}  // namespace pdq
