// Oracle: a plain, single-threaded CPU pattern-defeating quicksort, written
// from the paper (Peters, "Pattern-defeating Quicksort", arXiv 2106.05123).
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
// call this file; only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark do. It shares no code, header, table or constant with
// the GPU library.
//
// What it computes: the input keys (and, for pairs, their uint32 payloads)
// rearranged into ascending order of the canonical key order, by the paper's
// algorithm, step for step:
//   * driver loop, insertion-sort base case, heapsort fallback      (Sec. 2, 4.1, 5.1)
//   * partition_right / partition_left with their Figure 3 semantics (Sec. 3, Fig. 3)
//   * predecessor rule selecting partition_left                       (Sec. 3, end)
//   * bad-partition counter, p = 1/8 by a shift, log n initial value  (Sec. 4.1)
//   * fresh pivot candidates after a bad partition                    (Sec. 4.2)
//   * median-of-3 / Tukey's ninther, median moved to the start        (Sec. 2; Sec. 5.2 footnote)
//   * partial insertion sort on a swapless, non-bad partition         (Sec. 5.2)
//   * block (branchless) partitioning for partition_right, bsize 64   (Sec. 5.3)
//
// Readings where the paper is silent (thresholds, candidate layout, abort
// limit, leftover handling) are fixed constants below; each is listed with
// its reason in the design notes of the repository.
//
// Key order: uint32 and uint64 compare as unsigned integers; int32 as two's
// complement; float32 by the total order on bit patterns (-0.0 < +0.0;
// NaN is outside the contract). The comparison is done on a canonical
// unsigned image of the key; stored bits are never altered.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstddef>
#include <utility>

namespace {

// ---- readings of values the paper leaves open --------------------------
constexpr size_t kInsertionThreshold = 24;   // "<= 16-32 elements" (Sec. 5.1): sizes < 24
constexpr size_t kNintherThreshold = 128;    // "sufficiently large" (Sec. 2): sizes > 128
constexpr size_t kPartialInsertionLimit = 8; // "a tiny number of corrections" (Sec. 5.2)
constexpr int kBlockSize = 64;               // static block of 64 elements (Sec. 5.3 footnote)

// ---- canonical key images (total order on the stored bits) -------------
inline uint64_t canon(uint32_t x) { return x; }
inline uint64_t canon(uint64_t x) { return x; }
inline uint64_t canon(int32_t x) { return static_cast<uint32_t>(x) ^ 0x80000000u; }
inline uint64_t canon(int64_t x) { return static_cast<uint64_t>(x) ^ 0x8000000000000000ull; }
inline uint64_t canon(double f) {
  uint64_t b;
  std::memcpy(&b, &f, 8);
  // the same rule as for float, on 64 bits
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
inline uint64_t canon(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  // negative values: all bits flipped (larger magnitude -> smaller image);
  // non-negative values: sign bit set (above every negative value).
  return (b & 0x80000000u) ? static_cast<uint64_t>(~b) : static_cast<uint64_t>(b | 0x80000000u);
}

template <class K>
struct Pair {
  K key;
  uint32_t val;
};

template <class K> inline uint64_t key_image(const K& k) { return canon(k); }
template <class K> inline uint64_t key_image(const Pair<K>& p) { return canon(p.key); }

}  // namespace

extern "C" {

// Counters of what the algorithm did; filled when a pointer is supplied.
struct oracle_counters {
  uint64_t comparisons;        // every key comparison, all phases
  uint64_t partitions_right;
  uint64_t partitions_left;
  uint64_t bad_partitions;
  uint64_t heapsort_calls;
  uint64_t heapsort_elements;
  uint64_t insertion_sorts;
  uint64_t partial_insertion_ok;
  uint64_t partial_insertion_abort;
  uint64_t already_partitioned;  // partition_right calls with no swaps needed
  uint64_t max_depth;
  uint64_t max_bad_on_path;      // most bad partitions seen on one root-to-leaf path
  // optional pivot log: canonical image of each pivot and its mode (0 right, 1 left)
  uint64_t pivot_log_cap;
  uint64_t pivot_log_len;
  uint64_t* pivot_log_key;
  uint8_t* pivot_log_mode;
  // the first partition of the (first) call: pivot, left size, mode, no_swaps
  uint64_t first_pivot_image;
  int64_t first_left_size;
  int32_t first_mode;
  int32_t first_no_swaps;
  int32_t first_recorded;
  int32_t first_bad;       // whether that first partition_right was bad
};

struct oracle_options {
  int32_t block;         // 1: block partitioning in partition_right (bpdq); 0: Fig. 3 loop (pdq)
  int32_t force_budget;  // < 0: floor(log2 n); else the initial bad-partition budget
};

}  // extern "C"

namespace {

template <class T, bool COUNT>
class Sorter {
 public:
  Sorter(oracle_counters* c, bool block, int force_budget)
      : c_(c), block_(block), force_budget_(force_budget) {}

  void sort(T* b, T* e) {
    size_t n = static_cast<size_t>(e - b);
    if (n < 2) return;
    int budget = force_budget_ >= 0 ? force_budget_ : floor_log2(n);
    loop(b, e, budget, true, 1, 0);
  }

  // --- single routines exposed for unit pins -----------------------------
  void insertion(T* b, T* e) { insertion_sort(b, e); }
  void heap(T* b, T* e) { heapsort(b, e); }
  bool partial_insertion(T* b, T* e) { return partial_insertion_sort(b, e); }
  // pivot choice followed by one partition; returns the pivot position
  T* partition_once(T* b, T* e, bool left_mode, bool block, bool* no_swaps) {
    block_ = block;
    choose_pivot(b, e);
    if (left_mode) {
      *no_swaps = false;
      return partition_left(b, e);
    }
    return partition_right(b, e, no_swaps);
  }

 private:
  oracle_counters* c_;
  bool block_;
  int force_budget_;

  static int floor_log2(size_t n) {
    int r = 0;
    while (n > 1) {
      n >>= 1;
      ++r;
    }
    return r;
  }

  bool less(const T& a, const T& b) {
    if (COUNT && c_) ++c_->comparisons;
    return key_image(a) < key_image(b);
  }

  static void swap_elems(T* a, T* b) {
    T t = *a;
    *a = *b;
    *b = t;
  }

  // ---- Sec. 5.1: insertion sort with moves, guarded ----------------------
  void insertion_sort(T* b, T* e) {
    if (COUNT && c_) ++c_->insertion_sorts;
    if (e - b < 2) return;
    for (T* cur = b + 1; cur != e; ++cur) {
      T* hole = cur;
      if (!less(*hole, *(hole - 1))) continue;
      T tmp = *hole;
      do {
        *hole = *(hole - 1);
        --hole;
      } while (hole != b && less(tmp, *(hole - 1)));
      *hole = tmp;
    }
  }

  // Sec. 5.1: without bounds checks; the predecessor at b[-1] is no larger
  // than any element of [b, e) (it is an ancestor's pivot, Lemma 1), so the
  // inner loop always stops at or before b.
  void unguarded_insertion_sort(T* b, T* e) {
    if (COUNT && c_) ++c_->insertion_sorts;
    if (e - b < 2) return;
    for (T* cur = b + 1; cur != e; ++cur) {
      T* hole = cur;
      if (!less(*hole, *(hole - 1))) continue;
      T tmp = *hole;
      do {
        *hole = *(hole - 1);
        --hole;
      } while (less(tmp, *(hole - 1)));
      *hole = tmp;
    }
  }

  // Sec. 5.2: insertion sort that gives up after more than a few element
  // moves. Always leaves a permutation of the range. True when it finished.
  bool partial_insertion_sort(T* b, T* e) {
    if (e - b < 2) return true;
    size_t moves = 0;
    for (T* cur = b + 1; cur != e; ++cur) {
      T* hole = cur;
      if (!less(*hole, *(hole - 1))) continue;
      T tmp = *hole;
      do {
        *hole = *(hole - 1);
        --hole;
      } while (hole != b && less(tmp, *(hole - 1)));
      *hole = tmp;
      moves += static_cast<size_t>(cur - hole);
      if (moves > kPartialInsertionLimit) {
        if (COUNT && c_) ++c_->partial_insertion_abort;
        return false;
      }
    }
    if (COUNT && c_) ++c_->partial_insertion_ok;
    return true;
  }

  // ---- Sec. 2 / 4.1: Williams' heapsort as the O(n log n) fallback ---------
  void sift_down(T* a, size_t root, size_t n) {
    for (;;) {
      size_t child = 2 * root + 1;
      if (child >= n) return;
      if (child + 1 < n && less(a[child], a[child + 1])) ++child;
      if (!less(a[root], a[child])) return;
      swap_elems(a + root, a + child);
      root = child;
    }
  }
  void heapsort(T* b, T* e) {
    size_t n = static_cast<size_t>(e - b);
    if (COUNT && c_) {
      ++c_->heapsort_calls;
      c_->heapsort_elements += n;
    }
    if (n < 2) return;
    for (size_t i = n / 2; i-- > 0;) sift_down(b, i, n);
    for (size_t end = n - 1; end > 0; --end) {
      swap_elems(b, b + end);
      sift_down(b, 0, end);
    }
  }

  // ---- Sec. 2 and the Sec. 5.2 footnote: pivot choice ---------------------
  void sort2(T* a, T* b) {
    if (less(*b, *a)) swap_elems(a, b);
  }
  // Leaves the smallest of the three at a, the median at b, the largest at c.
  void sort3(T* a, T* b, T* c) {
    sort2(a, b);
    sort2(b, c);
    sort2(a, b);
  }
  // Median of first/middle/last, or Tukey's ninther for large ranges; the
  // chosen median ends at b[0]. For the median-of-3 the smallest candidate is
  // parked in the middle and the largest at the end, so that a swapless
  // partition of an ascending range puts every element back where it was.
  void choose_pivot(T* b, T* e) {
    size_t s = static_cast<size_t>(e - b);
    T* mid = b + s / 2;
    if (s > kNintherThreshold) {
      sort3(b, mid, e - 1);
      sort3(b + 1, mid - 1, e - 2);
      sort3(b + 2, mid + 1, e - 3);
      sort3(mid - 1, mid, mid + 1);
      swap_elems(b, mid);
    } else {
      sort3(mid, b, e - 1);
    }
  }

  // Sec. 4.2: after a bad partition, bring elements from around the 25% and
  // 75% points of a child into its pivot-candidate positions.
  void fresh_candidates(T* cb, T* ce) {
    size_t s = static_cast<size_t>(ce - cb);
    if (s < kInsertionThreshold) return;
    size_t q = s / 4;
    swap_elems(cb, cb + q);
    swap_elems(ce - 1, ce - 1 - q);
    if (s > kNintherThreshold) {
      swap_elems(cb + 1, cb + q + 1);
      swap_elems(cb + 2, cb + q + 2);
      swap_elems(ce - 2, ce - 2 - q);
      swap_elems(ce - 3, ce - 3 - q);
    }
  }

  // ---- Sec. 3, Fig. 3: partition_right -------------------------------------
  // The pivot p sits at b[0]. Afterwards [b, r) < p, *r == p, (r, e) >= p.
  // *no_swaps tells whether the range was already partitioned around p, found
  // by comparing the two scan positions once both initial scans are done.
  T* partition_right(T* b, T* e, bool* no_swaps) {
    if (COUNT && c_) ++c_->partitions_right;
    const T p = *b;
    // Scan up from b+1 for the first element not less than p. An element
    // >= p exists to the right (the largest pivot candidate), the bound is a
    // safety net only.
    T* i = b + 1;
    while (i < e && less(*i, p)) ++i;
    // Scan down for the last element less than p. When nothing below p was
    // found on the left the scan must not pass i; otherwise the element at
    // b+1 (< p) stops it.
    T* j = e;
    if (i == b + 1) {
      while (i < j) {
        --j;
        if (less(*j, p)) break;
      }
    } else {
      do {
        --j;
      } while (!less(*j, p));
    }
    *no_swaps = (i >= j);
    if (COUNT && c_ && *no_swaps) ++c_->already_partitioned;

    T* boundary;  // first position of the ">= p" part
    if (*no_swaps) {
      boundary = i;
    } else if (!block_) {
      // Fig. 3 swap loop: swap the two misplaced elements, rescan.
      while (i < j) {
        swap_elems(i, j);
        do {
          ++i;
        } while (less(*i, p));
        do {
          --j;
        } while (!less(*j, p));
      }
      boundary = i;
    } else {
      boundary = block_partition(i, j + 1, p);
    }
    T* r = boundary - 1;
    swap_elems(b, r);
    return r;
  }

  // Sec. 5.3: BlockQuicksort classification. [first, last) is unresolved;
  // everything before it is < p, everything from last on is >= p. Blocks of
  // kBlockSize elements are classified without branches into offset buffers
  // (left block: elements >= p; right block: elements < p) and misplaced
  // pairs are swapped unconditionally. A buffer that still holds offsets
  // keeps its block for the next round. Once fewer than two blocks remain the
  // rest is finished by a plain bounded two-pointer loop.
  T* block_partition(T* first, T* last, const T& p) {
    unsigned char off_l[kBlockSize];
    unsigned char off_r[kBlockSize];
    int num_l = 0, num_r = 0, start_l = 0, start_r = 0;
    while (last - first >= 2 * kBlockSize) {
      if (num_l == 0) {
        start_l = 0;
        for (int k = 0; k < kBlockSize; ++k) {
          off_l[num_l] = static_cast<unsigned char>(k);
          num_l += !less(first[k], p);
        }
      }
      if (num_r == 0) {
        start_r = 0;
        for (int k = 0; k < kBlockSize; ++k) {
          off_r[num_r] = static_cast<unsigned char>(k + 1);
          num_r += less(*(last - 1 - k), p);
        }
      }
      int m = num_l < num_r ? num_l : num_r;
      for (int q = 0; q < m; ++q) swap_elems(first + off_l[start_l + q], last - off_r[start_r + q]);
      num_l -= m;
      num_r -= m;
      start_l += m;
      start_r += m;
      if (num_l == 0) first += kBlockSize;
      if (num_r == 0) last -= kBlockSize;
    }
    T* lo = first;
    T* hi = last;
    for (;;) {
      while (lo < hi && less(*lo, p)) ++lo;
      while (lo < hi && !less(*(hi - 1), p)) --hi;
      if (lo >= hi) break;
      swap_elems(lo, hi - 1);
      ++lo;
      --hi;
    }
    return lo;
  }

  // ---- Sec. 3, Fig. 3: partition_left ---------------------------------------
  // The pivot p sits at b[0]. Afterwards [b, r) <= p, *r == p, (r, e) > p.
  T* partition_left(T* b, T* e) {
    if (COUNT && c_) ++c_->partitions_left;
    const T p = *b;
    // scan down for the last element <= p; p itself at b stops it
    T* j = e;
    do {
      --j;
    } while (less(p, *j));
    T* i = b;
    if (j + 1 == e) {
      // nothing above p at the end: the upward scan must not pass j
      while (i < j) {
        ++i;
        if (less(p, *i)) break;
      }
    } else {
      // the element at j+1 (> p) stops the upward scan
      do {
        ++i;
      } while (!less(p, *i));
    }
    while (i < j) {
      swap_elems(i, j);
      do {
        --j;
      } while (less(p, *j));
      do {
        ++i;
      } while (!less(p, *i));
    }
    swap_elems(b, j);
    return j;
  }

  void log_pivot(const T& p, int mode, T* b, T* r, bool no_swaps) {
    if (!(COUNT && c_)) return;
    if (c_->pivot_log_key && c_->pivot_log_len < c_->pivot_log_cap) {
      c_->pivot_log_key[c_->pivot_log_len] = key_image(p);
      if (c_->pivot_log_mode) c_->pivot_log_mode[c_->pivot_log_len] = static_cast<uint8_t>(mode);
    }
    ++c_->pivot_log_len;
    if (!c_->first_recorded) {
      c_->first_recorded = 1;
      c_->first_pivot_image = key_image(p);
      c_->first_left_size = static_cast<int64_t>(r - b);
      c_->first_mode = mode;
      c_->first_no_swaps = no_swaps ? 1 : 0;
    }
  }

  // ---- Sec. 2, 3, 4.1, 5.2: the driver loop ---------------------------------
  // Recurse on the left part, loop on the right part (the right part always
  // has a predecessor: the pivot just placed).
  void loop(T* b, T* e, int bad_allowed, bool leftmost, uint64_t depth, uint64_t bad_on_path) {
    for (;;) {
      if (COUNT && c_) {
        if (depth > c_->max_depth) c_->max_depth = depth;
        if (bad_on_path > c_->max_bad_on_path) c_->max_bad_on_path = bad_on_path;
      }
      size_t size = static_cast<size_t>(e - b);
      if (size < kInsertionThreshold) {
        if (leftmost)
          insertion_sort(b, e);
        else
          unguarded_insertion_sort(b, e);
        return;
      }
      if (bad_allowed == 0) {
        heapsort(b, e);
        return;
      }
      choose_pivot(b, e);
      // Sec. 3: a predecessor equal to the pivot selects partition_left. The
      // predecessor is never larger than the pivot (Lemma 1), so "not less"
      // means "equal".
      if (!leftmost && !less(*(b - 1), *b)) {
        const T p = *b;
        T* r = partition_left(b, e);
        log_pivot(p, 1, b, r, false);
        // everything left of r equals the pivot: no recursion there
        b = r + 1;
        continue;
      }
      const T p = *b;
      bool no_swaps = false;
      T* r = partition_right(b, e, &no_swaps);
      log_pivot(p, 0, b, r, no_swaps);
      size_t ls = static_cast<size_t>(r - b);
      size_t rs = static_cast<size_t>(e - r - 1);
      // Sec. 4.1: bad when a side holds less than 1/8 of the range
      bool bad = ls < (size >> 3) || rs < (size >> 3);
      if (COUNT && c_ && c_->pivot_log_len == 1 && c_->first_mode == 0) c_->first_bad = bad ? 1 : 0;
      if (bad) {
        if (COUNT && c_) ++c_->bad_partitions;
        --bad_allowed;
        ++bad_on_path;
        fresh_candidates(b, r);
        fresh_candidates(r + 1, e);
      } else if (no_swaps) {
        // Sec. 5.2: optimistic partial insertion sort of both sides
        if (partial_insertion_sort(b, r) && partial_insertion_sort(r + 1, e)) return;
      }
      loop(b, r, bad_allowed, leftmost, depth + 1, bad_on_path);
      b = r + 1;
      leftmost = false;
      ++depth;
    }
  }
};

template <class T>
void run_sort(T* b, uint64_t n, const oracle_options* opt, oracle_counters* c) {
  bool block = opt ? opt->block != 0 : true;
  int fb = opt ? opt->force_budget : -1;
  if (c) {
    Sorter<T, true> s(c, block, fb);
    s.sort(b, b + n);
  } else {
    Sorter<T, false> s(nullptr, block, fb);
    s.sort(b, b + n);
  }
}

template <class K>
int sort_typed(void* keys, uint32_t* vals, uint64_t n, const uint64_t* offsets, uint64_t nseg,
               const oracle_options* opt, oracle_counters* c) {
  K* k = static_cast<K*>(keys);
  uint64_t segs = offsets ? nseg : 1;
  if (!vals) {
    for (uint64_t s = 0; s < segs; ++s) {
      uint64_t lo = offsets ? offsets[s] : 0, hi = offsets ? offsets[s + 1] : n;
      run_sort<K>(k + lo, hi - lo, opt, c);
    }
    return 0;
  }
  // pairs: sort an array of (key, payload) records, then split back
  for (uint64_t s = 0; s < segs; ++s) {
    uint64_t lo = offsets ? offsets[s] : 0, hi = offsets ? offsets[s + 1] : n;
    uint64_t m = hi - lo;
    if (m == 0) continue;
    Pair<K>* tmp = new Pair<K>[m];
    for (uint64_t i = 0; i < m; ++i) tmp[i] = Pair<K>{k[lo + i], vals[lo + i]};
    run_sort<Pair<K>>(tmp, m, opt, c);
    for (uint64_t i = 0; i < m; ++i) {
      k[lo + i] = tmp[i].key;
      vals[lo + i] = tmp[i].val;
    }
    delete[] tmp;
  }
  return 0;
}

template <class K>
int routine_typed(int which, void* keys, uint64_t n, int arg, oracle_counters* c, int64_t* out) {
  K* b = static_cast<K*>(keys);
  Sorter<K, true> s(c, true, -1);
  switch (which) {
    case 0:
      s.insertion(b, b + n);
      return 0;
    case 1:
      s.heap(b, b + n);
      return 0;
    case 2:
      *out = s.partial_insertion(b, b + n) ? 1 : 0;
      return 0;
    case 3: {  // pivot choice + one partition (arg bit 0: left; bit 1: no block partitioning)
      if (n < 3) return -1;
      bool ns = false;
      K* r = s.partition_once(b, b + n, (arg & 1) != 0, (arg & 2) == 0, &ns);
      out[0] = static_cast<int64_t>(r - b);
      out[1] = ns ? 1 : 0;
      return 0;
    }
    default:
      return -1;
  }
}

}  // namespace

extern "C" {

// key_type: 1 uint32, 2 int32, 3 float32, 4 uint64. vals may be null.
int oracle_sort(int key_type, void* keys, uint32_t* vals, uint64_t n, const oracle_options* opt,
                oracle_counters* c) {
  switch (key_type) {
    case 1: return sort_typed<uint32_t>(keys, vals, n, nullptr, 0, opt, c);
    case 2: return sort_typed<int32_t>(keys, vals, n, nullptr, 0, opt, c);
    case 3: return sort_typed<float>(keys, vals, n, nullptr, 0, opt, c);
    case 4: return sort_typed<uint64_t>(keys, vals, n, nullptr, 0, opt, c);
    case 5: return sort_typed<int64_t>(keys, vals, n, nullptr, 0, opt, c);
    case 6: return sort_typed<double>(keys, vals, n, nullptr, 0, opt, c);
    default: return -2;
  }
}

// Each segment [offsets[s], offsets[s+1]) is sorted as its own call.
int oracle_segmented_sort(int key_type, void* keys, uint32_t* vals, uint64_t n,
                          const uint64_t* offsets, uint64_t nseg, const oracle_options* opt,
                          oracle_counters* c) {
  if (!offsets) return -1;
  switch (key_type) {
    case 1: return sort_typed<uint32_t>(keys, vals, n, offsets, nseg, opt, c);
    case 2: return sort_typed<int32_t>(keys, vals, n, offsets, nseg, opt, c);
    case 3: return sort_typed<float>(keys, vals, n, offsets, nseg, opt, c);
    case 4: return sort_typed<uint64_t>(keys, vals, n, offsets, nseg, opt, c);
    case 5: return sort_typed<int64_t>(keys, vals, n, offsets, nseg, opt, c);
    case 6: return sort_typed<double>(keys, vals, n, offsets, nseg, opt, c);
    default: return -2;
  }
}

// Single routines for unit pins. which: 0 insertion sort, 1 heapsort,
// 2 partial insertion sort (out[0] = 1 on success), 3 pivot choice + one
// partition (arg bit 0: partition_left; bit 1: Fig. 3 loop instead of block
// partitioning; out[0] = pivot position, out[1] = no_swaps).
int oracle_routine(int key_type, int which, void* keys, uint64_t n, int arg, oracle_counters* c,
                   int64_t* out) {
  switch (key_type) {
    case 1: return routine_typed<uint32_t>(which, keys, n, arg, c, out);
    case 2: return routine_typed<int32_t>(which, keys, n, arg, c, out);
    case 3: return routine_typed<float>(which, keys, n, arg, c, out);
    case 4: return routine_typed<uint64_t>(which, keys, n, arg, c, out);
    case 5: return routine_typed<int64_t>(which, keys, n, arg, c, out);
    case 6: return routine_typed<double>(which, keys, n, arg, c, out);
    default: return -2;
  }
}

// Canonical image of one key (for tests of the key order).
uint64_t oracle_key_image(int key_type, const void* key) {
  switch (key_type) {
    case 1: return canon(*static_cast<const uint32_t*>(key));
    case 2: return canon(*static_cast<const int32_t*>(key));
    case 3: return canon(*static_cast<const float*>(key));
    case 4: return canon(*static_cast<const uint64_t*>(key));
    case 5: return canon(*static_cast<const int64_t*>(key));
    case 6: return canon(*static_cast<const double*>(key));
    default: return 0;
  }
}

// Float32 prediction of the learned-splitter model (the numpy model in
// mlp_oracle.py defines it; this is its float32 evaluation, used wherever a
// float32 value decides an integer). Parameters: W1[32] b1[32] W2[32][32]
// (row v, column u) b2[32] W3[32] b3. Every dot product is a chain of fused
// multiply-adds in increasing index order, started from the bias; ReLU keeps
// values > 0; the residual input x is added last; the result is clamped to
// [0, 1].
void oracle_mlp_infer_f32(const float* p, const float* x, size_t n, int residual, float* y) {
  const float* W1 = p;
  const float* b1 = p + 32;
  const float* W2 = p + 64;
  const float* b2 = p + 64 + 1024;
  const float* W3 = p + 64 + 1024 + 32;
  const float b3 = p[64 + 1024 + 64];
  for (size_t i = 0; i < n; ++i) {
    float h1[32], h2[32];
    for (int u = 0; u < 32; ++u) {
      const float z = std::fmaf(W1[u], x[i], b1[u]);
      h1[u] = z > 0.0f ? z : 0.0f;
    }
    for (int v = 0; v < 32; ++v) {
      float acc = b2[v];
      for (int u = 0; u < 32; ++u) acc = std::fmaf(W2[v * 32 + u], h1[u], acc);
      h2[v] = acc > 0.0f ? acc : 0.0f;
    }
    float out = b3;
    for (int v = 0; v < 32; ++v) out = std::fmaf(W3[v], h2[v], out);
    if (residual) out = out + x[i];
    y[i] = out < 0.0f ? 0.0f : (out > 1.0f ? 1.0f : out);
  }
}

}  // extern "C"
