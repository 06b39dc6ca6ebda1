// Host driver and C ABI of the partition sort (declared in include/pdq.h).
//
// One call runs partition passes until no live segment is left. Every pass
// launches, on the caller's stream:
//   pivot    one lane per live segment: ninther + predecessor rule
//   tilemap  one lane per tile ticket: ticket -> segment, cleared status
//   partition  persistent tiles with decoupled look-back (the hot kernel)
//   bookkeep one lane per live segment: pivot placement, retirement,
//            budget, children filed as live / base case / heapsort / copy
// then reads a few counters back to size the next pass and runs the
// finishing kernels (base case, heapsort, copies) for what retired.
// Keys ping-pong between the user buffer and a scratch buffer of the same
// size inside the caller's workspace; everything that is final ends up in
// the user buffer.
#include <stdint.h>
#include <string.h>

#include <vector>

#include "pdq.h"
#include "pdq_internal.h"

namespace {

using namespace pdq;

thread_local int g_last_hip = 0;

constexpr size_t kAlign = 256;
constexpr uint32_t kMinTile = 1024;
constexpr uint32_t kDefaultTile = 32768;
constexpr uint32_t kMaxPasses = 20000;  // far above any reachable pass count; a guard against bugs

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t scratch_keys = 0, scratch_vals = 0, segs0 = 0, segs1 = 0, tilemap = 0, status = 0;
  size_t base[kBaseClasses] = {}, heap = 0, copy = 0, ctr = 0, total = 0;
  uint32_t max_active = 0, max_tiles = 0, max_items = 0;
};

Layout make_layout(size_t n, size_t nseg, uint32_t kt, bool vals) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  // live segments hold more than kBaseMax keys each and never overlap
  L.max_active = static_cast<uint32_t>(n / (kBaseMax + 1) + 2);
  L.max_tiles = static_cast<uint32_t>(n / kMinTile + 2ull * L.max_active + 64);
  size_t items = 2ull * L.max_active;
  if (nseg > items) items = nseg;
  L.max_items = static_cast<uint32_t>(items + 64);
  L.scratch_keys = take(n * key_bytes(kt));
  L.scratch_vals = take(vals ? n * 4 : 0);
  L.segs0 = take(sizeof(Seg) * L.max_active);
  L.segs1 = take(sizeof(Seg) * L.max_active);
  L.tilemap = take(4ull * L.max_tiles);
  L.status = take(8ull * L.max_tiles);
  for (int k = 0; k < kBaseClasses; ++k) L.base[k] = take(sizeof(Item) * L.max_items);
  L.heap = take(sizeof(Item) * L.max_items);
  L.copy = take(sizeof(Item) * L.max_items);
  L.ctr = take(sizeof(Counters));
  L.total = off + kAlign;  // room to align the caller's base pointer
  return L;
}

bool valid_key_type(int kt) { return kt >= PDQ_U32 && kt <= PDQ_U64; }

struct Opts {
  uint32_t flags = 0;
  int32_t force_budget = -1;
  uint32_t tile = 0;
  uint64_t seed = 0;
};

int read_opts(const pdq_options* o, Opts* out) {
  if (!o) return PDQ_OK;
  // struct_size 0 is taken as the current layout; smaller sizes keep defaults
  // for fields they do not cover
  const size_t sz = o->struct_size ? o->struct_size : sizeof(pdq_options);
  if (sz >= offsetof(pdq_options, flags) + sizeof(uint32_t)) out->flags = o->flags;
  if (sz >= offsetof(pdq_options, force_budget) + sizeof(int32_t)) out->force_budget = o->force_budget;
  if (sz >= offsetof(pdq_options, tile) + sizeof(uint32_t)) out->tile = o->tile;
  if (sz >= offsetof(pdq_options, seed) + sizeof(uint64_t)) out->seed = o->seed;
  if (out->flags & ~static_cast<uint32_t>(PDQ_VALIDATE | PDQ_PROFILE)) return PDQ_ERR_UNSUPPORTED;
  if (out->tile != 0 && out->tile != 1024 && out->tile != 2048 && out->tile != 4096 && out->tile != 8192 &&
      out->tile != 16384 && out->tile != 32768 && out->tile != 65536)
    return PDQ_ERR_UNSUPPORTED;
  return PDQ_OK;
}

#define HIP_TRY(expr)                                \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) {                          \
      g_last_hip = static_cast<int>(e_);             \
      return PDQ_ERR_HIP;                            \
    }                                                \
  } while (0)

struct Timed {
  hipEvent_t a = nullptr, b = nullptr;
  uint64_t bytes = 0;
};

int read_counters(const Ctx& c, Counters* snap, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(snap, c.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (snap->errors & kErrCapacity) return PDQ_ERR_INVALID;  // only bad offsets can overfill a list
  if (snap->errors) {
    g_last_hip = 0;
    return PDQ_ERR_HIP;
  }
  const uint32_t nact0 = static_cast<uint32_t>(snap->list[0] >> 32), nact1 = static_cast<uint32_t>(snap->list[1] >> 32);
  if (nact0 > c.max_active || nact1 > c.max_active || static_cast<uint32_t>(snap->list[0]) > c.max_tiles ||
      static_cast<uint32_t>(snap->list[1]) > c.max_tiles || snap->nheap > c.max_items || snap->ncopy > c.max_items)
    return PDQ_ERR_INVALID;
  for (int k = 0; k < kBaseClasses; ++k)
    if (snap->nbase[k] > c.max_items) return PDQ_ERR_INVALID;
  return PDQ_OK;
}

int finish_items(const Ctx& c, const Counters& snap, hipStream_t s) {
  for (int k = 0; k < kBaseClasses; ++k)
    if (snap.nbase[k]) HIP_TRY(launch_base(c, k, snap.nbase[k], s));
  if (snap.nheap) HIP_TRY(launch_heap(c, snap.nheap, s));
  if (snap.ncopy) HIP_TRY(launch_copy(c, snap.ncopy, s));
  return PDQ_OK;
}

int run_sort(void* keys, uint32_t* vals, size_t n, const uint64_t* offsets, size_t nseg, int kt, int order,
             void* ws, size_t ws_bytes, void* stream, const pdq_options* opt, pdq_stats* st) {
  g_last_hip = 0;
  if (!valid_key_type(kt) || order != PDQ_ASCENDING) return PDQ_ERR_UNSUPPORTED;
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc != PDQ_OK) return rc;
  if (n >= (1ull << 32)) return PDQ_ERR_UNSUPPORTED;
  const uint32_t kb = key_bytes(static_cast<uint32_t>(kt));
  if (st) {
    const uint32_t sz = st->struct_size;
    memset(st, 0, sizeof(pdq_stats));
    st->struct_size = sz;
    st->first_mode = -1;
  }
  if (offsets && nseg == 0) return n == 0 ? PDQ_OK : PDQ_ERR_INVALID;
  if (n <= 1 && !offsets) return PDQ_OK;
  if (n == 0) return PDQ_OK;
  if (!keys) return PDQ_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(keys) % kb) return PDQ_ERR_INVALID;
  if (vals && (reinterpret_cast<uintptr_t>(vals) % 4)) return PDQ_ERR_INVALID;
  if (offsets && (reinterpret_cast<uintptr_t>(offsets) % 8)) return PDQ_ERR_INVALID;
  if (nseg >= (1ull << 32)) return PDQ_ERR_UNSUPPORTED;
  const Layout L = make_layout(n, offsets ? nseg : 1, static_cast<uint32_t>(kt), vals != nullptr);
  if (!ws || ws_bytes < L.total) return PDQ_ERR_WORKSPACE;

  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + kAlign - 1) / kAlign * kAlign);
  Ctx c = {};
  c.keys[0] = keys;
  c.keys[1] = base + L.scratch_keys;
  c.vals[0] = vals;
  c.vals[1] = vals ? reinterpret_cast<uint32_t*>(base + L.scratch_vals) : nullptr;
  c.n = n;
  c.segs[0] = reinterpret_cast<Seg*>(base + L.segs0);
  c.segs[1] = reinterpret_cast<Seg*>(base + L.segs1);
  c.tilemap = reinterpret_cast<uint32_t*>(base + L.tilemap);
  c.status = reinterpret_cast<uint64_t*>(base + L.status);
  for (int k = 0; k < kBaseClasses; ++k) c.base[k] = reinterpret_cast<Item*>(base + L.base[k]);
  c.heap = reinterpret_cast<Item*>(base + L.heap);
  c.copy = reinterpret_cast<Item*>(base + L.copy);
  c.ctr = reinterpret_cast<Counters*>(base + L.ctr);
  c.offsets = offsets;
  c.nseg = offsets ? nseg : 1;
  c.tile = o.tile ? o.tile : kDefaultTile;
  c.max_active = L.max_active;
  c.max_tiles = L.max_tiles;
  c.max_items = L.max_items;
  c.force_budget = o.force_budget;
  c.key_type = static_cast<uint32_t>(kt);
  c.has_vals = vals ? 1u : 0u;
  c.single = offsets ? 0u : 1u;
  c.seed = o.seed;

  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool prof = (o.flags & PDQ_PROFILE) && st;
  std::vector<Timed> timed;
  auto cleanup = [&]() {
    for (auto& t : timed) {
      if (t.a) (void)hipEventDestroy(t.a);
      if (t.b) (void)hipEventDestroy(t.b);
    }
  };

  Counters snap = {};
  HIP_TRY(launch_reset(c, s));
  HIP_TRY(launch_init(c, s));
  rc = read_counters(c, &snap, s);
  if (rc != PDQ_OK) return rc;
  if ((o.flags & PDQ_VALIDATE) && snap.bad_offsets) return PDQ_ERR_INVALID;
  // base cases and heapsorts of the input segments themselves
  rc = finish_items(c, snap, s);
  if (rc != PDQ_OK) return rc;

  const uint64_t bytes_per_key = 2ull * kb + (vals ? 8ull : 0ull);
  int parity = 0;
  uint32_t src = 0;
  uint32_t pass = 0;
  uint64_t visits = 0;
  for (;;) {
    const uint32_t nact = static_cast<uint32_t>(snap.list[parity] >> 32);
    const uint32_t ntiles = static_cast<uint32_t>(snap.list[parity]);
    if (nact == 0) break;
    if (pass >= kMaxPasses) {
      cleanup();
      return PDQ_ERR_HIP;
    }
    visits += snap.elems[parity];
    int r2 = PDQ_OK;
    do {
      hipError_t e;
      if ((e = launch_pivot(c, parity, nact, src, s)) != hipSuccess) { g_last_hip = e; r2 = PDQ_ERR_HIP; break; }
      if ((e = launch_tilemap(c, parity, ntiles, s)) != hipSuccess) { g_last_hip = e; r2 = PDQ_ERR_HIP; break; }
      Timed tm;
      if (prof) {
        if (hipEventCreate(&tm.a) != hipSuccess || hipEventCreate(&tm.b) != hipSuccess) { r2 = PDQ_ERR_HIP; break; }
        tm.bytes = snap.elems[parity] * bytes_per_key;
        (void)hipEventRecord(tm.a, s);
      }
      if ((e = launch_partition(c, parity, ntiles, src, s)) != hipSuccess) { g_last_hip = e; r2 = PDQ_ERR_HIP; break; }
      if (prof) {
        (void)hipEventRecord(tm.b, s);
        timed.push_back(tm);
      }
      if ((e = launch_bookkeep(c, parity, nact, src, pass, s)) != hipSuccess) { g_last_hip = e; r2 = PDQ_ERR_HIP; break; }
    } while (0);
    if (r2 == PDQ_OK) r2 = read_counters(c, &snap, s);
    if (r2 == PDQ_OK) r2 = finish_items(c, snap, s);
    if (r2 != PDQ_OK) {
      cleanup();
      return r2;
    }
    parity ^= 1;
    src ^= 1u;
    ++pass;
  }

  if (st) {
    int r3 = read_counters(c, &snap, s);
    if (r3 != PDQ_OK) {
      cleanup();
      return r3;
    }
    st->passes = pass;
    st->element_visits = visits;
    st->partitions_right = snap.partitions_right;
    st->partitions_left = snap.partitions_left;
    st->bad_partitions = snap.bad_partitions;
    st->heapsort_segments = snap.heap_segments;
    st->heapsort_elements = snap.heap_elements;
    st->base_segments = snap.base_segments;
    st->base_elements = snap.base_elements;
    st->sorted_segments = snap.sorted_segments;
    st->sorted_elements = snap.sorted_elements;
    st->equal_elements = snap.equal_elements;
    st->first_pivot_image = snap.first_pivot_image;
    st->first_left_size = snap.first_left;
    st->first_mode = snap.first_mode;
    if (prof) {
      double total = 0;
      uint64_t bytes = 0;
      for (size_t i = 0; i < timed.size(); ++i) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, timed[i].a, timed[i].b);
        total += ms;
        bytes += timed[i].bytes;
        if (i == 0) {
          st->first_pass_ms = ms;
          st->first_pass_bytes = timed[i].bytes;
        }
      }
      st->partition_launches = static_cast<uint32_t>(timed.size());
      st->partition_ms = total;
      st->partition_bytes = bytes;
    }
  }
  cleanup();
  return PDQ_OK;
}

}  // namespace

extern "C" {

size_t pdq_workspace_bytes(size_t n, size_t nseg, pdq_key_type key_type, int has_vals, const pdq_options* opt) {
  (void)opt;
  if (!valid_key_type(key_type)) return 0;
  if (nseg == 0) nseg = 1;
  return make_layout(n, nseg, static_cast<uint32_t>(key_type), has_vals != 0).total;
}

int pdq_sort(void* d_keys, size_t n, pdq_key_type key_type, pdq_order order, void* d_ws, size_t ws_bytes,
             void* stream, const pdq_options* opt, pdq_stats* stats) {
  return run_sort(d_keys, nullptr, n, nullptr, 1, key_type, order, d_ws, ws_bytes, stream, opt, stats);
}

int pdq_sort_pairs(void* d_keys, uint32_t* d_vals, size_t n, pdq_key_type key_type, pdq_order order, void* d_ws,
                   size_t ws_bytes, void* stream, const pdq_options* opt, pdq_stats* stats) {
  if (n > 1 && !d_vals) return PDQ_ERR_INVALID;
  return run_sort(d_keys, d_vals, n, nullptr, 1, key_type, order, d_ws, ws_bytes, stream, opt, stats);
}

int pdq_segmented_sort(void* d_keys, uint32_t* d_vals, size_t n, const uint64_t* d_offsets, size_t nseg,
                       pdq_key_type key_type, pdq_order order, void* d_ws, size_t ws_bytes, void* stream,
                       const pdq_options* opt, pdq_stats* stats) {
  if (!d_offsets && nseg > 0) return PDQ_ERR_INVALID;
  if (!d_offsets) return n == 0 ? PDQ_OK : PDQ_ERR_INVALID;
  return run_sort(d_keys, d_vals, n, d_offsets, nseg, key_type, order, d_ws, ws_bytes, stream, opt, stats);
}

const char* pdq_status_string(int status) {
  switch (status) {
    case PDQ_OK: return "PDQ_OK: success";
    case PDQ_ERR_INVALID: return "PDQ_ERR_INVALID: invalid argument (null or misaligned pointer, bad offsets)";
    case PDQ_ERR_UNSUPPORTED: return "PDQ_ERR_UNSUPPORTED: unsupported key type, order, size or option";
    case PDQ_ERR_WORKSPACE: return "PDQ_ERR_WORKSPACE: workspace missing or smaller than pdq_workspace_bytes()";
    case PDQ_ERR_HIP: return "PDQ_ERR_HIP: a HIP launch or synchronisation failed";
    default: return "unknown pdq status";
  }
}

int pdq_last_hip_error(void) { return g_last_hip; }

int pdq_abi_version(void) { return PDQ_ABI_VERSION; }

}  // extern "C"
