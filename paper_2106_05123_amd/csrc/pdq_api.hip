// Host driver and C ABI of the partition sort (declared in include/pdq.h).
//
// One call runs partition passes until no live segment is left. Every pass
// launches, on the caller's stream:
//   pivot    one lane per live segment: ninther + predecessor rule
//   tilemap  one lane per tile ticket: ticket -> segment
//   partition  persistent tiles, each reserving its places in its segment
//            with one atomic (the hot kernel)
//   bookkeep one lane per live segment: pivot placement, retirement,
//            budget, children filed as live / base case / heapsort / copy
// then reads a few counters back to size the next pass and runs the
// finishing kernels (base case, heapsort, copies) for what retired.
// Keys ping-pong between the user buffer and a scratch buffer of the same
// size inside the caller's workspace; everything that is final ends up in
// the user buffer.
//
// With PDQ_LEARNED a single-range call first fits the splitter model on a
// key sample, counts the keys per bin, and -- if no range bin is too full --
// scatters the keys into their bins in the scratch buffer; the partition
// passes then start from the scratch buffer with one segment per range bin.
#include <stdint.h>
#include <string.h>

#include <math.h>

#include <stdio.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "batch_internal.h"
#include "learn_internal.h"
#include "pdq.h"
#include "pdq_learned.h"
#include "pdq_internal.h"
#include "runs_internal.h"

namespace {

using namespace pdq;

thread_local int g_last_hip = 0;

constexpr size_t kAlign = 256;
constexpr uint32_t kMinTile = 1024;
constexpr uint32_t kDefaultTile = 32768;

// Partition tile for segments of `avg` keys on average, when the caller did
// not fix one: large tiles while segments span many of them (fewer
// reservations on each segment's cursor), 8192 once they hold a few hundred
// thousand keys or less (less of each tile lies outside its segment).
// The partition tile of a pass over `elems` keys whose largest segment
// holds `maxlen`. Each tile makes one atomic on its segment's cursor, and
// atomics on one cache line run one after another (~12-16 ns apiece), so a
// segment that holds much of the pass takes larger tiles: 16384 tiles of
// 16384 keys cost one segment of 2^28 keys ~0.25 ms of atomics against a
// ~0.5 ms pass. Cursors of different segments work in parallel, so once no
// segment holds more than 1/kSpread of the keys the 8192-key tile (more
// workgroups per CU, faster per key) wins at any size.
constexpr uint64_t kSpread = 10;
uint32_t auto_tile(uint64_t elems, uint64_t maxlen) {
  if (maxlen * kSpread <= elems) return 8192u;
  return maxlen >= (1ull << 18) ? 16384u : 8192u;
}
constexpr uint32_t kMaxPasses = 20000;  // far above any reachable pass count; a guard against bugs

constexpr uint64_t kLearnSample = PDQ_LEARN_SAMPLE;
constexpr uint32_t kMaxTrainGrid = 64;
constexpr uint32_t kMaxLearnSteps = 65536;
constexpr uint32_t kStage1Steps = 32;  // the staged budget's short fit

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t scratch_keys = 0, scratch_vals = 0, segs0 = 0, segs1 = 0, cur = 0, tickets = 0, tilemap = 0, status = 0;
  size_t base[kBaseClasses] = {}, heap = 0, copy = 0, ctr = 0, total = 0;
  // the second item set of the pipelined pass loop (zero in the batched form)
  size_t base1[kBaseClasses] = {}, heap1 = 0, copy1 = 0;
  uint32_t max_active = 0, max_tiles = 0, max_items = 0;
  // learned first pass (zero sizes when not requested)
  size_t fit_out = 0, fit_scratch = 0, bucket = 0;
  // near-sorted path of single-range sorts (zero when not used)
  size_t runs = 0;
  // batched segmented sort: queue words, ring items, ring slot states, and
  // (autotuning only) a copy of the input
  size_t bq = 0, bitems = 0, bstate = 0, backup_keys = 0, backup_vals = 0;
  uint32_t bcap = 0;
};

// Offsets inside an area, built by the same bump allocator as the layout.
struct Bump {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off = (off + bytes + kAlign - 1) / kAlign * kAlign;
    return o;
  }
};

Layout make_layout(size_t n, size_t nseg, uint32_t kt, bool vals, bool batched);

// Outputs of the fit (sample, features, targets, prediction, parameters,
// losses, splitters, count, info).
struct FitOutLayout {
  size_t sample, x, t, y, params, losses, splitters, count, info, total;
};
FitOutLayout fit_out_layout(uint32_t steps) {
  FitOutLayout f;
  Bump b;
  f.sample = b.take(kLearnSample * 8);
  f.x = b.take(kLearnSample * 4);
  f.t = b.take(kLearnSample * 4);
  f.y = b.take(kLearnSample * 4);
  f.params = b.take(kParamStride * 4);
  f.losses = b.take(static_cast<size_t>(steps) * 4);
  f.splitters = b.take(256 * 8);
  f.count = b.take(4);
  f.info = b.take(kInfoWords * 8);
  f.total = b.off;
  return f;
}

// Scratch of the fit: running maximum, gradient partials, barrier words,
// the unsorted sample, and the second stage with its candidates.
struct FitScratchLayout {
  size_t runmax, partials, sync, raw, runmax2, yx, yy, leaf, cand, cand_count, est, total;
};
FitScratchLayout fit_scratch_layout(uint32_t grid) {
  FitScratchLayout f;
  Bump b;
  f.runmax = b.take(kLearnSample * 4);
  f.partials = b.take(2ull * grid * kParamStride * 4);
  f.sync = b.take(4 * 4);
  f.raw = b.take(kLearnSample * 8);
  f.runmax2 = b.take(2ull * kLearnSample * 4);
  f.yx = b.take(kLearnSample * 4);
  f.yy = b.take(kLearnSample * 4);
  f.leaf = b.take(2ull * kLeaves * 2 * 8);
  f.cand = b.take(static_cast<size_t>(kCandidates) * 256 * 8);
  f.cand_count = b.take(kCandidates * 4);
  f.est = b.take(kCandidates * 8);
  f.total = b.off;
  return f;
}

// Per-tile rows, chunk rows, bin totals and bin starts of the histogram.
struct BucketLayout {
  size_t rows, chunk, totals, begin, order, total;
};
BucketLayout bucket_layout(size_t n) {
  BucketLayout L;
  Bump b;
  L.rows = b.take(bucket_tiles(n) * kBinStride * 4);
  L.chunk = b.take(bucket_chunks(n) * kBinStride * 4);
  L.totals = b.take(kBinStride * 8);
  L.begin = b.take((kBinStride + 1) * 8);
  L.order = b.take(4);
  L.total = b.off;
  return L;
}

// Descent log, plan, gather list, outlier buffer and merge splits of the
// near-sorted path.
struct RunsLayout {
  size_t count, pos, plan, shorts, item, okeys, ovals, splits, total;
};
RunsLayout runs_layout(size_t n) {
  RunsLayout r;
  Bump b;
  r.count = b.take(8);
  r.pos = b.take(4ull * kRunMaxDescents);
  r.plan = b.take(sizeof(RunPlan));
  r.shorts = b.take(sizeof(RunSpan) * (kRunMaxDescents + 1ull));
  r.item = b.take(sizeof(Item));
  r.okeys = b.take(8ull * kRunMaxOutliers);
  r.ovals = b.take(4ull * kRunMaxOutliers);
  r.splits = b.take(8ull * (n / kRunMergeTile + 2));
  r.total = b.off;
  return r;
}

// Single-range sorts of at least kRunMinKeys keys try the near-sorted path
// (a call with one segment reserves its area too, whatever its flags, so
// that pdq_workspace_bytes and the call agree).
bool uses_runs(size_t n, size_t nseg) { return nseg == 1 && n >= kRunMinKeys; }

// Widest LDS class of the batched form: 16384 keys, 8192 for 64-bit keys
// with a payload (12 LDS bytes a slot).
uint32_t batch_base_max(uint32_t kt, bool vals) { return key_bytes(kt) == 8 && vals ? 8192u : kWideBaseMax; }

Layout make_layout(size_t n, size_t nseg, uint32_t kt, bool vals, bool batched) {
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
  if (batched) {
    // the item lists accumulate over the passes: the input segments, then at
    // most two children (or one ordered run and one equal run) for each of
    // the disjoint live segments of every pass
    items = nseg + 2ull * kMaxBatchPasses * (n / (batch_base_max(kt, vals) + 1) + 2);
  }
  // copy items cover at most kCopyChunk keys each: a retired range of r keys
  // takes up to r / kCopyChunk more slots, and retired ranges are disjoint
  L.max_items = static_cast<uint32_t>(items + n / kCopyChunk + 64);
  // the counter block comes first, so pdq_check finds it from d_ws alone
  L.ctr = take(sizeof(Counters));
  L.scratch_keys = take(n * key_bytes(kt));
  L.scratch_vals = take(vals ? n * 4 : 0);
  L.segs0 = take(sizeof(Seg) * L.max_active);
  L.segs1 = take(sizeof(Seg) * L.max_active);
  L.cur = take(sizeof(Cursor) * L.max_active);
  L.tickets = take(4ull * kTicketQueues * kTicketStride);
  L.tilemap = take(4ull * L.max_tiles);
  L.status = take(8ull * L.max_tiles);
  for (int k = 0; k < kBaseClasses; ++k) L.base[k] = take(sizeof(Item) * L.max_items);
  L.heap = take(sizeof(Item) * L.max_items);
  L.copy = take(sizeof(Item) * L.max_items);
  if (!batched) {
    // the pipelined pass loop finishes one pass's items while the next pass
    // fills the other set
    for (int k = 0; k < kBaseClasses; ++k) L.base1[k] = take(sizeof(Item) * L.max_items);
    L.heap1 = take(sizeof(Item) * L.max_items);
    L.copy1 = take(sizeof(Item) * L.max_items);
  }
  L.total = off + kAlign;  // room to align the caller's base pointer
  return L;
}

// Ring capacity of the batched queue: queued segments are disjoint and hold
// more than kBaseMax keys each, plus at most one parent per resident
// workgroup while it pushes its children.
uint32_t batch_capacity(size_t n) { return static_cast<uint32_t>(n / (kBaseMax + 1) + 4096); }

Layout make_layout_opts(size_t n, size_t nseg, uint32_t kt, bool vals, bool learned, uint32_t steps, uint32_t grid,
                        bool batched = false, bool tune = false) {
  Layout L = make_layout(n, nseg, kt, vals, batched);
  const bool runs = uses_runs(n, nseg);
  if (!learned && !batched && !runs) return L;
  Bump b;
  b.off = L.total - kAlign;
  if (runs) L.runs = b.take(runs_layout(n).total);
  if (learned) {
    L.fit_out = b.take(fit_out_layout(steps).total);
    L.fit_scratch = b.take(fit_scratch_layout(grid).total);
    L.bucket = b.take(bucket_layout(n).total);
  }
  if (batched) {
    L.bcap = batch_capacity(n);
    L.bq = b.take(sizeof(BatchQ));
    L.bitems = b.take(sizeof(BItem) * static_cast<size_t>(L.bcap));
    L.bstate = b.take(4ull * L.bcap);
    if (tune) {
      L.backup_keys = b.take(n * key_bytes(kt));
      L.backup_vals = b.take(vals ? n * 4 : 0);
    }
  }
  L.total = b.off + kAlign;
  return L;
}

bool valid_key_type(int kt) { return kt >= PDQ_U32 && kt <= PDQ_F64; }

struct Opts {
  uint32_t flags = 0;
  int32_t force_budget = -1;
  uint32_t tile = 0;
  uint64_t seed = 0;
  float limit = 2.0f;
  uint32_t steps = 128;
  bool staged = true;        // learn_steps 0: the staged budget (kStage1Steps, then `steps` if needed)
  uint32_t batch = 1024;
  uint32_t grid = 16;
  uint32_t batch_shape = 0;  // 0 = tuned or default, else shape index + 1
  uint32_t batch_passes = 0; // 0 = automatic, else passes + 1
  uint32_t waves = 0;        // 0 = default / tuned base-case shapes, else lanes / 64 for every class
  const char* tune_cache = nullptr;
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
  if (sz >= offsetof(pdq_options, learned_imbalance_limit) + sizeof(float) && o->learned_imbalance_limit != 0.0f)
    out->limit = o->learned_imbalance_limit;
  if (sz >= offsetof(pdq_options, learn_steps) + sizeof(uint32_t) && o->learn_steps) {
    out->steps = o->learn_steps;
    out->staged = false;
  }
  if (sz >= offsetof(pdq_options, learn_batch) + sizeof(uint32_t) && o->learn_batch) out->batch = o->learn_batch;
  if (sz >= offsetof(pdq_options, learn_grid) + sizeof(uint32_t) && o->learn_grid) out->grid = o->learn_grid;
  if (sz >= offsetof(pdq_options, batch_shape) + sizeof(uint32_t)) out->batch_shape = o->batch_shape;
  if (sz >= offsetof(pdq_options, batch_passes) + sizeof(uint32_t)) out->batch_passes = o->batch_passes;
  if (sz >= offsetof(pdq_options, waves) + sizeof(uint32_t)) out->waves = o->waves;
  if (sz >= offsetof(pdq_options, reserved_) + sizeof(uint32_t) && o->reserved_) return PDQ_ERR_UNSUPPORTED;
  if (sz >= offsetof(pdq_options, tune_cache_path) + sizeof(const char*)) out->tune_cache = o->tune_cache_path;
  if (out->flags &
      ~static_cast<uint32_t>(PDQ_VALIDATE | PDQ_PROFILE | PDQ_LEARNED | PDQ_BATCHED | PDQ_AUTOTUNE |
                             PDQ_DETERMINISTIC | PDQ_FRESH_FIXED | PDQ_VALS64 | PDQ_HOST_LOOP | PDQ_HEAPSORT))
    return PDQ_ERR_UNSUPPORTED;
  if (out->batch_shape > static_cast<uint32_t>(kBatchShapes)) return PDQ_ERR_UNSUPPORTED;
  if (out->waves != 0 && out->waves != 1 && out->waves != 2 && out->waves != 4 && out->waves != 8 &&
      out->waves != 16)
    return PDQ_ERR_UNSUPPORTED;
  if (out->batch_passes > kMaxBatchPasses + 1) return PDQ_ERR_UNSUPPORTED;
  if (out->steps > kMaxLearnSteps || out->grid > kMaxTrainGrid || out->batch > 65536 || out->batch % out->grid)
    return PDQ_ERR_UNSUPPORTED;
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

// A counter snapshot's consistency: device-side error bits, and counts that
// fit their lists (only bad offsets can overfill a list).
int check_snapshot(const Ctx& c, const Counters& snap) {
  if (snap.errors & kErrCapacity) return PDQ_ERR_INVALID;
  if (snap.errors) return PDQ_ERR_DEVICE;
  const uint32_t nact0 = static_cast<uint32_t>(snap.list[0] >> 32), nact1 = static_cast<uint32_t>(snap.list[1] >> 32);
  if (nact0 > c.max_active || nact1 > c.max_active || static_cast<uint32_t>(snap.list[0]) > c.max_tiles ||
      static_cast<uint32_t>(snap.list[1]) > c.max_tiles)
    return PDQ_ERR_INVALID;
  for (int set = 0; set < 2; ++set)
    for (int k = 0; k < kItemCounts; ++k)
      if (item_counts(&snap, set)[k] > c.max_items) return PDQ_ERR_INVALID;
  return PDQ_OK;
}

int read_counters(const Ctx& c, Counters* snap, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(snap, c.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return check_snapshot(c, *snap);
}

// The base cases, heapsorts and copies of one item set, with the counts of
// a snapshot (`cnt`: item_counts of that set); c's lists are that set's.
int finish_set(Ctx c, const uint32_t* cnt, hipStream_t s) {
  c.device_counts = 0;
  for (int k = 0; k < kBaseClasses; ++k)
    if (cnt[k]) HIP_TRY(launch_base(c, k, cnt[k], s));
  if (cnt[kItemHeap]) HIP_TRY(launch_heap(c, cnt[kItemHeap], s));
  if (cnt[kItemCopy]) HIP_TRY(launch_copy(c, cnt[kItemCopy], s));
  return PDQ_OK;
}

int finish_items(const Ctx& c, const Counters& snap, hipStream_t s) { return finish_set(c, item_counts(&snap, 0), s); }

// Host side of the pipelined pass loop: pinned host memory that counter
// snapshots are copied into asynchronously, with one completion event per
// slot. A call takes a block from the pool for its duration; blocks are
// created on first need (one per concurrent call and device) and kept until
// the process ends.
constexpr int kPinSlots = 4;
constexpr size_t kStageBytes = 8192;  // pinned staging for the few words a host decision reads
struct PinBlock {
  int dev = -1;
  Counters* host = nullptr;
  unsigned char* stage = nullptr;
  hipEvent_t ev[kPinSlots] = {};
};
std::mutex g_pin_mu;
std::vector<PinBlock*> g_pin_free;
// set while pdq_sort_noalloc runs (and sizes its call): it allocates
// nothing and its scratch array is sized for the host-driven loop, so it
// keeps that loop with one synchronisation per pass
thread_local bool t_noalloc = false;

PinBlock* pin_acquire() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    for (size_t i = 0; i < g_pin_free.size(); ++i)
      if (g_pin_free[i]->dev == dev) {
        PinBlock* b = g_pin_free[i];
        g_pin_free.erase(g_pin_free.begin() + static_cast<long>(i));
        return b;
      }
  }
  PinBlock* b = new PinBlock;
  b->dev = dev;
  bool ok = hipHostMalloc(reinterpret_cast<void**>(&b->host), kPinSlots * sizeof(Counters), hipHostMallocDefault) ==
            hipSuccess;
  ok = ok && hipHostMalloc(reinterpret_cast<void**>(&b->stage), kStageBytes, hipHostMallocDefault) == hipSuccess;
  for (int i = 0; ok && i < kPinSlots; ++i) ok = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();  // the failure must not be reported by a later launch
    for (auto& e : b->ev)
      if (e) (void)hipEventDestroy(e);
    if (b->host) (void)hipHostFree(b->host);
    if (b->stage) (void)hipHostFree(b->stage);
    delete b;
    return nullptr;
  }
  return b;
}

void pin_release(PinBlock* b) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.push_back(b);
}

// Holds a call's block and gives it back when the call returns.
struct PinGuard {
  PinBlock* p;
  ~PinGuard() {
    if (p) pin_release(p);
  }
};

// Device -> host reads of the few words a host decision needs. With a
// pinned staging block every copy queues behind the kernels and one
// synchronisation covers them all; into pageable memory (no block: the
// call allocates nothing) each copy waits on its own.
struct ReadItem {
  void* dst;
  const void* src;
  size_t bytes;
};
int read_to_host(PinBlock* pin, const ReadItem* it, int k, hipStream_t s) {
  size_t total = 0;
  for (int i = 0; i < k; ++i) total += (it[i].bytes + 7) & ~static_cast<size_t>(7);
  const bool staged = pin && pin->stage && total <= kStageBytes;
  size_t off = 0;
  for (int i = 0; i < k; ++i) {
    void* d = staged ? static_cast<void*>(pin->stage + off) : it[i].dst;
    HIP_TRY(hipMemcpyAsync(d, it[i].src, it[i].bytes, hipMemcpyDeviceToHost, s));
    off += (it[i].bytes + 7) & ~static_cast<size_t>(7);
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (staged) {
    off = 0;
    for (int i = 0; i < k; ++i) {
      memcpy(it[i].dst, pin->stage + off, it[i].bytes);
      off += (it[i].bytes + 7) & ~static_cast<size_t>(7);
    }
  }
  return PDQ_OK;
}

int run_sort(void* keys, uint32_t* vals, size_t n, const uint64_t* offsets, size_t nseg, int kt, int order,
             void* ws, size_t ws_bytes, void* stream, const pdq_options* opt, pdq_stats* st);

char* align_ptr(void* p) {
  return reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + kAlign - 1) / kAlign * kAlign);
}

FitBufs fit_bufs(char* out, char* scratch, uint32_t steps, uint32_t grid) {
  const FitOutLayout fo = fit_out_layout(steps);
  const FitScratchLayout fs = fit_scratch_layout(grid);
  FitBufs f;
  f.sample = reinterpret_cast<uint64_t*>(out + fo.sample);
  f.x = reinterpret_cast<float*>(out + fo.x);
  f.t = reinterpret_cast<float*>(out + fo.t);
  f.y = reinterpret_cast<float*>(out + fo.y);
  f.params = reinterpret_cast<float*>(out + fo.params);
  f.losses = reinterpret_cast<float*>(out + fo.losses);
  f.splitters = reinterpret_cast<uint64_t*>(out + fo.splitters);
  f.count = reinterpret_cast<uint32_t*>(out + fo.count);
  f.info = reinterpret_cast<uint64_t*>(out + fo.info);
  f.runmax = reinterpret_cast<float*>(scratch + fs.runmax);
  f.partials = reinterpret_cast<float*>(scratch + fs.partials);
  f.sync = reinterpret_cast<uint32_t*>(scratch + fs.sync);
  f.raw = reinterpret_cast<uint64_t*>(scratch + fs.raw);
  f.runmax2 = reinterpret_cast<float*>(scratch + fs.runmax2);
  f.yx = reinterpret_cast<float*>(scratch + fs.yx);
  f.yy = reinterpret_cast<float*>(scratch + fs.yy);
  f.leaf = reinterpret_cast<double*>(scratch + fs.leaf);
  f.cand = reinterpret_cast<uint64_t*>(scratch + fs.cand);
  f.cand_count = reinterpret_cast<uint32_t*>(scratch + fs.cand_count);
  f.est = reinterpret_cast<uint64_t*>(scratch + fs.est);
  return f;
}

// Sample, sample sort, features, training, inference, the second stage,
// three candidate splitter sets judged on the sample and the best one kept,
// all queued on the stream without a synchronisation. info[7] says whether
// the winner's sample judge is within `go_limit` sample keys (the histogram
// kernels run only then).
// The sample: m keys at hashed positions, sorted, with their features and
// targets.
int run_fit_sample(const void* keys, uint64_t n, uint32_t kt, const Opts& o, const FitBufs& f, hipStream_t s) {
  const uint64_t m = kLearnSample;
  HIP_TRY(launch_sample(kt, keys, n, m, o.seed, f.raw, s));
  HIP_TRY(launch_sample_sort(f.raw, m, f.sample, s));
  HIP_TRY(launch_features(f.sample, m, f.x, f.t, f.info, s));
  return PDQ_OK;
}

// Training of `steps` Adam steps from the seeded initial parameters,
// inference, the second stage, three candidate splitter sets judged on the
// sample and the best one kept, all queued without a synchronisation.
// info[7] says whether the winner's sample judge is within `go_limit`
// sample keys (the histogram kernels run only then).
int run_fit_model(const Opts& o, uint32_t steps, const FitBufs& f, hipStream_t s, uint64_t go_limit) {
  const uint64_t m = kLearnSample;
  TrainArgs a;
  a.x = f.x;
  a.t = f.t;
  a.m = m;
  a.seed = o.seed;
  a.steps = steps;
  a.batch = o.batch;
  a.grid = o.grid;
  a.residual = 1;
  a.init = nullptr;
  a.params = f.params;
  a.losses = f.losses;
  a.partials = f.partials;
  a.sync = f.sync;
  HIP_TRY(launch_train(a, s));
  HIP_TRY(launch_infer(f.params, f.x, m, 1u, f.y, s));
  // the running maximum of the network's prediction defines the leaves; then
  // the three candidates' splitters are extracted side by side
  HIP_TRY(launch_running_max(f.y, m, f.runmax, s));
  HIP_TRY(launch_leaves(f.x, f.t, f.y, f.runmax, m, f.leaf, f.yx, f.yy, s));
  const float* preds[kCandidates] = {f.y, f.yx, f.yy};
  float* maxima[kCandidates] = {f.runmax, f.runmax2, f.runmax2 + m};
  HIP_TRY(launch_extract_candidates(f.sample, m, preds, maxima, f.cand, 256, f.cand_count, s));
  HIP_TRY(launch_sample_judge(f.sample, m, f.cand, 256, f.cand_count, kCandidates, f.est, s));
  HIP_TRY(launch_pick(f.cand, 256, f.cand_count, f.est, kCandidates, go_limit, f.splitters, f.count, f.info, s));
  return PDQ_OK;
}

// Whether a short fit is kept: its fullest range bin holds at most
// 1.3 m / 256 sample keys (judge * 2560 <= 13 m), or more than 4 m / 256
// (judge * 64 > m), which longer training does not bring to the limit.
bool early_accept(uint64_t judge, uint64_t m) { return judge * 2560ull <= 13ull * m; }
bool hopeless(uint64_t judge, uint64_t m) { return judge * 64ull > m; }

// The whole fit. With the staged budget (learn_steps 0) a kStage1Steps fit
// is judged first (one synchronisation to read its sample judge) and kept
// when early_accept or hopeless holds; otherwise the model is trained again
// from the same initial parameters for o.steps steps. *steps_run receives
// the steps of the kept fit.
int run_fit(const void* keys, uint64_t n, uint32_t kt, const Opts& o, const FitBufs& f, hipStream_t s,
            uint64_t go_limit = ~0ull, uint32_t* steps_run = nullptr, PinBlock* pin = nullptr) {
  int rc = run_fit_sample(keys, n, kt, o, f, s);
  if (rc != PDQ_OK) return rc;
  uint32_t steps = o.steps;
  if (o.staged && kStage1Steps < o.steps) {
    rc = run_fit_model(o, kStage1Steps, f, s, go_limit);
    if (rc != PDQ_OK) return rc;
    uint64_t info[kInfoWords] = {};
    const ReadItem rd[] = {{info, f.info, sizeof(info)}};
    rc = read_to_host(pin, rd, 1, s);
    if (rc != PDQ_OK) return rc;
    const uint64_t choice = info[3] < kCandidates ? info[3] : 0;
    if (early_accept(info[4 + choice], kLearnSample) || hopeless(info[4 + choice], kLearnSample)) {
      if (steps_run) *steps_run = kStage1Steps;
      return PDQ_OK;
    }
  }
  rc = run_fit_model(o, steps, f, s, go_limit);
  if (rc == PDQ_OK && steps_run) *steps_run = steps;
  return rc;
}

BucketBufs bucket_bufs(char* area, uint64_t n, const uint64_t* splitters, const uint32_t* count) {
  const BucketLayout L = bucket_layout(n);
  BucketBufs b;
  b.splitters = splitters;
  b.count = count;
  b.rows = reinterpret_cast<uint32_t*>(area + L.rows);
  b.chunk = reinterpret_cast<uint32_t*>(area + L.chunk);
  b.totals = reinterpret_cast<uint64_t*>(area + L.totals);
  b.begin = reinterpret_cast<uint64_t*>(area + L.begin);
  b.ntiles = bucket_tiles(n);
  b.nchunks = bucket_chunks(n);
  b.errors = nullptr;
  b.order = reinterpret_cast<uint32_t*>(area + L.order);
  b.go = nullptr;
  return b;
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() = default;
  EventPair(const EventPair&) = delete;
  EventPair& operator=(const EventPair&) = delete;
  bool make() { return hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess; }
  double ms() const {
    float v = 0;
    if (a && b) (void)hipEventElapsedTime(&v, a, b);
    return v;
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// What the learned first pass found, for the statistics.
struct LearnedResult {
  uint32_t state = 0;  // 0 not run, 1 used, 2 fell back
  uint32_t splitters = 0, use_log = 0, ordered = 0, choice = 0, steps = 0;
  uint64_t sample_judge = 0;
  uint64_t max_range = 0, equal = 0;
  float loss = 0.0f;
  double fit_ms = 0, hist_ms = 0;
  uint64_t hist_bytes = 0, scatter_bytes = 0;
  // the scatter's events live as long as the result: they are read once the
  // whole sort has been waited for, so timing it costs no wait in the middle
  EventPair scat;
};

// Fit, histogram, judge and (if the judge agrees) scatter into bins.
// Returns with res.state 1 when the bins were set up as the first lists,
// 2 when the caller must start the plain path.
// `unordered`: the run scan has already seen both a descending and an
// ascending adjacent pair, so the order scan is skipped.
int run_learned(Ctx& c, const Opts& o, const Layout& L, char* base, bool prof, LearnedResult& res, hipStream_t s,
                bool unordered = false, PinBlock* pin = nullptr) {
  const uint32_t kt = c.key_type;
  const uint64_t n = c.n;
  const uint32_t kb = key_bytes(kt);
  const FitBufs f = fit_bufs(base + L.fit_out, base + L.fit_scratch, o.steps, o.grid);
  BucketBufs b = bucket_bufs(base + L.bucket, n, f.splitters, f.count);
  b.errors = &c.ctr->errors;
  EventPair e_fit, e_hist;
  EventPair& e_scat = res.scat;
  if (prof && !(e_fit.make() && e_hist.make() && e_scat.make())) return PDQ_ERR_HIP;
  if (!unordered) {
    // an input that is already non-decreasing or non-increasing is retired
    // by the plain path's first pass: find out before the fit is paid for
    uint32_t order_bits = 0;
    HIP_TRY(launch_order_scan(kt, c.keys[0], n, b.order, s));
    const ReadItem rd[] = {{&order_bits, b.order, 4}};
    const int rc0 = read_to_host(pin, rd, 1, s);
    if (rc0 != PDQ_OK) return rc0;
    if ((order_bits & 1u) == 0 || (order_bits & 2u) == 0) {
      res.ordered = 1;
      res.state = 2;
      return PDQ_OK;
    }
  }
  if (prof) HIP_TRY(hipEventRecord(e_fit.a, s));
  // the histogram runs only when the chosen splitters' sample judge is
  // within the limit with a 15 % margin for sampling error (the sample
  // holds m keys: a range bin at the limit holds limit * m / 256 of them)
  const double lim = o.limit >= 0.0f ? 1.15 * static_cast<double>(o.limit) * static_cast<double>(kLearnSample) / 256.0
                                     : -1.0;
  const uint64_t go_limit = lim >= 0.0 ? static_cast<uint64_t>(lim) : 0ull;
  b.go = f.info + 7;
  uint32_t steps_run = o.steps;
  int rc = run_fit(c.keys[0], n, kt, o, f, s, go_limit, &steps_run, pin);
  if (rc != PDQ_OK) return rc;
  res.steps = steps_run;
  if (prof) {
    HIP_TRY(hipEventRecord(e_fit.b, s));
    HIP_TRY(hipEventRecord(e_hist.a, s));
  }
  HIP_TRY(launch_bucket_hist(kt, c.keys[0], n, b, s));
  HIP_TRY(launch_bucket_scan(b, s));
  if (prof) HIP_TRY(hipEventRecord(e_hist.b, s));
  // judge on the host: bin totals, splitter count, trainer flag, last loss
  uint64_t totals[kBinStride];
  uint32_t count = 0, sync[2] = {0, 0};
  uint64_t info[kInfoWords] = {};
  float loss = 0.0f;
  {
    const ReadItem rd[] = {{totals, b.totals, sizeof(totals)},
                           {&count, f.count, 4},
                           {sync, f.sync, 8},
                           {info, f.info, sizeof(info)},
                           {&loss, f.losses + (steps_run - 1), 4}};
    rc = read_to_host(pin, rd, 5, s);
    if (rc != PDQ_OK) return rc;
  }
  res.splitters = count;
  res.use_log = static_cast<uint32_t>(info[2]);
  res.loss = loss;
  res.choice = static_cast<uint32_t>(info[3]);
  res.sample_judge = info[4 + (info[3] < kCandidates ? info[3] : 0)];
  if (info[7] == 0) {
    // the sample judge rejected every candidate: the histogram did not run
    res.state = 2;
    if (prof) res.fit_ms = e_fit.ms();
    return PDQ_OK;
  }
  uint64_t max_range = 0, equal = 0;
  for (uint32_t i = 0; i <= 2 * count && i < static_cast<uint32_t>(kBinStride); ++i) {
    if (i & 1u) equal += totals[i];
    else if (totals[i] > max_range) max_range = totals[i];
  }
  res.max_range = max_range;
  res.equal = equal;
  // (an ordered input never gets here: the order scan sent it to the plain
  // path, whose first pass retires it)
  const bool ok = sync[1] == 0 && isfinite(loss) && o.limit >= 0.0f &&
                  static_cast<double>(max_range) <= static_cast<double>(o.limit) * static_cast<double>(n) / 256.0;
  if (prof) {
    res.fit_ms = e_fit.ms();
    res.hist_ms = e_hist.ms();
    res.hist_bytes = n * kb;
  }
  if (!ok) {
    res.state = 2;
    return PDQ_OK;
  }
  if (prof) HIP_TRY(hipEventRecord(e_scat.a, s));
  HIP_TRY(launch_bucket_scatter(kt, c.has_vals != 0, c.keys[0], c.vals[0], c.keys[1], c.vals[1], n, b, s));
  if (prof) HIP_TRY(hipEventRecord(e_scat.b, s));
  HIP_TRY(launch_bucket_init(c, b.begin, s));
  if (prof) {
    res.scatter_bytes = n * 2ull * (kb + (c.has_vals ? 4u : 0u));
  }
  res.state = 1;
  return PDQ_OK;
}

// pdq_options.waves: every base-case class that has a shape of that many
// waves per workgroup takes it.
void apply_waves(Ctx& c, uint32_t waves) {
  if (!waves) return;
  const bool wide = key_bytes(c.key_type) == 8 && c.has_vals;
  for (int k = 0; k < kBaseClasses; ++k)
    for (int v = 0; v < kBaseVariants; ++v)
      if (kBaseThreads[wide ? 1 : 0][k][v] == 64u * waves) c.base_var[k] = static_cast<uint8_t>(v);
}

Ctx make_ctx(void* keys, uint32_t* vals, size_t n, const uint64_t* offsets, size_t nseg, int kt, const Opts& o,
             const Layout& L, char* base) {
  Ctx c = {};
  c.keys[0] = keys;
  c.keys[1] = base + L.scratch_keys;
  c.vals[0] = vals;
  c.vals[1] = vals ? reinterpret_cast<uint32_t*>(base + L.scratch_vals) : nullptr;
  c.n = n;
  c.segs[0] = reinterpret_cast<Seg*>(base + L.segs0);
  c.segs[1] = reinterpret_cast<Seg*>(base + L.segs1);
  c.tilemap = reinterpret_cast<uint32_t*>(base + L.tilemap);
  c.cur = reinterpret_cast<Cursor*>(base + L.cur);
  c.tickets = reinterpret_cast<uint32_t*>(base + L.tickets);
  c.status = reinterpret_cast<uint64_t*>(base + L.status);
  for (int k = 0; k < kBaseClasses; ++k) c.base[k] = reinterpret_cast<Item*>(base + L.base[k]);
  c.heap = reinterpret_cast<Item*>(base + L.heap);
  c.copy = reinterpret_cast<Item*>(base + L.copy);
  c.ctr = reinterpret_cast<Counters*>(base + L.ctr);
  c.icnt = item_counts(c.ctr, 0);
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
  c.base_max = kBaseMax;
  for (int k = 0; k < kBaseClasses; ++k) c.base_var[k] = 0;
  apply_waves(c, o.waves);
  c.lookback = (o.flags & PDQ_DETERMINISTIC) ? 1u : 0u;
  c.fresh_fixed = (o.flags & PDQ_FRESH_FIXED) ? 1u : 0u;
  c.heapsort = (o.flags & PDQ_HEAPSORT) ? 1u : 0u;
  return c;
}

// ---- near-sorted inputs -------------------------------------------------------

RunBufs run_bufs(const Layout& L, char* base, size_t n) {
  const RunsLayout r = runs_layout(n);
  char* a = base + L.runs;
  RunBufs rb;
  rb.count = reinterpret_cast<uint32_t*>(a + r.count);
  rb.pos = reinterpret_cast<uint32_t*>(a + r.pos);
  rb.plan = reinterpret_cast<RunPlan*>(a + r.plan);
  rb.shorts = reinterpret_cast<RunSpan*>(a + r.shorts);
  rb.item = reinterpret_cast<Item*>(a + r.item);
  rb.okeys = a + r.okeys;
  rb.ovals = reinterpret_cast<uint32_t*>(a + r.ovals);
  rb.splits = reinterpret_cast<uint64_t*>(a + r.splits);
  return rb;
}

// The GPU form of Section 5.2's partial insertion sort (k_runs.hip): one
// scan finds the runs; a range that is already sorted, one long run plus a
// few outliers, or two long runs is finished here by a merge and
// plan->state says so; otherwise (state kRunUnsorted) the partition passes
// sort it.
int run_near_sorted(const Ctx& c, const Layout& L, char* base, RunPlan* plan, hipStream_t s, PinBlock* pin = nullptr) {
  const RunBufs rb = run_bufs(L, base, c.n);
  HIP_TRY(launch_run_scan(c, rb, s));
  {
    const ReadItem rd[] = {{plan, rb.plan, sizeof(RunPlan)}};
    const int rc = read_to_host(pin, rd, 1, s);
    if (rc != PDQ_OK) return rc;
  }
  if (plan->state == kRunOutliers) {
    HIP_TRY(launch_run_gather(c, rb, plan->nshort, s));
    if (plan->outliers > 1) {
      // the LDS base case sorts the outlier buffer in place, as one item
      Ctx o = c;
      o.keys[0] = o.keys[1] = rb.okeys;
      o.vals[0] = o.vals[1] = c.has_vals ? rb.ovals : nullptr;
      const int cls = base_class(plan->outliers);
      o.base[cls] = rb.item;
      o.device_counts = 0;
      o.max_items = 1;
      HIP_TRY(launch_base(o, cls, 1, s));
    }
    HIP_TRY(launch_run_merge(c, rb, *plan, s));
  } else if (plan->state == kRunTwoRuns) {
    HIP_TRY(launch_run_merge(c, rb, *plan, s));
  }
  return PDQ_OK;
}

// ---- batched segmented sort --------------------------------------------------

// The batched form's configuration: the shape (partition tile) and the
// workgroup shape of every base-case class.
struct Tuned {
  int shape = 0;
  uint8_t var[kBaseClasses] = {};
};

// Autotuned configurations, remembered per (key type, payload, n, segment
// count) in process memory, and in pdq_options.tune_cache_path when given.
std::mutex g_tune_mu;
std::map<std::tuple<uint32_t, uint32_t, uint64_t, uint64_t>, Tuned> g_tune;

// "<gfx arch>/<compute units> <key type> <payload> <n> <segments>": a cache
// line is only taken on the same kind of device for the same problem.
std::string tune_key(const Ctx& c) {
  int dev = 0;
  hipDeviceProp_t prop = {};
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  char buf[256];
  snprintf(buf, sizeof(buf), "%s/%d %u %u %llu %llu", arch.c_str(), cus, c.key_type, c.has_vals,
           static_cast<unsigned long long>(c.n), static_cast<unsigned long long>(c.nseg));
  return buf;
}

// Cache file lines: "pdq-tune 1 <key> <shape> <variant of class 0> ... <class 6>".
bool cache_lookup(const char* path, const std::string& key, Tuned* out) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  const std::string prefix = "pdq-tune 1 " + key + " ";
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    if (strncmp(line, prefix.c_str(), prefix.size()) != 0) continue;
    int v[1 + kBaseClasses];
    if (sscanf(line + prefix.size(), "%d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6],
               &v[7]) != 1 + kBaseClasses)
      continue;
    bool ok = v[0] >= 0 && v[0] < kBatchShapes;
    for (int k = 0; k < kBaseClasses; ++k) ok = ok && v[1 + k] >= 0 && v[1 + k] < kBaseVariants;
    if (!ok) continue;
    out->shape = v[0];
    for (int k = 0; k < kBaseClasses; ++k) out->var[k] = static_cast<uint8_t>(v[1 + k]);
    found = true;  // the last matching line wins
  }
  fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const Tuned& t) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "pdq-tune 1 %s %d", key.c_str(), t.shape);
  for (int k = 0; k < kBaseClasses; ++k) fprintf(f, " %d", t.var[k]);
  fprintf(f, "\n");
  fclose(f);
}

// The configuration a batched call uses: an explicit batch_shape, else the
// tuned one of this process, else the cache file's, else the defaults; then
// pdq_options.waves, if set, for the base-case classes.
Tuned tuned_config(const Ctx& c, const Opts& o) {
  Tuned t;
  bool have = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(c.key_type, c.has_vals, c.n, c.nseg));
    if (it != g_tune.end()) {
      t = it->second;
      have = true;
    }
  }
  if (!have && o.tune_cache && cache_lookup(o.tune_cache, tune_key(c), &t)) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(c.key_type, c.has_vals, c.n, c.nseg)] = t;
  }
  if (o.batch_shape) {
    t = Tuned();
    t.shape = static_cast<int>(o.batch_shape) - 1;
    if (kShapes[t.shape].wide_e == 32) t.var[5] = t.var[6] = 1;  // the 32-slot widest classes
  }
  if (o.waves) {
    Ctx tmp = c;
    for (int k = 0; k < kBaseClasses; ++k) tmp.base_var[k] = t.var[k];
    apply_waves(tmp, o.waves);
    for (int k = 0; k < kBaseClasses; ++k) t.var[k] = tmp.base_var[k];
  }
  return t;
}

BatchArgs batch_args(const Layout& L, char* base) {
  BatchArgs b;
  b.q = reinterpret_cast<BatchQ*>(base + L.bq);
  b.items = reinterpret_cast<BItem*>(base + L.bitems);
  b.state = reinterpret_cast<uint32_t*>(base + L.bstate);
  return b;
}

// The batched form's context: device-side counts, accumulating item lists,
// the wide LDS classes, the shape's partition tile and the classes' shapes.
Ctx batch_ctx(Ctx c, const Opts& o, const Tuned& t) {
  c.device_counts = 1;
  c.accumulate = 1;
  c.base_max = batch_base_max(c.key_type, c.has_vals != 0);
  c.tile = o.tile ? o.tile : kShapes[t.shape].tile;
  for (int k = 0; k < kBaseClasses; ++k) c.base_var[k] = t.var[k];
  return c;
}

// Device-counted passes to queue for a largest segment of m keys: the
// halvings that bring it to base_max, plus 3 and half of them again
// (splits are uneven, so some paths need more passes; a pass that finds no
// live segment costs a few microseconds, while a segment left to the
// persistent tail is partitioned by a single workgroup). Anything deeper
// finishes in the persistent tail.
uint32_t batch_passes(uint64_t m, uint32_t base_max) {
  uint32_t p = 0;
  while (m > base_max && p < kMaxBatchPasses) {
    m = (m + 1) / 2;
    ++p;
  }
  if (p == 0) return 0;
  p += 3 + p / 2;
  return p < kMaxBatchPasses ? p : kMaxBatchPasses;
}

// First step, the same for every shape: counters, and the input segments
// filed into the item lists and live list 0.
int enqueue_batch_init(const Ctx& c, hipStream_t s) {
  HIP_TRY(launch_reset(c, s));
  HIP_TRY(launch_init(c, s));
  return PDQ_OK;
}

// Reads the counters after the first step: offsets, capacity, and the
// number of passes to queue.
int batch_probe(const Ctx& c, const Opts& o, hipStream_t s, uint32_t* passes) {
  Counters snap = {};
  HIP_TRY(hipMemcpyAsync(&snap, c.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (snap.bad_offsets || (snap.errors & kErrCapacity)) return PDQ_ERR_INVALID;
  *passes = o.batch_passes ? o.batch_passes - 1 : batch_passes(snap.max_seg, c.base_max);
  return PDQ_OK;
}

// The rest, with no host synchronisation (capturable): `passes` partition
// passes whose kernels read their counts on the device, the persistent tail
// over whatever is still live, then every item list finished once.
// `src0`: the buffer the live segments of list 0 are in. `timed`: events
// around every partition launch (PDQ_PROFILE).
int enqueue_batch_rest(const Ctx& c, const Layout& L, char* base, uint32_t passes, int tail, hipStream_t s,
                       EventPair* class_ev = nullptr, uint32_t src0 = 0, std::vector<Timed>* timed = nullptr) {
  const BatchArgs b = batch_args(L, base);
  const uint32_t grid = batch_grid(c, tail);
  if (grid == 0) return PDQ_ERR_HIP;
  int parity = 0;
  uint32_t src = src0;
  for (uint32_t p = 0; p < passes; ++p) {
    HIP_TRY(launch_pivot(c, parity, c.max_active, src, s));
    HIP_TRY(launch_tilemap(c, parity, c.max_tiles, s));
    if (timed) {
      Timed tm;
      HIP_TRY(hipEventCreate(&tm.a));
      timed->push_back(tm);
      HIP_TRY(hipEventCreate(&timed->back().b));
      HIP_TRY(hipEventRecord(timed->back().a, s));
    }
    HIP_TRY(launch_partition(c, parity, c.max_tiles, src, s));
    if (timed) HIP_TRY(hipEventRecord(timed->back().b, s));
    HIP_TRY(launch_bookkeep(c, parity, c.max_active, src, p, s));
    parity ^= 1;
    src ^= 1u;
  }
  HIP_TRY(launch_batch_zero(b, L.bcap, s));
  HIP_TRY(launch_batch_from_list(c, b, parity, src, s));
  HIP_TRY(launch_batch(c, b, tail, grid, s));
  HIP_TRY(launch_batch_fold(c, b, s));
  for (int k = 0; k < kBaseClasses; ++k) {
    if (k == 6 && c.base_max < kWideBaseMax) continue;
    if (class_ev) HIP_TRY(hipEventRecord(class_ev[k].a, s));
    HIP_TRY(launch_base(c, k, c.max_items, s));
    if (class_ev) HIP_TRY(hipEventRecord(class_ev[k].b, s));
  }
  HIP_TRY(launch_heap(c, c.max_items, s));
  HIP_TRY(launch_copy(c, c.max_items, s));
  return PDQ_OK;
}

// Whether a call runs the device-counted passes: single-range sorts, unless
// PDQ_HOST_LOOP asks for the host-driven loop or pdq_sort_noalloc runs (its
// scratch array is sized for the host loop's smaller workspace).
bool device_passes(const uint64_t* offsets, const Opts& o) {
  return !offsets && !(o.flags & PDQ_HOST_LOOP) && !t_noalloc;
}

// The statistics every form reads from the final counters.
void fill_pass_stats(pdq_stats* st, const Counters& snap) {
  st->element_visits = snap.visits;
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
}

void fill_learned_stats(pdq_stats* st, const LearnedResult& lres) {
  st->learned = lres.state;
  st->learned_splitters = lres.splitters;
  st->learned_max_range_bin = lres.max_range;
  st->learned_equal_elements = lres.state == 1 ? lres.equal : 0;
  st->learned_final_loss = lres.loss;
  st->learned_use_log = lres.use_log;
  st->learned_choice = lres.choice;
  st->learned_steps = lres.steps;
  st->learned_sample_judge = lres.sample_judge;
  st->learned_fit_ms = lres.fit_ms;
  st->learned_hist_ms = lres.hist_ms;
  st->learned_scatter_ms = lres.state == 1 ? lres.scat.ms() : 0.0;  // the sort has been waited for
  st->learned_hist_bytes = lres.hist_bytes;
  st->learned_scatter_bytes = lres.scatter_bytes;
}

// Partition launch times of PDQ_PROFILE: their sum, and the first launch.
void fill_profile_stats(pdq_stats* st, const std::vector<Timed>& timed, uint64_t total_bytes) {
  double total = 0;
  for (size_t i = 0; i < timed.size(); ++i) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, timed[i].a, timed[i].b);
    total += ms;
    if (i == 0) {
      st->first_pass_ms = ms;
      st->first_pass_bytes = timed[i].bytes;
    }
  }
  st->partition_launches = static_cast<uint32_t>(timed.size());
  st->partition_ms = total;
  st->partition_bytes = total_bytes;
}

// Statistics of a single-range sort that ran the device-counted passes (one
// synchronisation, here at the end). Device-side errors are reported now.
int device_pass_stats(const Ctx& c, const Layout& L, char* base, uint32_t kb, bool vals, const LearnedResult& lres,
                      bool prof, const std::vector<Timed>& timed, pdq_stats* st, hipStream_t s) {
  Counters snap = {};
  BatchQ q = {};
  HIP_TRY(hipMemcpyAsync(&snap, c.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&q, batch_args(L, base).q, sizeof(BatchQ), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (snap.errors & kErrCapacity) return PDQ_ERR_INVALID;
  if (snap.errors || q.error) return PDQ_ERR_DEVICE;
  fill_pass_stats(st, snap);
  st->passes = snap.live_passes;
  st->batch_items = q.tail;
  fill_learned_stats(st, lres);
  if (prof) {
    // the first launch's bytes are known for a plain single range (n keys);
    // after the learned split they depend on the bins and are left at 0
    std::vector<Timed> t = timed;
    const uint64_t bpk = 2ull * kb + (vals ? 8ull : 0ull);
    if (!t.empty() && lres.state != 1) t[0].bytes = c.n * bpk;
    fill_profile_stats(st, t, snap.visits * bpk);
  }
  return PDQ_OK;
}

int run_batched(const Ctx& c0, const Opts& o, const Layout& L, char* base, pdq_stats* st, hipStream_t s) {
  const Tuned tc = tuned_config(c0, o);
  const int shape = tc.shape;
  const Ctx c = batch_ctx(c0, o, tc);
  EventPair ev;
  const bool prof = (o.flags & PDQ_PROFILE) && st;
  if (prof && !ev.make()) return PDQ_ERR_HIP;
  int rc = enqueue_batch_init(c, s);
  if (rc != PDQ_OK) return rc;
  uint32_t passes = 0;
  rc = batch_probe(c, o, s, &passes);
  if (rc != PDQ_OK) return rc;
  if (prof) HIP_TRY(hipEventRecord(ev.a, s));
  rc = enqueue_batch_rest(c, L, base, passes, kShapes[shape].tail, s);
  if (rc != PDQ_OK) return rc;
  if (prof) HIP_TRY(hipEventRecord(ev.b, s));
  if (!st) return PDQ_OK;
  Counters snap = {};
  BatchQ q = {};
  HIP_TRY(hipMemcpyAsync(&snap, c.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&q, batch_args(L, base).q, sizeof(BatchQ), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (snap.errors & kErrCapacity) return PDQ_ERR_INVALID;
  if (snap.errors || q.error) return PDQ_ERR_DEVICE;
  fill_pass_stats(st, snap);
  st->passes = passes;
  st->batch_items = q.tail;
  st->batch_shape = static_cast<uint32_t>(shape);
  if (prof) st->batch_ms = ev.ms();
  return PDQ_OK;
}

// Pass loop with one host synchronisation per pass: the counters after a
// pass size the next one exactly. Used where pinned host memory is not to
// be allocated (pdq_sort_noalloc) or cannot be.
int run_passes_sync(Ctx& c, const Opts& o, Counters& snap, uint32_t src, bool prof, uint64_t bytes_per_key,
                    std::vector<Timed>& timed, uint32_t* passes, uint64_t* visits_out, hipStream_t s) {
  int parity = 0;
  uint32_t pass = 0;
  uint64_t visits = 0;
  for (;;) {
    const uint32_t nact = static_cast<uint32_t>(snap.list[parity] >> 32);
    const uint32_t ntiles = static_cast<uint32_t>(snap.list[parity]);
    if (nact == 0) break;
    if (pass >= kMaxPasses) return PDQ_ERR_HIP;
    visits += snap.elems[parity];
    HIP_TRY(launch_pivot(c, parity, nact, src, s));
    HIP_TRY(launch_tilemap(c, parity, ntiles, s));
    Timed tm;
    if (prof) {
      HIP_TRY(hipEventCreate(&tm.a));
      timed.push_back(tm);
      HIP_TRY(hipEventCreate(&timed.back().b));
      timed.back().bytes = snap.elems[parity] * bytes_per_key;
      HIP_TRY(hipEventRecord(timed.back().a, s));
    }
    HIP_TRY(launch_partition(c, parity, ntiles, src, s));
    if (prof) HIP_TRY(hipEventRecord(timed.back().b, s));
    // the children filed now are tiled for the next pass: about two per
    // segment, sharing its keys; the next pass's largest segment is taken as
    // half this pass's largest
    if (!o.tile) c.tile = auto_tile(snap.elems[parity], (snap.maxlen[parity] + 1) / 2);
    HIP_TRY(launch_bookkeep(c, parity, nact, src, pass, s));
    int r = read_counters(c, &snap, s);
    if (r == PDQ_OK) r = finish_items(c, snap, s);
    if (r != PDQ_OK) return r;
    parity ^= 1;
    src ^= 1u;
    ++pass;
  }
  *passes = pass;
  *visits_out = visits;
  return PDQ_OK;
}

// The context of item set `set`: its lists and its counts.
Ctx with_items(Ctx c, const Layout& L, char* base, int set) {
  for (int k = 0; k < kBaseClasses; ++k) c.base[k] = reinterpret_cast<Item*>(base + (set ? L.base1[k] : L.base[k]));
  c.heap = reinterpret_cast<Item*>(base + (set ? L.heap1 : L.heap));
  c.copy = reinterpret_cast<Item*>(base + (set ? L.copy1 : L.copy));
  c.icnt = item_counts(c.ctr, set);
  return c;
}

// Pass loop that keeps the GPU fed. Pass q + 1 is queued before the host
// has seen the counters after pass q: its kernels take their counts on the
// device, and their grids come from bounds on pass q's live list (at most
// two children per segment, no more keys), which the counters after pass
// q - 1 give. The counters after every pass are copied into pinned host
// memory as the pass's last step, and while the GPU runs pass q + 1 the
// host reads those of pass q, queues the finishing of pass q - 1's items
// and then pass q + 2. Passes alternate between two item sets, so the
// items of pass q - 1 are finished while pass q fills the other set; every
// item range is retired, so no later pass touches it. The loop ends when
// the counters show an empty live list: the pass already queued for it
// finds nothing to do.
int run_passes_pipelined(Ctx c, const Opts& o, const Layout& L, char* base, const Counters& init, uint32_t src0,
                         bool prof, uint64_t bytes_per_key, std::vector<Timed>& timed, uint32_t* passes,
                         uint64_t* visits_out, PinBlock* pin, hipStream_t s) {
  Ctx cp = c;
  cp.device_counts = 1;
  // tile_of[q % 4]: the tile of pass q (its segments were tiled for it by
  // the bookkeeping of pass q - 1)
  uint32_t tile_of[4];
  tile_of[0] = c.tile;
  int last = -1;  // the last slot a counter copy was queued into
  auto enqueue = [&](uint32_t q, uint32_t live_bound, uint32_t tile_bound) -> int {
    const int parity = static_cast<int>(q & 1u);
    const uint32_t src = src0 ^ (q & 1u);
    Ctx cq = with_items(cp, L, base, static_cast<int>((q + 1) & 1u));
    cq.tile = tile_of[q % 4];
    HIP_TRY(launch_pivot(cq, parity, live_bound, src, s));
    HIP_TRY(launch_tilemap(cq, parity, tile_bound, s));
    if (prof) {
      Timed tm;
      HIP_TRY(hipEventCreate(&tm.a));
      timed.push_back(tm);
      HIP_TRY(hipEventCreate(&timed.back().b));
      HIP_TRY(hipEventRecord(timed.back().a, s));
    }
    HIP_TRY(launch_partition(cq, parity, tile_bound, src, s));
    if (prof) HIP_TRY(hipEventRecord(timed.back().b, s));
    cq.tile = tile_of[(q + 1) % 4];
    HIP_TRY(launch_bookkeep(cq, parity, live_bound, src, q, s));
    const int slot = static_cast<int>(q % kPinSlots);
    HIP_TRY(hipMemcpyAsync(&pin->host[slot], c.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(pin->ev[slot], s));
    last = slot;
    return PDQ_OK;
  };
  // no copy may still be landing in the pinned block once it is handed back
  auto drain = [&](int rc) {
    if (last >= 0) (void)hipEventSynchronize(pin->ev[last]);
    return rc;
  };
  const uint32_t live0 = static_cast<uint32_t>(init.list[0] >> 32);
  if (live0 == 0) {
    *passes = 0;
    *visits_out = 0;
    return PDQ_OK;
  }
  tile_of[1] = o.tile ? o.tile : auto_tile(init.elems[0], (init.maxlen[0] + 1) / 2);
  int rc = enqueue(0, live0, static_cast<uint32_t>(init.list[0]));
  if (rc != PDQ_OK) return drain(rc);
  Counters prev = init;  // the counters after pass q - 1 (the initial lists for q = 0)
  uint64_t visits = 0;
  uint32_t q = 0;
  for (;;) {
    const int parity = static_cast<int>(q & 1u);
    // pass q - 1's items (set q & 1), queued before pass q + 1 clears that set
    if (q > 0) {
      rc = finish_set(with_items(c, L, base, parity), item_counts(&prev, parity), s);
      if (rc != PDQ_OK) return drain(rc);
    }
    const uint32_t live = static_cast<uint32_t>(prev.list[parity] >> 32);
    if (live == 0) break;  // pass q, already queued, runs empty
    if (q + 1 >= kMaxPasses) return drain(PDQ_ERR_HIP);
    visits += prev.elems[parity];
    if (prof && q < timed.size()) timed[q].bytes = prev.elems[parity] * bytes_per_key;
    // pass q + 1: at most two children per live segment of pass q, no more keys
    const uint64_t live_bound = 2ull * live < c.max_active ? 2ull * live : c.max_active;
    const uint32_t next_tile = tile_of[(q + 1) % 4];
    uint64_t tile_bound = prev.elems[parity] / next_tile + 1 + live_bound;
    if (tile_bound > c.max_tiles) tile_bound = c.max_tiles;
    // the tile pass q + 2 is filed with: its largest segment taken as a
    // quarter of pass q's largest
    tile_of[(q + 2) % 4] = o.tile ? o.tile : auto_tile(prev.elems[parity], (prev.maxlen[parity] + 3) / 4);
    rc = enqueue(q + 1, static_cast<uint32_t>(live_bound), static_cast<uint32_t>(tile_bound));
    if (rc != PDQ_OK) return drain(rc);
    // the counters after pass q
    const int slot = static_cast<int>(q % kPinSlots);
    if (hipEventSynchronize(pin->ev[slot]) != hipSuccess) return drain(PDQ_ERR_HIP);
    prev = pin->host[slot];
    rc = check_snapshot(c, prev);
    if (rc != PDQ_OK) return drain(rc);
    ++q;
  }
  // the last queued pass found its live list empty: not a pass
  if (prof && timed.size() > q) {
    for (size_t i = q; i < timed.size(); ++i) {
      (void)hipEventDestroy(timed[i].a);
      (void)hipEventDestroy(timed[i].b);
    }
    timed.resize(q);
  }
  *passes = q;
  *visits_out = visits;
  return drain(PDQ_OK);
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
  const bool learned = (o.flags & PDQ_LEARNED) && !offsets && n > kLearnSample;
  const bool batched = (o.flags & PDQ_BATCHED) && offsets;
  const bool dev_passes = device_passes(offsets, o);
  const Layout L = make_layout_opts(n, offsets ? nseg : 1, static_cast<uint32_t>(kt), vals != nullptr, learned,
                                    o.steps, o.grid, batched || dev_passes, false);
  if (!ws || ws_bytes < L.total) return PDQ_ERR_WORKSPACE;

  char* base = align_ptr(ws);
  Ctx c = make_ctx(keys, vals, n, offsets, nseg, kt, o, L, base);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batched) return run_batched(c, o, L, base, st, s);
  Tuned tc;
  if (dev_passes) {
    tc = tuned_config(c, o);
    c = batch_ctx(c, o, tc);
  }
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
  // pinned host memory for the call's reads (none in the call that allocates nothing)
  PinBlock* pin = t_noalloc ? nullptr : pin_acquire();
  const PinGuard pin_guard{pin};
  bool unordered = false;  // both a descending and an ascending pair seen
  if (!offsets && uses_runs(n, 1)) {
    RunPlan plan = {};
    rc = run_near_sorted(c, L, base, &plan, s, pin);
    unordered = plan.descents > 0 && plan.ascent != 0;
    if (rc != PDQ_OK) return rc;
    if (plan.state != kRunUnsorted) {
      if (st) {
        if (plan.state == kRunSorted) {
          st->sorted_segments = 1;
          st->sorted_elements = n;
        }
        st->near_sorted = plan.state;
        st->near_sorted_runs = plan.runs;
        st->near_sorted_outliers = plan.state == kRunOutliers ? plan.outliers : 0;
        HIP_TRY(hipStreamSynchronize(s));
      }
      return PDQ_OK;
    }
  }
  // the tile of the first pass, from the average size of its segments
  // (the learned bins hold at most 2n/256 keys each, or the fit is judged
  // failed; input segments are taken as equal until the first pass has run)
  if (!o.tile && !dev_passes) c.tile = auto_tile(n, learned ? n / 128 : n / (offsets ? nseg : 1));
  LearnedResult lres;
  uint32_t src = 0;
  if (learned) {
    c.single = 0;  // the first partition pass sees the bins, not the whole range
    rc = run_learned(c, o, L, base, prof, lres, s, unordered, pin);
    if (rc != PDQ_OK) return rc;
    if (lres.state == 1) src = 1;
    else if (!o.tile && !dev_passes) c.tile = auto_tile(n, n);  // judged and fell back: one segment [0, n)
  }
  if (src == 0) HIP_TRY(launch_init(c, s));
  if (dev_passes) {
    // the largest live segment: the fullest range bin, or the whole input
    const uint64_t maxseg = lres.state == 1 ? lres.max_range : n;
    const uint32_t passes = o.batch_passes ? o.batch_passes - 1 : batch_passes(maxseg, c.base_max);
    rc = enqueue_batch_rest(c, L, base, passes, kShapes[tc.shape].tail, s, nullptr, src, prof ? &timed : nullptr);
    if (rc == PDQ_OK && st) rc = device_pass_stats(c, L, base, kb, vals != nullptr, lres, prof, timed, st, s);
    cleanup();
    return rc;
  }
  rc = read_counters(c, &snap, s);
  if (rc != PDQ_OK) return rc;
  if ((o.flags & PDQ_VALIDATE) && snap.bad_offsets) return PDQ_ERR_INVALID;
  // base cases and heapsorts of the input segments themselves
  rc = finish_items(c, snap, s);
  if (rc != PDQ_OK) return rc;

  const uint64_t bytes_per_key = 2ull * kb + (vals ? 8ull : 0ull);
  uint32_t pass = 0;
  uint64_t visits = 0;
  if (pin) {
    rc = run_passes_pipelined(c, o, L, base, snap, src, prof, bytes_per_key, timed, &pass, &visits, pin, s);
  } else {
    rc = run_passes_sync(c, o, snap, src, prof, bytes_per_key, timed, &pass, &visits, s);
  }
  if (rc != PDQ_OK) {
    cleanup();
    return rc;
  }

  if (st) {
    int r3 = read_counters(c, &snap, s);
    if (r3 != PDQ_OK) {
      cleanup();
      return r3;
    }
    fill_pass_stats(st, snap);
    st->passes = pass;
    st->element_visits = visits;
    fill_learned_stats(st, lres);
    if (prof) {
      uint64_t bytes = 0;
      for (const Timed& t : timed) bytes += t.bytes;
      fill_profile_stats(st, timed, bytes);
    }
  }
  cleanup();
  return PDQ_OK;
}

// Runs a sort with statistics gathered in a current-layout struct and copied
// out up to the caller's struct_size (older, smaller layouts stay valid).
// Workspace of 64-bit payloads (PDQ_VALS64), after the call's layout: the
// 32-bit index payload the sort moves, and a copy of the payloads.
size_t vals64_bytes(size_t n) { return align_up(n * 4) + align_up(n * 8); }

// The layout a call uses (the same decisions as run_sort).
Layout call_layout(size_t n, const uint64_t* offsets, size_t nseg, int kt, bool vals, const Opts& o) {
  const bool learned = (o.flags & PDQ_LEARNED) && !offsets && n > kLearnSample;
  const bool batched = ((o.flags & PDQ_BATCHED) && offsets) || device_passes(offsets, o);
  return make_layout_opts(n, offsets ? nseg : 1, static_cast<uint32_t>(kt), vals, learned, o.steps, o.grid, batched,
                          false);
}

int sort_stats(void* keys, uint32_t* vals, size_t n, const uint64_t* offsets, size_t nseg, int kt, int order,
               void* ws, size_t ws_bytes, void* stream, const pdq_options* opt, pdq_stats* st) {
  if (!st) return run_sort(keys, vals, n, offsets, nseg, kt, order, ws, ws_bytes, stream, opt, nullptr);
  pdq_stats local;
  memset(&local, 0, sizeof(local));
  const uint32_t user_size = st->struct_size;
  const size_t copy = user_size == 0 || user_size > sizeof(pdq_stats) ? sizeof(pdq_stats) : user_size;
  const int rc = run_sort(keys, vals, n, offsets, nseg, kt, order, ws, ws_bytes, stream, opt, &local);
  local.struct_size = user_size;
  memcpy(st, &local, copy);
  return rc;
}

// Runs a sort with statistics gathered in a current-layout struct and copied
// out up to the caller's struct_size (older, smaller layouts stay valid).
// With PDQ_VALS64 the 64-bit payloads travel as 32-bit indices: the sort
// moves an index array in the workspace, and one gather places the payloads
// at the end (traffic: 12 bytes per key once, instead of 8 more bytes per
// key in every partition pass).
int sort_entry(void* keys, uint32_t* vals, size_t n, const uint64_t* offsets, size_t nseg, int kt, int order,
               void* ws, size_t ws_bytes, void* stream, const pdq_options* opt, pdq_stats* st) {
  Opts o;
  const int orc = read_opts(opt, &o);
  if (orc != PDQ_OK || !vals || !(o.flags & PDQ_VALS64) || n <= 1 || !valid_key_type(kt))
    return sort_stats(keys, vals, n, offsets, nseg, kt, order, ws, ws_bytes, stream, opt, st);
  g_last_hip = 0;
  if (reinterpret_cast<uintptr_t>(vals) % 8) return PDQ_ERR_INVALID;
  if (n >= (1ull << 32)) return PDQ_ERR_UNSUPPORTED;
  const Layout L = call_layout(n, offsets, nseg, kt, true, o);
  if (!ws || ws_bytes < L.total + vals64_bytes(n)) return PDQ_ERR_WORKSPACE;
  char* extra = align_ptr(ws) + (L.total - kAlign);
  uint32_t* idx = reinterpret_cast<uint32_t*>(extra);
  uint64_t* vcopy = reinterpret_cast<uint64_t*>(extra + align_up(n * 4));
  uint64_t* v64 = reinterpret_cast<uint64_t*>(vals);
  const hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_vals64_prepare(v64, n, idx, vcopy, s));
  const int rc = sort_stats(keys, idx, n, offsets, nseg, kt, order, ws, ws_bytes, stream, opt, st);
  if (rc != PDQ_OK) return rc;
  HIP_TRY(launch_vals64_gather(v64, n, idx, vcopy, s));
  if (st) HIP_TRY(hipStreamSynchronize(s));
  return PDQ_OK;
}

// ---- scratch of pdq_sort_noalloc ---------------------------------------------

constexpr size_t kNoAllocBytes = PDQ_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

}  // namespace

// The workspace of pdq_sort_noalloc: one copy of this array on every GPU the
// library runs on. Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol); it uses the device address
// that noalloc_scratch looks up once per device.
static __device__ __align__(256) unsigned char scratch[PDQ_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current and kept for later calls.
int noalloc_scratch(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return PDQ_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return PDQ_ERR_HIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PDQ_OK;
}

}  // namespace

extern "C" {

size_t pdq_workspace_bytes(size_t n, size_t nseg, pdq_key_type key_type, int has_vals, const pdq_options* opt) {
  if (!valid_key_type(key_type)) return 0;
  Opts o;
  if (read_opts(opt, &o) != PDQ_OK) return 0;
  if (nseg == 0) nseg = 1;
  const bool learned = (o.flags & PDQ_LEARNED) && nseg == 1 && n > kLearnSample;
  // one segment: enough for pdq_sort's device-counted passes as well
  const bool batched = (o.flags & (PDQ_BATCHED | PDQ_AUTOTUNE)) != 0 ||
                       (nseg == 1 && !(o.flags & PDQ_HOST_LOOP) && !t_noalloc);
  const size_t total = make_layout_opts(n, nseg, static_cast<uint32_t>(key_type), has_vals != 0, learned, o.steps,
                                        o.grid, batched, (o.flags & PDQ_AUTOTUNE) != 0)
                           .total;
  return total + (has_vals && (o.flags & PDQ_VALS64) ? vals64_bytes(n) : 0);
}

int pdq_sort(void* d_keys, size_t n, pdq_key_type key_type, pdq_order order, void* d_ws, size_t ws_bytes,
             void* stream, const pdq_options* opt, pdq_stats* stats) {
  return sort_entry(d_keys, nullptr, n, nullptr, 1, key_type, order, d_ws, ws_bytes, stream, opt, stats);
}

int pdq_sort_pairs(void* d_keys, uint32_t* d_vals, size_t n, pdq_key_type key_type, pdq_order order, void* d_ws,
                   size_t ws_bytes, void* stream, const pdq_options* opt, pdq_stats* stats) {
  if (n > 1 && !d_vals) return PDQ_ERR_INVALID;
  return sort_entry(d_keys, d_vals, n, nullptr, 1, key_type, order, d_ws, ws_bytes, stream, opt, stats);
}

int pdq_segmented_sort(void* d_keys, uint32_t* d_vals, size_t n, const uint64_t* d_offsets, size_t nseg,
                       pdq_key_type key_type, pdq_order order, void* d_ws, size_t ws_bytes, void* stream,
                       const pdq_options* opt, pdq_stats* stats) {
  if (!d_offsets && nseg > 0) return PDQ_ERR_INVALID;
  if (!d_offsets) return n == 0 ? PDQ_OK : PDQ_ERR_INVALID;
  return sort_entry(d_keys, d_vals, n, d_offsets, nseg, key_type, order, d_ws, ws_bytes, stream, opt, stats);
}

const char* pdq_status_string(int status) {
  switch (status) {
    case PDQ_OK: return "PDQ_OK: success";
    case PDQ_ERR_INVALID: return "PDQ_ERR_INVALID: invalid argument (null or misaligned pointer, bad offsets)";
    case PDQ_ERR_UNSUPPORTED: return "PDQ_ERR_UNSUPPORTED: unsupported key type, order, size or option";
    case PDQ_ERR_WORKSPACE: return "PDQ_ERR_WORKSPACE: workspace missing or smaller than pdq_workspace_bytes()";
    case PDQ_ERR_HIP: return "PDQ_ERR_HIP: a HIP launch or synchronisation failed";
    case PDQ_ERR_DEVICE:
      return "PDQ_ERR_DEVICE: a kernel found an internal inconsistency (or a bounded wait timed out) and skipped "
             "its writes; the output is not sorted";
    case PDQ_ERR_SCRATCH:
      return "PDQ_ERR_SCRATCH: pdq_sort_noalloc needs more scratch than PDQ_NOALLOC_SCRATCH_BYTES for this size";
    default: return "unknown pdq status";
  }
}

int pdq_last_hip_error(void) { return g_last_hip; }

int pdq_abi_version(void) { return PDQ_ABI_VERSION; }

int pdq_check(const void* d_ws, void* stream) {
  g_last_hip = 0;
  if (!d_ws) return PDQ_ERR_INVALID;
  // every layout starts with the counter block (make_layout)
  const Counters* ctr = reinterpret_cast<const Counters*>(align_ptr(const_cast<void*>(d_ws)));
  uint32_t words[2] = {0, 0};
  const hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(words, &ctr->bad_offsets, sizeof(words), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (words[0] || (words[1] & kErrCapacity)) return PDQ_ERR_INVALID;
  return words[1] ? PDQ_ERR_DEVICE : PDQ_OK;
}

int pdq_sort_noalloc(void* d_keys, uint32_t* d_vals, size_t n, pdq_key_type key_type, pdq_order order,
                     void* stream, const pdq_options* opt, pdq_stats* stats) {
  g_last_hip = 0;
  Opts o;
  const int rc = read_opts(opt, &o);
  if (rc != PDQ_OK) return rc;
  if (o.flags & (PDQ_PROFILE | PDQ_BATCHED | PDQ_AUTOTUNE)) return PDQ_ERR_UNSUPPORTED;
  if (!valid_key_type(key_type) || order != PDQ_ASCENDING || n >= (1ull << 32)) return PDQ_ERR_UNSUPPORTED;
  if (n > 1) {
    if (!d_keys) return PDQ_ERR_INVALID;
    // the size check comes before anything touches the GPU (the layout of
    // the host-driven pass loop, which this entry point runs)
    t_noalloc = true;
    const size_t need = pdq_workspace_bytes(n, 1, key_type, d_vals != nullptr, opt);
    t_noalloc = false;
    if (need == 0 || need > kNoAllocBytes) return PDQ_ERR_SCRATCH;
  }
  void* ws = nullptr;
  if (n > 1) {
    const int r2 = noalloc_scratch(&ws);
    if (r2 != PDQ_OK) return r2;
  }
  t_noalloc = true;
  const int r3 = sort_entry(d_keys, d_vals, n, nullptr, 1, key_type, order, ws, kNoAllocBytes, stream, opt, stats);
  t_noalloc = false;
  return r3;
}

// ---- captured batched sort --------------------------------------------------

struct pdq_plan {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t shape = 0;
  uint32_t passes = 0;
  double ms[kBatchShapes] = {};
  uint8_t var[kBaseClasses] = {};
  uint32_t threads[kBaseClasses] = {};
  double class_ms[kBaseClasses][kBaseVariants] = {};
};

int pdq_plan_create(pdq_plan** plan, void* d_keys, uint32_t* d_vals, size_t n, const uint64_t* d_offsets,
                    size_t nseg, pdq_key_type key_type, void* d_ws, size_t ws_bytes, void* stream,
                    const pdq_options* opt) {
  g_last_hip = 0;
  if (!plan) return PDQ_ERR_INVALID;
  *plan = nullptr;
  if (!valid_key_type(key_type)) return PDQ_ERR_UNSUPPORTED;
  Opts o;
  int rc = read_opts(opt, &o);
  if (rc != PDQ_OK) return rc;
  if (n == 0 || n >= (1ull << 32) || nseg == 0 || nseg >= (1ull << 32)) return PDQ_ERR_UNSUPPORTED;
  const uint32_t kb = key_bytes(static_cast<uint32_t>(key_type));
  const bool v64 = d_vals && (o.flags & PDQ_VALS64);
  // d_offsets NULL with nseg 1: one range [0, n)
  if (!d_keys || (!d_offsets && nseg != 1) || reinterpret_cast<uintptr_t>(d_keys) % kb ||
      reinterpret_cast<uintptr_t>(d_offsets) % 8 || (d_vals && reinterpret_cast<uintptr_t>(d_vals) % (v64 ? 8 : 4)))
    return PDQ_ERR_INVALID;
  const bool tune = (o.flags & PDQ_AUTOTUNE) != 0;
  const Layout L = make_layout_opts(n, nseg, static_cast<uint32_t>(key_type), d_vals != nullptr, false, o.steps,
                                    o.grid, true, tune);
  if (!d_ws || ws_bytes < L.total + (v64 ? vals64_bytes(n) : 0)) return PDQ_ERR_WORKSPACE;
  char* base = align_ptr(d_ws);
  // 64-bit payloads: the plan sorts 32-bit indices and gathers at the end
  uint64_t* const vals64 = v64 ? reinterpret_cast<uint64_t*>(d_vals) : nullptr;
  uint32_t* const idx = v64 ? reinterpret_cast<uint32_t*>(base + (L.total - kAlign)) : nullptr;
  uint64_t* const vcopy = v64 ? reinterpret_cast<uint64_t*>(base + (L.total - kAlign) + align_up(n * 4)) : nullptr;
  if (v64) d_vals = idx;
  const Ctx c = make_ctx(d_keys, d_vals, n, d_offsets, nseg, key_type, o, L, base);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (v64 && launch_vals64_prepare(vals64, n, idx, vcopy, s) != hipSuccess) return PDQ_ERR_HIP;
  pdq_plan* p = new pdq_plan();
  auto fail = [&](int code) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
    return code;
  };
  Tuned tc = tuned_config(c, o);
  // the first step (shape-independent) gives the number of passes to capture
  uint32_t passes = 0;
  {
    const Ctx c0 = batch_ctx(c, o, tc);
    rc = enqueue_batch_init(c0, s);
    if (rc == PDQ_OK) rc = batch_probe(c0, o, s, &passes);
    if (rc != PDQ_OK) return fail(rc);
  }
  const std::string key = o.tune_cache ? tune_key(c) : std::string();
  Tuned cached;
  const bool from_cache = tune && !o.batch_shape && cache_lookup(o.tune_cache, key, &cached);
  if (from_cache) {
    tc = cached;
  } else if (tune) {
    // On a copy of the caller's data: first the partition tile of the
    // passes (every tile shape with the default base-case shapes, the
    // whole sequence timed), then the base-case classes (every variant
    // for all classes at once with that tile, each class's launch timed
    // by its own events); the fastest of each is kept. The first run of
    // every configuration warms its kernels up and is not counted.
    void* bk = base + L.backup_keys;
    uint32_t* bv = d_vals ? reinterpret_cast<uint32_t*>(base + L.backup_vals) : nullptr;
    if (hipMemcpyAsync(bk, d_keys, n * kb, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(PDQ_ERR_HIP);
    if (bv && hipMemcpyAsync(bv, d_vals, n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(PDQ_ERR_HIP);
    auto timed_run = [&](const Tuned& t, EventPair* class_ev, double* total) -> int {
      const Ctx cs = batch_ctx(c, o, t);
      for (int rep = 0; rep < 2; ++rep) {
        if (hipMemcpyAsync(d_keys, bk, n * kb, hipMemcpyDeviceToDevice, s) != hipSuccess) return PDQ_ERR_HIP;
        if (bv && hipMemcpyAsync(d_vals, bv, n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return PDQ_ERR_HIP;
        EventPair ev;
        if (!ev.make() || hipEventRecord(ev.a, s) != hipSuccess) return PDQ_ERR_HIP;
        int r = enqueue_batch_init(cs, s);
        if (r == PDQ_OK)
          r = enqueue_batch_rest(cs, L, base, passes, kShapes[t.shape].tail, s, rep == 1 ? class_ev : nullptr);
        if (r != PDQ_OK) return r;
        if (hipEventRecord(ev.b, s) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess) return PDQ_ERR_HIP;
        if (rep == 1) *total = ev.ms();
      }
      return PDQ_OK;
    };
    Tuned best;
    double best_ms = 1e300;
    for (int sh = 0; sh < kTunedShapes; ++sh) {
      Tuned t;
      t.shape = sh;
      double total = 0;
      rc = timed_run(t, nullptr, &total);
      if (rc != PDQ_OK) return fail(rc);
      p->ms[sh] = total;
      if (total < best_ms) {
        best_ms = total;
        best.shape = sh;
      }
    }
    double class_best[kBaseClasses];
    for (int k = 0; k < kBaseClasses; ++k) class_best[k] = 1e300;
    const bool wide = kb == 8 && d_vals;
    for (int v = 0; v < kBaseVariants; ++v) {
      Tuned t = best;
      for (int k = 0; k < kBaseClasses; ++k) t.var[k] = kBaseThreads[wide ? 1 : 0][k][v] ? v : 0;
      EventPair class_ev[kBaseClasses];
      for (auto& e2 : class_ev)
        if (!e2.make()) return fail(PDQ_ERR_HIP);
      double total = 0;
      rc = timed_run(t, class_ev, &total);
      if (rc != PDQ_OK) return fail(rc);
      for (int k = 0; k < kBaseClasses; ++k) {
        if (!kBaseThreads[wide ? 1 : 0][k][v] || (k == 6 && batch_base_max(c.key_type, d_vals != nullptr) < kWideBaseMax))
          continue;
        const double ms = class_ev[k].ms();
        p->class_ms[k][v] = ms > 0 ? ms : 1e-6;  // nonzero marks a measured shape
        if (ms < class_best[k]) {
          class_best[k] = ms;
          best.var[k] = static_cast<uint8_t>(v);
        }
      }
    }
    if (hipMemcpyAsync(d_keys, bk, n * kb, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(PDQ_ERR_HIP);
    if (bv && hipMemcpyAsync(d_vals, bv, n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(PDQ_ERR_HIP);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(PDQ_ERR_HIP);
    tc = best;
    cache_store(o.tune_cache, key, tc);
  }
  if (tune || from_cache) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(c.key_type, c.has_vals, c.n, c.nseg)] = tc;
  }
  const bool wide = kb == 8 && d_vals;
  for (int k = 0; k < kBaseClasses; ++k) {
    p->var[k] = tc.var[k];
    p->threads[k] = static_cast<uint32_t>(base_threads(wide, k, tc.var[k]));
  }
  const int shape = tc.shape;
  p->shape = static_cast<uint32_t>(shape);
  p->passes = passes;
  // capture the launch sequence on a private stream
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(PDQ_ERR_HIP);
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const Ctx cc = batch_ctx(c, o, tc);
    rc = PDQ_OK;
    if (v64 && launch_vals64_prepare(vals64, n, idx, vcopy, cs) != hipSuccess) rc = PDQ_ERR_HIP;
    if (rc == PDQ_OK) rc = enqueue_batch_init(cc, cs);
    if (rc == PDQ_OK) rc = enqueue_batch_rest(cc, L, base, passes, kShapes[shape].tail, cs);
    if (rc == PDQ_OK && v64 && launch_vals64_gather(vals64, n, idx, vcopy, cs) != hipSuccess) rc = PDQ_ERR_HIP;
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    p->graph = g;
    if (rc == PDQ_OK && e2 != hipSuccess) {
      g_last_hip = static_cast<int>(e2);
      rc = PDQ_ERR_HIP;
    }
    if (rc == PDQ_OK && (e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0)) != hipSuccess) {
      g_last_hip = static_cast<int>(e);
      rc = PDQ_ERR_HIP;
    }
  } else {
    g_last_hip = static_cast<int>(e);
    rc = PDQ_ERR_HIP;
  }
  (void)hipStreamDestroy(cs);
  if (rc != PDQ_OK) return fail(rc);
  *plan = p;
  return PDQ_OK;
}

int pdq_plan_launch(pdq_plan* plan, void* stream) {
  g_last_hip = 0;
  if (!plan || !plan->exec) return PDQ_ERR_INVALID;
  HIP_TRY(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
  return PDQ_OK;
}

int pdq_plan_info(const pdq_plan* plan, uint32_t* shape, double* ms) {
  if (!plan) return PDQ_ERR_INVALID;
  if (shape) *shape = plan->shape;
  if (ms)
    for (int i = 0; i < kBatchShapes; ++i) ms[i] = plan->ms[i];
  return PDQ_OK;
}

int pdq_plan_classes(const pdq_plan* plan, uint32_t* threads, double* ms) {
  if (!plan) return PDQ_ERR_INVALID;
  for (int k = 0; k < kBaseClasses; ++k) {
    if (threads) threads[k] = plan->threads[k];
    if (ms)
      for (int v = 0; v < kBaseVariants; ++v) ms[k * kBaseVariants + v] = plan->class_ms[k][v];
  }
  return PDQ_OK;
}

void pdq_plan_destroy(pdq_plan* plan) {
  if (!plan) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
}

// ---- learned first pass, step by step (pdq_learned.h) ----------------------

int pdq_mlp_infer(const float* d_params, const float* d_x, size_t m, int residual, float* d_y, void* stream) {
  g_last_hip = 0;
  if (m == 0) return PDQ_OK;
  if (!d_params || !d_x || !d_y) return PDQ_ERR_INVALID;
  HIP_TRY(launch_infer(d_params, d_x, m, residual ? 1u : 0u, d_y, static_cast<hipStream_t>(stream)));
  return PDQ_OK;
}

int pdq_mlp_gradient(const float* d_params, const float* d_x, const float* d_t, uint32_t batch, int residual,
                     float* d_grad, float* d_loss, void* stream) {
  g_last_hip = 0;
  if (batch == 0 || batch > 65536) return PDQ_ERR_UNSUPPORTED;
  if (!d_params || !d_x || !d_t || !d_grad || !d_loss) return PDQ_ERR_INVALID;
  HIP_TRY(launch_gradient(d_params, d_x, d_t, batch, residual ? 1u : 0u, d_grad, d_loss,
                          static_cast<hipStream_t>(stream)));
  return PDQ_OK;
}

size_t pdq_mlp_train_workspace_bytes(uint32_t grid) {
  Bump b;
  b.take(2ull * grid * kParamStride * 4);
  b.take(4 * 4);
  return b.off + kAlign;
}

int pdq_mlp_train(const float* d_x, const float* d_t, size_t m, uint64_t seed, uint32_t steps, uint32_t batch,
                  uint32_t grid, int residual, const float* d_init, float* d_params, float* d_losses, void* d_ws,
                  size_t ws_bytes, void* stream) {
  g_last_hip = 0;
  if (grid == 0 || grid > kMaxTrainGrid || batch == 0 || batch > 65536 || batch % grid || steps == 0 ||
      steps > kMaxLearnSteps || m == 0 || m >= (1ull << 32))
    return PDQ_ERR_UNSUPPORTED;
  if (!d_x || !d_t || !d_params || !d_losses) return PDQ_ERR_INVALID;
  if (!d_ws || ws_bytes < pdq_mlp_train_workspace_bytes(grid)) return PDQ_ERR_WORKSPACE;
  char* base = align_ptr(d_ws);
  Bump b;
  const size_t partials = b.take(2ull * grid * kParamStride * 4);
  const size_t sync = b.take(4 * 4);
  TrainArgs a;
  a.x = d_x;
  a.t = d_t;
  a.m = m;
  a.seed = seed;
  a.steps = steps;
  a.batch = batch;
  a.grid = grid;
  a.residual = residual ? 1u : 0u;
  a.init = d_init;
  a.params = d_params;
  a.losses = d_losses;
  a.partials = reinterpret_cast<float*>(base + partials);
  a.sync = reinterpret_cast<uint32_t*>(base + sync);
  HIP_TRY(launch_train(a, static_cast<hipStream_t>(stream)));
  return PDQ_OK;
}

int pdq_learned_features(const uint64_t* d_sorted, size_t m, float* d_x, float* d_t, uint64_t* d_info,
                         void* stream) {
  g_last_hip = 0;
  if (m == 0) return PDQ_OK;
  if (!d_sorted || !d_x || !d_t || !d_info) return PDQ_ERR_INVALID;
  HIP_TRY(launch_features(d_sorted, m, d_x, d_t, d_info, static_cast<hipStream_t>(stream)));
  return PDQ_OK;
}

int pdq_learned_extract(const uint64_t* d_sorted, const float* d_pred, size_t m, float* d_runmax,
                        uint64_t* d_splitters, uint32_t* d_count, void* stream) {
  g_last_hip = 0;
  if (m == 0 || m >= (1ull << 32)) return PDQ_ERR_UNSUPPORTED;
  if (!d_sorted || !d_pred || !d_runmax || !d_splitters || !d_count) return PDQ_ERR_INVALID;
  HIP_TRY(launch_extract(d_sorted, d_pred, m, d_runmax, d_splitters, d_count, static_cast<hipStream_t>(stream)));
  return PDQ_OK;
}

int pdq_learned_leaves(const float* d_x, const float* d_t, const float* d_pred, size_t m, float* d_runmax,
                       double* d_leaf, float* d_pred_x, float* d_pred_y, void* stream) {
  g_last_hip = 0;
  if (m == 0) return PDQ_OK;
  if (m >= (1ull << 32)) return PDQ_ERR_UNSUPPORTED;
  if (!d_x || !d_t || !d_pred || !d_runmax || !d_leaf || !d_pred_x || !d_pred_y) return PDQ_ERR_INVALID;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_running_max(d_pred, m, d_runmax, s));
  HIP_TRY(launch_leaves(d_x, d_t, d_pred, d_runmax, m, d_leaf, d_pred_x, d_pred_y, s));
  return PDQ_OK;
}

int pdq_sample_judge(const uint64_t* d_sorted, size_t m, const uint64_t* d_splitters, const uint32_t* d_count,
                     uint64_t* d_max_range, void* stream) {
  g_last_hip = 0;
  if (m == 0 || m >= (1ull << 32)) return PDQ_ERR_UNSUPPORTED;
  if (!d_sorted || !d_splitters || !d_count || !d_max_range) return PDQ_ERR_INVALID;
  HIP_TRY(launch_sample_judge(d_sorted, m, d_splitters, 0, d_count, 1, d_max_range,
                              static_cast<hipStream_t>(stream)));
  return PDQ_OK;
}

size_t pdq_bucket_workspace_bytes(size_t n) { return bucket_layout(n).total + kAlign; }

int pdq_bucket_histogram(const void* d_keys, size_t n, pdq_key_type key_type, const uint64_t* d_splitters,
                         const uint32_t* d_count, uint64_t* d_hist, void* d_ws, size_t ws_bytes, void* stream) {
  g_last_hip = 0;
  if (!valid_key_type(key_type)) return PDQ_ERR_UNSUPPORTED;
  if (n == 0 || n >= (1ull << 32)) return PDQ_ERR_UNSUPPORTED;
  if (!d_keys || !d_splitters || !d_count || !d_hist) return PDQ_ERR_INVALID;
  if (!d_ws || ws_bytes < pdq_bucket_workspace_bytes(n)) return PDQ_ERR_WORKSPACE;
  BucketBufs b = bucket_bufs(align_ptr(d_ws), n, d_splitters, d_count);
  b.totals = d_hist;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_bucket_hist(static_cast<uint32_t>(key_type), d_keys, n, b, s));
  HIP_TRY(launch_bucket_scan(b, s));
  return PDQ_OK;
}

size_t pdq_learned_fit_workspace_bytes(const pdq_options* opt) {
  Opts o;
  if (read_opts(opt, &o) != PDQ_OK) return 0;
  return fit_scratch_layout(o.grid).total + kAlign;
}

int pdq_learned_fit(const void* d_keys, size_t n, pdq_key_type key_type, void* d_ws, size_t ws_bytes,
                    void* stream, const pdq_options* opt, const pdq_fit_buffers* out) {
  g_last_hip = 0;
  if (!valid_key_type(key_type)) return PDQ_ERR_UNSUPPORTED;
  Opts o;
  const int rc = read_opts(opt, &o);
  if (rc != PDQ_OK) return rc;
  if (n == 0 || n >= (1ull << 32)) return PDQ_ERR_UNSUPPORTED;
  if (!d_keys || !out || !out->d_sample || !out->d_x || !out->d_t || !out->d_pred || !out->d_params ||
      !out->d_losses || !out->d_splitters || !out->d_count || !out->d_info)
    return PDQ_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(d_keys) % key_bytes(static_cast<uint32_t>(key_type))) return PDQ_ERR_INVALID;
  if (!d_ws || ws_bytes < pdq_learned_fit_workspace_bytes(opt)) return PDQ_ERR_WORKSPACE;
  char* scratch = align_ptr(d_ws);
  const FitScratchLayout fs = fit_scratch_layout(o.grid);
  FitBufs f;
  f.sample = out->d_sample;
  f.x = out->d_x;
  f.t = out->d_t;
  f.y = out->d_pred;
  f.params = out->d_params;
  f.losses = out->d_losses;
  f.splitters = out->d_splitters;
  f.count = out->d_count;
  f.info = out->d_info;
  f.runmax = reinterpret_cast<float*>(scratch + fs.runmax);
  f.partials = reinterpret_cast<float*>(scratch + fs.partials);
  f.sync = reinterpret_cast<uint32_t*>(scratch + fs.sync);
  f.raw = reinterpret_cast<uint64_t*>(scratch + fs.raw);
  f.runmax2 = reinterpret_cast<float*>(scratch + fs.runmax2);
  f.yx = reinterpret_cast<float*>(scratch + fs.yx);
  f.yy = reinterpret_cast<float*>(scratch + fs.yy);
  f.leaf = reinterpret_cast<double*>(scratch + fs.leaf);
  f.cand = reinterpret_cast<uint64_t*>(scratch + fs.cand);
  f.cand_count = reinterpret_cast<uint32_t*>(scratch + fs.cand_count);
  f.est = reinterpret_cast<uint64_t*>(scratch + fs.est);
  return run_fit(d_keys, n, static_cast<uint32_t>(key_type), o, f, static_cast<hipStream_t>(stream));
}

}  // extern "C"
