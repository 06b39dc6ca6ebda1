/*
 * pdq.h -- C ABI of the MI355X (gfx950) partition sort.
 *
 * The operation is the one of "Pattern-defeating Quicksort" (Peters,
 * arXiv 2106.05123): an unstable, in-place, ascending sort of a contiguous
 * range (Sections 1 and 3: a [begin, end) range, a comparison order, no
 * stability). Its data-parallel hot path -- the partition step -- runs as
 * out-of-place passes over all live segments at once:
 *   - pivot: Tukey's ninther, with fresh (hashed, seeded) candidates
 *     after a bad partition (Sections 2 and 4.2);
 *   - partition_right, or partition_left when the pivot equals the
 *     predecessor, so k distinct keys need O(k) passes (Section 3,
 *     Lemmas 1-4, Theorem 1);
 *   - branchless block classification (Section 5.3) as wave ballots and
 *     LDS prefix sums with a decoupled look-back scatter;
 *   - bad-partition budget with an O(n log n) fallback sort (Section 4.1;
 *     by default one workgroup merge-sorts the segment, lanes sharing every
 *     merge; PDQ_HEAPSORT selects the paper's in-place heapsort);
 *   - detection of already ordered segments (Section 5.2);
 *   - an LDS-resident base case for segments of at most 4096 keys, 16384
 *     with device-counted passes (Section 5.1's small-case sort: a sorting
 *     network below 1024 keys; from 2048 keys an LDS bucket sort when the
 *     keys spread evenly over their range, else an LDS merge sort).
 * With PDQ_LEARNED a multiway first pass runs before the partition passes
 * (the multiway partitioning Section 2 mentions as the road not taken): a
 * small MLP fitted to the CDF of a key sample proposes up to 255
 * splitters, one histogram pass judges the bins they induce, and one
 * scatter splits the input into up to 511 bins; a bin holding too many keys
 * sends the whole call back to the plain ninther path. The building blocks
 * of that pass have entry points of their own in pdq_learned.h.
 *
 * Key order ("canonical order"): uint32 / uint64 as unsigned integers,
 * int32 as two's complement, float32 by the total order on its bit
 * patterns: -inf < ... < -0.0 < +0.0 < ... < +inf. NaN inputs are outside
 * the contract (they are placed by bit pattern, nothing more is promised).
 * Sorted keys are unique bit for bit. Payloads (uint32, or uint64 with
 * PDQ_VALS64) travel with their keys; the sort is unstable, so the order of
 * payloads of equal keys is not specified (any permutation consistent with
 * the keys is valid).
 *
 * Memory and ownership: every pointer argument named d_* is a device
 * pointer owned by the caller. The library never allocates device memory:
 * all scratch lives in the caller's workspace d_ws (size from
 * pdq_workspace_bytes; 256-byte alignment recommended). d_ws must stay
 * allocated until the work queued on `stream` has finished. No pointer is
 * kept after a call returns. `stream` is a hipStream_t (NULL = the default
 * stream). pdq_sort and pdq_sort_pairs queue their partition passes with
 * device-side counts (see pdq_sort). The host-driven pass loop
 * (pdq_segmented_sort without PDQ_BATCHED, PDQ_HOST_LOOP) reads the number
 * of live segments after each pass: each pass ends with an asynchronous
 * copy of the pass counters into pinned host memory (a few small blocks the
 * library allocates on first use, one per concurrent call and device, kept
 * until the process ends), and the host waits for one pass's counters while
 * the next pass already runs. Calls return once their work is queued (it
 * may still run) unless `stats` is non-NULL or PDQ_VALIDATE is set, which
 * synchronise `stream` at the end; pdq_check reports device-side errors of
 * a call that returned early.
 *
 * Errors: every entry point returns PDQ_OK (0) or a negative status; no
 * exception crosses the ABI. n <= 1 is a no-op returning PDQ_OK.
 * Concurrent calls on different streams need different workspaces.
 */
#ifndef PDQ_H
#define PDQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDQ_ABI_VERSION 3

/* Largest segment that goes straight to the LDS base case. */
#define PDQ_BASE_CASE_MAX 4096

typedef enum pdq_key_type {
  PDQ_U32 = 1,
  PDQ_I32 = 2,
  PDQ_F32 = 3,
  PDQ_U64 = 4,
  PDQ_I64 = 5, /* signed 64-bit integers */
  PDQ_F64 = 6  /* IEEE doubles: -0.0 before +0.0, NaN outside the contract (as for PDQ_F32) */
} pdq_key_type;

/* The comparison order is supplied by the caller but fixed to ascending
 * canonical order; any other value returns PDQ_ERR_UNSUPPORTED. */
typedef enum pdq_order { PDQ_ASCENDING = 0 } pdq_order;

enum pdq_status {
  PDQ_OK = 0,
  PDQ_ERR_INVALID = -1,     /* null pointer with n > 0, misaligned pointer, bad offsets (validate mode) */
  PDQ_ERR_UNSUPPORTED = -2, /* key type, order, n >= 2^32, unknown flag */
  PDQ_ERR_WORKSPACE = -3,   /* d_ws NULL or ws_bytes below pdq_workspace_bytes() */
  PDQ_ERR_HIP = -4,         /* a HIP launch or synchronisation failed (see pdq_last_hip_error) */
  PDQ_ERR_SCRATCH = -5,     /* pdq_sort_noalloc: the call needs more scratch than
                               PDQ_NOALLOC_SCRATCH_BYTES */
  PDQ_ERR_DEVICE = -6       /* a kernel caught an internal inconsistency (a reservation or split
                               that does not fit its segment, a lost queue item) or a bounded wait
                               timed out, and skipped its writes: the output is not sorted.
                               Reported by the call itself when it synchronises (stats requested,
                               or a host-driven pass loop), else by pdq_check afterwards */
};

enum pdq_flags {
  PDQ_VALIDATE = 1u << 0, /* check offsets on the device before sorting (synchronises) */
  PDQ_PROFILE = 1u << 1,  /* time every partition launch with HIP events (needs stats) */
  PDQ_LEARNED = 1u << 2,  /* learned multiway first pass (pdq_sort / pdq_sort_pairs with
                             n > 65536; other calls ignore it); pass the same options to
                             pdq_workspace_bytes */
  PDQ_BATCHED = 1u << 3,  /* pdq_segmented_sort: device-counted partition passes and one
                             persistent launch over a device work queue; the host synchronises
                             once, after the first kernel, to size the passes (pdq_plan_launch
                             not at all), and once more at the end only when stats are
                             requested: without stats, device-side errors are reported by
                             pdq_check. Meant for many segments of up to ~2^20 keys each; pass
                             the same options to pdq_workspace_bytes */
  PDQ_AUTOTUNE = 1u << 4, /* pdq_plan_create: on the caller's data, time every partition tile of
                             the batched passes (8192, 16384, 32768 keys), then every workgroup
                             shape of each LDS base-case size class (1 to 16 waves), and keep the
                             fastest of each (needs the workspace pdq_workspace_bytes gives with
                             this flag); see tune_cache_path */
  PDQ_DETERMINISTIC = 1u << 5, /* partition tiles take their places in tile order by a decoupled
                             look-back instead of one atomic reservation each: every run then
                             arranges the keys (and the payloads of equal keys) identically.
                             Slower. The learned pass's scatter still orders keys inside a bin
                             by LDS atomics, so with PDQ_LEARNED it covers the passes only */
  PDQ_VALS64 = 1u << 7,   /* the payload pointer d_vals of pdq_sort_pairs, pdq_segmented_sort,
                             pdq_plan_create and pdq_sort_noalloc points to uint64_t payloads
                             (8-byte aligned) instead of uint32_t; pass the same options to
                             pdq_workspace_bytes (12 more bytes per key) */
  PDQ_HOST_LOOP = 1u << 8, /* pdq_sort / pdq_sort_pairs: the host-driven pass loop (the host reads
                             each pass's counters, one pass behind) instead of the default
                             device-counted passes; needs less workspace */
  PDQ_HEAPSORT = 1u << 9, /* the fallback of segments out of bad-partition budget (Section 4.1)
                             is the paper's heapsort, one lane per segment in the user buffer,
                             instead of the default workgroup merge sort (also O(n log n)) */
  PDQ_FRESH_FIXED = 1u << 6 /* after a bad partition take the fresh pivot candidates at the fixed
                             quarter offsets of Section 4.2's deterministic rule instead of the
                             default hashed positions (Section 4.2's randomised rule; the hash
                             is keyed by pdq_options.seed, so a caller facing adversarial
                             inputs should pass a secret seed) */
};

typedef struct pdq_options {
  uint32_t struct_size;  /* sizeof(pdq_options); 0 or a smaller value = older layout */
  uint32_t flags;        /* pdq_flags */
  int32_t force_budget;  /* < 0: floor(log2 size) per segment (Section 4.1); >= 0: that budget */
  uint32_t tile;         /* keys per partition tile: 0 = chosen per pass (8192 once no segment
                            holds more than a tenth of the pass's keys, else 16384 for segments
                            of 2^18 keys or more), else 1024 ... 65536, a power of two;
                            PDQ_BATCHED uses its shape's tile unless this is set */
  uint64_t seed;         /* seeds the hashed pivot candidates taken after a bad partition, and
                            the sample, initial weights and minibatches of PDQ_LEARNED */
  float learned_imbalance_limit; /* PDQ_LEARNED: fall back to the plain path when a range bin holds
                                    more than limit * n / 256 keys; 0 = 2.0; < 0 = always fall back */
  uint32_t learn_steps;  /* PDQ_LEARNED: Adam steps (at most 65536); 0 = the staged budget: a
                            32-step fit, kept when its chosen splitters put at most 1.3 m/256 of
                            the m sample keys into one range bin (or more than 4 m/256: too
                            uneven to rescue, and rejected), else a 128-step fit from the same
                            initial parameters (one synchronisation between the two) */
  uint32_t learn_batch;  /* PDQ_LEARNED: minibatch, 0 = 1024; a multiple of learn_grid, at most 65536 */
  uint32_t learn_grid;   /* PDQ_LEARNED: cooperating trainer workgroups, 0 = 16 (1 ... 64) */
  uint32_t batch_shape;  /* PDQ_BATCHED: 0 = the tuned (or default) shape; 1 ... 4 = shape
                            (partition tile, slots per lane of the two widest LDS classes):
                            (8192, 16), (16384, 16), (32768, 16), (8192, 32) */
  uint32_t batch_passes; /* device-counted passes (PDQ_BATCHED, and pdq_sort without
                            PDQ_HOST_LOOP): 0 = automatic (h + 3 + h/2, h the halvings that
                            bring the largest segment to the widest LDS class); k > 0 = k - 1
                            passes (at most 32); segments still live after them finish in the
                            persistent tail */
  uint32_t waves;        /* 0 = each LDS base-case size class takes its default (or tuned)
                            workgroup shape; 1, 2, 4, 8 or 16 = every class that has a shape of
                            that many waves per workgroup takes it (pdq_plan_classes lists the
                            shapes a plan uses) */
  uint32_t reserved_;    /* must be 0 */
  const char* tune_cache_path; /* NULL, or a text file that remembers autotuned configurations
                            across processes: pdq_plan_create with PDQ_AUTOTUNE reads a line
                            for this device kind and problem (key type, payload, n, segment
                            count) and skips the timing when it finds one, else tunes and
                            appends one; batched calls without PDQ_AUTOTUNE use a line if one is
                            there. File errors only skip the cache */
} pdq_options;

/* Filled on request (forces a synchronisation at the end of the call). */
typedef struct pdq_stats {
  uint32_t struct_size;           /* set by the caller: sizeof(pdq_stats) */
  uint32_t passes;                /* partition passes run */
  uint64_t element_visits;        /* sum over passes of keys partitioned */
  uint64_t partitions_right;
  uint64_t partitions_left;
  uint64_t bad_partitions;
  uint64_t heapsort_segments;     /* segments out of bad-partition budget, given to the fallback
                                     sort (Section 4.1's heapsort; a workgroup merge sort here) */
  uint64_t heapsort_elements;
  uint64_t base_segments;         /* segments sorted by the LDS base case */
  uint64_t base_elements;
  uint64_t sorted_segments;       /* segments found already ascending or descending */
  uint64_t sorted_elements;
  uint64_t equal_elements;        /* keys retired by partition_left (equal to their pivot) */
  uint64_t first_pivot_image;     /* first partition of a single-range sort: canonical pivot */
  int64_t first_left_size;        /*   ... its left-side size (pivot excluded) */
  int32_t first_mode;             /*   ... 0 partition_right, 1 partition_left, -1 none */
  uint32_t partition_launches;    /* PDQ_PROFILE: partition kernel launches timed */
  double partition_ms;            /* PDQ_PROFILE: summed duration of those launches */
  uint64_t partition_bytes;       /* PDQ_PROFILE: algorithmic bytes moved by them (read + write) */
  double first_pass_ms;           /* PDQ_PROFILE: duration of the first partition launch */
  uint64_t first_pass_bytes;      /* PDQ_PROFILE: its algorithmic bytes */
  uint32_t learned;               /* 0 not run, 1 learned first pass used, 2 judged and fell back */
  uint32_t learned_splitters;     /* splitters after duplicates were removed */
  uint64_t learned_max_range_bin; /* keys in the largest range bin */
  uint64_t learned_equal_elements;/* keys retired in equality bins */
  float learned_final_loss;       /* mean squared error of the last training step */
  uint32_t learned_use_log;       /* 1: piecewise-linear log2 feature, 0: linear feature */
  double learned_fit_ms;          /* PDQ_PROFILE: sample, sample sort, features, training, splitters */
  double learned_hist_ms;         /* PDQ_PROFILE: histogram and scans */
  double learned_scatter_ms;      /* PDQ_PROFILE: scatter into the bins */
  uint64_t learned_hist_bytes;    /* PDQ_PROFILE: algorithmic bytes of the histogram pass */
  uint64_t learned_scatter_bytes; /* PDQ_PROFILE: algorithmic bytes of the scatter */
  uint32_t batch_items;           /* PDQ_BATCHED: segments that went through the device queue */
  uint32_t batch_shape;           /* PDQ_BATCHED: persistent-kernel shape used (0 ... 3) */
  double batch_ms;                /* PDQ_BATCHED + PDQ_PROFILE: duration of the whole launch sequence */
  uint32_t near_sorted;           /* single-range sorts finished before any partition pass (Section
                                     5.2): 0 no, 1 one long run with at most 8192 keys in short runs
                                     (sorted, then merged into it), 2 two long runs merged, 3 already
                                     non-decreasing */
  uint32_t pad_;
  uint64_t near_sorted_runs;      /* maximal non-decreasing runs found (near_sorted != 0) */
  uint64_t near_sorted_outliers;  /* keys in short runs (near_sorted == 1) */
  uint32_t learned_choice;        /* PDQ_LEARNED: splitters taken from 0 the network, 1 its x-leaves,
                                     2 its y-leaves (pdq_learned.h) */
  uint32_t learned_steps;         /* PDQ_LEARNED: Adam steps of the kept fit (with learn_steps 0: 32
                                     when the short fit was kept, else 128) */
  uint64_t learned_sample_judge;  /* PDQ_LEARNED: sample keys in the fullest range bin of the chosen
                                     splitters (of PDQ_LEARN_SAMPLE) */
} pdq_stats;

/* Bytes of device workspace needed for a call with these sizes and options
 * (PDQ_LEARNED and its learn_* fields enlarge it). nseg is the number of
 * segments (1 for pdq_sort / pdq_sort_pairs). */
size_t pdq_workspace_bytes(size_t n, size_t nseg, pdq_key_type key_type, int has_vals,
                           const pdq_options* opt);

/* Sort d_keys[0..n) ascending in place (Sections 3-5; the paper's pdqsort on
 * one range). By default the partition passes take their counts on the
 * device: after the near-sorted check (a single synchronisation for n >=
 * 16384) and, with PDQ_LEARNED, the fit and the judge, the passes, the
 * persistent tail and the finishing kernels are queued without reading
 * anything back. PDQ_HOST_LOOP selects the host-driven pass loop. */
int pdq_sort(void* d_keys, size_t n, pdq_key_type key_type, pdq_order order, void* d_ws,
             size_t ws_bytes, void* stream, const pdq_options* opt, pdq_stats* stats);

/* Sort d_keys[0..n) ascending in place, moving d_vals[i] with d_keys[i]. */
int pdq_sort_pairs(void* d_keys, uint32_t* d_vals, size_t n, pdq_key_type key_type,
                   pdq_order order, void* d_ws, size_t ws_bytes, void* stream,
                   const pdq_options* opt, pdq_stats* stats);

/* Sort each segment [d_offsets[s], d_offsets[s+1]) independently, for
 * s < nseg. d_offsets is a device array of nseg+1 non-decreasing uint64
 * with d_offsets[0] = 0 and d_offsets[nseg] = n (checked only with
 * PDQ_VALIDATE). Empty segments are allowed. d_vals may be NULL. */
int pdq_segmented_sort(void* d_keys, uint32_t* d_vals, size_t n, const uint64_t* d_offsets,
                       size_t nseg, pdq_key_type key_type, pdq_order order, void* d_ws,
                       size_t ws_bytes, void* stream, const pdq_options* opt, pdq_stats* stats);

/* A captured batched segmented sort: the launch sequence of
 * pdq_segmented_sort with PDQ_BATCHED for these exact buffers, instantiated
 * once as a HIP graph and replayed by pdq_plan_launch; with d_offsets NULL
 * and nseg 1 the sort of the one range [0, n) (the device-counted passes of
 * pdq_sort without the near-sorted check). The plan owns host
 * memory and the graph only; the caller keeps d_keys, d_vals, d_offsets and
 * d_ws alive and unchanged in size while the plan exists, and may refill
 * them between launches. With PDQ_AUTOTUNE in opt->flags the persistent
 * kernel's shape is first chosen by timing every shape on the caller's data
 * (the keys and payloads are restored afterwards; synchronises `stream`);
 * the choice is remembered for later calls with the same key type, payload
 * flag, n and segment count. */
typedef struct pdq_plan pdq_plan;

int pdq_plan_create(pdq_plan** plan, void* d_keys, uint32_t* d_vals, size_t n, const uint64_t* d_offsets,
                    size_t nseg, pdq_key_type key_type, void* d_ws, size_t ws_bytes, void* stream,
                    const pdq_options* opt);

/* Replays the plan's graph on `stream`. */
int pdq_plan_launch(pdq_plan* plan, void* stream);

/* Shape index used (0 ... 3) and, after autotuning, the measured ms per
 * shape (ms[4]; 0 where not measured). Either pointer may be NULL. */
int pdq_plan_info(const pdq_plan* plan, uint32_t* shape, double* ms);

/* Workgroup shape of each of the seven LDS base-case size classes the plan
 * uses (threads[7]: lanes per workgroup; classes of at most 64, 256, 1024,
 * 2048, 4096, 8192 and 16384 keys) and, after autotuning, the measured ms of
 * each class under each of its three candidate shapes (ms[7 * 3], 0 where
 * not measured or the shape does not exist). Either pointer may be NULL. */
int pdq_plan_classes(const pdq_plan* plan, uint32_t* threads, double* ms);

void pdq_plan_destroy(pdq_plan* plan);

/* Bytes of the library's own device scratch array used by pdq_sort_noalloc
 * (one copy per GPU, held until the process ends). */
#define PDQ_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* pdq_sort / pdq_sort_pairs without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). The scratch that pdq_sort keeps in
 * d_ws (second key and payload buffer, segment lists, counters) lives instead
 * in a file-scope device array of PDQ_NOALLOC_SCRATCH_BYTES inside the
 * library; this call allocates nothing (no hipMalloc, no events, no library
 * allocation). d_vals may be NULL (keys only, as pdq_sort) or a uint32
 * (uint64 with PDQ_VALS64) payload moved with the keys (as pdq_sort_pairs).
 * A call whose
 * pdq_workspace_bytes(n, 1, key_type, d_vals != NULL, opt with PDQ_HOST_LOOP added) exceeds
 * PDQ_NOALLOC_SCRATCH_BYTES returns PDQ_ERR_SCRATCH before touching the GPU
 * (without PDQ_LEARNED: up to 15,637,440 uint32 keys, 8,072,320 uint32 keys
 * with payloads, 8,072,352 uint64 keys, 5,440,704 uint64 keys with
 * payloads). Unlike pdq_sort, it runs the host-driven pass loop with one host
 * synchronisation per partition pass (its smaller workspace fits more keys
 * into the array, and it allocates no pinned host memory). PDQ_PROFILE, PDQ_BATCHED and PDQ_AUTOTUNE return
 * PDQ_ERR_UNSUPPORTED. Every call on one GPU shares that GPU's array, which
 * keeps the previous call's contents (the call clears what must start at
 * zero): calls that overlap in time on one GPU -- on different streams, or
 * from different threads -- race and corrupt each other's results;
 * serialise them. The first call on each device looks up the array's
 * address on that device (the device must be current). Results, errors and
 * synchronisation are those of pdq_sort / pdq_sort_pairs. */
int pdq_sort_noalloc(void* d_keys, uint32_t* d_vals, size_t n, pdq_key_type key_type, pdq_order order,
                     void* stream, const pdq_options* opt, pdq_stats* stats);

/* Device-side error state of the last call (or plan launch) that used the
 * workspace d_ws: waits for `stream` and returns PDQ_OK, PDQ_ERR_INVALID
 * (the segment offsets were found inconsistent) or PDQ_ERR_DEVICE. Calls that
 * return before their work has finished (PDQ_BATCHED without stats,
 * pdq_plan_launch) cannot report these themselves. */
int pdq_check(const void* d_ws, void* stream);

/* Human-readable text of a status code (static storage). */
const char* pdq_status_string(int status);

/* The hipError_t value behind the last PDQ_ERR_HIP of this thread (0 if none). */
int pdq_last_hip_error(void);

/* PDQ_ABI_VERSION of the library. */
int pdq_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PDQ_H */
