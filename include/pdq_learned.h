/*
 * pdq_learned.h -- building blocks of the learned multiway first pass of the
 * MI355X (gfx950) partition sort, exposed one by one so that each step can
 * be called and checked on its own. pdq_sort with PDQ_LEARNED (pdq.h) runs
 * them in this order:
 *
 *   1. sample m = PDQ_LEARN_SAMPLE keys at positions SplitMix64(seed ^ j)
 *      mod n, as order-preserving key images, and sort them;
 *   2. pdq_learned_features: feature x and mid-rank CDF target t of every
 *      sorted sample key;
 *   3. pdq_mlp_train: Adam on the 1 -> 32 -> 32 -> 1 ReLU MLP
 *      y = x + W3 . relu(W2 relu(W1 x + b1) + b2) + b3 (by default 32
 *      steps, and 128 when steps 4-5 judge the 32-step fit too uneven);
 *   4. pdq_mlp_infer, then pdq_learned_leaves: a second stage of 64 linear
 *      leaves (a two-level learned CDF model, as in learned index
 *      structures) refines the network's prediction two ways;
 *   5. pdq_learned_extract on each of the three predictions, and
 *      pdq_sample_judge: the splitter set whose fullest range bin holds the
 *      fewest sample keys is kept; if even that one is over the imbalance
 *      limit (with a 15 % margin), the call goes back to the plain path
 *      without a histogram;
 *   6. pdq_bucket_histogram: keys per bin; a range bin above the imbalance
 *      limit sends the call back to the plain path;
 *   7. scatter into the bins, then partition passes inside the range bins.
 *
 * The paper ("Pattern-defeating Quicksort", Peters, arXiv 2106.05123) has
 * no learned component; its Section 2 names multiway partitioning as the
 * alternative pdqsort did not take. This pass is that alternative, with
 * splitters from a fitted CDF instead of from a sorted sample's quantiles.
 *
 * Definitions shared by every entry point:
 *   key image   the unsigned integer with the canonical key order (pdq.h):
 *               uint32 / uint64 as is, int32 with the sign bit flipped,
 *               float32 with all bits flipped when negative, else the sign
 *               bit set; widened to uint64.
 *   parameters  1153 floats: W1[32] b1[32] W2[32][32] (row v, column u)
 *               b2[32] W3[32] b3.
 *   float32 inference  every dot product is a chain of fused multiply-adds
 *               in increasing index order, started from the bias; ReLU keeps
 *               values > 0; the residual x is added last; the result is
 *               clamped to [0, 1].
 *   bins        for u sorted, distinct splitters s[0..u): a key with image v
 *               and b = #{i : s[i] <= v} falls into equality bin 2b - 1 when
 *               b > 0 and v == s[b - 1], else into range bin 2b; there are
 *               2u + 1 bins, and bins are ordered like the keys they hold.
 *
 * All d_* pointers are device pointers owned by the caller; nothing is
 * allocated or kept. Calls are asynchronous on `stream` (a hipStream_t,
 * NULL = default stream) unless stated. Status codes are those of pdq.h.
 */
#ifndef PDQ_LEARNED_H
#define PDQ_LEARNED_H

#include "pdq.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PDQ_MLP_PARAMS 1153
#define PDQ_MAX_SPLITTERS 255
#define PDQ_MAX_BINS 511
#define PDQ_LEARN_SAMPLE 65536

/* Float32 inference (definition above) of d_x[0..m) into d_y[0..m).
 * residual: 1 adds x to the network output, 0 does not. */
int pdq_mlp_infer(const float* d_params, const float* d_x, size_t m, int residual, float* d_y, void* stream);

/* Gradient of L = (1/batch) sum_i (y_i - t_i)^2 over d_x[0..batch),
 * d_t[0..batch) at d_params (unclamped y), in float32, into
 * d_grad[PDQ_MLP_PARAMS]; d_loss[0] = L. One workgroup; the arithmetic of
 * one training step. batch 1 ... 65536. */
int pdq_mlp_gradient(const float* d_params, const float* d_x, const float* d_t, uint32_t batch, int residual,
                     float* d_grad, float* d_loss, void* stream);

/* Workspace of pdq_mlp_train for `grid` cooperating workgroups. */
size_t pdq_mlp_train_workspace_bytes(uint32_t grid);

/* Adam (beta1 0.9, beta2 0.999, eps 1e-8; learning rate cosine from 1e-2 at
 * step 1 to 1e-4 at step `steps`) on the mean squared error of minibatches
 * of `batch` samples drawn with replacement at positions
 * SplitMix64(seed ^ (0xBA7C0000 + step * batch + i)) mod m, step = 1 ...
 * steps. Initial parameters: d_init when non-NULL, else the seeded
 * initialisation (each first-layer knot -b1/W1 at a sample quantile of the
 * sorted features d_x). Writes the parameters after the last step to
 * d_params[PDQ_MLP_PARAMS] and the minibatch losses to d_losses[steps].
 * One cooperative launch of `grid` workgroups (1 ... 64); batch must be a
 * multiple of grid. Deterministic: the gradient partials of the workgroups
 * are summed in a fixed order. Returns PDQ_ERR_HIP if the grid cannot be
 * co-resident. */
int pdq_mlp_train(const float* d_x, const float* d_t, size_t m, uint64_t seed, uint32_t steps, uint32_t batch,
                  uint32_t grid, int residual, const float* d_init, float* d_params, float* d_losses, void* d_ws,
                  size_t ws_bytes, void* stream);

/* Features and targets of a sorted sample of key images d_sorted[0..m):
 * L(v) = e + (4 f - f^2) / 3 with f = (v - 2^e) / 2^e, e = floor(log2 v)
 * and L(0) = -1 (a pseudo-log2 within 0.0098 of log2 whose slope is
 * continuous across powers of two; operations in the order f * f,
 * 4 f - f * f, / 3, + e);
 * xl = (L(v) - L(lo)) / (L(hi) - L(lo)), xn = (v - lo) / (hi - lo) with lo
 * and hi the first and last sample key, all in double with correctly
 * rounded operations; the scaling with the smaller max_j |x_j - (j+1/2)/m|
 * is used (the log one on ties; x = 0.5 when lo == hi) and rounded once to
 * float. t_j = (first + last + 1) / (2m) over the run of keys equal to the
 * j-th. d_info[4] receives the two deviations' bit patterns and the choice
 * (1 = log). */
int pdq_learned_features(const uint64_t* d_sorted, size_t m, float* d_x, float* d_t, uint64_t* d_info,
                         void* stream);

/* Splitters from clamped predictions d_pred[0..m) of the sorted sample
 * d_sorted: r = running maximum of d_pred (written to d_runmax[0..m)); for
 * k = 1 ... 255 the candidate is the sample key at index floor(k m / 256)
 * when that key fills at least m / 256 sample slots (a heavy key: a smooth
 * model cannot isolate it, and it gets an equality bin), else the sample key
 * at the first j with r_j >= k / 256, if any. Writes the u <= 255 sorted,
 * distinct candidates to d_splitters and u to d_count[0]. */
int pdq_learned_extract(const uint64_t* d_sorted, const float* d_pred, size_t m, float* d_runmax,
                        uint64_t* d_splitters, uint32_t* d_count, void* stream);

/* Second stage of the splitter model, over the sorted sample's features
 * d_x, targets d_t and clamped float32 predictions d_pred (all [m]). The
 * running maximum r of d_pred (written to d_runmax[m]) assigns sample j to
 * leaf min(63, floor(64 r_j)); each leaf fits t = a + b u by least squares,
 * u = x for the x-leaves and u = the prediction for the y-leaves, with the
 * sums k, sum u, sum t, sum u^2, sum u t taken in index order in double,
 * b = (k sum u t - sum u sum t) / (k sum u^2 - (sum u)^2) and
 * a = (sum t - b sum u) / k (b = 0, a = mean t when the leaf has fewer than
 * two samples or no spread). d_leaf[2][64][2] receives (a, b) of every
 * leaf (x-leaves first); d_pred_x[j] and d_pred_y[j] the float32 of
 * a + b u_j of sample j's leaf. */
int pdq_learned_leaves(const float* d_x, const float* d_t, const float* d_pred, size_t m, float* d_runmax,
                       double* d_leaf, float* d_pred_x, float* d_pred_y, void* stream);

/* The largest number of keys of the sorted sample d_sorted[0..m) that fall
 * into one range bin of the d_count[0] sorted, distinct splitters
 * d_splitters, written to d_max_range[0]. */
int pdq_sample_judge(const uint64_t* d_sorted, size_t m, const uint64_t* d_splitters, const uint32_t* d_count,
                     uint64_t* d_max_range, void* stream);

/* Workspace of pdq_bucket_histogram for n keys. */
size_t pdq_bucket_workspace_bytes(size_t n);

/* Keys of d_keys[0..n) per bin (definition above) for the d_count[0] <=
 * 255 sorted, distinct splitter images d_splitters (images of this key
 * type, so below 2^32 for 32-bit keys): d_hist[0 .. 2u] get the counts,
 * d_hist[2u+1 .. 512) zero. */
int pdq_bucket_histogram(const void* d_keys, size_t n, pdq_key_type key_type, const uint64_t* d_splitters,
                         const uint32_t* d_count, uint64_t* d_hist, void* d_ws, size_t ws_bytes, void* stream);

/* Outputs of pdq_learned_fit; every pointer is required. */
typedef struct pdq_fit_buffers {
  uint64_t* d_sample;    /* [PDQ_LEARN_SAMPLE] sorted sample key images */
  float* d_x;            /* [PDQ_LEARN_SAMPLE] features */
  float* d_t;            /* [PDQ_LEARN_SAMPLE] targets */
  float* d_pred;         /* [PDQ_LEARN_SAMPLE] float32 predictions after training */
  float* d_params;       /* [PDQ_MLP_PARAMS] trained parameters */
  float* d_losses;       /* [learn_steps, or 128 with the staged budget] minibatch losses of the
                            kept fit */
  uint64_t* d_splitters; /* [PDQ_MAX_SPLITTERS] the chosen splitters */
  uint32_t* d_count;     /* [1] number of splitters */
  uint64_t* d_info;      /* [8]: [0..2] as in pdq_learned_features; [3] the chosen candidate (0 the
                            network, 1 its x-leaves, 2 its y-leaves); [4..6] the sample judge of each
                            candidate; [7] 1 when the histogram would run (always here) */
} pdq_fit_buffers;

/* Workspace of pdq_learned_fit with these options (learn_* fields). */
size_t pdq_learned_fit_workspace_bytes(const pdq_options* opt);

/* Steps 1-5 on d_keys[0..n) (n >= 1) with opt's seed and learn_* fields:
 * the whole fit that PDQ_LEARNED runs before its histogram, queued on
 * `stream` without a synchronisation when learn_steps is set; with
 * learn_steps 0 it runs the staged budget (pdq.h), which synchronises
 * `stream` once to judge the 32-step fit. d_losses needs 128 entries then. */
int pdq_learned_fit(const void* d_keys, size_t n, pdq_key_type key_type, void* d_ws, size_t ws_bytes,
                    void* stream, const pdq_options* opt, const pdq_fit_buffers* out);

#ifdef __cplusplus
}
#endif

#endif /* PDQ_LEARNED_H */
