"""Oracle of the learned first pass: a 1 -> 32 -> 32 -> 1 ReLU MLP fitted to
the CDF of a key sample with Adam, and the splitters and bins it induces.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

The paper has no learned component. Its Section 2 names multiway
partitioning as the route pdqsort did not take; this is the project's
multiway first pass in that spirit: one histogram pass and one scatter into
up to 511 bins replace the top eight levels of binary partitioning. Every
definition is written out plainly in numpy (float64 unless a function says
float32), so that it can be read against this summary:

  sample     position j = SplitMix64(seed ^ j) mod n, j < m, with replacement;
             keys are taken as their order-preserving unsigned images
  feature    of a sorted sample image v: a smooth pseudo-log2
             L(v) = e + (4 f - f^2) / 3 with f = (v - 2^e) / 2^e in [0, 1) and
             e = floor(log2 v) for v >= 1, L(0) = -1 (within 0.0098 of log2,
             increasing, and with a continuous slope across every power of
             two), scaled by the sample's min and max onto [0, 1]; or a
             linear scaling (v - lo) / (hi - lo). The scaling whose sample is
             closer to uniform (smaller max |x_j - (j + 1/2) / m|) is used.
             Computed in float64 with correctly rounded operations only, then
             rounded once to float32.
  target     mid-rank CDF of each sample key, (first + last + 1) / (2 m) over
             its run of equal keys
  model      y = x + W3 . relu(W2 relu(W1 x + b1) + b2) + b3   (residual form)
             1153 parameters: W1[32] b1[32] W2[32][32] (row v, column u) b2[32]
             W3[32] b3
  init       from SplitMix64(seed ^ (0x5EED0000 + i)) with a_i uniform in
             [-1, 1): |W1| in [1, 4] with a random sign, each first-layer knot
             -b1/W1 at a sample quantile of x, W2 ~ a * sqrt(6/32),
             W3 ~ a * sqrt(6/32) / 8, b2 = 0.1, b3 = 0
  loss       mean over the minibatch of (y - t)^2
  optimiser  Adam (beta1 0.9, beta2 0.999, eps 1e-8), learning rate cosine
             from lr0 to lr1 over S steps, minibatch positions
             SplitMix64(seed ^ (0xBA7C0000 + step * B + i)) mod m
  splitters  for k = 1..255: the sample key at index k m / 256 if it fills at
             least m / 256 sample slots (a heavy key, which a smooth model
             cannot isolate; it gets an equality bin), else the first sample
             key whose running maximum of the clamped float32 prediction
             reaches k / 256; sorted, duplicates removed
  leaves     second stage of the model (a two-level learned CDF, as in
             learned index structures): the running maximum r of the clamped
             prediction puts sample j in leaf min(63, floor(64 r_j)); every
             leaf fits t = a + b u by least squares over its samples, with u
             the feature x (x-leaves) or the clamped prediction (y-leaves);
             sums run in index order in float64, a leaf of fewer than two
             samples (or no spread) predicts its mean target
  choice     the splitters of the prediction, of the x-leaves and of the
             y-leaves are each judged on the sample (largest count of sample
             keys in a range bin); the smallest wins, ties in that order
  bins       b = number of splitters <= key; equality bin 2b - 1 when
             key == s[b - 1], range bin 2b otherwise (2u + 1 bins)
  budget     staged: a fit of 32 steps first; it is kept when its chosen
             splitters put at most 1.3 m / 256 sample keys into one range bin
             (in integers: judge * 2560 <= 13 m), and also when they put more
             than 4 m / 256 there (judge * 64 > m: longer training does not
             rescue such a fit, and the judge will reject it); otherwise the
             fit is redone from the same initial parameters with 128 steps

Where a float32 result decides an integer (the splitters), the float32
inference is the C routine oracle_mlp_infer_f32 (pdq_oracle.cpp), which
evaluates every dot product as a chain of fused multiply-adds in index order.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

H = 32
NPARAM = H + H + H * H + H + H + 1  # 1153
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 32, 64, 64 + 1024, 64 + 1024 + 32, 64 + 1024 + 64
NSPLIT = 255
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8
LR0, LR1 = 1e-2, 1e-4
SALT_INIT = 0x5EED0000
SALT_BATCH = 0xBA7C0000

M64 = (1 << 64) - 1


# ----------------------------------------------------------------- random numbers

def splitmix64(x: int) -> int:
    """SplitMix64 output function applied to x (Steele, Lea, Flood 2014)."""
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix64_np(x) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = np.asarray(x).astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def sample_positions(seed: int, m: int, n: int) -> np.ndarray:
    j = np.arange(m, dtype=np.uint64)
    return (splitmix64_np(np.uint64(seed) ^ j) % np.uint64(n)).astype(np.int64)


def batch_positions(seed: int, step: int, batch: int, m: int) -> np.ndarray:
    j = np.uint64(step) * np.uint64(batch) + np.arange(batch, dtype=np.uint64)
    with np.errstate(over="ignore"):
        h = splitmix64_np(np.uint64(seed) ^ (np.uint64(SALT_BATCH) + j))
    return (h % np.uint64(m)).astype(np.int64)


# ----------------------------------------------------------------- key images

def key_images(keys: np.ndarray) -> np.ndarray:
    """Order-preserving unsigned image of each key, as uint64."""
    if keys.dtype == np.uint32 or keys.dtype == np.uint64:
        return keys.astype(np.uint64)
    if keys.dtype == np.int32:
        return (keys.view(np.uint32) ^ np.uint32(0x80000000)).astype(np.uint64)
    if keys.dtype == np.float32:
        b = keys.view(np.uint32)
        neg = (b >> np.uint32(31)) == 1
        return np.where(neg, ~b, b | np.uint32(0x80000000)).astype(np.uint64)
    raise TypeError(keys.dtype)


# ----------------------------------------------------------------- features and targets

def floor_log2_u64(v: np.ndarray) -> np.ndarray:
    """Exact floor(log2 v) for v >= 1 (bit length - 1), by counting shifts."""
    v = v.astype(np.uint64)
    e = np.zeros(v.shape, dtype=np.int64)
    for k in range(1, 64):
        e += (v >> np.uint64(k)) > 0
    return e


def pseudo_log2(v: np.ndarray) -> np.ndarray:
    """L(v) = e + (4 f - f^2) / 3 with f = (v - 2^e) / 2^e, L(0) = -1.
    On [0, 1) the polynomial p(f) = (4 f - f^2) / 3 has p(0) = 0, p(1) = 1 and
    p'(1) = p'(0) / 2, so L is increasing with a slope that is continuous
    across each power of two (a chord per octave, the first version, kinks
    there, which a small network follows badly). float64, correctly rounded
    operations in this order: f (exact scaling of the converted difference),
    f * f, 4 f - f * f, / 3, + e."""
    v = v.astype(np.uint64)
    out = np.full(v.shape, -1.0)
    nz = v > 0
    e = floor_log2_u64(v[nz])
    d = (v[nz] - (np.uint64(1) << e.astype(np.uint64))).astype(np.float64)
    f = np.ldexp(d, -e)
    out[nz] = (4.0 * f - f * f) / 3.0 + e.astype(np.float64)
    return out


def features(sorted_images: np.ndarray):
    """Feature of each sorted sample image; returns (x float32, use_log)."""
    v = sorted_images.astype(np.uint64)
    m = v.size
    lo, hi = v[0], v[-1]
    if hi == lo:
        return np.full(m, 0.5, dtype=np.float32), True
    L = pseudo_log2(v)
    xl = (L - L[0]) / (L[-1] - L[0])
    xn = (v - lo).astype(np.float64) / np.float64(hi - lo)
    ref = (np.arange(m, dtype=np.float64) + 0.5) / m
    use_log = bool(np.max(np.abs(xl - ref)) <= np.max(np.abs(xn - ref)))
    return (xl if use_log else xn).astype(np.float32), use_log


def midrank_targets(sorted_keys: np.ndarray) -> np.ndarray:
    """(first index + last index + 1) / (2 m) over each key's run of equals."""
    m = sorted_keys.size
    first = np.searchsorted(sorted_keys, sorted_keys, side="left")
    last = np.searchsorted(sorted_keys, sorted_keys, side="right") - 1
    return ((first + last + 1) / (2.0 * m)).astype(np.float32)


# ----------------------------------------------------------------- model

def unpack(p):
    return (p[OFF_W1:OFF_B1], p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(H, H), p[OFF_B2:OFF_W3],
            p[OFF_W3:OFF_B3], p[OFF_B3])


def init_params(seed: int, x_sorted: np.ndarray) -> np.ndarray:
    """Initial float32 parameters. Every value is computed exactly in float64
    and rounded once to float32."""
    idx = np.arange(NPARAM, dtype=np.uint64)
    h = splitmix64_np(np.uint64(seed) ^ (np.uint64(SALT_INIT) + idx))
    a = (h >> np.uint64(40)).astype(np.float64) * 2.0 ** -23 - 1.0   # in [-1, 1), 24 bits
    lim = np.float64(np.float32(math.sqrt(6.0 / H)))
    p = np.zeros(NPARAM, dtype=np.float32)
    w1 = np.where(a[OFF_W1:OFF_B1] >= 0, 1.0, -1.0) * (1.0 + 3.0 * np.abs(a[OFF_W1:OFF_B1]))
    p[OFF_W1:OFF_B1] = w1.astype(np.float32)
    m = x_sorted.size
    q = x_sorted[((2 * np.arange(H) + 1) * m) // (2 * H)].astype(np.float64)
    p[OFF_B1:OFF_W2] = (-(p[OFF_W1:OFF_B1].astype(np.float64) * q)).astype(np.float32)
    p[OFF_W2:OFF_B2] = (a[OFF_W2:OFF_B2] * lim).astype(np.float32)
    p[OFF_B2:OFF_W3] = np.float32(0.1)
    p[OFF_W3:OFF_B3] = (a[OFF_W3:OFF_B3] * lim / 8.0).astype(np.float32)
    p[OFF_B3] = 0.0
    return p


def forward(p: np.ndarray, x: np.ndarray, residual: bool = True):
    """float64 forward pass; returns y and (z1, h1, z2, h2)."""
    W1, b1, W2, b2, W3, b3 = unpack(p.astype(np.float64))
    x = np.asarray(x, dtype=np.float64)
    z1 = np.outer(x, W1) + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    if residual:
        y = y + x
    return y, (z1, h1, z2, h2)


def loss(p, x, t, residual: bool = True) -> float:
    y, _ = forward(p, x, residual)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(p, x, t, residual: bool = True):
    """Analytic gradient of the minibatch mean squared error (float64), by the
    chain rule; the ReLU derivative is taken as 1 where its input is > 0."""
    W1, b1, W2, b2, W3, b3 = unpack(p.astype(np.float64))
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    y, (z1, h1, z2, h2) = forward(p, x, residual)
    B = x.size
    dy = 2.0 * (y - t) / B
    g = np.zeros(NPARAM, dtype=np.float64)
    g[OFF_W3:OFF_B3] = h2.T @ dy
    g[OFF_B3] = dy.sum()
    dz2 = np.outer(dy, W3) * (z2 > 0)
    g[OFF_W2:OFF_B2] = (dz2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    g[OFF_W1:OFF_B1] = dz1.T @ x
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    return g, float(np.mean((y - t) ** 2))


def numeric_grad(p, x, t, residual: bool = True, h: float = 1e-6) -> np.ndarray:
    """Central finite differences of `loss` in float64."""
    p64 = p.astype(np.float64)
    g = np.zeros(NPARAM)
    for i in range(NPARAM):
        a = p64.copy()
        b = p64.copy()
        a[i] += h
        b[i] -= h
        g[i] = (loss(a, x, t, residual) - loss(b, x, t, residual)) / (2 * h)
    return g


def lr_at(step: int, steps: int, lr0: float = LR0, lr1: float = LR1) -> float:
    """Cosine schedule: lr0 at step 1, lr1 at step `steps`."""
    if steps <= 1:
        return lr0
    return lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * (step - 1) / (steps - 1)))


def adam_train(p0: np.ndarray, x: np.ndarray, t: np.ndarray, seed: int, steps: int, batch: int,
               residual: bool = True):
    """Adam from p0 over `steps` minibatches; returns (float32 params, losses)."""
    p = p0.astype(np.float64)
    mom = np.zeros(NPARAM)
    vel = np.zeros(NPARAM)
    losses = []
    for s in range(1, steps + 1):
        pos = batch_positions(seed, s, batch, x.size)
        g, L = grad(p, x[pos], t[pos], residual)
        losses.append(L)
        mom = BETA1 * mom + (1 - BETA1) * g
        vel = BETA2 * vel + (1 - BETA2) * g * g
        mh = mom / (1 - BETA1 ** s)
        vh = vel / (1 - BETA2 ** s)
        p = p - lr_at(s, steps) * mh / (np.sqrt(vh) + EPS)
    return p.astype(np.float32), np.array(losses)


# ----------------------------------------------------------------- float32 inference (C)

def infer_f32(p: np.ndarray, x: np.ndarray, residual: bool = True) -> np.ndarray:
    """Clamped float32 prediction, fused multiply-adds in index order (C)."""
    import oracle

    lib = oracle.lib()
    p = np.ascontiguousarray(p, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty(x.size, dtype=np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.oracle_mlp_infer_f32(p.ctypes.data_as(fp), x.ctypes.data_as(fp), ctypes.c_size_t(x.size),
                             ctypes.c_int(1 if residual else 0), y.ctypes.data_as(fp))
    return y


# ----------------------------------------------------------------- splitters and bins

def splitters(sorted_images: np.ndarray, pred: np.ndarray, nsplit: int = NSPLIT) -> np.ndarray:
    """Candidate k (k = 1..nsplit): the sample key at index q = floor(k m /
    (nsplit + 1)) when that key fills at least m / (nsplit + 1) sample slots
    (a heavy key: it gets an equality bin), else the first sample key whose
    running maximum of the clamped float32 prediction reaches
    k / (nsplit + 1), if any. Splitters: the sorted distinct candidates."""
    m = sorted_images.size
    r = np.maximum.accumulate(np.clip(pred.astype(np.float32), np.float32(0), np.float32(1)))
    first = np.searchsorted(sorted_images, sorted_images, side="left")
    end = np.searchsorted(sorted_images, sorted_images, side="right")
    out = []
    for k in range(1, nsplit + 1):
        q = (k * m) // (nsplit + 1)
        if (end[q] - first[q]) * (nsplit + 1) >= m:
            out.append(sorted_images[q])
            continue
        thr = np.float32(k) / np.float32(nsplit + 1)
        j = int(np.searchsorted(r, thr, side="left"))
        if j < m:
            out.append(sorted_images[j])
    return np.unique(np.array(out, dtype=np.uint64))


LEAVES = 64


def leaf_predictions(x: np.ndarray, t: np.ndarray, pred: np.ndarray, leaves: int = LEAVES):
    """Second stage of the splitter model: returns the float32 predictions
    of the x-leaves and of the y-leaves (see the module summary)."""
    p32 = np.clip(np.asarray(pred, dtype=np.float32), np.float32(0), np.float32(1))
    r = np.maximum.accumulate(p32)
    leaf = np.minimum((r * np.float32(leaves)).astype(np.int64), leaves - 1)  # exact scaling, then floor
    t64 = np.asarray(t, dtype=np.float32).astype(np.float64)
    outs = []
    for u32 in (np.asarray(x, dtype=np.float32), p32):
        u = u32.astype(np.float64)
        out = np.zeros(u.size, dtype=np.float32)
        for j in range(leaves):
            idx = np.nonzero(leaf == j)[0]
            if idx.size == 0:
                continue
            uj, tj = u[idx], t64[idx]
            k = float(idx.size)
            # float32 * float32 is exact in float64, so only the additions round
            sx = np.add.accumulate(uj)[-1]
            st = np.add.accumulate(tj)[-1]
            sxx = np.add.accumulate(uj * uj)[-1]
            sxt = np.add.accumulate(uj * tj)[-1]
            den = k * sxx - sx * sx
            if idx.size < 2 or not den > 0.0:
                b = 0.0
                a = st / k
            else:
                b = (k * sxt - sx * st) / den
                a = (st - b * sx) / k
            out[idx] = (np.float64(a) + np.float64(b) * uj).astype(np.float32)
        outs.append(out)
    return outs[0], outs[1]


def sample_judge(sorted_images: np.ndarray, split: np.ndarray) -> int:
    """Largest number of sample keys in one range bin of these splitters."""
    return int(histogram(sorted_images, split)[0::2].max())


def choose_splitters(sorted_images: np.ndarray, x: np.ndarray, t: np.ndarray, pred: np.ndarray):
    """Splitters of the prediction, the x-leaves and the y-leaves; the one
    with the smallest sample judge wins (the first on ties). Returns
    (splitters, choice, estimates, leaf predictions)."""
    px, py = leaf_predictions(x, t, pred)
    cands = [splitters(sorted_images, c) for c in (pred, px, py)]
    est = [sample_judge(sorted_images, c) for c in cands]
    best = int(np.argmin(est))
    return cands[best], best, est, (px, py)


def bins_of(images: np.ndarray, split: np.ndarray) -> np.ndarray:
    """Bin of every key image: range bin 2b, equality bin 2b - 1."""
    images = images.astype(np.uint64)
    split = split.astype(np.uint64)
    b = np.searchsorted(split, images, side="right")
    eq = np.zeros(images.size, dtype=bool)
    nz = b > 0
    eq[nz] = images[nz] == split[b[nz] - 1]
    return np.where(eq, 2 * b - 1, 2 * b).astype(np.int64)


def histogram(images: np.ndarray, split: np.ndarray) -> np.ndarray:
    return np.bincount(bins_of(images, split), minlength=2 * split.size + 1).astype(np.uint64)


def judge(hist: np.ndarray, n: int, limit: float = 2.0) -> bool:
    """True when every range bin holds at most limit * n / 256 keys (equality
    bins are final and are not judged)."""
    return bool(np.all(hist[0::2].astype(np.float64) <= limit * n / 256.0))


# ----------------------------------------------------------------- whole fit

def fit(keys: np.ndarray, seed: int = 0, m: int = 1 << 16, steps: int = 128, batch: int = 1024,
        residual: bool = True):
    """Sample, sort, features, targets, Adam, float32 inference, leaves,
    the sample-judged choice of splitters. Returns a dict of every
    intermediate."""
    img = key_images(keys)
    pos = sample_positions(seed, m, img.size)
    samp = np.sort(img[pos])
    x, use_log = features(samp)
    t = midrank_targets(samp)
    p0 = init_params(seed, x)
    p, losses = adam_train(p0, x, t, seed, steps, batch, residual)
    y = infer_f32(p, x, residual)
    sp, choice, est, leaves = choose_splitters(samp, x, t, y)
    return dict(sample=samp, x=x, use_log=use_log, t=t, p0=p0, params=p, losses=losses, pred=y, splitters=sp,
                choice=choice, estimates=est, leaf_pred=leaves, root_splitters=splitters(samp, y))


STAGE1_STEPS = 32
STAGE2_STEPS = 128


def early_accept(judge: int, m: int) -> bool:
    """Whether a short fit is kept: its fullest range bin holds at most
    1.3 m / 256 sample keys."""
    return judge * 2560 <= 13 * m


def hopeless(judge: int, m: int) -> bool:
    """Whether a short fit is too uneven for longer training to rescue: its
    fullest range bin holds more than 4 m / 256 sample keys."""
    return judge * 64 > m


def fit_staged(keys: np.ndarray, seed: int = 0, m: int = 1 << 16, batch: int = 1024, residual: bool = True):
    """The default budget: a 32-step fit, kept if early_accept or hopeless
    holds for its chosen splitters, else a 128-step fit from the same initial
    parameters. Adds `stage` (1 or 2) to fit's dict."""
    f = fit(keys, seed, m, STAGE1_STEPS, batch, residual)
    judge = f["estimates"][f["choice"]]
    if early_accept(judge, m) or hopeless(judge, m):
        f["stage"] = 1
        return f
    f = fit(keys, seed, m, STAGE2_STEPS, batch, residual)
    f["stage"] = 2
    return f
