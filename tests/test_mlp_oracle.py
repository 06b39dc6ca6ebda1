"""Pins of the learned-splitter oracle (oracle/mlp_oracle.py) against facts
that do not come from the oracle itself: published SplitMix64 outputs,
finite differences, hand-derived derivatives, Adam's closed-form first
step, exact values of the piecewise-linear log, brute-force ranks and bins,
and the closed-form splitters of a perfect CDF."""
import math

import numpy as np
import pytest

import gen.workloads as W
import oracle
from oracle import mlp_oracle as M


# ----------------------------------------------------------------- SplitMix64

def test_splitmix64_published_outputs():
    # the first outputs of SplitMix64 seeded with 0 (state advances by the
    # golden gamma before each output)
    g = 0x9E3779B97F4A7C15
    assert M.splitmix64(0) == 0xE220A8397B1DCDAF
    assert M.splitmix64(g) == 0x6E789E6AA1B965F4
    assert M.splitmix64((2 * g) & M.M64) == 0x06C45D188009454F
    xs = np.array([0, g, 12345, 2**63 + 7], dtype=np.uint64)
    assert [int(v) for v in M.splitmix64_np(xs)] == [M.splitmix64(int(x)) for x in xs]


def test_sample_and_batch_positions_in_range():
    pos = M.sample_positions(3, 1000, 777)
    assert pos.min() >= 0 and pos.max() < 777
    assert int(pos[5]) == M.splitmix64(3 ^ 5) % 777
    b = M.batch_positions(9, 4, 64, 1000)
    assert int(b[10]) == M.splitmix64(9 ^ (M.SALT_BATCH + 4 * 64 + 10)) % 1000


# ----------------------------------------------------------------- gradient

def _rand_params(seed, scale=0.7):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(M.NPARAM) * scale).astype(np.float32)


@pytest.mark.parametrize("residual", [True, False])
def test_gradient_matches_finite_differences(residual):
    rng = np.random.default_rng(1)
    p = _rand_params(2)
    x = rng.random(12)
    t = rng.random(12)
    g, _ = M.grad(p, x, t, residual)
    gn = M.numeric_grad(p, x, t, residual)
    # ReLU kinks are measure-zero for random inputs; central differences with
    # h = 1e-6 are good to ~1e-8 here
    assert np.max(np.abs(g - gn)) <= 1e-6 * max(1.0, np.max(np.abs(gn)))


def test_gradient_only_output_bias():
    # all weights zero: y = b3 + x, so only dL/db3 = 2 mean(b3 + x - t) is non-zero
    p = np.zeros(M.NPARAM, dtype=np.float32)
    p[M.OFF_B3] = 0.25
    x = np.array([0.1, 0.5, 0.9])
    t = np.array([0.2, 0.4, 0.3])
    g, L = M.grad(p, x, t)
    assert g[M.OFF_B3] == pytest.approx(2 * np.mean(0.25 + x - t), abs=1e-15)
    assert np.count_nonzero(np.delete(g, M.OFF_B3)) == 0
    assert L == pytest.approx(np.mean((0.25 + x - t) ** 2), abs=1e-15)


def test_gradient_single_path_by_hand():
    # one live path x -> h1[3] -> h2[5] -> y, every other weight zero:
    # y = e * (c * (a x + b) + d) + b3 + x ; L = (y - t)^2 for one sample
    a, b, c, d, e, b3 = 1.5, 0.25, -0.75, 2.0, 0.5, 0.125
    p = np.zeros(M.NPARAM, dtype=np.float32)
    p[M.OFF_W1 + 3], p[M.OFF_B1 + 3] = a, b
    p[M.OFF_W2 + 5 * 32 + 3], p[M.OFF_B2 + 5] = c, d
    p[M.OFF_W3 + 5], p[M.OFF_B3] = e, b3
    x, t = 0.5, 0.3
    z1 = a * x + b
    z2 = c * z1 + d
    y = e * z2 + b3 + x
    r = 2 * (y - t)
    g, _ = M.grad(p, np.array([x]), np.array([t]))
    assert g[M.OFF_B3] == pytest.approx(r)
    assert g[M.OFF_W3 + 5] == pytest.approx(r * z2)
    assert g[M.OFF_B2 + 5] == pytest.approx(r * e)
    assert g[M.OFF_W2 + 5 * 32 + 3] == pytest.approx(r * e * z1)
    assert g[M.OFF_B1 + 3] == pytest.approx(r * e * c)
    assert g[M.OFF_W1 + 3] == pytest.approx(r * e * c * x)
    # a dead first-layer unit (z1 <= 0) passes no gradient
    p[M.OFF_B1 + 3] = -10.0
    g2, _ = M.grad(p, np.array([x]), np.array([t]))
    assert g2[M.OFF_W1 + 3] == 0 and g2[M.OFF_B1 + 3] == 0 and g2[M.OFF_W2 + 5 * 32 + 3] == 0


# ----------------------------------------------------------------- Adam

def test_adam_first_step_closed_form():
    # after one step Adam's bias-corrected moments are g and g^2, so the
    # update is -lr0 * g / (|g| + eps)
    rng = np.random.default_rng(4)
    x = np.sort(rng.random(4096)).astype(np.float32)
    t = ((np.arange(4096) + 0.5) / 4096).astype(np.float32)
    p0 = M.init_params(7, x)
    p1, losses = M.adam_train(p0, x, t, seed=7, steps=1, batch=256)
    pos = M.batch_positions(7, 1, 256, x.size)
    g, L = M.grad(p0, x[pos], t[pos])
    want = p0.astype(np.float64) - M.LR0 * g / (np.abs(g) + M.EPS)
    assert np.allclose(p1, want.astype(np.float32), rtol=0, atol=1e-7)
    assert losses[0] == pytest.approx(L)


def test_learning_rate_schedule_endpoints():
    assert M.lr_at(1, 257) == pytest.approx(M.LR0)
    assert M.lr_at(257, 257) == pytest.approx(M.LR1)
    assert M.lr_at(129, 257) == pytest.approx((M.LR0 + M.LR1) / 2)


def test_training_reduces_loss_and_beats_untrained_splitters():
    keys = W.uniform_u32(1 << 20, seed=0)
    f = M.fit(keys, steps=256, batch=1024)
    assert f["losses"][-1] < f["losses"][0] / 100
    img = M.key_images(keys)
    h = M.histogram(img, f["splitters"])
    y0 = M.infer_f32(f["p0"], f["x"])
    h0 = M.histogram(img, M.splitters(f["sample"], y0))
    assert M.judge(h, keys.size)
    assert h[0::2].max() < h0[0::2].max()


# ----------------------------------------------------------------- features and targets

def test_pseudo_log2_exact_values():
    # p(f) = (4 f - f^2) / 3 at f = 0, 1/4, 1/2, 3/4: 0, 5/16, 7/12, 13/16
    e = np.arange(64, dtype=np.uint64)
    pw = np.uint64(1) << e
    assert np.array_equal(M.pseudo_log2(pw), np.arange(64, dtype=np.float64))
    three_halves = (np.uint64(3) << (e[1:] - np.uint64(1)))
    assert np.array_equal(M.pseudo_log2(three_halves), np.arange(1, 64) + 7.0 / 12.0)
    five_quarters = (np.uint64(5) << (e[2:] - np.uint64(2)))
    assert np.array_equal(M.pseudo_log2(five_quarters), np.arange(2, 64) + 5.0 / 16.0)
    seven_quarters = (np.uint64(7) << (e[2:] - np.uint64(2)))
    assert np.array_equal(M.pseudo_log2(seven_quarters), np.arange(2, 64) + 13.0 / 16.0)
    assert M.pseudo_log2(np.array([0], dtype=np.uint64))[0] == -1.0
    assert np.array_equal(M.floor_log2_u64(np.array([1, 2, 3, 2**63, 2**64 - 1], dtype=np.uint64)),
                          [0, 1, 1, 63, 63])


def test_pseudo_log2_monotone_and_close_to_log2():
    v = np.sort(W.uniform_u64(100000, seed=3) >> np.uint64(np.random.default_rng(0).integers(0, 63)))
    L = M.pseudo_log2(v)
    assert np.all(np.diff(L) >= 0)
    nz = v > 0
    # log2(1 + f) - (4 f - f^2) / 3 on [0, 1) lies in [-0.005342, 0.009709]
    d = np.log2(v[nz].astype(np.float64)) - L[nz]
    assert d.max() <= 0.00971 and d.min() >= -0.00535


def test_pseudo_log2_slope_continuous_across_powers_of_two():
    """The chord-per-octave form doubled its slope at every power of two;
    this one keeps it: finite-difference slopes just below and just above
    2^e agree, and equal (2/3) / 2^(e-1) (p'(1) / 2^(e-1) = p'(0) / 2^e)."""
    for e in (20, 33, 47):
        v = np.uint64(1) << np.uint64(e)
        h = np.uint64(1) << np.uint64(e - 12)
        L = M.pseudo_log2(np.array([v - h, v, v + h], dtype=np.uint64))
        left = (L[1] - L[0]) / float(h)
        right = (L[2] - L[1]) / float(h)
        want = (2.0 / 3.0) / 2.0 ** (e - 1)
        assert abs(left / want - 1) < 2e-3 and abs(right / want - 1) < 2e-3


def test_features_choose_scaling():
    m = 4096
    lin = np.arange(m, dtype=np.uint64) * np.uint64(1000) + np.uint64(5)
    x, use_log = M.features(lin)
    assert not use_log
    assert np.array_equal(x, (np.arange(m) / (m - 1)).astype(np.float32))
    geo = np.unique((2.0 ** (np.arange(m) * 60.0 / m)).astype(np.uint64))
    xg, use_log_g = M.features(geo)
    assert use_log_g and xg[0] == 0 and xg[-1] == 1 and np.all(np.diff(xg) >= 0)
    xe, _ = M.features(np.full(10, 7, dtype=np.uint64))
    assert np.all(xe == 0.5)


def test_midrank_targets_brute_force():
    rng = np.random.default_rng(5)
    s = np.sort(rng.integers(0, 20, 300)).astype(np.uint64)
    t = M.midrank_targets(s)
    for j in range(s.size):
        eq = np.nonzero(s == s[j])[0]
        assert t[j] == np.float32((eq[0] + eq[-1] + 1) / (2 * s.size))


def test_key_images_match_c_oracle():
    for kt in ("u32", "i32", "f32", "u64"):
        a = W.random_keys(kt, 200, seed=2)
        img = M.key_images(a)
        assert [int(v) for v in img] == [oracle.key_image(kt, v) for v in a]


# ----------------------------------------------------------------- init

def test_init_knots_at_sample_quantiles():
    x = np.sort(np.random.default_rng(2).random(1 << 12)).astype(np.float32)
    p = M.init_params(11, x)
    W1, b1, W2, b2, W3, b3 = M.unpack(p)
    assert np.all((np.abs(W1) >= 1) & (np.abs(W1) <= 4))
    q = x[((2 * np.arange(32) + 1) * x.size) // 64]
    assert np.allclose(-b1 / W1, q, rtol=1e-6, atol=1e-7)
    lim = math.sqrt(6 / 32)
    assert np.all(np.abs(W2) <= lim * (1 + 1e-6)) and np.all(np.abs(W3) <= lim / 8 * (1 + 1e-6))
    assert np.all(b2 == np.float32(0.1)) and b3 == 0
    assert np.array_equal(M.init_params(11, x), p)
    assert not np.array_equal(M.init_params(12, x), p)


# ----------------------------------------------------------------- float32 inference (C)

def test_infer_f32_close_to_float64_forward():
    rng = np.random.default_rng(6)
    for residual in (True, False):
        p = (_rand_params(8, 0.3)).astype(np.float32)
        x = rng.random(5000).astype(np.float32)
        y32 = M.infer_f32(p, x, residual)
        y64, _ = M.forward(p, x, residual)
        assert np.max(np.abs(y32 - np.clip(y64, 0, 1))) < 2e-5


def test_infer_f32_exact_dyadic_case():
    # dyadic weights keep every intermediate exact in float32
    p = np.zeros(M.NPARAM, dtype=np.float32)
    p[M.OFF_W1:M.OFF_B1] = 1.0
    p[M.OFF_B1:M.OFF_W2] = -np.arange(32) / 32.0
    p[M.OFF_W2 + np.arange(32) * 33] = 1.0          # W2 = identity
    p[M.OFF_W3:M.OFF_B3] = 1.0 / 64
    x = np.array([0.0, 0.25, 0.5, 1.0], dtype=np.float32)
    y = M.infer_f32(p, x, residual=False)
    want = [sum(max(v - u / 32.0, 0.0) for u in range(32)) / 64 for v in x]
    assert np.array_equal(y, np.array(want, dtype=np.float32))
    assert np.all(M.infer_f32(p, np.array([1e6], dtype=np.float32)) == 1.0)


# ----------------------------------------------------------------- splitters and bins

def test_splitters_of_perfect_cdf_are_sample_quantiles():
    m = 1 << 16
    samp = np.sort(W.uniform_u64(m, seed=4))
    assert np.unique(samp).size == m
    pred = M.midrank_targets(samp)
    sp = M.splitters(samp, pred)
    assert np.array_equal(sp, samp[np.arange(1, 256) * (m // 256)])


def test_splitters_constant_and_duplicates():
    # distinct keys, constant prediction 0.5: thresholds <= 1/2 all map to the
    # first key, higher ones are never reached
    samp = np.sort(W.uniform_u64(4096, seed=2))
    sp = M.splitters(samp, np.full(4096, 0.5, dtype=np.float32))
    assert np.array_equal(sp, samp[:1])
    # five values, each far above m/256 copies: every one is a splitter, whatever the prediction
    dup = np.sort(np.random.default_rng(1).integers(0, 5, 1000)).astype(np.uint64)
    assert np.array_equal(M.splitters(dup, np.full(1000, 0.5, dtype=np.float32)), np.arange(5, dtype=np.uint64))
    assert np.array_equal(M.splitters(dup, M.midrank_targets(dup)), np.arange(5, dtype=np.uint64))


def test_heavy_key_becomes_splitter():
    # one key with exactly m/256 + 1 copies in the middle of distinct keys is a
    # splitter even when the prediction is useless (constant 0)
    m = 1 << 16
    samp = np.sort(np.concatenate([W.uniform_u64(m - 257, seed=3) | np.uint64(1), np.full(257, 2**62, np.uint64)]))
    sp = M.splitters(samp, np.zeros(m, dtype=np.float32))
    assert np.array_equal(sp, np.array([2**62], dtype=np.uint64))
    # with m/256 - 1 copies it is not heavy
    samp2 = np.sort(np.concatenate([W.uniform_u64(m - 255, seed=3) | np.uint64(1), np.full(255, 2**62, np.uint64)]))
    assert M.splitters(samp2, np.zeros(m, dtype=np.float32)).size == 0


def test_bins_brute_force_and_histogram():
    rng = np.random.default_rng(9)
    split = np.array([3, 7, 8, 20], dtype=np.uint64)
    keys = rng.integers(0, 25, 2000).astype(np.uint64)
    bins = M.bins_of(keys, split)
    for k, b in zip(keys, bins):
        below = sum(1 for s in split if s <= k)
        want = 2 * below - 1 if below and split[below - 1] == k else 2 * below
        assert b == want
    h = M.histogram(keys, split)
    assert h.size == 9 and int(h.sum()) == keys.size
    assert int(h[1]) == int(np.count_nonzero(keys == 3))
    assert M.judge(np.array([10, 500, 10], dtype=np.uint64), 256 * 5, limit=2.0)
    assert not M.judge(np.array([11, 0, 10], dtype=np.uint64), 256 * 5, limit=2.0)


# ----------------------------------------------------------------- leaves, sample judge, choice

def test_leaves_reproduce_a_linear_cdf_exactly():
    """t = x on dyadic x: every leaf (on x or on the prediction t) fits
    slope 1 and intercept 0 with exact sums, so both leaf predictions are
    x itself."""
    m = 1 << 14
    x = (np.arange(m, dtype=np.float64) / m).astype(np.float32)
    px, py = M.leaf_predictions(x, x, x)
    assert np.array_equal(px, x) and np.array_equal(py, x)


def test_leaves_match_least_squares_per_leaf():
    """Against numpy's polyfit on each leaf's samples (leaves from the
    running maximum of the clamped prediction)."""
    rng = np.random.default_rng(12)
    m = 1 << 13
    x = np.sort(rng.random(m)).astype(np.float32)
    t = np.sort(rng.random(m)).astype(np.float32)
    pred = (t + rng.normal(0, 0.01, m)).astype(np.float32)
    px, py = M.leaf_predictions(x, t, pred, leaves=16)
    r = np.maximum.accumulate(np.clip(pred, 0, 1))
    leaf = np.minimum(np.floor(r.astype(np.float64) * 16).astype(np.int64), 15)
    for u, got in ((x, px), (np.clip(pred, 0, 1), py)):
        for j in range(16):
            sel = leaf == j
            if sel.sum() < 2:
                continue
            b, a = np.polyfit(u[sel].astype(np.float64), t[sel].astype(np.float64), 1)
            assert np.allclose(got[sel], a + b * u[sel], rtol=0, atol=2e-6)


def test_leaf_of_one_sample_predicts_its_target():
    x = np.array([0.1, 0.2, 0.3, 0.9], dtype=np.float32)
    t = np.array([0.125, 0.375, 0.625, 0.875], dtype=np.float32)
    pred = np.array([0.05, 0.06, 0.07, 0.95], dtype=np.float32)  # leaves {0,1,2} and {3} for 2 leaves
    px, py = M.leaf_predictions(x, t, pred, leaves=2)
    assert px[3] == t[3] and py[3] == t[3]


def test_sample_judge_brute_force():
    rng = np.random.default_rng(13)
    s = np.sort(rng.integers(0, 500, 4000)).astype(np.uint64)
    sp = np.unique(rng.choice(s, 40))
    counts = {}
    for k in s:
        below = int(np.sum(sp <= k))
        if below and sp[below - 1] == k:
            continue  # equality bin
        counts[below] = counts.get(below, 0) + 1
    assert M.sample_judge(s, sp) == max(counts.values())


def test_choice_takes_the_smallest_sample_judge_first_on_ties():
    m = 1 << 12
    s = np.arange(m, dtype=np.uint64) * np.uint64(3)
    x = (np.arange(m) / m).astype(np.float32)
    t = ((np.arange(m) + 0.5) / m).astype(np.float32)
    # a root prediction that is far off (a square): the leaves repair it
    pred = (x.astype(np.float64) ** 2).astype(np.float32)
    sp, choice, est, _ = M.choose_splitters(s, x, t, pred)
    assert est[choice] == min(est) and choice != 0 and est[0] > est[choice]
    assert M.sample_judge(s, sp) == est[choice]
    # a perfect root: all three candidates tie and the root wins
    sp2, choice2, est2, _ = M.choose_splitters(s, x, t, t)
    assert choice2 == 0 and est2[0] == min(est2)


def test_early_accept_threshold():
    """The short fit is kept while its fullest range bin holds at most
    1.3 m / 256 sample keys: 332.8 for m = 65536, so 332 passes and 333 does
    not; m = 2560 gives exactly 13."""
    assert M.early_accept(332, 1 << 16) and not M.early_accept(333, 1 << 16)
    assert M.early_accept(13, 2560) and not M.early_accept(14, 2560)
    assert M.early_accept(0, 1)
    # retraining is skipped above 4 m / 256: 1024 for m = 65536
    assert not M.hopeless(1024, 1 << 16) and M.hopeless(1025, 1 << 16)


def test_staged_budget_keeps_the_short_fit_or_redoes_the_long_one():
    """Uniform keys are split well after 32 steps, so the staged fit is the
    32-step fit; lognormal keys are not, so it is the 128-step fit from the
    same initial parameters (same splitters, same losses)."""
    n = 1 << 20
    keys = W.uniform_u32(n, seed=0)
    f = M.fit_staged(keys, seed=0)
    short = M.fit(keys, seed=0, steps=M.STAGE1_STEPS)
    assert f["stage"] == 1
    assert np.array_equal(f["splitters"], short["splitters"])
    assert M.early_accept(short["estimates"][short["choice"]], 1 << 16)
    keys = W.lognormal_u64(n, seed=0)
    f = M.fit_staged(keys, seed=0)
    short = M.fit(keys, seed=0, steps=M.STAGE1_STEPS)
    long = M.fit(keys, seed=0, steps=M.STAGE2_STEPS)
    assert f["stage"] == 2
    assert not M.early_accept(short["estimates"][short["choice"]], 1 << 16)
    assert np.array_equal(f["splitters"], long["splitters"])
    assert np.array_equal(f["losses"], long["losses"])
    # the paper's dup8 keys: the short fit is far over the limit (about 4.9
    # times the fair share), so it is kept without retraining
    keys = W.paper_pattern_u64("dup8", n, seed=0)
    f = M.fit_staged(keys, seed=0)
    short = M.fit(keys, seed=0, steps=M.STAGE1_STEPS)
    assert f["stage"] == 1 and M.hopeless(short["estimates"][short["choice"]], 1 << 16)
    assert np.array_equal(f["splitters"], short["splitters"])
