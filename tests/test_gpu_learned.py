"""Parity of the learned multiway first pass with its oracle
(oracle/mlp_oracle.py), step by step through the C ABI, and of the whole
learned sort with the CPU pdqsort oracle.

Exact (bit for bit): the sorted sample, features, targets and the scaling
choice; float32 inference; running maximum and splitters; bin histograms;
sorted keys. Within tolerance: the float32 gradient against the float64
oracle (|g - g_ref| <= 1e-4 |g_ref| + 1e-6, from float32 rounding of sums
over at most 65536 samples), and the training trajectory (see its test)."""
import numpy as np
import pytest

import gen.workloads as W
import oracle
from oracle import mlp_oracle as M
import paper_2106_05123_amd as pdq
from tests._util import as_bytes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pdq.lib()
    return torch.device("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


DISTS = {
    "uniform_u32": lambda n, s: W.uniform_u32(n, seed=s),
    "i32": lambda n, s: W.random_keys("i32", n, seed=s),
    "f32": lambda n, s: W.random_keys("f32", n, seed=s),
    "lognormal_u64": lambda n, s: W.lognormal_u64(n, seed=s),
    "zipf_u64": lambda n, s: W.zipf_u64(n, seed=s),
    "gmm_u64": lambda n, s: W.gmm_u64(n, seed=s),
}


# ----------------------------------------------------------------- fit steps

@pytest.mark.parametrize("dist", list(DISTS))
def test_fit_sample_features_targets_exact(dist):
    n = (1 << 20) + 333
    keys = DISTS[dist](n, 1)
    f = pdq.learned_fit(dev(keys), seed=5, learn_steps=8)
    img = M.key_images(keys)
    samp = np.sort(img[M.sample_positions(5, pdq.LEARN_SAMPLE, n)])
    assert np.array_equal(host(f["sample"]), samp)
    x, use_log = M.features(samp)
    assert int(host(f["info"])[2]) == int(use_log)
    assert np.array_equal(host(f["x"]).view(np.uint32), x.view(np.uint32))
    assert np.array_equal(host(f["t"]), M.midrank_targets(samp))


def test_features_entry_point_degenerate_and_small():
    s = np.full(1000, 42, dtype=np.uint64)
    x, t, info = pdq.learned_features(dev(s))
    assert np.all(host(x) == 0.5) and np.all(host(t) == np.float32(0.5))
    s2 = np.sort(W.uniform_u64(777, seed=3))
    x2, t2, info2 = pdq.learned_features(dev(s2))
    xr, ul = M.features(s2)
    assert np.array_equal(host(x2), xr) and int(host(info2)[2]) == int(ul)
    assert np.array_equal(host(t2), M.midrank_targets(s2))


@pytest.mark.parametrize("residual", [True, False])
@pytest.mark.parametrize("batch", [1, 63, 64, 1000, 4096])
def test_gradient_within_float32_tolerance(residual, batch):
    rng = np.random.default_rng(batch)
    x = np.sort(rng.random(batch)).astype(np.float32)
    t = ((np.arange(batch) + 0.5) / batch + rng.normal(0, 0.01, batch)).astype(np.float32)
    p = M.init_params(3, x)
    p[M.OFF_W3:M.OFF_B3] *= 8  # stronger output weights so every gradient block is exercised
    g, L = pdq.mlp_gradient(dev(p), dev(x), dev(t), residual=residual)
    gr, Lr = M.grad(p, x, t, residual)
    gg = host(g).astype(np.float64)
    assert np.all(np.abs(gg - gr) <= 1e-4 * np.abs(gr) + 1e-6), np.max(np.abs(gg - gr))
    assert abs(float(host(L)[0]) - Lr) <= 1e-4 * Lr + 1e-7


@pytest.mark.parametrize("residual", [True, False])
def test_inference_bit_exact(residual):
    rng = np.random.default_rng(2)
    x = np.concatenate([np.sort(rng.random(70000)), [0.0, 1.0, 2.0, -1.0]]).astype(np.float32)
    p, _ = M.adam_train(M.init_params(4, x[:70000]), x[:70000],
                        ((np.arange(70000) + 0.5) / 70000).astype(np.float32), seed=4, steps=16, batch=256,
                        residual=residual)
    y = pdq.mlp_infer(dev(p), dev(x), residual=residual)
    assert np.array_equal(host(y).view(np.uint32), M.infer_f32(p, x, residual).view(np.uint32))


@pytest.mark.parametrize("dist", ["uniform_u32", "zipf_u64", "gmm_u64"])
def test_extract_bit_exact(dist):
    n = 1 << 20
    keys = DISTS[dist](n, 7)
    samp = np.sort(M.key_images(keys)[M.sample_positions(7, pdq.LEARN_SAMPLE, n)])
    x, _ = M.features(samp)
    t = M.midrank_targets(samp)
    p, _ = M.adam_train(M.init_params(7, x), x, t, seed=7, steps=32, batch=512)
    pred = M.infer_f32(p, x)
    sp, r = pdq.learned_extract(dev(samp), dev(pred))
    assert np.array_equal(host(r), np.maximum.accumulate(pred))
    assert np.array_equal(host(sp), M.splitters(samp, pred))
    # perfect CDF: the splitters are the sample quantiles
    if dist == "uniform_u32":
        sp2, _ = pdq.learned_extract(dev(samp), dev(t))
        assert np.array_equal(host(sp2), M.splitters(samp, t))


def test_extract_heavy_keys_exact():
    m = pdq.LEARN_SAMPLE
    samp = np.sort(W.k_distinct_u64(m, 64, seed=2))
    for pred in (np.zeros(m, np.float32), M.midrank_targets(samp)):
        sp, _ = pdq.learned_extract(dev(samp), dev(pred))
        assert np.array_equal(host(sp), M.splitters(samp, pred))
        assert host(sp).size == 64  # every value fills far more than m/256 slots


def test_train_trajectory_close_to_oracle_and_deterministic():
    """float32 Adam against the float64 oracle from identical initial
    parameters and minibatches. Adam divides by the running gradient scale,
    so rounding differences do not shrink with the gradient; the loss curves
    agree to a few percent over the first steps and the final losses agree
    within a factor of 2. Runs are bitwise reproducible for a fixed grid."""
    n = 1 << 20
    keys = W.uniform_u32(n, seed=0)
    samp = np.sort(M.key_images(keys)[M.sample_positions(0, pdq.LEARN_SAMPLE, n)])
    x, _ = M.features(samp)
    t = M.midrank_targets(samp)
    steps, batch = 128, 1024
    p_ref, l_ref = M.adam_train(M.init_params(0, x), x, t, seed=0, steps=steps, batch=batch)
    p1, l1 = pdq.mlp_train(dev(x), dev(t), seed=0, steps=steps, batch=batch, grid=16)
    p2, l2 = pdq.mlp_train(dev(x), dev(t), seed=0, steps=steps, batch=batch, grid=16)
    l1, l2 = host(l1), host(l2)
    assert np.array_equal(host(p1), host(p2)) and np.array_equal(l1, l2)
    assert abs(l1[0] - l_ref[0]) <= 1e-4 * l_ref[0]   # identical parameters at step 1
    assert np.all(np.abs(l1[:8] - l_ref[:8]) <= 0.05 * l_ref[:8])
    assert 0.5 * l_ref[-8:].mean() <= l1[-8:].mean() <= 2.0 * l_ref[-8:].mean()
    # seeded initialisation on the device equals the oracle's
    p0, _ = pdq.mlp_train(dev(x), dev(t), seed=0, steps=1, batch=batch, grid=16)
    g, _ = M.grad(M.init_params(0, x), x[M.batch_positions(0, 1, batch, x.size)],
                  t[M.batch_positions(0, 1, batch, x.size)])
    want = M.init_params(0, x).astype(np.float64) - M.LR0 * g / (np.abs(g) + M.EPS)
    big = np.abs(g) > 1e-5
    assert np.allclose(host(p0)[big], want[big], atol=2e-6)


def test_train_grid_one_and_init_argument():
    rng = np.random.default_rng(1)
    x = np.sort(rng.random(4096)).astype(np.float32)
    t = ((np.arange(4096) + 0.5) / 4096).astype(np.float32)
    p0 = M.init_params(9, x)
    pa, la = pdq.mlp_train(dev(x), dev(t), seed=9, steps=16, batch=128, grid=1, init=dev(p0))
    pb, lb = pdq.mlp_train(dev(x), dev(t), seed=9, steps=16, batch=128, grid=1)
    assert np.array_equal(host(pa), host(pb))  # explicit init == seeded init
    _, l_ref = M.adam_train(p0, x, t, seed=9, steps=16, batch=128)
    assert np.all(np.abs(host(la) - l_ref) <= 0.05 * l_ref)


# ----------------------------------------------------------------- histogram

@pytest.mark.parametrize("dist", list(DISTS))
@pytest.mark.parametrize("n", [1, 8191, 8192, 8193, (1 << 20) + 77])
def test_histogram_exact(dist, n):
    keys = DISTS[dist](n, n)
    img = M.key_images(keys)
    rng = np.random.default_rng(n)
    srt = np.sort(img)
    for u in (0, 1, 17, 255):
        sp = np.unique(srt[rng.integers(0, n, u)]) if u else np.zeros(0, dtype=np.uint64)
        h = pdq.bucket_histogram(dev(keys), dev(sp))
        assert np.array_equal(host(h), M.histogram(img, sp)), u


def test_histogram_extreme_splitters():
    keys = np.array([0, 1, 2**64 - 1, 2**64 - 1, 5, 2**63], dtype=np.uint64)
    for sp in ([2**64 - 1], [0], [0, 2**64 - 1], [1, 5, 2**63]):
        sp = np.array(sp, dtype=np.uint64)
        assert np.array_equal(host(pdq.bucket_histogram(dev(keys), dev(sp))), M.histogram(keys, sp))


# ----------------------------------------------------------------- whole learned sort

def gpu_sort(a, vals=None, **kw):
    t = dev(a)
    if vals is None:
        st = pdq.sort_(t, stats=True, **kw)
        return host(t), None, st
    v = dev(vals)
    st = pdq.sort_pairs_(t, v, stats=True, **kw)
    return host(t), host(v), st


@pytest.mark.parametrize("dist", list(DISTS))
def test_learned_sort_bit_exact(dist):
    n = (1 << 22) + 5
    a = DISTS[dist](n, 3)
    out, _, st = gpu_sort(a, learned=True)
    assert np.array_equal(as_bytes(out), as_bytes(oracle.sort(a)[0]))
    print(dist, {k: st[k] for k in ("learned", "learned_choice", "learned_sample_judge", "learned_max_range_bin",
                                    "learned_splitters")})
    assert st["learned"] in (1, 2)
    if dist in ("lognormal_u64", "zipf_u64"):
        assert st["learned"] == 1  # the leaf stage brings the worst bin under the judge's limit
    if dist == "uniform_u32":
        assert st["learned"] == 1 and st["learned_splitters"] >= 200
    if dist == "gmm_u64":
        assert st["learned"] == 2  # narrow components: the fit is judged too coarse


@pytest.mark.parametrize("kt", ["i64", "f64"])
def test_learned_sort_wide_signed_and_double(kt):
    # 64-bit signed and double keys through the learned pass: bit-exact
    # whether the fit is used or judged and sent to the plain path
    n = (1 << 21) + 11
    a = W.random_keys(kt, n, seed=12)
    out, _, st = gpu_sort(a, learned=True)
    assert st["learned"] in (1, 2)
    assert np.array_equal(as_bytes(out), as_bytes(oracle.sort(a)[0]))


@pytest.mark.parametrize("kt", ["u32", "i32", "f32", "u64"])
def test_learned_sort_pairs(kt):
    n = (1 << 21) + 11
    a = W.random_keys(kt, n, seed=12)
    if kt == "u64":
        a = a % np.uint64(1 << 40)
    v = np.random.default_rng(2).permutation(n).astype(np.uint32)
    out, vo, st = gpu_sort(a, v, learned=True)
    # normal float32 keys have a two-banded CDF in key-image space (negative
    # and positive halves far apart); the fit is used when the judge accepts it
    assert st["learned"] == 1 if kt != "f32" else st["learned"] in (1, 2)
    assert np.array_equal(as_bytes(out), as_bytes(oracle.sort(a)[0]))
    inv = np.empty(n, dtype=np.int64)
    inv[v] = np.arange(n)
    assert np.array_equal(as_bytes(out), as_bytes(a[inv[vo]]))
    assert np.array_equal(np.sort(vo), np.arange(n, dtype=np.uint32))


def test_learned_equality_bins_and_fallback():
    n = 1 << 21
    a = W.k_distinct_u64(n, 64, seed=1)  # 64 heavy values: each one gets an equality bin
    out, _, st = gpu_sort(a, learned=True)
    assert np.array_equal(out, np.sort(a))
    assert st["learned"] == 1 and st["learned_equal_elements"] == n and st["passes"] == 0
    b = (W.uniform_u32(n, seed=3) % np.uint32(300)).astype(np.uint32)  # 300 values, none heavy
    out_b, _, st_b = gpu_sort(b, learned=True)
    assert np.array_equal(out_b, np.sort(b)) and st_b["learned"] == 1
    # ordered input: the run scan finds an ascending one sorted before anything
    # else; a descending one goes through the order scan to the plain path,
    # whose first pass retires it
    o = W.pattern_i32("ascending", n, seed=0)
    out_o, _, st_o = gpu_sort(o, learned=True)
    assert np.array_equal(out_o, o) and st_o["learned"] == 0 and st_o["near_sorted"] == 3 and st_o["passes"] == 0
    o = W.pattern_i32("descending", n, seed=0)
    out_o, _, st_o = gpu_sort(o, learned=True)
    assert np.array_equal(out_o, np.sort(o)) and st_o["learned"] == 2 and st_o["passes"] == 1
    mix = W.one_value_mix_u64(n, seed=4)  # 90% one value, the rest spread thinly
    out_m, _, st_m = gpu_sort(mix, learned=True)
    assert np.array_equal(out_m, np.sort(mix)) and st_m["learned"] in (1, 2)
    out2, _, st2 = gpu_sort(W.uniform_u32(n, seed=5), learned=True, imbalance_limit=-1.0)
    assert st2["learned"] == 2 and np.all(out2[1:] >= out2[:-1])
    same = np.full(n, 9, dtype=np.uint32)
    out3, _, st3 = gpu_sort(same, learned=True)
    assert np.array_equal(out3, same)
    small = W.uniform_u32(50000, seed=6)   # below the sample size: plain path
    out4, _, st4 = gpu_sort(small, learned=True)
    assert st4["learned"] == 0 and np.array_equal(out4, np.sort(small))


# budget 0: range bins above the LDS base case go to heapsort (above 16384
# keys with the device-counted passes, above 4096 with the host-driven loop)
@pytest.mark.parametrize("n,host_loop", [(1 << 21, True), (1 << 23, False)])
def test_learned_forced_heapsort_inside_bins(n, host_loop):
    a = W.uniform_u32(n, seed=8)
    out, _, st = gpu_sort(a, learned=True, force_budget=0, host_loop=host_loop)
    assert st["learned"] == 1 and st["heapsort_segments"] >= 1
    assert np.array_equal(out, np.sort(a))


@pytest.mark.parametrize("dist", ["uniform_u32", "lognormal_u64"])
def test_trained_network_gains_over_untrained(dist):
    """What training buys: on the same sample and the same extraction, the
    trained network's own splitters (before the leaf stage) have a much
    emptier worst range bin than the initial network's; the
    splitters the fit keeps stay under the judge's 2n/256; and the learned
    sort partitions far fewer keys than the plain path."""
    n = 1 << 22
    keys = DISTS[dist](n, 0)
    f = pdq.learned_fit(dev(keys), seed=0, learn_steps=128)
    sp_tr, _ = pdq.learned_extract(f["sample"], f["pred"])
    h_tr = host(pdq.bucket_histogram(dev(keys), sp_tr))
    p0 = M.init_params(0, host(f["x"]))
    y0 = pdq.mlp_infer(dev(p0), f["x"])
    sp0, _ = pdq.learned_extract(f["sample"], y0)
    h_un = host(pdq.bucket_histogram(dev(keys), sp0))
    h_kept = host(pdq.bucket_histogram(dev(keys), f["splitters"]))
    print(dist, "worst range bin / fair: trained network", h_tr[0::2].max() / (n / 256), "untrained",
          h_un[0::2].max() / (n / 256), "kept", h_kept[0::2].max() / (n / 256), "choice", int(host(f["info"])[3]))
    assert h_tr[0::2].max() * 1.2 < h_un[0::2].max()
    assert h_kept[0::2].max() <= 2 * n / 256
    _, _, st_l = gpu_sort(keys, learned=True)
    _, _, st_p = gpu_sort(keys)
    assert st_l["learned"] == 1
    assert st_l["element_visits"] < 0.6 * st_p["element_visits"]
    assert st_l["passes"] < st_p["passes"]


@pytest.mark.parametrize("dist", ["uniform_u32", "lognormal_u64", "zipf_u64", "gmm_u64"])
def test_staged_budget_follows_the_rule(dist):
    """The default budget: the 32-step fit is kept exactly when its sample
    judge passes the early-accept rule or is hopeless (checked with the
    oracle's rules on the GPU's own 32-step judge), else the fit is the
    128-step fit; parameters and splitters are bitwise those of the
    corresponding single-budget fit, and the sort reports the steps it kept."""
    n = 1 << 22
    keys = DISTS[dist](n, 0)
    short = pdq.learned_fit(dev(keys), seed=0, learn_steps=M.STAGE1_STEPS)
    info = host(short["info"])
    judge = int(info[4 + int(info[3])])
    keep = M.early_accept(judge, pdq.LEARN_SAMPLE) or M.hopeless(judge, pdq.LEARN_SAMPLE)
    staged = pdq.learned_fit(dev(keys), seed=0)
    want = short if keep else pdq.learned_fit(dev(keys), seed=0, learn_steps=M.STAGE2_STEPS)
    assert np.array_equal(host(staged["splitters"]), host(want["splitters"]))
    assert np.array_equal(host(staged["params"]).view(np.uint32), host(want["params"]).view(np.uint32))
    out, _, st = gpu_sort(keys, learned=True)
    assert st["learned_steps"] == (M.STAGE1_STEPS if keep else M.STAGE2_STEPS)
    assert np.array_equal(out, np.sort(keys))
    if dist == "uniform_u32":
        assert keep  # uniform keys are split evenly after the short fit
    if dist == "lognormal_u64":
        assert not keep
    if dist == "gmm_u64":
        # far over the limit after 32 steps: kept as it is, and judged failed
        assert keep and st["learned"] == 2


@pytest.mark.parametrize("dist", ["uniform_u32", "lognormal_u64", "zipf_u64", "gmm_u64"])
def test_leaves_and_sample_judge_bit_exact(dist):
    """The second stage and the sample judge against the oracle, on the
    GPU fit's own sample, features, targets and predictions; and the fit's
    choice among the three candidates is the oracle's."""
    n = (1 << 21) + 17
    keys = DISTS[dist](n, 4)
    f = pdq.learned_fit(dev(keys), seed=4)
    samp, x, t, pred = (host(f[k]) for k in ("sample", "x", "t", "pred"))
    px, py = pdq.learned_leaves(f["x"], f["t"], f["pred"])
    rx, ry = M.leaf_predictions(x, t, pred)
    assert np.array_equal(host(px).view(np.uint32), rx.view(np.uint32))
    assert np.array_equal(host(py).view(np.uint32), ry.view(np.uint32))
    sp, choice, est, _ = M.choose_splitters(samp, x, t, pred)
    for c, arr in enumerate((pred, rx, ry)):
        spc = M.splitters(samp, arr)
        assert pdq.sample_judge(f["sample"], dev(spc)) == est[c] == M.sample_judge(samp, spc)
    info = host(f["info"])
    assert int(info[3]) == choice and [int(v) for v in info[4:7]] == est
    assert np.array_equal(host(f["splitters"]), sp)


def test_sample_judge_edge_cases():
    s = np.sort(W.uniform_u64(4096, seed=1))
    assert pdq.sample_judge(dev(s), dev(np.zeros(0, dtype=np.uint64))) == 4096   # no splitter: one range bin
    sp = np.array([s[0], s[-1]], dtype=np.uint64)  # keys equal to splitters go to equality bins
    assert pdq.sample_judge(dev(s), dev(sp)) == M.sample_judge(s, sp) == 4094


def test_learned_full_size_u32_sampled():
    """2^28 uint32 uniform keys, learned path, benchmark launch
    configuration: sortedness, multiset hash, sampled order statistics."""
    from tests._util import multiset_hash
    n = 1 << 28
    a = W.uniform_u32(n, seed=0)
    t = dev(a)
    st = pdq.sort_(t, learned=True, stats=True)
    out = host(t)
    del t
    torch.cuda.empty_cache()
    assert st["learned"] == 1
    assert np.all(out[1:] >= out[:-1])
    assert multiset_hash(out) == multiset_hash(a)
    rng = np.random.default_rng(1)
    for r in list(rng.integers(0, n, 8)) + [0, n - 1]:
        v = out[r]
        assert int(np.count_nonzero(a < v)) <= r < int(np.count_nonzero(a <= v))
