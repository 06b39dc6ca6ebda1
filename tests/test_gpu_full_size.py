"""Every benchmark configuration at its full size, in the benchmark's launch
configuration, checked through the C ABI by properties that hold at any
size (the oracle would take too long per case here):

  * keys: non-decreasing in canonical order, the same multiset as the input
    (order-independent SplitMix64 hash), and order statistics at sampled
    ranks counted by brute force over the input;
  * payloads: a permutation, and keys_out[j] == keys_in[vals_out[j]];
  * the O(nk) behaviour of the equal-key scheme (Theorem 1) as bounds on the
    passes and on the keys partitioned.

Sizes: 2^28 int32 in each of the paper's patterns (plain and learned
forms), 2^27 uint64 with k equal values plus payloads, 2^29 uint64 skewed
mixtures through the learned pass, and the 2^28 uint32 headline input in
both forms. Keys are also compared element by element with numpy's sort of
the same input: the sorted key sequence is unique, so any correct sort pins
it. The 65,536-segment batch has a full-size test of its own."""
import numpy as np
import pytest

import gen.workloads as W
import paper_2106_05123_amd as pdq
from tests._util import multiset_hash

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pdq.lib()
    return torch.device("cuda:0")


def sort_on_gpu(a, vals=None, **kw):
    t = torch.from_numpy(a).to("cuda:0")
    v = torch.from_numpy(vals).to("cuda:0") if vals is not None else None
    if v is None:
        st = pdq.sort_(t, stats=True, **kw)
    else:
        st = pdq.sort_pairs_(t, v, stats=True, **kw)
    torch.cuda.synchronize()
    out = t.cpu().numpy()
    vo = v.cpu().numpy() if v is not None else None
    del t, v
    torch.cuda.empty_cache()
    return out, vo, st


def check_sorted_permutation(a, out, h_in, nranks=4, seed=0):
    assert np.all(out[1:] >= out[:-1])
    assert multiset_hash(out) == h_in
    rng = np.random.default_rng(seed)
    n = a.size
    for r in list(rng.integers(0, n, nranks)) + [0, n - 1]:
        v = out[r]
        assert int(np.count_nonzero(a < v)) <= r < int(np.count_nonzero(a <= v))


@pytest.mark.parametrize("pattern", [p for p in W.C2_PATTERNS if p != "random"])
def test_full_size_patterns_i32_plain_and_learned(pattern):
    n = 1 << 28
    a = W.pattern_i32(pattern, n, seed=0)
    h = multiset_hash(a)
    out, _, st = sort_on_gpu(a)
    check_sorted_permutation(a, out, h)
    if pattern == "ascending":
        assert st["passes"] == 0 and st["near_sorted"] == 3 and st["sorted_elements"] == n
    if pattern == "descending":
        assert st["passes"] == 1 and st["sorted_elements"] == n
    if pattern == "ascending_random_tail":
        # the GPU form of the partial insertion sort (Section 5.2): one scan
        # finds one long run and 2^10 outliers, sorts them and merges
        assert st["passes"] == 0 and st["near_sorted"] == 1
    out_l, _, st_l = sort_on_gpu(a, learned=True)
    assert np.array_equal(out_l, out)
    assert np.array_equal(out, np.sort(a))  # element by element (an independent sort)
    print(pattern, "plain passes", st["passes"], "learned state", st_l["learned"], "passes", st_l["passes"])


@pytest.mark.parametrize("k", [2, 16, 1024, 65536, "mix"])
def test_full_size_equal_keys_u64_pairs(k):
    n = 1 << 27
    a = W.one_value_mix_u64(n, seed=0) if k == "mix" else W.k_distinct_u64(n, k, seed=0)
    vals = W.index_payload(n)
    h = multiset_hash(a)
    out, vo, st = sort_on_gpu(a, vals)
    assert np.all(out[1:] >= out[:-1])
    assert multiset_hash(out) == h
    assert np.array_equal(np.bincount(vo, minlength=n), np.ones(n, dtype=np.int64))
    assert np.array_equal(out, a[vo])
    assert np.array_equal(out, np.sort(a))  # element by element (an independent sort)
    print("k", k, {x: st[x] for x in ("passes", "element_visits", "partitions_right", "partitions_left",
                                      "equal_elements", "base_segments", "heapsort_segments")})
    if k != "mix" and k <= 16:
        # every value is a pivot at most twice (Lemma 4), so a key is
        # partitioned at most 2k + 2 times and the recursion is that deep
        assert st["passes"] <= 2 * k + 2
        assert st["element_visits"] <= (2 * k + 2) * n
    assert st["heapsort_segments"] == 0


def zipf_full(n, seed=0):
    """zipf_u64 with the inverse-CDF lookup done on the GPU (same uniforms,
    same float64 table, so the same keys)."""
    cdf = torch.from_numpy(W.zipf_cdf()).to("cuda:0")
    u = torch.from_numpy(W.zipf_uniforms(n, seed)).to("cuda:0")
    r = torch.searchsorted(cdf, u, right=True) + 1
    out = torch.clamp(r, max=cdf.numel()).to(torch.int64).cpu().numpy().view(np.uint64)
    del cdf, u, r
    torch.cuda.empty_cache()
    return out


def test_zipf_gpu_lookup_matches_generator():
    n = 1 << 20
    assert np.array_equal(zipf_full(n, seed=5), W.zipf_u64(n, seed=5))


@pytest.mark.parametrize("dist", ["lognormal", "zipf", "gmm"])
def test_full_size_learned_u64_mixtures(dist):
    n = 1 << 29
    a = {"lognormal": lambda: W.lognormal_u64(n, seed=0), "zipf": lambda: zipf_full(n, seed=0),
         "gmm": lambda: W.gmm_u64(n, seed=0)}[dist]()
    h = multiset_hash(a)
    out, _, st = sort_on_gpu(a, learned=True)
    check_sorted_permutation(a, out, h, nranks=3)
    assert np.array_equal(out, np.sort(a))  # element by element (an independent sort)
    assert st["learned"] in (1, 2)
    print(dist, {x: st[x] for x in ("learned", "learned_splitters", "learned_max_range_bin", "passes",
                                    "element_visits", "equal_elements", "learned_equal_elements")})


@pytest.mark.parametrize("learned", [False, True])
def test_full_size_headline_u32_element_by_element(learned):
    """The headline input (2^28 uint32 keys uniform over [0, 2^32), seed 0)
    in the benchmark's launch configuration, both forms, compared key by key
    with numpy's sort."""
    n = 1 << 28
    a = W.uniform_u32(n, seed=0)
    out, _, st = sort_on_gpu(a, learned=learned)
    assert np.array_equal(out, np.sort(a))
    assert st["heapsort_segments"] == 0
    if learned:
        assert st["learned"] == 1
