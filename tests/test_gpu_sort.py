"""Parity of the HIP partition sort with the CPU oracle, through the C ABI.

Keys must match the oracle bit for bit. Payloads must form a valid
permutation that travels with the keys (the sort is unstable, so payload
order among equal keys is not compared). At the full benchmark size the
oracle would take too long per case, so there the checks are properties
that hold at any size: sortedness, an order-independent multiset hash, and
sampled order statistics counted by brute force."""
import math

import numpy as np
import pytest

import gen.workloads as W
import oracle
import paper_2106_05123_amd as pdq
from tests._util import as_bytes, multiset_hash

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pdq.lib()  # fail loudly when the library is missing
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def gpu_sort(a, vals=None, **kw):
    t = to_dev(a)
    if vals is None:
        st = pdq.sort_(t, stats=True, **kw)
        torch.cuda.synchronize()
        return t.cpu().numpy(), None, st
    v = to_dev(vals)
    st = pdq.sort_pairs_(t, v, stats=True, **kw)
    torch.cuda.synchronize()
    return t.cpu().numpy(), v.cpu().numpy(), st


def check_pairs(keys_in, keys_out, vals_out):
    assert np.array_equal(as_bytes(keys_out), as_bytes(keys_in[vals_out]))
    cnt = np.bincount(vals_out.astype(np.int64), minlength=keys_in.size)
    assert cnt.size == keys_in.size and np.all(cnt == 1)


# ------------------------------------------------------------------ plain keys

def test_uniform_u32_2p20_bit_exact_and_first_pass():
    """Small config: 2^20 uint32 uniform keys, seed 0."""
    a = W.uniform_u32(1 << 20, seed=0)
    out, _, st = gpu_sort(a)
    ref, _, c, _ = oracle.sort(a, count=True)
    assert np.array_equal(as_bytes(out), as_bytes(ref))
    # the first partition uses the same ninther on the same input, so its
    # pivot and its left size (count of keys below it) are identical
    assert st["first_pivot_image"] == c["first_pivot_image"]
    assert st["first_left_size"] == c["first_left_size"]
    assert st["first_mode"] == 0
    assert st["heapsort_segments"] == 0


@pytest.mark.parametrize("pattern", W.C2_PATTERNS)
def test_patterns_i32(pattern):
    a = W.pattern_i32(pattern, 1 << 22, seed=0, period=1 << 12, tail=1 << 10)
    out, _, st = gpu_sort(a)
    ref, _, c, _ = oracle.sort(a, count=True)
    assert np.array_equal(out, ref)
    if pattern == "ascending":
        # no descent: the run scan finds it sorted, no partition pass runs
        assert st["passes"] == 0 and st["near_sorted"] == 3 and st["sorted_elements"] == a.size
    if pattern == "descending":
        # the first pass finds the one segment ordered and retires it reversed
        assert st["passes"] == 1 and st["sorted_elements"] == a.size
    if pattern == "ascending_random_tail":
        # one long run and 2^10 outliers: sorted and merged, no partition pass
        assert st["passes"] == 0 and st["near_sorted"] == 1 and 0 < st["near_sorted_outliers"] <= 1 << 10


@pytest.mark.parametrize("kt", ["u32", "i32", "f32", "u64", "i64", "f64"])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 100, 4095, 4096, 4097, 4098, 8191, 8192, 8193, 12289, 65537, 1000003])
def test_sizes_and_key_types(kt, n):
    a = W.random_keys(kt, n, seed=n + 17)
    out, _, _ = gpu_sort(a)
    ref, _, _, _ = oracle.sort(a) if n else (a.copy(), None, None, None)
    assert np.array_equal(as_bytes(out), as_bytes(ref))


@pytest.mark.parametrize("tile", [1024, 2048, 4096, 8192, 16384, 32768, 65536])
@pytest.mark.parametrize("pattern", ["random", "organ_pipe", "sawtooth"])
def test_tile_sizes_same_keys(tile, pattern):
    a = W.pattern_i32(pattern, (1 << 21) + 12345, seed=3, period=1 << 9)
    out, _, _ = gpu_sort(a, tile=tile)
    assert np.array_equal(out, oracle.sort(a)[0])


@pytest.mark.parametrize("learned", [False, True])
@pytest.mark.parametrize("pattern", W.PAPER_PATTERNS)
def test_paper_distributions_u64(pattern, learned):
    # the paper's remaining distributions (Section 6.1) on 64-bit keys, a
    # ragged size above the learned pass's sample: bit-exact in both forms
    n = (1 << 20) + 4099
    a = W.paper_pattern_u64(pattern, n, seed=7)
    out, _, st = gpu_sort(a, learned=learned)
    assert np.array_equal(out, oracle.sort(a)[0])
    if pattern == "ones":
        assert st["passes"] <= 1  # one pass retires the constant input


def test_float_edge_bit_patterns():
    bits = np.array([0xFF800000, 0xFF7FFFFF, 0xBF800000, 0x80800000, 0x807FFFFF, 0x80000001, 0x80000000,
                     0x00000000, 0x00000001, 0x007FFFFF, 0x00800000, 0x3F800000, 0x7F7FFFFF, 0x7F800000],
                    dtype=np.uint32)
    rng = np.random.default_rng(5)
    reps = 3000
    a = np.tile(bits, reps)[rng.permutation(bits.size * reps)].view(np.float32)
    out, _, _ = gpu_sort(a)
    assert np.array_equal(out.view(np.uint32), np.repeat(bits, reps))


def test_all_equal_and_two_values():
    for a in (np.full(1 << 20, 7, np.uint32), W.k_distinct_u64(1 << 20, 2, seed=1)):
        out, _, st = gpu_sort(a)
        assert np.array_equal(out, np.sort(a))


# ------------------------------------------------------------------ LDS base case paths

def _base_case_keys(kind, n, seed):
    """Single segments that go to the LDS base case whole, shaped for each
    path of its block sort: keys that spread over their range (bucket sort),
    keys that cluster (the sample test sends them to the merge sort), few
    distinct values (a bucket overflows), exactly 16, 17, 32 and 33 copies of
    evenly spaced values (the largest bucket at and just past the two finishes'
    caps: ties inside buckets, buckets over two lanes' runs), and 64-bit and
    floating-point images. Float blocks cut their range of values when every
    key is finite (normal keys, keys on both sides of zero) and their range of
    images otherwise (infinities and NaNs)."""
    rng = np.random.default_rng(seed)
    if kind == "uniform_u32":
        return rng.integers(0, 1 << 32, n, dtype=np.uint32)
    if kind == "narrow_u32":
        return (1000 + rng.integers(0, 3 * n, n)).astype(np.uint32)
    if kind == "normal_f32":
        return rng.standard_normal(n, dtype=np.float32)
    if kind == "unit_f32":
        return (1.0 + rng.random(n, dtype=np.float32)).astype(np.float32)
    if kind == "few_u32":
        return rng.integers(0, 40, n).astype(np.uint32)
    if kind.startswith("copies"):
        c = int(kind[len("copies"):].split("_")[0])
        a = np.repeat(np.arange(-(-n // c), dtype=np.uint64) * 1000003, c)[:n].astype(np.uint32)
        return rng.permutation(a)
    if kind == "spanzero_f32":
        # values on both sides of zero with both zeros: a sliver of the image range each
        a = (rng.standard_normal(n) * 1e-3).astype(np.float32)
        a[rng.integers(0, n, 16)] = np.float32(0.0)
        a[rng.integers(0, n, 16)] = np.float32(-0.0)
        return a
    if kind == "normal_inf_nan_f32":
        # non-finite keys send the block back to image buckets
        a = rng.standard_normal(n, dtype=np.float32)
        a[rng.integers(0, n, 3)] = np.inf
        a[rng.integers(0, n, 3)] = -np.inf
        a[rng.integers(0, n, 2)] = np.float32("nan")
        a[rng.integers(0, n, 1)] = -np.float32("nan")
        return a
    if kind == "normal_f64":
        return rng.standard_normal(n)
    if kind == "signed_i64":
        return rng.integers(-(1 << 62), 1 << 62, n, dtype=np.int64)
    if kind == "uniform_f64":
        return rng.standard_normal(n) * 1e-3 + 5.0
    raise ValueError(kind)


BASE_KINDS = ("uniform_u32", "narrow_u32", "normal_f32", "unit_f32", "spanzero_f32", "normal_inf_nan_f32",
              "few_u32", "copies16_u32", "copies17_u32", "copies32_u32", "copies33_u32", "signed_i64",
              "uniform_f64", "normal_f64")


@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("host_loop", [False, True])
@pytest.mark.parametrize("n", [2049, 4096, 8193, 16384])
@pytest.mark.parametrize("kind", BASE_KINDS)
def test_lds_base_case_block_sort_paths(kind, n, host_loop, pairs):
    a = _base_case_keys(kind, n, seed=n)
    v = W.index_payload(n) if pairs else None
    out, vo, st = gpu_sort(a, v, host_loop=host_loop)
    ref = oracle.sort(a)[0]
    assert np.array_equal(as_bytes(out), as_bytes(ref))
    if pairs:
        check_pairs(a, out, vo)


# ------------------------------------------------------------------ pairs / equal keys

@pytest.mark.parametrize("k", [2, 16, 1024, 65536, "mix"])
def test_k_distinct_u64_pairs(k):
    n = 1 << 21
    a = W.one_value_mix_u64(n, seed=2) if k == "mix" else W.k_distinct_u64(n, k, seed=k)
    v = W.index_payload(n)
    out, vo, st = gpu_sort(a, v)
    ref, _, c, _ = oracle.sort(a, count=True)
    assert np.array_equal(out, ref)
    check_pairs(a, out, vo)
    if k != "mix" and k <= 16:
        # Theorem 1: each distinct value is a pivot at most twice
        assert st["passes"] <= 2 * k + 2
        assert st["element_visits"] <= n * (2 * k + 2)


@pytest.mark.parametrize("kt", ["u32", "i32", "f32", "u64", "i64", "f64"])
def test_pairs_key_types(kt):
    n = (1 << 20) + 77
    a = W.random_keys(kt, n, seed=8)
    if kt in ("u32", "u64"):
        a = a % a.dtype.type(5000)
    elif kt in ("i32", "i64"):
        a = (a % 5000).astype(a.dtype) - a.dtype.type(2500)
    elif kt == "f64":
        a = np.round(a, 2)  # many equal keys, both signs, the zeros and infinities kept
    v = np.random.default_rng(1).permutation(n).astype(np.uint32)
    out, vo, _ = gpu_sort(a, v)
    assert np.array_equal(as_bytes(out), as_bytes(oracle.sort(a)[0]))
    assert np.array_equal(as_bytes(out), as_bytes(a[np.argsort(v)][vo]))
    assert np.array_equal(np.sort(vo), np.arange(n, dtype=np.uint32))


# ------------------------------------------------------------------ near-sorted inputs (Section 5.2)

def near_sorted_input(kind, n, kt, seed):
    """Ascending keys of type kt with a disturbance: 'append1' one random key
    appended, 'tail' a random tail of 2^10 keys, 'insert1' one random key
    inserted in the middle, 'merge' two ascending runs concatenated,
    'tail_cap' exactly 8192 keys in short runs, 'tail_over' 8193, 'three'
    two long runs and a short one, 'sorted' nothing."""
    rng = np.random.default_rng(seed)
    # ascending in canonical order (-0.0 before +0.0), which np.sort does not promise
    base = oracle.sort(W.random_keys(kt, n, seed=seed))[0]
    if kind == "sorted":
        return base
    if kind == "append1":
        return np.concatenate([base[: n - 1], W.random_keys(kt, 1, seed=seed + 1)])
    if kind == "tail":
        t = 1 << 10
        return np.concatenate([base[: n - t], W.random_keys(kt, t, seed=seed + 1)])
    if kind in ("tail_cap", "tail_over"):
        # the t smallest keys, descending, after the t largest: every tail key
        # is a run of its own (or of two equal keys), all of them short
        t = 8192 if kind == "tail_cap" else 8193
        return np.concatenate([base[t:], base[:t][::-1]])
    if kind == "insert1":
        m = n // 2
        return np.concatenate([base[:m], W.random_keys(kt, 1, seed=seed + 1), base[m: n - 1]])
    if kind == "merge":
        return np.concatenate([oracle.sort(base[rng.permutation(n)[: n // 3]])[0],
                               oracle.sort(base[rng.permutation(n)[: n - n // 3]])[0]])
    if kind == "three":
        # [run, largest key] [one key above the next run's start] [run]
        m = n // 2
        return np.concatenate([base[:m], base[-1:], base[m + 5: m + 6], base[m: n - 2]])
    raise ValueError(kind)


NEAR_EXPECT = {"sorted": 3, "append1": 1, "tail": 1, "insert1": (1, 2), "merge": 2, "tail_cap": 1,
               "tail_over": 0, "three": 0}


@pytest.mark.parametrize("kind", list(NEAR_EXPECT))
@pytest.mark.parametrize("kt", ["i32", "u64", "f32", "f64"])
@pytest.mark.parametrize("pairs", [False, True])
def test_near_sorted_inputs(kind, kt, pairs):
    n = (1 << 20) + 321
    a = near_sorted_input(kind, n, kt, seed=31)
    v = W.index_payload(a.size) if pairs else None
    out, vo, st = gpu_sort(a, v)
    ref = oracle.sort(a)[0]
    assert np.array_equal(as_bytes(out), as_bytes(ref))
    if pairs:
        check_pairs(a, out, vo)
    want = NEAR_EXPECT[kind]
    assert st["near_sorted"] in (want if isinstance(want, tuple) else (want,))
    if st["near_sorted"]:
        assert st["passes"] == 0
    if kind == "append1" and st["near_sorted"] == 1:
        assert st["near_sorted_outliers"] == 1
    if kind == "tail_cap":
        assert st["near_sorted_outliers"] == 8192


@pytest.mark.parametrize("learned", [False, True])
def test_near_sorted_both_forms_and_sizes(learned):
    """The run scan is tried before the learned pass too; ranges below
    16384 keys skip it; a random input falls through to the passes."""
    for n, kind in ((16384, "append1"), (16383, "append1"), (70001, "tail"), (1 << 21, "merge")):
        a = near_sorted_input(kind, n, "u32", seed=n)
        out, _, st = gpu_sort(a, learned=learned)
        assert np.array_equal(out, np.sort(a))
        assert (st["near_sorted"] != 0) == (n >= 16384)
    a = W.uniform_u32(1 << 20, seed=2)
    out, _, st = gpu_sort(a, learned=learned)
    assert np.array_equal(out, np.sort(a)) and st["near_sorted"] == 0
    if learned:
        # the learned split ran; its bins (~4096 keys) fit the LDS classes
        assert st["learned"] == 1
    else:
        assert st["passes"] > 0


# ------------------------------------------------------------------ fresh candidates (Section 4.2)

def planted_bad_first_pivot(n, seed):
    """Uniform keys >= 1000 with the nine ninther candidate positions of the
    whole range (first, mid, last and their neighbours) holding nine keys
    below 10: the first pivot has rank < 9, so the first partition is bad
    (L < n/8) and both children take fresh candidates."""
    rng = np.random.default_rng(seed)
    a = rng.integers(1000, 2**32, n, dtype=np.uint32)
    m = n // 2
    pos = [0, m, n - 1, 1, m - 1, n - 2, 2, m + 1, n - 3]
    a[pos] = rng.permutation(9).astype(np.uint32)
    return a


@pytest.mark.parametrize("fixed", [False, True])
@pytest.mark.parametrize("deterministic", [False, True])
def test_fresh_candidate_rules_after_bad_partition(fixed, deterministic):
    """Both fresh-candidate rules (hashed positions by default; the paper's
    fixed quarter offsets with PDQ_FRESH_FIXED) run after a planted bad
    first partition: the budget is charged, no segment falls to heapsort,
    and the keys are bit-exact."""
    n = (1 << 21) + 999
    a = planted_bad_first_pivot(n, seed=4)
    v = W.index_payload(n)
    t = to_dev(a)
    tv = to_dev(v)
    st = pdq.sort_pairs_(t, tv, stats=True, fresh_fixed=fixed, deterministic=deterministic)
    torch.cuda.synchronize()
    out, vo = t.cpu().numpy(), tv.cpu().numpy()
    ref, _, c, _ = oracle.sort(a, count=True)
    assert np.array_equal(out, ref)
    check_pairs(a, out, vo)
    assert st["first_left_size"] == c["first_left_size"] < n // 8
    assert st["bad_partitions"] >= 1
    assert st["heapsort_segments"] == 0


def test_fresh_rules_differ_only_below_the_bad_partition():
    """With the look-back form every run arranges the keys identically, so
    each rule repeats its own statistics exactly; the first partition (before
    any fresh candidate) is the same for both rules."""
    n = (1 << 21) + 999
    a = planted_bad_first_pivot(n, seed=5)
    runs = {}
    for fixed in (False, True, False, True):
        out, _, st = gpu_sort(a, deterministic=True, fresh_fixed=fixed)
        assert np.array_equal(out, np.sort(a))
        runs.setdefault(fixed, []).append(st)
    for fixed, (s1, s2) in runs.items():
        assert {k: s1[k] for k in DET_STATS} == {k: s2[k] for k in DET_STATS}
    assert runs[False][0]["first_left_size"] == runs[True][0]["first_left_size"]


def test_check_after_sort_reports_no_device_error():
    a = W.uniform_u32((1 << 20) + 3, seed=3)
    t = to_dev(a)
    ws = torch.empty(pdq.workspace_bytes(a.size, 1, "u32"), dtype=torch.uint8, device="cuda:0")
    pdq.sort_(t, workspace=ws)
    pdq.check(ws)
    assert np.array_equal(t.cpu().numpy(), np.sort(a))


# ------------------------------------------------------------------ segmented

def test_segmented_f32_pairs():
    keys, off, vals = W.segmented_f32(500, max_log2=16, seed=4)
    t, o, v = to_dev(keys), to_dev(off), to_dev(vals)
    st = pdq.segmented_sort_(t, o, v, stats=True, validate=True)
    out, vo = t.cpu().numpy(), v.cpu().numpy()
    ref, _, _ = oracle.segmented_sort(keys, off)
    assert np.array_equal(as_bytes(out), as_bytes(ref))
    check_pairs(keys, out, vo)
    seg_of = np.searchsorted(off, np.arange(keys.size, dtype=np.uint64), side="right") - 1
    assert np.array_equal(seg_of[vo], seg_of)  # payloads stay inside their segment


def test_segmented_empty_and_tiny_segments():
    sizes = np.array([0, 1, 0, 2, 3, 4096, 4097, 0, 1, 9000, 0], dtype=np.int64)
    off = W.offsets_from_sizes(sizes)
    a = W.uniform_u32(int(off[-1]), seed=9)
    t = to_dev(a)
    pdq.segmented_sort_(t, to_dev(off), validate=True)
    assert np.array_equal(t.cpu().numpy(), oracle.segmented_sort(a, off)[0])


@pytest.mark.parametrize("tile", [1024, 8192])
def test_segmented_tiles_straddling_segments(tile):
    # segments just below, at and just above multiples of the tile, in a
    # shuffled order: every segment's tiles start at its first key and only
    # its last tile is partial; the pass hands tiles out over a permutation
    # that interleaves segments and over one ticket queue per XCD
    rng = np.random.default_rng(tile)
    base = np.array([1, 2, tile - 1, tile, tile + 1, 2 * tile - 1, 2 * tile + 1, 5 * tile + 7, 40 * tile + 3])
    sizes = rng.permutation(np.repeat(base, 37)).astype(np.int64)
    off = W.offsets_from_sizes(sizes)
    n = int(off[-1])
    a = W.uniform_u32(n, seed=tile + 1)
    vals = np.arange(n, dtype=np.uint32)
    t, o, v = to_dev(a), to_dev(off), to_dev(vals)
    pdq.segmented_sort_(t, o, v, tile=tile, validate=True)
    out, vo = t.cpu().numpy(), v.cpu().numpy()
    assert np.array_equal(out, oracle.segmented_sort(a, off)[0])
    check_pairs(a, out, vo)
    seg_of = np.searchsorted(off, np.arange(n, dtype=np.uint64), side="right") - 1
    assert np.array_equal(seg_of[vo], seg_of)


def test_segmented_validate_rejects_bad_offsets():
    a = W.uniform_u32(1000, seed=1)
    bad = np.array([0, 600, 400, 1000], dtype=np.uint64)  # not monotone
    with pytest.raises(pdq.PdqError) as ei:
        pdq.segmented_sort_(to_dev(a), to_dev(bad), validate=True)
    assert ei.value.status == -1
    short = np.array([0, 500, 900], dtype=np.uint64)      # does not end at n
    with pytest.raises(pdq.PdqError):
        pdq.segmented_sort_(to_dev(a), to_dev(short), validate=True)


# ------------------------------------------------------------------ fallbacks

# a budget of 0 sends every segment above the LDS base case to heapsort: above
# 4096 keys in the host-driven loop, above 16384 in the device-counted passes
@pytest.mark.parametrize("n,host_loop", [(4097, True), (5000, True), (20000, True), (16385, False),
                                         (20000, False), (100003, False), ((1 << 21) + 3, False)])
@pytest.mark.parametrize("kt", ["u32", "f64"])
def test_forced_heapsort(n, host_loop, kt):
    """The fallback sort (a workgroup merge sort: LDS-sorted chunks of 2048
    keys, then merge passes between the two buffers) on a whole input whose
    budget is 0: one item, keys bit-exact, payloads travel with them."""
    a = W.random_keys(kt, n, seed=n)
    v = W.index_payload(n)
    out, vo, st = gpu_sort(a, v, force_budget=0, host_loop=host_loop)
    assert st["heapsort_segments"] == 1 and st["heapsort_elements"] == n
    assert np.array_equal(as_bytes(out), as_bytes(oracle.sort(a)[0]))
    check_pairs(a, out, vo)


@pytest.mark.parametrize("n,host_loop", [(5000, True), (100003, True), (20000, False), (100003, False)])
def test_paper_heapsort_fallback_option(n, host_loop):
    """PDQ_HEAPSORT: the fallback is the paper's heapsort (Section 4.1), one
    lane per segment in the user buffer; same keys as the oracle."""
    a = W.uniform_u32(n, seed=n + 1)
    v = W.index_payload(n)
    out, vo, st = gpu_sort(a, v, force_budget=0, host_loop=host_loop, heapsort=True)
    assert st["heapsort_segments"] == 1 and st["heapsort_elements"] == n
    assert np.array_equal(out, oracle.sort(a)[0])
    check_pairs(a, out, vo)


def test_fallback_sort_of_segments_out_of_budget_in_the_tail():
    """With no device-counted pass, the persistent tail partitions the
    input; its planted bad first partition uses up a budget of 1, so the
    big child is filed for the fallback sort, which runs after the tail."""
    n = (1 << 20) + 99
    a = planted_bad_first_pivot(n, seed=7)
    v = W.index_payload(n)
    out, vo, st = gpu_sort(a, v, force_budget=1, batch_passes=0)
    assert st["heapsort_segments"] >= 1 and st["heapsort_elements"] > n // 2
    assert np.array_equal(out, oracle.sort(a)[0])
    check_pairs(a, out, vo)


@pytest.mark.parametrize("n,host_loop", [(1 << 16, True), (1 << 18, False)])
def test_budget_one_reaches_heapsort_after_bad_partition(n, host_loop):
    a = W.pattern_i32("organ_pipe", n)
    out, _, st = gpu_sort(a, force_budget=1, host_loop=host_loop)
    assert st["bad_partitions"] >= 1 and st["heapsort_segments"] >= 1
    assert np.array_equal(out, oracle.sort(a)[0])


# ------------------------------------------------------------------ pass loops

@pytest.mark.parametrize("kt", ["u32", "f32", "u64", "i64"])
@pytest.mark.parametrize("pairs", [False, True])
def test_host_loop_and_device_passes_agree(kt, pairs):
    """The host-driven pass loop (PDQ_HOST_LOOP) and the default
    device-counted passes give the oracle's keys, and payloads that travel
    with their keys."""
    n = (1 << 21) + 4321
    a = W.random_keys(kt, n, seed=31)
    v = W.index_payload(n) if pairs else None
    ref = oracle.sort(a)[0]
    for host_loop in (False, True):
        out, vo, st = gpu_sort(a, v, host_loop=host_loop)
        assert np.array_equal(as_bytes(out), as_bytes(ref)), f"host_loop={host_loop}"
        if pairs:
            check_pairs(a, out, vo)
        assert st["passes"] > 0 and st["heapsort_segments"] == 0


@pytest.mark.parametrize("passes", [0, 1, 3, 8])
@pytest.mark.parametrize("pairs", [False, True])
def test_device_passes_cut_short_leave_the_rest_to_the_tail(passes, pairs):
    """With fewer device-counted passes than the recursion needs, the
    persistent tail partitions what is still live (single workgroups, a
    device queue) and sorts the small pieces in LDS: keys still bit-exact."""
    n = (1 << 20) + 77
    a = W.uniform_u32(n, seed=passes)
    v = W.index_payload(n) if pairs else None
    out, vo, st = gpu_sort(a, v, batch_passes=passes)
    assert np.array_equal(out, oracle.sort(a)[0])
    if pairs:
        check_pairs(a, out, vo)
    assert st["passes"] <= passes
    if passes < 3:
        assert st["batch_items"] > 0


def test_single_range_plan_replays_bit_exact():
    """pdq_plan_create with no offsets captures the device-counted sort of
    one range as a HIP graph: three replays on refilled buffers (eager work
    and synchronisation between them) equal the oracle and the eager call."""
    n = (1 << 22) + 1234
    keys0 = W.uniform_u32(n, seed=40)
    vals0 = W.index_payload(n)
    tk, tv = to_dev(keys0), to_dev(vals0)
    plan = pdq.Plan(tk, None, tv)
    for rep in range(3):
        keys = W.uniform_u32(n, seed=41 + rep)
        tk.copy_(to_dev(keys))
        tv.copy_(to_dev(vals0))
        plan.launch()
        torch.cuda.synchronize()
        out, vo = tk.cpu().numpy(), tv.cpu().numpy()
        assert np.array_equal(out, oracle.sort(keys)[0])
        check_pairs(keys, out, vo)
        eager, _, _ = gpu_sort(keys)
        assert np.array_equal(eager, out)
        _ = torch.ones(1000, device="cuda:0").sum().item()
    plan.destroy()


# ------------------------------------------------------------------ full size, sampled

def test_full_size_random_i32_sampled():
    """2^28 int32 uniform keys in the benchmark's launch configuration:
    sortedness, multiset hash, and order statistics at sampled ranks
    (count of keys below / not above the output key, by brute force)."""
    n = 1 << 28
    a = W.pattern_i32("random", n, seed=0)
    t = to_dev(a)
    pdq.sort_(t)
    torch.cuda.synchronize()
    out = t.cpu().numpy()
    del t
    torch.cuda.empty_cache()
    assert np.all(out[1:] >= out[:-1])
    assert multiset_hash(out) == multiset_hash(a)
    rng = np.random.default_rng(0)
    for r in list(rng.integers(0, n, 12)) + [0, n // 2, n - 1]:
        v = out[r]
        lt = int(np.count_nonzero(a < v))
        le = int(np.count_nonzero(a <= v))
        assert lt <= r < le


# ------------------------------------------------------------------ deterministic (look-back) form

DET_STATS = ("passes", "element_visits", "partitions_right", "partitions_left", "bad_partitions",
             "base_segments", "sorted_segments", "equal_elements")


@pytest.mark.parametrize("tile", [0, 8192, 32768, 65536])
@pytest.mark.parametrize("kt", ["u32", "u64"])
def test_deterministic_pairs_repeat_exactly(kt, tile):
    """PDQ_DETERMINISTIC: keys bit-exact against the oracle, and two runs give
    the same payload order (also among equal keys) and the same recursion."""
    n = (1 << 21) + 4321
    if kt == "u64":
        a = W.k_distinct_u64(n, 16, seed=3)
    else:
        a = (W.uniform_u32(n, seed=3) % np.uint32(1000)).astype(np.uint32)
    vals = W.index_payload(n)
    out1, v1, st1 = gpu_sort(a, vals, tile=tile, deterministic=True)
    out2, v2, st2 = gpu_sort(a, vals, tile=tile, deterministic=True)
    assert np.array_equal(as_bytes(out1), as_bytes(oracle.sort(a)[0]))
    check_pairs(a, out1, v1)
    assert np.array_equal(v1, v2)
    assert np.array_equal(as_bytes(out1), as_bytes(out2))
    assert {k: st1[k] for k in DET_STATS} == {k: st2[k] for k in DET_STATS}


def test_deterministic_segmented_repeat_exactly():
    keys, off, vals = W.segmented_f32(800, max_log2=17, seed=8)
    res = []
    for _ in range(2):
        t, o, v = to_dev(keys), to_dev(off), to_dev(vals)
        pdq.segmented_sort_(t, o, v, deterministic=True)
        torch.cuda.synchronize()
        res.append((t.cpu().numpy(), v.cpu().numpy()))
    ref, _, _ = oracle.segmented_sort(keys, off)
    assert np.array_equal(as_bytes(res[0][0]), as_bytes(ref))
    assert np.array_equal(res[0][1], res[1][1])


def test_default_form_agrees_with_deterministic_on_keys_and_first_pass():
    """The default (reservation) form and the look-back form sort to the same
    keys, and their first partitions coincide (same pivot, same left size)."""
    a = W.uniform_u32((1 << 22) + 77, seed=12)
    o1, _, s1 = gpu_sort(a)
    o2, _, s2 = gpu_sort(a, deterministic=True)
    assert np.array_equal(o1, o2)
    assert s1["first_pivot_image"] == s2["first_pivot_image"]
    assert s1["first_left_size"] == s2["first_left_size"]


# ------------------------------------------------------------------ 64-bit payloads (PDQ_VALS64)

def check_pairs64(keys_in, vals_in, keys_out, vals_out):
    """Keys bit-exact against the oracle; every output (key, payload) pair is
    an input pair, each used once (payloads of equal keys in any order)."""
    assert np.array_equal(as_bytes(keys_out), as_bytes(oracle.sort(keys_in)[0]))
    kb_in, kb_out = bits_u64(keys_in), bits_u64(keys_out)
    a = np.lexsort((vals_in, kb_in))
    b = np.lexsort((vals_out, kb_out))
    assert np.array_equal(kb_in[a], kb_out[b]) and np.array_equal(vals_in[a], vals_out[b])


def bits_u64(a):
    return a.view(np.uint32).astype(np.uint64) if a.dtype.itemsize == 4 else a.view(np.uint64)


@pytest.mark.parametrize("kt", ["u32", "i32", "f32", "u64", "i64", "f64"])
@pytest.mark.parametrize("learned", [False, True])
def test_pairs_u64_payloads(kt, learned):
    n = (1 << 20) + 4097
    a = W.random_keys(kt, n, seed=40)
    if kt in ("u32", "i32", "u64", "i64"):
        a = (a % a.dtype.type(70000)).astype(a.dtype)  # equal keys with different payloads
    v = np.random.default_rng(41).integers(0, 2**64, n, dtype=np.uint64)
    t, tv = to_dev(a), to_dev(v)
    st = pdq.sort_pairs_(t, tv, stats=True, learned=learned)
    torch.cuda.synchronize()
    check_pairs64(a, v, t.cpu().numpy(), tv.cpu().numpy())
    if learned:
        assert st["learned"] in (1, 2)


@pytest.mark.parametrize("batched", [False, True])
def test_segmented_u64_payloads(batched):
    sizes = np.array([0, 1, 5, 4096, 4097, 20000, 70001, 300000, 1000, 9000], dtype=np.int64)
    off = W.offsets_from_sizes(sizes)
    n = int(off[-1])
    a = W.random_keys("f64", n, seed=42)
    v = np.random.default_rng(43).integers(0, 2**64, n, dtype=np.uint64)
    t, tv, to = to_dev(a), to_dev(v), to_dev(off)
    pdq.segmented_sort_(t, to, tv, batched=batched)
    torch.cuda.synchronize()
    ko, vo = t.cpu().numpy(), tv.cpu().numpy()
    ref = oracle.segmented_sort(a, off)[0]
    assert np.array_equal(as_bytes(ko), as_bytes(ref))
    for s in range(sizes.size):
        lo, hi = int(off[s]), int(off[s + 1])
        if hi > lo:
            x = np.lexsort((v[lo:hi], bits_u64(a[lo:hi])))
            y = np.lexsort((vo[lo:hi], bits_u64(ko[lo:hi])))
            assert np.array_equal(v[lo:hi][x], vo[lo:hi][y])


def test_plan_and_noalloc_u64_payloads():
    keys, off, _ = W.segmented_f32(300, max_log2=16, seed=12)
    n = keys.size
    v = np.random.default_rng(44).integers(0, 2**64, n, dtype=np.uint64)
    t, tv, to = to_dev(keys), to_dev(v), to_dev(off)
    plan = pdq.Plan(t, to, tv, autotune=True)
    for rep in range(2):
        t.copy_(to_dev(keys))
        tv.copy_(to_dev(v))
        plan.launch()
        plan.check()
        ko, vo = t.cpu().numpy(), tv.cpu().numpy()
        assert np.array_equal(as_bytes(ko), as_bytes(oracle.segmented_sort(keys, off)[0]))
        assert np.array_equal(np.sort(vo), np.sort(v))
    plan.destroy()
    a = W.random_keys("u64", 200003, seed=45)
    v2 = np.random.default_rng(46).integers(0, 2**64, a.size, dtype=np.uint64)
    t2, tv2 = to_dev(a), to_dev(v2)
    pdq.sort_noalloc_(t2, tv2)
    torch.cuda.synchronize()
    check_pairs64(a, v2, t2.cpu().numpy(), tv2.cpu().numpy())


# ------------------------------------------------------------------ LDS base case: radix and merge forms

@pytest.mark.parametrize("kt", ["u32", "i32", "f32", "u64"])
@pytest.mark.parametrize("pairs", [False, True])
def test_base_case_key_spans(kt, pairs):
    """Segments of 1000 ... 4096 keys whose images span 0, 1, 5, 6, 7, 12,
    13, 18, 19 and all bits: the radix form takes 0, 1, 1, 1, 2, 2, 3, 3
    passes, the merge form the rest; both bit-exact against the oracle."""
    rng = np.random.default_rng(47)
    spans = [0, 1, 5, 6, 7, 12, 13, 18, 19, 64]
    sizes, parts = [], []
    for sp in spans:
        for size in (1000, 1024, 2048, 2049, 3000, 4095, 4096):
            lo = int(rng.integers(0, 2**20))
            width = min(sp, 31)
            r = rng.integers(0, 2 ** width, size, dtype=np.uint64) if width else np.zeros(size, np.uint64)
            img = (np.uint64(lo) + r) if sp < 64 else rng.integers(0, 2**63, size, dtype=np.uint64)
            parts.append(img)
            sizes.append(size)
    img = np.concatenate(parts)
    off = W.offsets_from_sizes(np.array(sizes, dtype=np.int64))
    dt = W.key_dtype(kt)
    if dt().itemsize == 4:
        a = (img & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        if kt == "f32":
            a = np.where(a >> np.uint32(23) >= np.uint32(0xFF), a & np.uint32(0x3FFFFFFF), a)  # no NaN
        a = a.view(dt)
    else:
        a = img.view(dt)
    v = W.index_payload(a.size) if pairs else None
    t, to = to_dev(a), to_dev(off)
    tv = to_dev(v) if pairs else None
    pdq.segmented_sort_(t, to, tv)
    torch.cuda.synchronize()
    out = t.cpu().numpy()
    assert np.array_equal(as_bytes(out), as_bytes(oracle.segmented_sort(a, off)[0]))
    if pairs:
        vo = tv.cpu().numpy()
        assert np.array_equal(as_bytes(out), as_bytes(a[vo]))
        assert np.array_equal(np.sort(vo), v)
