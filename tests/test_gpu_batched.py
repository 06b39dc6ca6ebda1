"""The batched segmented sort (partition passes with device-side counts, the
wide LDS classes, the persistent tail over a device queue, and the captured
HIP-graph plan) against the CPU oracle, through the C ABI.

Keys must match the oracle bit for bit; payloads must be a valid
permutation that stays inside its segment. Segment sizes cover every size
class (<= 64 ... 16384 keys, 8192 for 64-bit keys with payloads), segments
that need partition passes, and, with the passes cut short, the persistent
tail: LDS networks of its workgroup, single-workgroup partitions and queued
children."""
import numpy as np
import pytest

import gen.workloads as W
import oracle
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


EDGE_SIZES = [0, 1, 2, 3, 63, 64, 65, 256, 1000, 4095, 4096, 4097, 5000, 8191, 8192, 8193, 16383, 16384, 16385,
              20000, 65536, 100003, 300000]


def mixed_sizes(seed, extra=300, max_log2=16):
    rng = np.random.default_rng(seed)
    sizes = np.concatenate([EDGE_SIZES, W.segment_sizes_loguniform(extra, max_log2, seed)])
    return sizes[rng.permutation(sizes.size)].astype(np.int64)


def check_segmented(keys, off, out, vals_out=None):
    ref, _, _ = oracle.segmented_sort(keys, off)
    assert np.array_equal(as_bytes(out), as_bytes(ref))
    if vals_out is not None:
        cnt = np.bincount(vals_out.astype(np.int64), minlength=keys.size)
        assert cnt.size == keys.size and np.all(cnt == 1)
        assert np.array_equal(as_bytes(out), as_bytes(keys[vals_out]))
        seg_of = np.searchsorted(off, np.arange(keys.size, dtype=np.uint64), side="right") - 1
        assert np.array_equal(seg_of[vals_out], seg_of)


def run_batched(keys, off, vals=None, **kw):
    t, o = dev(keys), dev(off)
    v = dev(vals) if vals is not None else None
    st = pdq.segmented_sort_(t, o, v, batched=True, stats=True, **kw)
    return host(t), (host(v) if v is not None else None), st


@pytest.mark.parametrize("kt", ["u32", "i32", "f32", "u64", "i64", "f64"])
@pytest.mark.parametrize("pairs", [False, True])
def test_batched_mixed_sizes(kt, pairs):
    off = W.offsets_from_sizes(mixed_sizes(7))
    n = int(off[-1])
    keys = W.random_keys(kt, n, seed=5)
    vals = W.index_payload(n) if pairs else None
    out, vo, st = run_batched(keys, off, vals)
    check_segmented(keys, off, out, vo)
    assert st["passes"] >= 1 and st["element_visits"] > 0


@pytest.mark.parametrize("kt", ["f32", "u64"])
@pytest.mark.parametrize("passes", [0, 1, 2])
def test_batched_tail(kt, passes):
    """Passes cut short: the persistent tail takes every segment still live."""
    off = W.offsets_from_sizes(mixed_sizes(13, extra=120, max_log2=17))
    n = int(off[-1])
    keys = W.random_keys(kt, n, seed=6)
    vals = W.index_payload(n)
    out, vo, st = run_batched(keys, off, vals, batch_passes=passes)
    check_segmented(keys, off, out, vo)
    assert st["passes"] == passes
    assert st["batch_items"] > 0


@pytest.mark.parametrize("kt", ["u64", "f64", "i32"])
@pytest.mark.parametrize("passes", [0, 1])
def test_batched_deep_tail(kt, passes):
    """Segments far above the persistent kernel's LDS size with the passes cut
    to 0 or 1: the tail partitions each of them over several levels (a child
    it queued is partitioned again by another workgroup, possibly on another
    XCD), then sorts the leaves. Bit-exact against the oracle."""
    sizes = np.array([3_000_001, 1_500_000, 700_003, 64, 4097, 0, 250_000, 9000], dtype=np.int64)
    off = W.offsets_from_sizes(sizes)
    n = int(off[-1])
    keys = W.random_keys(kt, n, seed=21)
    vals = W.index_payload(n)
    out, vo, st = run_batched(keys, off, vals, batch_passes=passes)
    check_segmented(keys, off, out, vo)
    assert st["passes"] == passes
    # a 3M-key segment needs at least log2(3M / 16384) > 7 levels of halving
    assert st["batch_items"] >= 8


def test_batched_without_stats_then_check():
    """Without stats the batched call does not wait for its work; pdq_check
    on the same workspace reports its device-side state afterwards."""
    off = W.offsets_from_sizes(mixed_sizes(3, extra=50))
    n = int(off[-1])
    keys = W.random_keys("u32", n, seed=1)
    t, o = dev(keys), dev(off)
    opt_ws = pdq.workspace_bytes(n, off.size - 1, "u32", options=pdq._options(-1, 0, pdq.FLAG_BATCHED))
    ws = torch.empty(opt_ws, dtype=torch.uint8, device="cuda:0")
    pdq.segmented_sort_(t, o, batched=True, workspace=ws)
    pdq.check(ws)
    check_segmented(keys, off, host(t))


@pytest.mark.parametrize("shape", [1, 2, 3, 4])
def test_batched_every_shape(shape):
    off = W.offsets_from_sizes(mixed_sizes(11, extra=100))
    n = int(off[-1])
    keys = W.random_keys("f32", n, seed=2)
    vals = W.index_payload(n)
    out, vo, st = run_batched(keys, off, vals, batch_shape=shape)
    assert st["batch_shape"] == shape - 1
    check_segmented(keys, off, out, vo)


def test_batched_segmented_f32_workload():
    keys, off, vals = W.segmented_f32(3000, max_log2=16, seed=4)
    out, vo, st = run_batched(keys, off, vals)
    check_segmented(keys, off, out, vo)


@pytest.mark.parametrize("pattern", ["ascending", "descending", "equal", "organ_pipe", "two_values", "sawtooth"])
def test_batched_patterns_and_equal_keys(pattern):
    sizes = np.array([5000, 20000, 70000, 131072, 3000, 17000], dtype=np.int64)
    off = W.offsets_from_sizes(sizes)
    n = int(off[-1])
    parts = []
    rng = np.random.default_rng(1)
    for sz in sizes:
        if pattern == "ascending":
            parts.append(np.arange(sz, dtype=np.int32))
        elif pattern == "descending":
            parts.append(np.arange(sz, dtype=np.int32)[::-1].copy())
        elif pattern == "equal":
            parts.append(np.full(sz, 7, dtype=np.int32))
        elif pattern == "organ_pipe":
            i = np.arange(sz)
            parts.append(np.where(i < sz // 2, i, sz - 1 - i).astype(np.int32))
        elif pattern == "two_values":
            parts.append(rng.integers(0, 2, sz).astype(np.int32))
        else:
            parts.append((np.arange(sz) % 1000).astype(np.int32))
    keys = np.concatenate(parts)
    vals = W.index_payload(n)
    out, vo, st = run_batched(keys, off, vals)
    check_segmented(keys, off, out, vo)
    if pattern in ("ascending", "descending"):
        assert st["sorted_segments"] >= 3  # the queued segments were retired as ordered runs


def test_batched_forced_heapsort():
    sizes = np.array([17000, 5000, 20000, 300], dtype=np.int64)
    off = W.offsets_from_sizes(sizes)
    keys = W.uniform_u32(int(off[-1]), seed=3)
    vals = W.index_payload(keys.size)
    out, vo, st = run_batched(keys, off, vals, force_budget=0)
    assert st["heapsort_segments"] >= 2
    check_segmented(keys, off, out, vo)


def test_batched_validate_rejects_bad_offsets():
    a = W.uniform_u32(1000, seed=1)
    bad = np.array([0, 600, 400, 1000], dtype=np.uint64)
    with pytest.raises(pdq.PdqError) as ei:
        pdq.segmented_sort_(dev(a), dev(bad), batched=True, validate=True)
    assert ei.value.status == -1


def test_plan_graph_replays_with_refilled_inputs():
    """One captured plan (autotuned), replayed on three different inputs in
    the same buffers, with eager work and synchronisation between replays;
    every replay is checked against the oracle and against the eager
    batched call."""
    keys0, off, vals0 = W.segmented_f32(1500, max_log2=16, seed=9)
    n = keys0.size
    tk, to, tv = dev(keys0), dev(off), dev(vals0)
    plan = pdq.Plan(tk, to, tv, autotune=True)
    shape, ms = plan.info()
    assert 0 <= shape < 4 and ms[shape] > 0 and ms[shape] == min(m for m in ms if m > 0)
    # autotuning restored the caller's data
    assert np.array_equal(host(tk).view(np.uint32), keys0.view(np.uint32))
    assert np.array_equal(host(tv), vals0)
    for rep in range(3):
        keys = W.random_keys("f32", n, seed=100 + rep)  # new keys, same segments
        tk.copy_(dev(keys))
        tv.copy_(dev(vals0))
        plan.launch()
        out, vo = host(tk), host(tv)
        check_segmented(keys, off, out, vo)
        ek, ev = dev(keys), dev(vals0)
        pdq.segmented_sort_(ek, to, ev, batched=True, batch_shape=shape + 1)
        assert np.array_equal(host(ek).view(np.uint32), out.view(np.uint32))
        _ = torch.ones(1000, device="cuda:0").sum().item()  # eager work between replays
    plan.destroy()


def test_batched_full_workload_sampled():
    """The 65,536-segment float32 + payload workload in the benchmark's
    configuration: every segment sorted by canonical order, payloads a
    permutation that stays in its segment, keys a permutation (hash)."""
    from tests._util import multiset_hash
    keys, off, vals = W.segmented_f32(65536, max_log2=16, seed=0)
    tk, to, tv = dev(keys), dev(off), dev(vals)
    st = pdq.segmented_sort_(tk, to, tv, batched=True, stats=True)
    out, vo = host(tk), host(tv)
    del tk, tv
    torch.cuda.empty_cache()
    img = np.where(out.view(np.uint32) >> 31 == 1, ~out.view(np.uint32), out.view(np.uint32) | np.uint32(0x80000000))
    desc = img[1:] < img[:-1]
    starts = np.zeros(out.size, dtype=bool)
    starts[off[:-1][off[:-1] < out.size].astype(np.int64)] = True
    assert not np.any(desc & ~starts[1:])
    assert multiset_hash(out) == multiset_hash(keys)
    assert np.array_equal(np.sort(vo), np.arange(out.size, dtype=np.uint32))
    assert np.array_equal(out.view(np.uint32), keys[vo].view(np.uint32))
    assert st["passes"] > 0


def test_batched_deterministic_repeat_exactly():
    """PDQ_DETERMINISTIC with the batched form: the captured passes use the
    look-back partition, and the tail and LDS classes are deterministic
    anyway, so two runs agree on every payload."""
    off = W.offsets_from_sizes(mixed_sizes(21, extra=150, max_log2=17))
    n = int(off[-1])
    keys = (W.uniform_u32(n, seed=9) % np.uint32(50)).astype(np.uint32)
    vals = W.index_payload(n)
    o1, v1, s1 = run_batched(keys, off, vals, deterministic=True)
    o2, v2, s2 = run_batched(keys, off, vals, deterministic=True)
    check_segmented(keys, off, o1, v1)
    assert np.array_equal(v1, v2)
    assert s1["element_visits"] == s2["element_visits"]


# lanes per workgroup of each base-case size class under each of its three
# launcher variants (0 = the variant does not exist), for 32-bit slots and
# 64-bit keys alone, and for 64-bit keys with a payload
CLASS_SHAPES = {
    False: [(64, 0, 0), (64, 128, 256), (64, 128, 256), (128, 256, 64), (256, 512, 128), (512, 256, 1024),
            (1024, 512, 0)],
    True: [(64, 0, 0), (64, 128, 256), (128, 256, 0), (256, 512, 0), (512, 1024, 0), (1024, 0, 0), (0, 0, 0)],
}


@pytest.mark.parametrize("waves", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("kt,pairs", [("u32", True), ("f64", False), ("u64", True)])
def test_batched_waves_option(kt, pairs, waves):
    """pdq_options.waves forces every base-case class that has a shape of that
    many waves to take it; results match the oracle whatever the shapes."""
    off = W.offsets_from_sizes(mixed_sizes(40 + waves, extra=120, max_log2=15))
    n = int(off[-1])
    keys = W.random_keys(kt, n, seed=waves)
    vals = W.index_payload(n) if pairs else None
    out, vo, _ = run_batched(keys, off, vals, waves=waves)
    check_segmented(keys, off, out, vo)


@pytest.mark.parametrize("waves", [1, 4, 16])
@pytest.mark.parametrize("kt", ["u32", "i64"])
def test_sort_waves_option(kt, waves):
    """The single-array sort takes the same option for its base case."""
    n = 300007
    keys = W.random_keys(kt, n, seed=7 + waves)
    t = dev(keys)
    pdq.sort_(t, waves=waves)
    assert np.array_equal(as_bytes(host(t)), as_bytes(oracle.sort(keys)[0]))
    v = dev(W.index_payload(n))
    t = dev(keys)
    pdq.sort_pairs_(t, v, waves=waves)
    out, vo = host(t), host(v)
    assert np.array_equal(as_bytes(out), as_bytes(oracle.sort(keys)[0]))
    assert np.array_equal(as_bytes(keys[vo]), as_bytes(out))


def test_waves_option_rejects_other_values():
    t = dev(W.random_keys("u32", 1000, seed=1))
    o = dev(np.array([0, 1000], dtype=np.uint64))
    for w in (3, 5, 32):
        with pytest.raises(pdq.PdqError) as ei:
            pdq.segmented_sort_(t, o, batched=True, waves=w)
        assert ei.value.status == -2


@pytest.mark.parametrize("kt,pairs", [("f32", True), ("u64", True)])
def test_plan_autotune_per_class_and_cache_file(tmp_path, kt, pairs):
    """PDQ_AUTOTUNE times every shape of every base-case class and keeps the
    fastest of each; with a cache file it appends one line, and a second plan
    for the same problem takes that line without timing anything (no new
    line, no class timings). A later invalid line for the same problem is
    ignored. Every replay matches the oracle."""
    off = W.offsets_from_sizes(mixed_sizes(77, extra=400, max_log2=15))
    n = int(off[-1])
    keys = W.random_keys(kt, n, seed=3)
    vals = W.index_payload(n) if pairs else None
    wide = kt in ("u64", "i64", "f64") and pairs
    cache = tmp_path / "tune.txt"
    tk, to = dev(keys), dev(off)
    tv = dev(vals) if pairs else None
    plan = pdq.Plan(tk, to, tv, autotune=True, tune_cache_path=str(cache))
    threads, ms = plan.classes()
    for k in range(7):
        shapes = CLASS_SHAPES[wide][k]
        if not shapes[0]:
            continue
        assert threads[k] in shapes
        # every existing variant was timed, and the kept one is the fastest
        for v in range(3):
            assert (ms[k][v] > 0) == (shapes[v] > 0), (k, v, ms[k])
        assert ms[k][shapes.index(threads[k])] == min(m for m in ms[k] if m > 0)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("pdq-tune 1 ")
    fields = lines[0].split()
    assert len(fields) == 2 + 5 + 1 + 7  # tag, version, arch/CUs, type, payload, n, segments, shape, 7 variants
    assert int(fields[5]) == n and int(fields[6]) == off.size - 1
    # the caller's data is back in place after the timing runs
    assert np.array_equal(as_bytes(host(tk)), as_bytes(keys))
    plan.launch()
    check_segmented(keys, off, host(tk), host(tv) if pairs else None)
    plan.destroy()
    # an invalid line after the valid one: skipped by the reader
    with open(cache, "a") as f:
        f.write(" ".join(fields[:8]) + " 9 9 9 9 9 9 9\n")
    tk2 = dev(keys)
    tv2 = dev(vals) if pairs else None
    plan2 = pdq.Plan(tk2, to, tv2, autotune=True, tune_cache_path=str(cache))
    threads2, ms2 = plan2.classes()
    assert threads2 == threads
    assert all(m == 0 for row in ms2 for m in row)
    assert len(cache.read_text().splitlines()) == 2
    plan2.launch()
    check_segmented(keys, off, host(tk2), host(tv2) if pairs else None)
    plan2.destroy()
    # the eager batched call with the same cache: same keys as the plan
    tk3 = dev(keys)
    tv3 = dev(vals) if pairs else None
    pdq.segmented_sort_(tk3, to, tv3, batched=True, tune_cache_path=str(cache))
    check_segmented(keys, off, host(tk3), host(tv3) if pairs else None)
