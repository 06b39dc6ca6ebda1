"""pdq_sort_noalloc (the entry point that allocates nothing) against
pdq_sort / pdq_sort_pairs, through the C ABI: two calls in a row on one GPU,
the second smaller, so the second runs over the scratch array the first left
behind. Keys must be bit-exact; payloads a permutation that travels with its
keys (the sort is unstable, Section 1)."""
import ctypes

import numpy as np
import pytest

import gen.workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2106_05123_amd as pdq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, pdq


def _noalloc(torch, pdq, keys_t, vals_t, kt):
    L = pdq.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.pdq_sort_noalloc(ctypes.c_void_p(keys_t.data_ptr()),
                            ctypes.c_void_p(vals_t.data_ptr()) if vals_t is not None else None,
                            keys_t.numel(), kt, 0, stream, None, None)
    assert rc == 0, pdq.status_string(rc)


def _with_workspace(torch, pdq, keys_t, vals_t, kt):
    L = pdq.lib()
    n = keys_t.numel()
    need = pdq.workspace_bytes(n, 1, kt, vals_t is not None)
    ws = torch.empty(need, dtype=torch.uint8, device=keys_t.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if vals_t is None:
        rc = L.pdq_sort(ctypes.c_void_p(keys_t.data_ptr()), n, kt, 0, ctypes.c_void_p(ws.data_ptr()), need,
                        stream, None, None)
    else:
        rc = L.pdq_sort_pairs(ctypes.c_void_p(keys_t.data_ptr()), ctypes.c_void_p(vals_t.data_ptr()), n, kt, 0,
                              ctypes.c_void_p(ws.data_ptr()), need, stream, None, None)
    assert rc == 0, pdq.status_string(rc)


def _inputs(kind, n, seed):
    if kind == "i32":
        return W.pattern_i32("sawtooth", n, seed=seed), 2
    return W.random_keys(kind, n, seed=seed), {"u32": 1, "f32": 3, "u64": 4, "f64": 6}[kind]


@pytest.mark.parametrize("kind,pairs", [("u32", True), ("u32", False), ("i32", True), ("f32", False),
                                        ("u64", True), ("f64", False)])
def test_noalloc_matches_workspace_entry_point(env, kind, pairs):
    torch, pdq = env
    dev = torch.device("cuda:0")
    # the first call near the scratch array's limit for uint32 pairs, the second smaller
    sizes = {"u32": (5_000_000 + 77, 300_001), "i32": (3_000_000 + 5, 65_536 + 3), "f32": (2_000_003, 4099),
             "u64": (2_500_001, 100_003), "f64": (1_500_007, 70_001)}[kind]
    for i, n in enumerate(sizes):
        print(f"noalloc case kind={kind} pairs={pairs} n={n}", flush=True)
        keys, kt = _inputs(kind, n, seed=11 + i)
        vals = W.index_payload(n)
        a_k = torch.from_numpy(keys).to(dev)
        b_k = a_k.clone()
        a_v = torch.from_numpy(vals).to(dev) if pairs else None
        b_v = a_v.clone() if pairs else None
        _noalloc(torch, pdq, a_k, a_v, kt)
        _with_workspace(torch, pdq, b_k, b_v, kt)
        torch.cuda.synchronize()
        out_a = a_k.cpu().numpy()
        out_b = b_k.cpu().numpy()
        assert np.array_equal(out_a.view(np.uint8), out_b.view(np.uint8)), f"keys differ (n={n})"
        if pairs:
            va = a_v.cpu().numpy()
            assert np.array_equal(np.sort(va), vals), "payloads are not a permutation"
            assert np.array_equal(keys[va].view(np.uint8), out_a.view(np.uint8)), "payloads left their keys"
