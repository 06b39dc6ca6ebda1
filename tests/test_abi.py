"""The C ABI library loads, exports every entry point of include/pdq.h and
include/pdq_learned.h, and rejects bad arguments before touching the GPU (no
compute call here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdq.h")
HEADERS = [HEADER, os.path.join(ROOT, "include", "pdq_learned.h")]


def header_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(pdq_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def pdq():
    import paper_2106_05123_amd as p
    if not os.path.exists(p.LIB_PATH):
        from paper_2106_05123_amd import build as b
        b.build()
    return p


def test_exports_every_declared_function(pdq):
    names = header_functions()
    assert {"pdq_sort", "pdq_sort_pairs", "pdq_segmented_sort", "pdq_workspace_bytes", "pdq_mlp_train",
            "pdq_learned_fit", "pdq_bucket_histogram"} <= set(names)
    L = pdq.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", pdq.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (pdq_\w+)", out))
    assert set(names) <= exported


def test_abi_version_matches_header(pdq):
    m = re.search(r"#define PDQ_ABI_VERSION (\d+)", open(HEADER).read())
    assert pdq.abi_version() == int(m.group(1))


def test_status_strings(pdq):
    for code, name in ((0, "PDQ_OK"), (-1, "PDQ_ERR_INVALID"), (-2, "PDQ_ERR_UNSUPPORTED"),
                       (-3, "PDQ_ERR_WORKSPACE"), (-4, "PDQ_ERR_HIP"), (-5, "PDQ_ERR_SCRATCH"),
                       (-6, "PDQ_ERR_DEVICE")):
        assert pdq.status_string(code).startswith(name)
    assert "unknown" in pdq.status_string(12345)


def test_workspace_bytes(pdq):
    for kt, kb in (("u32", 4), ("i32", 4), ("f32", 4), ("u64", 8)):
        prev = 0
        for n in (0, 1, 4096, 4097, 1 << 20, 1 << 28):
            w = pdq.workspace_bytes(n, 1, kt)
            assert w >= n * kb and w >= prev
            assert pdq.workspace_bytes(n, 1, kt, has_vals=True) >= w + 4 * n
            prev = w
    assert pdq.workspace_bytes(1 << 20, 1 << 16, "u32") >= pdq.workspace_bytes(1 << 20, 1, "u32")
    assert pdq.lib().pdq_workspace_bytes(10, 1, 9, 0, None) == 0


def _call_sort(pdq, keys, n, kt=1, order=0, ws=0x100000, ws_bytes=1 << 40, opt=None):
    L = pdq.lib()
    return L.pdq_sort(ctypes.c_void_p(keys), n, kt, order, ctypes.c_void_p(ws), ws_bytes, None,
                      ctypes.byref(opt) if opt else None, None)


def test_argument_errors_without_gpu(pdq):
    L = pdq.lib()
    Opt = pdq.Options
    assert _call_sort(pdq, 0x1000, 10, order=1) == -2
    assert _call_sort(pdq, 0x1000, 10, kt=0) == -2
    assert _call_sort(pdq, 0x1000, 10, kt=7) == -2  # 1 ... 6 are the key types
    assert _call_sort(pdq, 0, 10) == -1                      # null keys
    assert _call_sort(pdq, 0x1002, 10) == -1                 # misaligned u32 keys
    assert _call_sort(pdq, 0x1004, 10, kt=4) == -1           # misaligned u64 keys
    assert _call_sort(pdq, 0x1000, 1 << 32) == -2            # n >= 2^32
    assert _call_sort(pdq, 0x1000, 10, ws=0) == -3           # no workspace
    assert _call_sort(pdq, 0x1000, 1 << 20, ws_bytes=100) == -3
    assert _call_sort(pdq, 0, 0) == 0                        # n <= 1 is a no-op
    assert _call_sort(pdq, 0, 1) == 0
    assert _call_sort(pdq, 0x1000, 10, opt=Opt(ctypes.sizeof(Opt), 0x400, -1, 0, 0)) == -2  # unknown flag
    assert _call_sort(pdq, 0x1000, 10, opt=Opt(ctypes.sizeof(Opt), 0, -1, 3000, 0)) == -2  # bad tile
    # pairs without payload, segmented without offsets
    assert L.pdq_sort_pairs(ctypes.c_void_p(0x1000), None, 10, 1, 0, ctypes.c_void_p(0x10000), 1 << 40, None,
                            None, None) == -1
    assert L.pdq_segmented_sort(ctypes.c_void_p(0x1000), None, 10, None, 3, 1, 0, ctypes.c_void_p(0x10000),
                                1 << 40, None, None, None) == -1
    assert L.pdq_segmented_sort(ctypes.c_void_p(0x1000), None, 10, ctypes.c_void_p(0x1004), 3, 1, 0,
                                ctypes.c_void_p(0x10000), 1 << 40, None, None, None) == -1  # misaligned offsets


def test_noalloc_limits_without_gpu(pdq):
    """pdq_sort_noalloc rejects what does not fit its scratch array, and the
    options it does not serve, before anything touches the GPU."""
    L = pdq.lib()
    Opt = pdq.Options
    m = re.search(r"#define PDQ_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", open(HEADER).read())
    limit = int(m.group(1)) << int(m.group(2))
    assert limit == pdq.NOALLOC_SCRATCH_BYTES
    k = ctypes.c_void_p(0x1000)
    v = ctypes.c_void_p(0x2000)
    for kt, has_v in ((1, False), (1, True), (4, False), (4, True)):
        # the largest n whose workspace fits, and the next one
        lo, hi = 2, 1 << 30
        while lo < hi:
            mid = (lo + hi + 1) // 2
            # the entry point runs the host-driven pass loop: its workspace
            host_loop = pdq._options(-1, 0, pdq.FLAG_HOST_LOOP)
            if pdq.workspace_bytes(mid, 1, kt, has_v, host_loop) <= limit:
                lo = mid
            else:
                hi = mid - 1
        assert L.pdq_sort_noalloc(k, v if has_v else None, lo + 1, kt, 0, None, None, None) == -5
    assert L.pdq_sort_noalloc(k, None, 1 << 31, 1, 0, None, None, None) == -5
    assert L.pdq_sort_noalloc(k, None, 1 << 32, 1, 0, None, None, None) == -2
    assert L.pdq_sort_noalloc(None, None, 10, 1, 0, None, None, None) == -1
    assert L.pdq_sort_noalloc(k, None, 10, 1, 1, None, None, None) == -2   # order
    assert L.pdq_sort_noalloc(k, None, 10, 9, 0, None, None, None) == -2   # key type
    assert L.pdq_sort_noalloc(None, None, 1, 1, 0, None, None, None) == 0  # n <= 1 is a no-op
    for flag in (pdq.FLAG_PROFILE, pdq.FLAG_BATCHED, pdq.FLAG_AUTOTUNE):
        o = Opt(ctypes.sizeof(Opt), flag, -1, 0, 0)
        assert L.pdq_sort_noalloc(k, None, 10, 1, 0, None, ctypes.byref(o), None) == -2


def test_vals64_workspace_and_alignment_without_gpu(pdq):
    """PDQ_VALS64: 12 more workspace bytes per key (the 32-bit index payload
    the sort moves and a copy of the 64-bit payloads), and 8-byte alignment
    of the payload pointer."""
    Opt = pdq.Options
    o64 = Opt(ctypes.sizeof(Opt), pdq.FLAG_VALS64, -1, 0, 0)
    for kt in ("u32", "u64"):
        for n in (1000, 1 << 20):
            base = pdq.workspace_bytes(n, 1, kt, has_vals=True)
            assert pdq.workspace_bytes(n, 1, kt, has_vals=True, options=o64) >= base + 12 * n
            assert pdq.workspace_bytes(n, 1, kt, has_vals=False, options=o64) == pdq.workspace_bytes(n, 1, kt)
    L = pdq.lib()
    rc = L.pdq_sort_pairs(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2004), 10, 1, 0, ctypes.c_void_p(0x100000),
                          1 << 40, None, ctypes.byref(o64), None)
    assert rc == -1
    rc = L.pdq_sort_pairs(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 1 << 20, 1, 0, ctypes.c_void_p(0x100000),
                          pdq.workspace_bytes(1 << 20, 1, "u32", has_vals=True), None, ctypes.byref(o64), None)
    assert rc == -3  # the workspace of 32-bit payloads is too small for 64-bit ones


def test_check_argument_error_without_gpu(pdq):
    assert pdq.lib().pdq_check(None, None) == -1


def test_binding_has_no_fallback(pdq, monkeypatch):
    """The Python layer never sorts by itself: without the library it raises."""
    monkeypatch.setattr(pdq, "_lib", None)
    monkeypatch.setattr(pdq, "LIB_PATH", "/nonexistent/libpdq.so")
    with pytest.raises(RuntimeError):
        pdq.lib()


def test_learned_workspace_and_option_errors(pdq):
    Opt = pdq.Options
    plain = pdq.workspace_bytes(1 << 20, 1, "u32")
    lo = Opt(ctypes.sizeof(Opt), pdq.FLAG_LEARNED, -1, 0, 0, 0.0, 0, 0, 0)
    learned = pdq.workspace_bytes(1 << 20, 1, "u32", options=lo)
    # sample (8 B) + features, targets, predictions, running max (4 x 4 B) per sample key,
    # plus one histogram row of 512 counts per 8192-key tile
    assert learned >= plain + pdq.LEARN_SAMPLE * 24 + ((1 << 20) // 8192) * 512 * 4
    assert pdq.workspace_bytes(pdq.LEARN_SAMPLE, 1, "u32", options=lo) == pdq.workspace_bytes(pdq.LEARN_SAMPLE, 1, "u32")
    bad = Opt(ctypes.sizeof(Opt), pdq.FLAG_LEARNED, -1, 0, 0, 0.0, 0, 1000, 16)   # batch % grid != 0
    assert _call_sort(pdq, 0x1000, 1 << 20, opt=bad) == -2
    bad2 = Opt(ctypes.sizeof(Opt), pdq.FLAG_LEARNED, -1, 0, 0, 0.0, 0, 1024, 65)  # grid > 64
    assert _call_sort(pdq, 0x1000, 1 << 20, opt=bad2) == -2
    older = Opt(24, pdq.FLAG_LEARNED, -1, 0, 0, 0.0, 0, 1000, 16)  # fields past struct_size are ignored
    assert pdq.workspace_bytes(1 << 20, 1, "u32", options=older) == learned


def test_learned_entry_point_errors_without_gpu(pdq):
    L = pdq.lib()
    vp = ctypes.c_void_p
    # trainer: grid 0, batch not a multiple of grid, zero steps, null pointers, small workspace
    args = lambda grid, batch, steps, x=0x1000, ws_bytes=1 << 30: (
        vp(x), vp(0x2000), 65536, 0, steps, batch, grid, 1, None, vp(0x3000), vp(0x4000), vp(0x100000), ws_bytes, None)
    assert L.pdq_mlp_train(*args(0, 1024, 256)) == -2
    assert L.pdq_mlp_train(*args(16, 1000, 256)) == -2
    assert L.pdq_mlp_train(*args(16, 1024, 0)) == -2
    assert L.pdq_mlp_train(*args(16, 1024, 256, x=0)) == -1
    assert L.pdq_mlp_train(*args(16, 1024, 256, ws_bytes=16)) == -3
    assert L.pdq_mlp_train_workspace_bytes(16) >= 2 * 16 * 1153 * 4
    assert L.pdq_mlp_gradient(vp(0x1000), vp(0x2000), vp(0x3000), 0, 1, vp(0x4000), vp(0x5000), None) == -2
    assert L.pdq_mlp_gradient(None, vp(0x2000), vp(0x3000), 10, 1, vp(0x4000), vp(0x5000), None) == -1
    assert L.pdq_mlp_infer(vp(0x1000), vp(0x2000), 0, 1, vp(0x3000), None) == 0
    assert L.pdq_mlp_infer(None, vp(0x2000), 10, 1, vp(0x3000), None) == -1
    assert L.pdq_learned_features(None, 10, vp(0x2000), vp(0x3000), vp(0x4000), None) == -1
    assert L.pdq_learned_extract(vp(0x1000), vp(0x2000), 0, vp(0x3000), vp(0x4000), vp(0x5000), None) == -2
    n = 1 << 20
    need = L.pdq_bucket_workspace_bytes(n)
    assert need >= (n // 8192) * 512 * 4
    assert L.pdq_bucket_histogram(vp(0x1000), n, 9, vp(0x2000), vp(0x3000), vp(0x4000), vp(0x5000), need, None) == -2
    assert L.pdq_bucket_histogram(vp(0x1000), 0, 1, vp(0x2000), vp(0x3000), vp(0x4000), vp(0x5000), need, None) == -2
    assert L.pdq_bucket_histogram(vp(0x1000), n, 1, None, vp(0x3000), vp(0x4000), vp(0x5000), need, None) == -1
    assert L.pdq_bucket_histogram(vp(0x1000), n, 1, vp(0x2000), vp(0x3000), vp(0x4000), vp(0x5000), 100, None) == -3
    fb = pdq.FitBuffers()
    assert L.pdq_learned_fit(vp(0x1000), n, 1, vp(0x100000), 1 << 30, None, None, ctypes.byref(fb)) == -1
    assert L.pdq_learned_fit_workspace_bytes(None) > 0


def test_struct_layouts_match_header(pdq, tmp_path):
    """The ctypes mirrors of pdq_options / pdq_stats have the header's size and
    field offsets (compiled with the host C compiler)."""
    import ctypes
    fields_o = [f for f, _ in pdq.Options._fields_]
    fields_s = [f for f, _ in pdq.Stats._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pdq.h"', 'int main(void) {',
             'printf("%zu %zu\\n", sizeof(pdq_options), sizeof(pdq_stats));']
    lines += [f'printf("%zu\\n", offsetof(pdq_options, {f}));' for f in fields_o]
    lines += [f'printf("%zu\\n", offsetof(pdq_stats, {f}));' for f in fields_s]
    lines += ["return 0; }"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(pdq.Options) and vals[1] == ctypes.sizeof(pdq.Stats)
    offs = vals[2:]
    assert offs[:len(fields_o)] == [getattr(pdq.Options, f).offset for f in fields_o]
    assert offs[len(fields_o):] == [getattr(pdq.Stats, f).offset for f in fields_s]
