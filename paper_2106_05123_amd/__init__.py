"""MI355X (gfx950) partition sort: the partition step of pattern-defeating
quicksort (Peters, arXiv 2106.05123) as HIP kernels behind a C ABI.

This module only marshals arguments: every step of the sort runs in the HIP
library ``libpdq.so`` (C ABI declared in ``include/pdq.h``). PyTorch supplies
device memory and the stream. There is no fallback: if the library is not
built, every call raises.

    import torch, paper_2106_05123_amd as pdq
    x = torch.randint(-2**31, 2**31 - 1, (1 << 20,), dtype=torch.int32, device="cuda")
    pdq.sort_(x)                      # in place, ascending
    pdq.sort_pairs_(keys, vals)       # vals: uint32 payload moved with keys (unstable)
    pdq.segmented_sort_(keys, offsets, vals=None)
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "PdqError", "Options", "Stats", "lib", "workspace_bytes", "sort_", "sort_pairs_",
    "segmented_sort_", "status_string", "abi_version", "KEY_TYPES", "FLAG_VALIDATE", "FLAG_PROFILE",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdq.so")

PDQ_OK = 0
FLAG_VALIDATE = 1
FLAG_PROFILE = 2
KEY_TYPES = {"u32": 1, "i32": 2, "f32": 3, "u64": 4}


class Options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("force_budget", ctypes.c_int32),
        ("tile", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("passes", ctypes.c_uint32),
        ("element_visits", ctypes.c_uint64),
        ("partitions_right", ctypes.c_uint64),
        ("partitions_left", ctypes.c_uint64),
        ("bad_partitions", ctypes.c_uint64),
        ("heapsort_segments", ctypes.c_uint64),
        ("heapsort_elements", ctypes.c_uint64),
        ("base_segments", ctypes.c_uint64),
        ("base_elements", ctypes.c_uint64),
        ("sorted_segments", ctypes.c_uint64),
        ("sorted_elements", ctypes.c_uint64),
        ("equal_elements", ctypes.c_uint64),
        ("first_pivot_image", ctypes.c_uint64),
        ("first_left_size", ctypes.c_int64),
        ("first_mode", ctypes.c_int32),
        ("partition_launches", ctypes.c_uint32),
        ("partition_ms", ctypes.c_double),
        ("partition_bytes", ctypes.c_uint64),
        ("first_pass_ms", ctypes.c_double),
        ("first_pass_bytes", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "struct_size"}


class PdqError(RuntimeError):
    def __init__(self, status: int, text: str, hip_error: int = 0):
        super().__init__(f"{text} (status {status}, hip error {hip_error})")
        self.status = status
        self.hip_error = hip_error


_lib = None


def lib():
    """Load libpdq.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, u32p = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p
        L.pdq_workspace_bytes.argtypes = [sz, sz, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Options)]
        L.pdq_workspace_bytes.restype = sz
        L.pdq_sort.argtypes = [vp, sz, ctypes.c_int, ctypes.c_int, vp, sz, vp, ctypes.POINTER(Options),
                               ctypes.POINTER(Stats)]
        L.pdq_sort.restype = ctypes.c_int
        L.pdq_sort_pairs.argtypes = [vp, u32p, sz, ctypes.c_int, ctypes.c_int, vp, sz, vp,
                                     ctypes.POINTER(Options), ctypes.POINTER(Stats)]
        L.pdq_sort_pairs.restype = ctypes.c_int
        L.pdq_segmented_sort.argtypes = [vp, u32p, sz, vp, sz, ctypes.c_int, ctypes.c_int, vp, sz, vp,
                                         ctypes.POINTER(Options), ctypes.POINTER(Stats)]
        L.pdq_segmented_sort.restype = ctypes.c_int
        L.pdq_status_string.argtypes = [ctypes.c_int]
        L.pdq_status_string.restype = ctypes.c_char_p
        L.pdq_last_hip_error.argtypes = []
        L.pdq_last_hip_error.restype = ctypes.c_int
        L.pdq_abi_version.argtypes = []
        L.pdq_abi_version.restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().pdq_status_string(status).decode()


def abi_version() -> int:
    return lib().pdq_abi_version()


def _check(status: int):
    if status != PDQ_OK:
        raise PdqError(status, status_string(status), lib().pdq_last_hip_error())


def _key_type(t) -> int:
    import torch
    m = {torch.uint32: 1, torch.int32: 2, torch.float32: 3, torch.uint64: 4}
    if t.dtype not in m:
        raise TypeError(f"unsupported key dtype {t.dtype}; use uint32, int32, float32 or uint64")
    return m[t.dtype]


def _options(force_budget: int, tile: int, flags: int) -> Options:
    return Options(ctypes.sizeof(Options), flags, force_budget, tile, 0)


def workspace_bytes(n: int, nseg: int = 1, key_type: int | str = "u32", has_vals: bool = False,
                    options: Options | None = None) -> int:
    kt = KEY_TYPES[key_type] if isinstance(key_type, str) else int(key_type)
    return int(lib().pdq_workspace_bytes(n, max(1, nseg), kt, 1 if has_vals else 0,
                                         ctypes.byref(options) if options else None))


def _prepare(keys, vals, nseg, force_budget, tile, flags, workspace):
    import torch
    if not keys.is_cuda:
        raise ValueError("keys must be a device tensor")
    if not keys.is_contiguous():
        raise ValueError("keys must be contiguous")
    if vals is not None:
        if vals.dtype != torch.uint32 or not vals.is_cuda or not vals.is_contiguous():
            raise ValueError("vals must be a contiguous uint32 device tensor")
        if vals.numel() != keys.numel():
            raise ValueError("vals must have as many elements as keys")
    kt = _key_type(keys)
    opt = _options(force_budget, tile, flags)
    need = workspace_bytes(keys.numel(), nseg, kt, vals is not None, opt)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
    stream = torch.cuda.current_stream(keys.device).cuda_stream
    return kt, opt, workspace, need, ctypes.c_void_p(stream)


def _finish(st, want):
    return st.as_dict() if want else None


def sort_(keys, *, force_budget: int = -1, tile: int = 0, profile: bool = False, stats: bool = False,
          workspace=None):
    """Sort a 1-D device tensor in place (ascending canonical order)."""
    kt, opt, ws, need, stream = _prepare(keys, None, 1, force_budget, tile, FLAG_PROFILE if profile else 0,
                                         workspace)
    st = Stats(ctypes.sizeof(Stats)) if (stats or profile) else None
    rc = lib().pdq_sort(ctypes.c_void_p(keys.data_ptr()), keys.numel(), kt, 0, ctypes.c_void_p(ws.data_ptr()),
                        need, stream, ctypes.byref(opt), ctypes.byref(st) if st is not None else None)
    _check(rc)
    return _finish(st, st is not None)


def sort_pairs_(keys, vals, *, force_budget: int = -1, tile: int = 0, profile: bool = False,
                stats: bool = False, workspace=None):
    """Sort keys in place and move the uint32 payload `vals` with them."""
    kt, opt, ws, need, stream = _prepare(keys, vals, 1, force_budget, tile, FLAG_PROFILE if profile else 0,
                                         workspace)
    st = Stats(ctypes.sizeof(Stats)) if (stats or profile) else None
    rc = lib().pdq_sort_pairs(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()), keys.numel(),
                              kt, 0, ctypes.c_void_p(ws.data_ptr()), need, stream, ctypes.byref(opt),
                              ctypes.byref(st) if st is not None else None)
    _check(rc)
    return _finish(st, st is not None)


def segmented_sort_(keys, offsets, vals=None, *, force_budget: int = -1, tile: int = 0,
                    validate: bool = False, profile: bool = False, stats: bool = False, workspace=None):
    """Sort each segment [offsets[s], offsets[s+1]) of keys in place.
    offsets: uint64 device tensor of nseg+1 entries."""
    import torch
    if offsets.dtype != torch.uint64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous uint64 device tensor")
    nseg = offsets.numel() - 1
    flags = (FLAG_VALIDATE if validate else 0) | (FLAG_PROFILE if profile else 0)
    kt, opt, ws, need, stream = _prepare(keys, vals, nseg, force_budget, tile, flags, workspace)
    st = Stats(ctypes.sizeof(Stats)) if (stats or profile) else None
    rc = lib().pdq_segmented_sort(ctypes.c_void_p(keys.data_ptr()),
                                  ctypes.c_void_p(vals.data_ptr()) if vals is not None else None,
                                  keys.numel(), ctypes.c_void_p(offsets.data_ptr()), max(nseg, 0), kt, 0,
                                  ctypes.c_void_p(ws.data_ptr()), need, stream, ctypes.byref(opt),
                                  ctypes.byref(st) if st is not None else None)
    _check(rc)
    return _finish(st, st is not None)
