"""CPU oracle for the partition sort: a plain single-threaded pdqsort written
from the paper (see ``pdq_oracle.cpp``) plus the numpy model of the learned
splitter pass (``mlp_oracle``).

TEST INFRASTRUCTURE ONLY: the product path never imports this package. Only
the tests, the smoke check and the benchmark's CPU-baseline leg use it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdq_oracle.cpp")
_LIB = os.path.join(_HERE, "libpdq_oracle.so")

KEY_TYPES = {"u32": 1, "i32": 2, "f32": 3, "u64": 4, "i64": 5, "f64": 6}
_DTYPES = {"u32": np.uint32, "i32": np.int32, "f32": np.float32, "u64": np.uint64, "i64": np.int64,
           "f64": np.float64}


class Counters(ctypes.Structure):
    _fields_ = [
        ("comparisons", ctypes.c_uint64),
        ("partitions_right", ctypes.c_uint64),
        ("partitions_left", ctypes.c_uint64),
        ("bad_partitions", ctypes.c_uint64),
        ("heapsort_calls", ctypes.c_uint64),
        ("heapsort_elements", ctypes.c_uint64),
        ("insertion_sorts", ctypes.c_uint64),
        ("partial_insertion_ok", ctypes.c_uint64),
        ("partial_insertion_abort", ctypes.c_uint64),
        ("already_partitioned", ctypes.c_uint64),
        ("max_depth", ctypes.c_uint64),
        ("max_bad_on_path", ctypes.c_uint64),
        ("pivot_log_cap", ctypes.c_uint64),
        ("pivot_log_len", ctypes.c_uint64),
        ("pivot_log_key", ctypes.POINTER(ctypes.c_uint64)),
        ("pivot_log_mode", ctypes.POINTER(ctypes.c_uint8)),
        ("first_pivot_image", ctypes.c_uint64),
        ("first_left_size", ctypes.c_int64),
        ("first_mode", ctypes.c_int32),
        ("first_no_swaps", ctypes.c_int32),
        ("first_recorded", ctypes.c_int32),
        ("first_bad", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_
                if f not in ("pivot_log_key", "pivot_log_mode")}


class Options(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("force_budget", ctypes.c_int32)]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, as in the paper's setup; generic
    x86-64 so that the library runs on any host it is copied to)."""
    stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_sort.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                  ctypes.POINTER(Options), ctypes.POINTER(Counters)]
        L.oracle_sort.restype = ctypes.c_int
        L.oracle_segmented_sort.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                            ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Options),
                                            ctypes.POINTER(Counters)]
        L.oracle_segmented_sort.restype = ctypes.c_int
        L.oracle_routine.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                     ctypes.POINTER(Counters), ctypes.POINTER(ctypes.c_int64)]
        L.oracle_routine.restype = ctypes.c_int
        L.oracle_key_image.argtypes = [ctypes.c_int, ctypes.c_void_p]
        L.oracle_key_image.restype = ctypes.c_uint64
        fp = ctypes.POINTER(ctypes.c_float)
        L.oracle_mlp_infer_f32.argtypes = [fp, fp, ctypes.c_size_t, ctypes.c_int, fp]
        L.oracle_mlp_infer_f32.restype = None
        _lib = L
    return _lib


def key_type_of(a: np.ndarray) -> str:
    for k, d in _DTYPES.items():
        if a.dtype == d:
            return k
    raise TypeError(f"unsupported key dtype {a.dtype}")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def sort(keys: np.ndarray, vals: np.ndarray | None = None, *, block: bool = True,
         force_budget: int = -1, count: bool = False, pivot_log: int = 0):
    """Sort copies of `keys` (and `vals`) with the oracle. Returns
    (keys_sorted, vals_sorted_or_None, counters_dict_or_None, pivot_log)."""
    k = np.ascontiguousarray(keys).copy()
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    kt = KEY_TYPES[key_type_of(k)]
    opt = Options(1 if block else 0, force_budget)
    c = None
    log_k = log_m = None
    if count or pivot_log:
        c = Counters()
        if pivot_log:
            log_k = np.zeros(pivot_log, dtype=np.uint64)
            log_m = np.zeros(pivot_log, dtype=np.uint8)
            c.pivot_log_cap = pivot_log
            c.pivot_log_key = log_k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
            c.pivot_log_mode = log_m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    rc = lib().oracle_sort(kt, _ptr(k), _ptr(v), k.size, ctypes.byref(opt),
                           ctypes.byref(c) if c is not None else None)
    if rc != 0:
        raise RuntimeError(f"oracle_sort failed: {rc}")
    plog = None
    if pivot_log:
        m = min(c.pivot_log_len, pivot_log)
        plog = (log_k[:m].copy(), log_m[:m].copy())
    return k, v, (c.as_dict() if c is not None else None), plog


def segmented_sort(keys: np.ndarray, offsets: np.ndarray, vals: np.ndarray | None = None, *,
                   block: bool = True, force_budget: int = -1, count: bool = False):
    k = np.ascontiguousarray(keys).copy()
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    kt = KEY_TYPES[key_type_of(k)]
    opt = Options(1 if block else 0, force_budget)
    c = Counters() if count else None
    rc = lib().oracle_segmented_sort(kt, _ptr(k), _ptr(v), k.size, _ptr(off), off.size - 1,
                                     ctypes.byref(opt), ctypes.byref(c) if c is not None else None)
    if rc != 0:
        raise RuntimeError(f"oracle_segmented_sort failed: {rc}")
    return k, v, (c.as_dict() if c is not None else None)


def routine(which: str, keys: np.ndarray, arg: int = 0, block: bool = True):
    """Run one routine on a copy: 'insertion', 'heapsort', 'partial_insertion'
    (returns success flag), 'partition_right' / 'partition_left' (pivot
    choice + one partition; returns (pivot_pos, no_swaps)). Returns
    (array, result, counters)."""
    k = np.ascontiguousarray(keys).copy()
    kt = KEY_TYPES[key_type_of(k)]
    code = {"insertion": 0, "heapsort": 1, "partial_insertion": 2,
            "partition_right": 3, "partition_left": 3}[which]
    if which == "partition_left":
        arg = 1
    if code == 3 and not block:
        arg |= 2
    out = (ctypes.c_int64 * 2)()
    c = Counters()
    rc = lib().oracle_routine(kt, code, _ptr(k), k.size, arg, ctypes.byref(c), out)
    if rc != 0:
        raise RuntimeError(f"oracle_routine failed: {rc}")
    res = None
    if code == 2:
        res = bool(out[0])
    elif code == 3:
        res = (int(out[0]), bool(out[1]))
    return k, res, c.as_dict()


def key_image(key_type: str, value) -> int:
    a = np.array([value], dtype=_DTYPES[key_type])
    return int(lib().oracle_key_image(KEY_TYPES[key_type], _ptr(a)))
