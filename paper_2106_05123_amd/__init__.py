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
    pdq.sort_(x, learned=True)        # learned multiway first pass (include/pdq_learned.h)

The learned pass's building blocks (MLP inference, gradient, fused trainer,
features, splitter extraction, bin histogram, the whole fit) are bound
one by one below with the names of their C entry points.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "PdqError", "Options", "Stats", "lib", "workspace_bytes", "sort_", "sort_pairs_",
    "segmented_sort_", "status_string", "abi_version", "KEY_TYPES", "FLAG_VALIDATE", "FLAG_PROFILE",
    "FLAG_LEARNED", "MLP_PARAMS", "LEARN_SAMPLE", "mlp_infer", "mlp_gradient", "mlp_train",
    "learned_features", "learned_extract", "bucket_histogram", "learned_fit", "learned_leaves", "sample_judge", "FLAG_BATCHED", "FLAG_AUTOTUNE", "FLAG_DETERMINISTIC",
    "Plan", "sort_noalloc_", "NOALLOC_SCRATCH_BYTES", "check", "FLAG_FRESH_FIXED", "FLAG_VALS64", "FLAG_HOST_LOOP", "FLAG_HEAPSORT",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdq.so")

PDQ_OK = 0
PDQ_ERR_SCRATCH = -5
PDQ_ERR_DEVICE = -6
NOALLOC_SCRATCH_BYTES = 64 << 20  # PDQ_NOALLOC_SCRATCH_BYTES
FLAG_VALIDATE = 1
FLAG_PROFILE = 2
FLAG_LEARNED = 4
FLAG_BATCHED = 8
FLAG_AUTOTUNE = 16
FLAG_DETERMINISTIC = 32
FLAG_FRESH_FIXED = 64
FLAG_VALS64 = 128
FLAG_HOST_LOOP = 256
FLAG_HEAPSORT = 512
# batched shapes: (partition tile, slots per lane of the 8192 / 16384-key LDS classes)
BATCH_SHAPES = ((8192, 16), (16384, 16), (32768, 16), (8192, 32))
MLP_PARAMS = 1153
MAX_SPLITTERS = 255
LEARN_SAMPLE = 65536
KEY_TYPES = {"u32": 1, "i32": 2, "f32": 3, "u64": 4, "i64": 5, "f64": 6}


class Options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("force_budget", ctypes.c_int32),
        ("tile", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("learned_imbalance_limit", ctypes.c_float),
        ("learn_steps", ctypes.c_uint32),
        ("learn_batch", ctypes.c_uint32),
        ("learn_grid", ctypes.c_uint32),
        ("batch_shape", ctypes.c_uint32),
        ("batch_passes", ctypes.c_uint32),
        ("waves", ctypes.c_uint32),
        ("reserved_", ctypes.c_uint32),
        ("tune_cache_path", ctypes.c_char_p),
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
        ("learned", ctypes.c_uint32),
        ("learned_splitters", ctypes.c_uint32),
        ("learned_max_range_bin", ctypes.c_uint64),
        ("learned_equal_elements", ctypes.c_uint64),
        ("learned_final_loss", ctypes.c_float),
        ("learned_use_log", ctypes.c_uint32),
        ("learned_fit_ms", ctypes.c_double),
        ("learned_hist_ms", ctypes.c_double),
        ("learned_scatter_ms", ctypes.c_double),
        ("learned_hist_bytes", ctypes.c_uint64),
        ("learned_scatter_bytes", ctypes.c_uint64),
        ("batch_items", ctypes.c_uint32),
        ("batch_shape", ctypes.c_uint32),
        ("batch_ms", ctypes.c_double),
        ("near_sorted", ctypes.c_uint32),
        ("pad_", ctypes.c_uint32),
        ("near_sorted_runs", ctypes.c_uint64),
        ("near_sorted_outliers", ctypes.c_uint64),
        ("learned_choice", ctypes.c_uint32),
        ("learned_steps", ctypes.c_uint32),
        ("learned_sample_judge", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f not in ("struct_size", "pad_")}


class FitBuffers(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("d_sample", "d_x", "d_t", "d_pred", "d_params", "d_losses", "d_splitters", "d_count", "d_info")]


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
        L.pdq_sort_noalloc.argtypes = [vp, u32p, sz, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(Options),
                                       ctypes.POINTER(Stats)]
        L.pdq_sort_noalloc.restype = ctypes.c_int
        L.pdq_check.argtypes = [vp, vp]
        L.pdq_check.restype = ctypes.c_int
        L.pdq_status_string.argtypes = [ctypes.c_int]
        L.pdq_status_string.restype = ctypes.c_char_p
        L.pdq_last_hip_error.argtypes = []
        L.pdq_last_hip_error.restype = ctypes.c_int
        L.pdq_abi_version.argtypes = []
        L.pdq_abi_version.restype = ctypes.c_int
        i, u32, u64 = ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64
        L.pdq_mlp_infer.argtypes = [vp, vp, sz, i, vp, vp]
        L.pdq_mlp_gradient.argtypes = [vp, vp, vp, u32, i, vp, vp, vp]
        L.pdq_mlp_train_workspace_bytes.argtypes = [u32]
        L.pdq_mlp_train_workspace_bytes.restype = sz
        L.pdq_mlp_train.argtypes = [vp, vp, sz, u64, u32, u32, u32, i, vp, vp, vp, vp, sz, vp]
        L.pdq_learned_features.argtypes = [vp, sz, vp, vp, vp, vp]
        L.pdq_learned_extract.argtypes = [vp, vp, sz, vp, vp, vp, vp]
        L.pdq_learned_leaves.argtypes = [vp, vp, vp, sz, vp, vp, vp, vp, vp]
        L.pdq_learned_leaves.restype = ctypes.c_int
        L.pdq_sample_judge.argtypes = [vp, sz, vp, vp, vp, vp]
        L.pdq_sample_judge.restype = ctypes.c_int
        L.pdq_bucket_workspace_bytes.argtypes = [sz]
        L.pdq_bucket_workspace_bytes.restype = sz
        L.pdq_bucket_histogram.argtypes = [vp, sz, i, vp, vp, vp, vp, sz, vp]
        L.pdq_learned_fit_workspace_bytes.argtypes = [ctypes.POINTER(Options)]
        L.pdq_learned_fit_workspace_bytes.restype = sz
        L.pdq_learned_fit.argtypes = [vp, sz, i, vp, sz, vp, ctypes.POINTER(Options), ctypes.POINTER(FitBuffers)]
        L.pdq_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), vp, vp, sz, vp, sz, i, vp, sz, vp,
                                      ctypes.POINTER(Options)]
        L.pdq_plan_launch.argtypes = [vp, vp]
        L.pdq_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_double)]
        L.pdq_plan_classes.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_double)]
        L.pdq_plan_classes.restype = ctypes.c_int
        L.pdq_plan_destroy.argtypes = [vp]
        L.pdq_plan_destroy.restype = None
        for f in ("pdq_plan_create", "pdq_plan_launch", "pdq_plan_info"):
            getattr(L, f).restype = ctypes.c_int
        for f in ("pdq_mlp_infer", "pdq_mlp_gradient", "pdq_mlp_train", "pdq_learned_features",
                  "pdq_learned_extract", "pdq_bucket_histogram", "pdq_learned_fit"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().pdq_status_string(status).decode()


def abi_version() -> int:
    return lib().pdq_abi_version()


def _check(status: int):
    if status != PDQ_OK:
        raise PdqError(status, status_string(status), lib().pdq_last_hip_error())


def check(workspace):
    """pdq_check: wait for the current stream and raise if the last call that
    used this workspace (tensor) found a device-side error."""
    import torch
    _check(lib().pdq_check(ctypes.c_void_p(workspace.data_ptr()),
                           ctypes.c_void_p(torch.cuda.current_stream(workspace.device).cuda_stream)))


def _key_type(t) -> int:
    import torch
    m = {torch.uint32: 1, torch.int32: 2, torch.float32: 3, torch.uint64: 4, torch.int64: 5, torch.float64: 6}
    if t.dtype not in m:
        raise TypeError(f"unsupported key dtype {t.dtype}; use uint32, int32, float32, uint64, int64 or float64")
    return m[t.dtype]


def _options(force_budget: int, tile: int, flags: int, seed: int = 0, imbalance_limit: float = 0.0,
             learn_steps: int = 0, learn_batch: int = 0, learn_grid: int = 0, batch_shape: int = 0,
             batch_passes: int | None = None, waves: int = 0, tune_cache_path: str | None = None) -> Options:
    return Options(ctypes.sizeof(Options), flags, force_budget, tile, seed, imbalance_limit, learn_steps,
                   learn_batch, learn_grid, batch_shape, 0 if batch_passes is None else batch_passes + 1, waves, 0,
                   tune_cache_path.encode() if tune_cache_path else None)


def workspace_bytes(n: int, nseg: int = 1, key_type: int | str = "u32", has_vals: bool = False,
                    options: Options | None = None) -> int:
    kt = KEY_TYPES[key_type] if isinstance(key_type, str) else int(key_type)
    return int(lib().pdq_workspace_bytes(n, max(1, nseg), kt, 1 if has_vals else 0,
                                         ctypes.byref(options) if options else None))


def _prepare(keys, vals, nseg, force_budget, tile, flags, workspace, learn=None):
    import torch
    if not keys.is_cuda:
        raise ValueError("keys must be a device tensor")
    if not keys.is_contiguous():
        raise ValueError("keys must be contiguous")
    if vals is not None:
        if vals.dtype not in (torch.uint32, torch.uint64) or not vals.is_cuda or not vals.is_contiguous():
            raise ValueError("vals must be a contiguous uint32 or uint64 device tensor")
        if vals.numel() != keys.numel():
            raise ValueError("vals must have as many elements as keys")
        if vals.dtype == torch.uint64:
            flags |= FLAG_VALS64
    kt = _key_type(keys)
    opt = _options(force_budget, tile, flags, **(learn or {}))
    need = workspace_bytes(keys.numel(), nseg, kt, vals is not None, opt)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
    stream = torch.cuda.current_stream(keys.device).cuda_stream
    return kt, opt, workspace, need, ctypes.c_void_p(stream)


def _finish(st, want):
    return st.as_dict() if want else None


def _learn_opts(learned, seed, imbalance_limit, learn_steps, learn_batch, learn_grid):
    flags = FLAG_LEARNED if learned else 0
    return flags, dict(seed=seed, imbalance_limit=imbalance_limit, learn_steps=learn_steps,
                       learn_batch=learn_batch, learn_grid=learn_grid)


def sort_(keys, *, force_budget: int = -1, tile: int = 0, profile: bool = False, stats: bool = False,
          workspace=None, learned: bool = False, seed: int = 0, imbalance_limit: float = 0.0,
          learn_steps: int = 0, learn_batch: int = 0, learn_grid: int = 0, deterministic: bool = False,
          fresh_fixed: bool = False, waves: int = 0, host_loop: bool = False, batch_passes: int | None = None,
          heapsort: bool = False):
    """Sort a 1-D device tensor in place (ascending canonical order).
    learned=True runs the learned multiway first pass (see pdq_learned.h);
    deterministic=True selects the look-back partition (PDQ_DETERMINISTIC);
    fresh_fixed=True takes fresh pivot candidates at fixed offsets after a
    bad partition (PDQ_FRESH_FIXED) instead of hashed positions; waves
    (1, 2, 4, 8, 16) sets the workgroup shape of the LDS base-case classes;
    host_loop=True runs the host-driven pass loop (PDQ_HOST_LOOP) instead of
    the device-counted passes, whose number batch_passes overrides;
    heapsort=True makes the fallback of segments out of budget the paper's
    heapsort (PDQ_HEAPSORT)."""
    lf, learn = _learn_opts(learned, seed, imbalance_limit, learn_steps, learn_batch, learn_grid)
    kt, opt, ws, need, stream = _prepare(keys, None, 1, force_budget, tile,
                                         (FLAG_PROFILE if profile else 0) | lf |
                                         (FLAG_DETERMINISTIC if deterministic else 0) |
                                         (FLAG_FRESH_FIXED if fresh_fixed else 0) |
                                         (FLAG_HOST_LOOP if host_loop else 0) |
                                         (FLAG_HEAPSORT if heapsort else 0), workspace,
                                         dict(learn, waves=waves, batch_passes=batch_passes))
    st = Stats(ctypes.sizeof(Stats)) if (stats or profile) else None
    rc = lib().pdq_sort(ctypes.c_void_p(keys.data_ptr()), keys.numel(), kt, 0, ctypes.c_void_p(ws.data_ptr()),
                        need, stream, ctypes.byref(opt), ctypes.byref(st) if st is not None else None)
    _check(rc)
    return _finish(st, st is not None)


def sort_pairs_(keys, vals, *, force_budget: int = -1, tile: int = 0, profile: bool = False,
                stats: bool = False, workspace=None, learned: bool = False, seed: int = 0,
                imbalance_limit: float = 0.0, learn_steps: int = 0, learn_batch: int = 0, learn_grid: int = 0,
                deterministic: bool = False, fresh_fixed: bool = False, waves: int = 0, host_loop: bool = False,
                batch_passes: int | None = None, heapsort: bool = False):
    """Sort keys in place and move the payload `vals` (uint32, or uint64:
    PDQ_VALS64) with them."""
    lf, learn = _learn_opts(learned, seed, imbalance_limit, learn_steps, learn_batch, learn_grid)
    kt, opt, ws, need, stream = _prepare(keys, vals, 1, force_budget, tile,
                                         (FLAG_PROFILE if profile else 0) | lf |
                                         (FLAG_DETERMINISTIC if deterministic else 0) |
                                         (FLAG_FRESH_FIXED if fresh_fixed else 0) |
                                         (FLAG_HOST_LOOP if host_loop else 0) |
                                         (FLAG_HEAPSORT if heapsort else 0), workspace,
                                         dict(learn, waves=waves, batch_passes=batch_passes))
    st = Stats(ctypes.sizeof(Stats)) if (stats or profile) else None
    rc = lib().pdq_sort_pairs(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()), keys.numel(),
                              kt, 0, ctypes.c_void_p(ws.data_ptr()), need, stream, ctypes.byref(opt),
                              ctypes.byref(st) if st is not None else None)
    _check(rc)
    return _finish(st, st is not None)


def segmented_sort_(keys, offsets, vals=None, *, force_budget: int = -1, tile: int = 0,
                    validate: bool = False, profile: bool = False, stats: bool = False, workspace=None,
                    batched: bool = False, batch_shape: int = 0, batch_passes: int | None = None,
                    deterministic: bool = False, fresh_fixed: bool = False, waves: int = 0,
                    tune_cache_path: str | None = None):
    """Sort each segment [offsets[s], offsets[s+1]) of keys in place.
    offsets: uint64 device tensor of nseg+1 entries. batched=True runs the
    batched form (batch_shape 1..4 forces a shape, batch_passes the number of
    partition passes before the persistent tail; None = automatic)."""
    import torch
    if offsets.dtype != torch.uint64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous uint64 device tensor")
    nseg = offsets.numel() - 1
    flags = (FLAG_VALIDATE if validate else 0) | (FLAG_PROFILE if profile else 0) | (FLAG_BATCHED if batched else 0) \
        | (FLAG_DETERMINISTIC if deterministic else 0) | (FLAG_FRESH_FIXED if fresh_fixed else 0)
    kt, opt, ws, need, stream = _prepare(keys, vals, nseg, force_budget, tile, flags, workspace,
                                         dict(batch_shape=batch_shape, batch_passes=batch_passes, waves=waves,
                                              tune_cache_path=tune_cache_path))
    st = Stats(ctypes.sizeof(Stats)) if (stats or profile) else None
    rc = lib().pdq_segmented_sort(ctypes.c_void_p(keys.data_ptr()),
                                  ctypes.c_void_p(vals.data_ptr()) if vals is not None else None,
                                  keys.numel(), ctypes.c_void_p(offsets.data_ptr()), max(nseg, 0), kt, 0,
                                  ctypes.c_void_p(ws.data_ptr()), need, stream, ctypes.byref(opt),
                                  ctypes.byref(st) if st is not None else None)
    _check(rc)
    return _finish(st, st is not None)


def sort_noalloc_(keys, vals=None, *, force_budget: int = -1, tile: int = 0, stats: bool = False,
                  learned: bool = False, seed: int = 0, deterministic: bool = False):
    """pdq_sort_noalloc: sort keys (and move the uint32 payload vals, if
    given) in place using the library's own device scratch array instead of
    a workspace; nothing is allocated. Sizes beyond PDQ_NOALLOC_SCRATCH_BYTES
    raise PdqError (PDQ_ERR_SCRATCH); calls on one GPU must not overlap."""
    import torch
    if not keys.is_cuda or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous device tensor")
    if vals is not None and (vals.dtype not in (torch.uint32, torch.uint64) or not vals.is_cuda
                             or not vals.is_contiguous() or vals.numel() != keys.numel()):
        raise ValueError("vals must be a contiguous uint32 or uint64 device tensor with as many elements as keys")
    kt = _key_type(keys)
    flags = (FLAG_LEARNED if learned else 0) | (FLAG_DETERMINISTIC if deterministic else 0)
    if vals is not None and vals.dtype == torch.uint64:
        flags |= FLAG_VALS64
    opt = _options(force_budget, tile, flags, seed=seed)
    st = Stats(ctypes.sizeof(Stats)) if stats else None
    stream = ctypes.c_void_p(torch.cuda.current_stream(keys.device).cuda_stream)
    rc = lib().pdq_sort_noalloc(_ptr(keys), _ptr(vals), keys.numel(), kt, 0, stream, ctypes.byref(opt),
                                ctypes.byref(st) if st is not None else None)
    _check(rc)
    return _finish(st, st is not None)


# ---------------------------------------------------------------- learned pass, step by step

def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def mlp_infer(params, x, residual: bool = True):
    """float32 clamped prediction of the splitter model for features x."""
    import torch
    y = torch.empty_like(x)
    _check(lib().pdq_mlp_infer(_ptr(params), _ptr(x), x.numel(), 1 if residual else 0, _ptr(y), _stream(x)))
    return y


def mlp_gradient(params, x, t, residual: bool = True):
    """Gradient of the mean squared error over (x, t); returns (grad, loss)."""
    import torch
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(lib().pdq_mlp_gradient(_ptr(params), _ptr(x), _ptr(t), x.numel(), 1 if residual else 0, _ptr(g),
                                  _ptr(loss), _stream(x)))
    return g, loss


def mlp_train(x, t, *, seed: int = 0, steps: int = 256, batch: int = 1024, grid: int = 16, residual: bool = True,
              init=None):
    """Fused Adam training on sorted features x and targets t; returns (params, losses)."""
    import torch
    p = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    losses = torch.empty(steps, dtype=torch.float32, device=x.device)
    need = int(lib().pdq_mlp_train_workspace_bytes(grid))
    ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    _check(lib().pdq_mlp_train(_ptr(x), _ptr(t), x.numel(), seed, steps, batch, grid, 1 if residual else 0,
                               _ptr(init), _ptr(p), _ptr(losses), _ptr(ws), need, _stream(x)))
    return p, losses


def learned_features(sorted_images):
    """Features, targets and info words of a sorted uint64 sample of key images."""
    import torch
    m = sorted_images.numel()
    x = torch.empty(m, dtype=torch.float32, device=sorted_images.device)
    t = torch.empty_like(x)
    info = torch.zeros(4, dtype=torch.uint64, device=sorted_images.device)
    _check(lib().pdq_learned_features(_ptr(sorted_images), m, _ptr(x), _ptr(t), _ptr(info), _stream(x)))
    return x, t, info


def learned_extract(sorted_images, pred):
    """Splitters (uint64 images) from clamped predictions of a sorted sample."""
    import torch
    dev = pred.device
    r = torch.empty_like(pred)
    sp = torch.zeros(MAX_SPLITTERS, dtype=torch.uint64, device=dev)
    cnt = torch.zeros(1, dtype=torch.uint32, device=dev)
    _check(lib().pdq_learned_extract(_ptr(sorted_images), _ptr(pred), pred.numel(), _ptr(r), _ptr(sp), _ptr(cnt),
                                     _stream(pred)))
    u = int(cnt.cpu().item())
    return sp[:u].clone(), r


def learned_leaves(x, t, pred):
    """Second stage of the splitter model: (x-leaf, y-leaf) float32
    predictions of the sorted sample's features x, targets t and clamped
    network predictions pred."""
    import torch
    m = x.numel()
    r = torch.empty_like(x)
    px = torch.empty_like(x)
    py = torch.empty_like(x)
    leaf = torch.empty(2 * 64 * 2, dtype=torch.float64, device=x.device)
    _check(lib().pdq_learned_leaves(_ptr(x), _ptr(t), _ptr(pred), m, _ptr(r), _ptr(leaf), _ptr(px), _ptr(py),
                                    _stream(x)))
    return px, py


def sample_judge(sorted_images, splitters):
    """Largest number of sorted sample keys in one range bin of splitters."""
    import torch
    dev = sorted_images.device
    u = splitters.numel()
    sp = torch.zeros(MAX_SPLITTERS, dtype=torch.uint64, device=dev)
    sp[:u] = splitters
    cnt = torch.tensor([u], dtype=torch.uint32, device=dev)
    out = torch.zeros(1, dtype=torch.uint64, device=dev)
    _check(lib().pdq_sample_judge(_ptr(sorted_images), sorted_images.numel(), _ptr(sp), _ptr(cnt), _ptr(out),
                                  _stream(sorted_images)))
    return int(out.cpu().item())


def bucket_histogram(keys, splitters):
    """Keys per bin (2u + 1 bins) for sorted, distinct uint64 splitter images."""
    import torch
    dev = keys.device
    u = splitters.numel()
    sp = torch.zeros(MAX_SPLITTERS, dtype=torch.uint64, device=dev)
    sp[:u] = splitters
    cnt = torch.tensor([u], dtype=torch.uint32, device=dev)
    hist = torch.zeros(512, dtype=torch.uint64, device=dev)
    need = int(lib().pdq_bucket_workspace_bytes(keys.numel()))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(lib().pdq_bucket_histogram(_ptr(keys), keys.numel(), _key_type(keys), _ptr(sp), _ptr(cnt), _ptr(hist),
                                      _ptr(ws), need, _stream(keys)))
    return hist[:2 * u + 1]


def learned_fit(keys, *, seed: int = 0, learn_steps: int = 0, learn_batch: int = 0, learn_grid: int = 0):
    """The whole fit of the learned pass; returns a dict of device tensors."""
    import torch
    dev = keys.device
    opt = _options(-1, 0, 0, seed=seed, learn_steps=learn_steps, learn_batch=learn_batch, learn_grid=learn_grid)
    steps = learn_steps or 128
    m = LEARN_SAMPLE
    out = dict(sample=torch.empty(m, dtype=torch.uint64, device=dev),
               x=torch.empty(m, dtype=torch.float32, device=dev),
               t=torch.empty(m, dtype=torch.float32, device=dev),
               pred=torch.empty(m, dtype=torch.float32, device=dev),
               params=torch.empty(MLP_PARAMS, dtype=torch.float32, device=dev),
               losses=torch.empty(steps, dtype=torch.float32, device=dev),
               splitters=torch.zeros(MAX_SPLITTERS, dtype=torch.uint64, device=dev),
               count=torch.zeros(1, dtype=torch.uint32, device=dev),
               info=torch.zeros(8, dtype=torch.uint64, device=dev))
    fb = FitBuffers(*[_ptr(out[k]) for k in ("sample", "x", "t", "pred", "params", "losses", "splitters",
                                             "count", "info")])
    need = int(lib().pdq_learned_fit_workspace_bytes(ctypes.byref(opt)))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(lib().pdq_learned_fit(_ptr(keys), keys.numel(), _key_type(keys), _ptr(ws), need, _stream(keys),
                                 ctypes.byref(opt), ctypes.byref(fb)))
    u = int(out["count"].cpu().item())
    out["splitters"] = out["splitters"][:u]
    return out


_live_plans = None


def _destroy_live_plans():
    """atexit: destroy every plan still alive while the HIP runtime is still
    up (a graph destroyed from __del__ during interpreter teardown could run
    after the runtime's own exit handlers)."""
    if _live_plans is not None:
        for p in list(_live_plans):
            p.destroy()


class Plan:
    """A captured batched segmented sort bound to these tensors (see
    pdq_plan_create); offsets=None captures the sort of one range [0, n).
    launch() replays the graph on the current stream."""

    def __init__(self, keys, offsets, vals=None, *, autotune: bool = False, batch_shape: int = 0,
                 batch_passes: int | None = None, force_budget: int = -1, workspace=None, waves: int = 0,
                 tune_cache_path: str | None = None):
        # the workspace must be sized with the same flags (batched, autotune)
        import torch
        if offsets is not None and (offsets.dtype != torch.uint64 or not offsets.is_cuda or
                                    not offsets.is_contiguous()):
            raise ValueError("offsets must be a contiguous uint64 device tensor")
        nseg = offsets.numel() - 1 if offsets is not None else 1
        flags = FLAG_BATCHED | (FLAG_AUTOTUNE if autotune else 0)
        kt, opt, ws, need, stream = _prepare(keys, vals, nseg, force_budget, 0, flags, workspace,
                                             dict(batch_shape=batch_shape, batch_passes=batch_passes, waves=waves,
                                                  tune_cache_path=tune_cache_path))
        self._keep = (keys, offsets, vals, ws, opt)
        self._h = ctypes.c_void_p()
        _check(lib().pdq_plan_create(ctypes.byref(self._h), _ptr(keys), _ptr(vals), keys.numel(), _ptr(offsets),
                                     nseg, kt, _ptr(ws), need, stream, ctypes.byref(opt)))
        global _live_plans
        if _live_plans is None:
            import atexit
            import weakref
            _live_plans = weakref.WeakSet()
            atexit.register(_destroy_live_plans)
        _live_plans.add(self)

    def launch(self):
        import torch
        _check(lib().pdq_plan_launch(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def check(self):
        """Raise if the last launch found a device-side error (waits for the stream)."""
        check(self._keep[3])

    def info(self):
        shape = ctypes.c_uint32()
        ms = (ctypes.c_double * 4)()
        _check(lib().pdq_plan_info(self._h, ctypes.byref(shape), ms))
        return int(shape.value), list(ms)

    def classes(self):
        """(lanes per workgroup of each base-case size class, measured ms of
        each class under each candidate shape [7][3])."""
        th = (ctypes.c_uint32 * 7)()
        ms = (ctypes.c_double * 21)()
        _check(lib().pdq_plan_classes(self._h, th, ms))
        return list(th), [list(ms[3 * k:3 * k + 3]) for k in range(7)]

    def destroy(self):
        if self._h:
            lib().pdq_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
