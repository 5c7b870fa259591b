"""Python binding of libfastpc (the C ABI in include/fastpc.h).

Argument marshalling only: every step of the skeleton runs in the HIP
library.  PyTorch provides device memory and the stream.  Importing this
module fails if the library has not been built (python
paper_2109_04626_amd/build.py); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from collections.abc import Mapping

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastpc.so")

FPC_OK, FPC_EINVAL, FPC_ENONFINITE, FPC_ESINGULAR, FPC_EBUDGET, FPC_ENOMEM, FPC_EDEVICE, FPC_ESCRATCH, FPC_ETOOLARGE = range(9)
FPC_NOALLOC_MAX_P = 512
FPC_F64, FPC_F32 = 0, 1
FPC_CORR_FP64, FPC_CORR_BF16X3, FPC_CORR_BF16X6, FPC_CORR_FP32 = 0, 1, 2, 3
FPC_PREC_FP64, FPC_PREC_MIXED = 0, 1
FPC_REVERSE, FPC_FORWARD = 0, 1
FPC_ORDER_LEX, FPC_ORDER_LEARNED = 0, 1
FPC_SEP_NONE, FPC_SEP_LIST, FPC_SEP_ALL_BUT = 0, 1, 2
FPC_FLAG_PER_TEST_KERNEL = 1
FPC_FLAG_LOG_FEATURES = 2
FPC_FLAG_GRAPH = 4
FPC_KERNEL_AUTO, FPC_KERNEL_PER_TEST, FPC_KERNEL_PAIR, FPC_KERNEL_TRIPLE, FPC_KERNEL_GLOBAL = range(5)

EXPORTED = ["fpc_create", "fpc_destroy", "fpc_strerror", "fpc_last_hip_error", "fpc_quantile",
            "fpc_corr", "fpc_first_level", "fpc_ci_batch", "fpc_candidates", "fpc_skeleton", "fpc_skeleton_batch",
            "fpc_result_free", "fpc_orient", "fpc_mlp_bytes", "fpc_mlp_params", "fpc_mlp_init", "fpc_mlp_get",
            "fpc_mlp_forward", "fpc_mlp_grad", "fpc_mlp_train_step", "fpc_get_tuning", "fpc_set_tuning",
            "fpc_set_recheck_queue", "fpc_level_series", "fpc_first_level_noalloc", "fpc_checkpoint_of"]
FPC_TUNE_LEVELS = 17
TUNING_FIELDS = ("test_ranks_per_wave", "shared_ranks_per_wave", "window_growth", "first_window_items",
                 "max_blocks_per_cu", "shared_prefix_depth")
# launch-shape table written by the autotuner (python -m paper_2109_04626_amd.autotune)
TUNING_TABLE = os.path.join(_HERE, "tuning_gfx950.json")


class FastPCError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = f"{where}: {_strerror(code)}"
        if code == FPC_EDEVICE:
            msg += f" [{_lib.fpc_last_hip_error().decode()}]"
        super().__init__(msg)
        self.code = code


class fpc_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("p", ctypes.c_int32), ("X", ctypes.c_void_p),
                ("x_dtype", ctypes.c_int32), ("x_on_device", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("max_level", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("recheck_margin", ctypes.c_double),
                ("schedule", ctypes.c_int32), ("order", ctypes.c_int32),
                ("order_model", ctypes.c_void_p), ("max_tests", ctypes.c_int64),
                ("q_override", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("ill_cond_tau", ctypes.c_double), ("c32_method", ctypes.c_int32),
                ("stop_after_levels", ctypes.c_int32), ("resume", ctypes.c_void_p)]


class fpc_level_stats(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("max_cand", ctypes.c_int32),
                ("edges_eligible", ctypes.c_int64), ("tests_possible", ctypes.c_int64),
                ("tests_executed", ctypes.c_int64), ("tests_rechecked", ctypes.c_int64),
                ("deleted", ctypes.c_int64), ("kernel_ms", ctypes.c_double),
                ("test_kernel_ms", ctypes.c_double), ("test_launches", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("level_ms", ctypes.c_double),
                ("tests_required", ctypes.c_int64)]


class fpc_result(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("adj", ctypes.POINTER(ctypes.c_uint8)), ("sep_level", ctypes.POINTER(ctypes.c_int32)),
                ("sep_kind", ctypes.POINTER(ctypes.c_int8)), ("sep_off", ctypes.POINTER(ctypes.c_int64)),
                ("sep_nodes", ctypes.POINTER(ctypes.c_int32)),
                ("levels", ctypes.POINTER(fpc_level_stats)), ("total_tests", ctypes.c_int64),
                ("q", ctypes.c_double), ("corr_ms", ctypes.c_double),
                ("first_level_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("corr_max_abs_err", ctypes.c_double), ("log_rows", ctypes.c_int64),
                ("log_x", ctypes.POINTER(ctypes.c_float)), ("log_y", ctypes.POINTER(ctypes.c_uint8)),
                ("log_group", ctypes.POINTER(ctypes.c_int32)), ("log_level", ctypes.POINTER(ctypes.c_int32)),
                ("n_lists", ctypes.c_int64), ("list_pairs", ctypes.POINTER(ctypes.c_int64)),
                ("next_level", ctypes.c_int32)]


class fpc_checkpoint(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("next_level", ctypes.c_int32), ("adj", ctypes.c_void_p),
                ("sep_level", ctypes.c_void_p), ("sep_kind", ctypes.c_void_p), ("sep_off", ctypes.c_void_p),
                ("sep_nodes", ctypes.c_void_p), ("n_levels", ctypes.c_int32), ("levels", ctypes.c_void_p)]


class fpc_tuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32 * FPC_TUNE_LEVELS) for f in TUNING_FIELDS]


class fpc_instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("p", ctypes.c_int32), ("X", ctypes.c_void_p), ("x_rows", ctypes.c_int64),
                ("rows", ctypes.c_void_p)]


def _load():
    # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one
    # the library binds to.  Loaded the other way round, torch would bring a
    # second runtime into the process and the library's would see no device.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python paper_2109_04626_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, i64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.fpc_create.argtypes = [ctypes.POINTER(vp), i, vp]
    lib.fpc_create.restype = i
    lib.fpc_destroy.argtypes = [vp]
    lib.fpc_destroy.restype = i
    lib.fpc_strerror.argtypes = [i]
    lib.fpc_strerror.restype = ctypes.c_char_p
    lib.fpc_last_hip_error.argtypes = []
    lib.fpc_last_hip_error.restype = ctypes.c_char_p
    lib.fpc_quantile.argtypes = [d]
    lib.fpc_quantile.restype = d
    lib.fpc_corr.argtypes = [vp, vp, i, i, i, i, vp]
    lib.fpc_corr.restype = i
    lib.fpc_first_level.argtypes = [vp, vp, i, i, d, vp, vp]
    lib.fpc_first_level.restype = i
    lib.fpc_first_level_noalloc.argtypes = [vp, vp, i, i, d, vp, vp]
    lib.fpc_first_level_noalloc.restype = i
    lib.fpc_ci_batch.argtypes = [vp, vp, i, i, i, i, vp, i64, d, vp, vp]
    lib.fpc_ci_batch.restype = i
    lib.fpc_level_series.argtypes = [vp, vp, i, i, i, i, i, i, vp, i, i64, i64, i, i, i, d, d, d, d, vp, vp]
    lib.fpc_level_series.restype = i
    lib.fpc_candidates.argtypes = [vp, i, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp, vp, vp]
    lib.fpc_candidates.restype = i
    lib.fpc_skeleton.argtypes = [vp, ctypes.POINTER(fpc_params), ctypes.POINTER(ctypes.POINTER(fpc_result))]
    lib.fpc_skeleton.restype = i
    lib.fpc_skeleton_batch.argtypes = [vp, ctypes.POINTER(fpc_params), i, ctypes.POINTER(fpc_instance),
                                       ctypes.POINTER(ctypes.POINTER(fpc_result))]
    lib.fpc_skeleton_batch.restype = i
    lib.fpc_get_tuning.argtypes = [vp, ctypes.POINTER(fpc_tuning)]
    lib.fpc_get_tuning.restype = i
    lib.fpc_set_tuning.argtypes = [vp, ctypes.POINTER(fpc_tuning)]
    lib.fpc_set_tuning.restype = i
    lib.fpc_set_recheck_queue.argtypes = [vp, i64, i64]
    lib.fpc_set_recheck_queue.restype = i
    lib.fpc_result_free.argtypes = [ctypes.POINTER(fpc_result)]
    lib.fpc_result_free.restype = None
    lib.fpc_checkpoint_of.argtypes = [ctypes.POINTER(fpc_result), ctypes.POINTER(fpc_checkpoint)]
    lib.fpc_checkpoint_of.restype = None
    lib.fpc_orient.argtypes = [i, vp, vp, vp, vp, vp, vp]
    lib.fpc_orient.restype = i
    lib.fpc_mlp_bytes.argtypes = []
    lib.fpc_mlp_bytes.restype = ctypes.c_size_t
    lib.fpc_mlp_params.argtypes = []
    lib.fpc_mlp_params.restype = i
    lib.fpc_mlp_init.argtypes = [vp, vp, vp]
    lib.fpc_mlp_init.restype = i
    lib.fpc_mlp_get.argtypes = [vp, vp, vp]
    lib.fpc_mlp_get.restype = i
    lib.fpc_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    lib.fpc_mlp_forward.restype = i
    lib.fpc_mlp_grad.argtypes = [vp, vp, vp, i64, vp, vp]
    lib.fpc_mlp_grad.restype = i
    lib.fpc_mlp_train_step.argtypes = [vp, vp, vp, i64, vp, ctypes.c_float, vp]
    lib.fpc_mlp_train_step.restype = i
    return lib


_lib = _load()


def _strerror(code: int) -> str:
    return _lib.fpc_strerror(code).decode()


def _check(code: int, where: str):
    if code != FPC_OK:
        raise FastPCError(code, where)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _t_ptr(t):
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ host calls
def fpc_strerror(code: int) -> str:
    return _strerror(code)


def fpc_last_hip_error() -> str:
    return _lib.fpc_last_hip_error().decode()


def fpc_result_free(res) -> None:
    """Result dicts free their C buffers themselves once no array taken from
    them is left; this accepts a raw POINTER(fpc_result) for completeness."""
    if res:
        _lib.fpc_result_free(res)


def fpc_quantile(alpha: float) -> float:
    return float(_lib.fpc_quantile(float(alpha)))


def fpc_candidates(adj: np.ndarray):
    """(edge_i, edge_j, off, nodes) of adj(G,i,j) n path(G,i,j) per edge."""
    adj = np.ascontiguousarray(adj, dtype=np.uint8)
    p = adj.shape[0]
    E, N = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.fpc_candidates(_np_ptr(adj), p, ctypes.byref(E), ctypes.byref(N), None, None, None, None),
           "fpc_candidates")
    ei = np.empty(E.value, np.int32)
    ej = np.empty(E.value, np.int32)
    off = np.empty(E.value + 1, np.int64)
    nodes = np.empty(max(N.value, 1), np.int32)
    _check(_lib.fpc_candidates(_np_ptr(adj), p, ctypes.byref(E), ctypes.byref(N), _np_ptr(ei), _np_ptr(ej),
                               _np_ptr(off), _np_ptr(nodes)), "fpc_candidates")
    return ei, ej, off, nodes[: N.value]


def fpc_orient(res: dict) -> np.ndarray:
    """CPDAG marks (p x p uint8) of a fpc_skeleton result: [a, b] = 1 when
    the edge a-b may point a -> b."""
    p = res["p"]
    adj = np.ascontiguousarray(res["adj"], dtype=np.uint8)
    lev = np.ascontiguousarray(res["sep_level"], dtype=np.int32)
    kind = np.ascontiguousarray(res["sep_kind"], dtype=np.int8)
    off = np.ascontiguousarray(res["sep_off"], dtype=np.int64)
    nodes = np.ascontiguousarray(res["sep_nodes"], dtype=np.int32)
    out = np.empty((p, p), dtype=np.uint8)
    _check(_lib.fpc_orient(p, _np_ptr(adj), _np_ptr(lev), _np_ptr(kind), _np_ptr(off),
                           _np_ptr(nodes) if nodes.size else None, _np_ptr(out)), "fpc_orient")
    return out


# ------------------------------------------------------------------ device calls
class Context:
    """An fpc_ctx on a HIP device, enqueuing on torch's current stream.

    ``tuning``: "table" loads the autotuned launch shapes shipped with the
    package (when present), "default" keeps the library defaults, a dict
    {field: [per-level values]} sets them explicitly."""

    def __init__(self, device: int = 0, stream=None, tuning="table"):
        import torch

        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = ctypes.c_void_p()
        _check(_lib.fpc_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream.cuda_stream)), "fpc_create")
        self._h = h
        if isinstance(tuning, dict):
            fpc_set_tuning(self, tuning)
        elif tuning == "table" and os.path.exists(TUNING_TABLE):
            import json

            with open(TUNING_TABLE) as f:
                fpc_set_tuning(self, json.load(f)["tuning"])

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.fpc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def fpc_get_tuning(ctx: Context) -> dict:
    t = fpc_tuning()
    _check(_lib.fpc_get_tuning(ctx.handle, ctypes.byref(t)), "fpc_get_tuning")
    return {f: list(getattr(t, f)) for f in TUNING_FIELDS}


def fpc_set_recheck_queue(ctx: Context, initial: int = 1 << 23, maximum: int = 1 << 28) -> None:
    """First and largest size (entries) of the mixed form's FP64 recheck
    queue; results do not depend on them."""
    _check(_lib.fpc_set_recheck_queue(ctx.handle, int(initial), int(maximum)), "fpc_set_recheck_queue")


def fpc_set_tuning(ctx: Context, tuning) -> None:
    """tuning: dict of per-level lists (missing fields keep their values),
    or None for the library defaults."""
    if tuning is None:
        _check(_lib.fpc_set_tuning(ctx.handle, None), "fpc_set_tuning")
        return
    cur = fpc_get_tuning(ctx)
    t = fpc_tuning()
    for f in TUNING_FIELDS:
        vals = list(tuning.get(f, cur[f]))
        if len(vals) != FPC_TUNE_LEVELS:
            raise ValueError(f"{f}: {FPC_TUNE_LEVELS} values expected")
        getattr(t, f)[:] = [int(v) for v in vals]
    _check(_lib.fpc_set_tuning(ctx.handle, ctypes.byref(t)), "fpc_set_tuning")


def fpc_create(device: int = 0, stream=None) -> Context:
    return Context(device, stream)


def fpc_destroy(ctx: Context) -> None:
    ctx.close()


def _dtype_code(t):
    import torch

    if t.dtype == torch.float64:
        return FPC_F64
    if t.dtype == torch.float32:
        return FPC_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def fpc_corr(ctx: Context, X, method: int = FPC_CORR_FP64):
    """Correlation matrix of the device tensor X (n x p, row-major)."""
    import torch

    X = X.contiguous()
    n, p = X.shape
    out = torch.empty((p, p), dtype=torch.float64 if method == FPC_CORR_FP64 else torch.float32, device=X.device)
    _check(_lib.fpc_corr(ctx.handle, _t_ptr(X), _dtype_code(X), n, p, int(method), _t_ptr(out)), "fpc_corr")
    return out


def fpc_first_level(ctx: Context, C, n: int, q: float):
    """(r, indep) of the l = p-2 level on the FP64 device matrix C."""
    import torch

    C = C.contiguous()
    p = C.shape[0]
    r = torch.empty((p, p), dtype=torch.float64, device=C.device)
    ind = torch.empty((p, p), dtype=torch.uint8, device=C.device)
    _check(_lib.fpc_first_level(ctx.handle, _t_ptr(C), p, int(n), float(q), _t_ptr(r), _t_ptr(ind)),
           "fpc_first_level")
    return r, ind


def fpc_first_level_noalloc(ctx: Context, C, n: int, q: float, r_out, indep_out) -> None:
    """fpc_first_level into caller-allocated device outputs r_out (FP64 p x p)
    and indep_out (uint8 p x p), with the library's static workspace: the
    call allocates no device memory (p <= FPC_NOALLOC_MAX_P)."""
    p = C.shape[0]
    _check(_lib.fpc_first_level_noalloc(ctx.handle, _t_ptr(C), p, int(n), float(q), _t_ptr(r_out),
                                        _t_ptr(indep_out)), "fpc_first_level_noalloc")


def fpc_ci_batch(ctx: Context, C, n: int, B, q: float):
    """(z, indep) for the rows [i, j, k_1..k_l] of the int32 device matrix B."""
    import torch

    C = C.contiguous()
    B = B.contiguous()
    assert B.dtype == torch.int32 and B.dim() == 2
    b, w = B.shape
    l = w - 2
    z = torch.empty(b, dtype=torch.float64, device=C.device)
    ind = torch.empty(b, dtype=torch.uint8, device=C.device)
    _check(_lib.fpc_ci_batch(ctx.handle, _t_ptr(C), _dtype_code(C), C.shape[0], int(n), l, _t_ptr(B), b,
                             float(q), _t_ptr(z), _t_ptr(ind)), "fpc_ci_batch")
    return z, ind


def fpc_level_series(ctx: Context, C, n: int, l: int, i: int, j: int, cand, rank_lo: int, rank_hi: int, q: float,
                     kernel: int = FPC_KERNEL_AUTO, ranks_per_wave: int = 0, pair_table: int = -1,
                     band_z: float = 1e-3, c_err: float = 0.0, ill_cond_tau: float = 1e-4):
    """(r, dec) of the level-l tests ranked rank_lo..rank_hi-1 of the pair
    (i, j) with candidate list ``cand`` (host sequence), run by the level
    kernels on the device matrix C (FP64: FP64 kernels; FP32: the mixed
    form's FP32 kernels).  r: FP64 device tensor (NaN = degenerate); dec:
    uint8 device tensor (0 dependent, 1 independent, 2 FP64 re-run)."""
    import torch

    C = C.contiguous()
    cand = np.ascontiguousarray(np.asarray(cand, dtype=np.int32).reshape(-1))
    k = int(rank_hi) - int(rank_lo)
    r = torch.empty(max(k, 1), dtype=torch.float64, device=C.device)
    dec = torch.empty(max(k, 1), dtype=torch.uint8, device=C.device)
    _check(_lib.fpc_level_series(ctx.handle, _t_ptr(C), _dtype_code(C), C.shape[0], int(n), int(l), int(i), int(j),
                                 _np_ptr(cand) if cand.size else None, cand.size, int(rank_lo), int(rank_hi),
                                 int(kernel), int(ranks_per_wave), int(pair_table), float(q), float(band_z),
                                 float(c_err), float(ill_cond_tau), _t_ptr(r), _t_ptr(dec)), "fpc_level_series")
    return r[:k], dec[:k]


def fpc_mlp_bytes() -> int:
    return int(_lib.fpc_mlp_bytes())


def fpc_mlp_params() -> int:
    return int(_lib.fpc_mlp_params())


def fpc_mlp_init(ctx: Context, params: np.ndarray, model=None):
    """A device model buffer (torch uint8 tensor) holding ``params`` (FP32)."""
    import torch

    params = np.ascontiguousarray(params, dtype=np.float32)
    assert params.size == fpc_mlp_params()
    if model is None:
        model = torch.empty(fpc_mlp_bytes(), dtype=torch.uint8, device=f"cuda:{ctx.device}")
    _check(_lib.fpc_mlp_init(ctx.handle, _t_ptr(model), _np_ptr(params)), "fpc_mlp_init")
    return model


def fpc_mlp_get(ctx: Context, model) -> np.ndarray:
    out = np.empty(fpc_mlp_params(), dtype=np.float32)
    _check(_lib.fpc_mlp_get(ctx.handle, _t_ptr(model), _np_ptr(out)), "fpc_mlp_get")
    return out


def fpc_mlp_forward(ctx: Context, X, model):
    import torch

    X = X.contiguous()
    out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(_lib.fpc_mlp_forward(ctx.handle, _t_ptr(X), X.shape[0], _t_ptr(model), _t_ptr(out)), "fpc_mlp_forward")
    return out


def fpc_mlp_grad(ctx: Context, X, y, model):
    """(gradient of the mean BCE loss (FP32 vector), loss)."""
    import torch

    X, y = X.contiguous(), y.contiguous()
    out = torch.empty(fpc_mlp_params() + 1, dtype=torch.float32, device=X.device)
    _check(_lib.fpc_mlp_grad(ctx.handle, _t_ptr(X), _t_ptr(y), X.shape[0], _t_ptr(model), _t_ptr(out)),
           "fpc_mlp_grad")
    g = out.cpu().numpy()
    return g[:-1], float(g[-1])


def fpc_mlp_train_step(ctx: Context, X, y, model, lr: float) -> float:
    X, y = X.contiguous(), y.contiguous()
    loss = ctypes.c_float()
    _check(_lib.fpc_mlp_train_step(ctx.handle, _t_ptr(X), _t_ptr(y), X.shape[0], _t_ptr(model), float(lr),
                                   ctypes.byref(loss)), "fpc_mlp_train_step")
    return float(loss.value)


def fpc_skeleton(ctx: Context, X, alpha: float = 0.01, max_level: int = -1, precision: int = FPC_PREC_FP64,
                 recheck_margin: float = 1e-3, schedule: int = FPC_REVERSE, max_tests: int = 0,
                 q_override: float = float("nan"), flags: int = 0, order_model=None, ill_cond_tau: float = 1e-4,
                 c32_method: int = FPC_CORR_BF16X6, stop_after_levels: int = 0, resume: dict | None = None) -> dict:
    """Skeleton and separating sets of the data X (torch tensor on the
    device, or a host numpy array), n x p row-major.

    stop_after_levels > 0 returns at the level boundary after that many
    levels of this call (result["next_level"] >= 0 if the run is not
    complete); resume continues from such a result (or one loaded with
    load_checkpoint) on the same data and parameters."""
    prm = fpc_params()
    keep = X
    if isinstance(X, np.ndarray):
        keep = np.ascontiguousarray(X)
        n, p = keep.shape
        prm.X = _np_ptr(keep)
        prm.x_dtype = FPC_F64 if keep.dtype == np.float64 else FPC_F32
        if keep.dtype not in (np.float64, np.float32):
            raise TypeError(keep.dtype)
        prm.x_on_device = 0
    else:
        keep = X.contiguous()
        n, p = keep.shape
        prm.X = _t_ptr(keep).value
        prm.x_dtype = _dtype_code(keep)
        prm.x_on_device = 1
    prm.n, prm.p = n, p
    prm.alpha = float(alpha)
    prm.max_level = int(max_level)
    prm.precision = int(precision)
    prm.recheck_margin = float(recheck_margin)
    prm.schedule = int(schedule)
    prm.order = FPC_ORDER_LEX if order_model is None else FPC_ORDER_LEARNED
    prm.order_model = None if order_model is None else _t_ptr(order_model).value
    prm.max_tests = int(max_tests)
    prm.q_override = float(q_override)
    prm.flags = int(flags)
    prm.ill_cond_tau = float(ill_cond_tau)
    prm.c32_method = int(c32_method)
    prm.stop_after_levels = int(stop_after_levels)
    if resume is not None:
        ck, ck_keep = _checkpoint(resume)
        prm.resume = ctypes.cast(ctypes.pointer(ck), ctypes.c_void_p)
    res = ctypes.POINTER(fpc_result)()
    _check(_lib.fpc_skeleton(ctx.handle, ctypes.byref(prm), ctypes.byref(res)), "fpc_skeleton")
    return _unpack(res)


_CK_ARRAYS = (("adj", np.uint8), ("sep_level", np.int32), ("sep_kind", np.int8), ("sep_off", np.int64),
              ("sep_nodes", np.int32))


def _checkpoint(state: dict):
    """A fpc_checkpoint over the arrays of a result (or loaded) dict, and
    the arrays it borrows."""
    arrs = {k: np.ascontiguousarray(state[k], dtype=t) for k, t in _CK_ARRAYS}
    lv = state["levels"]
    levels = (fpc_level_stats * max(len(lv), 1))()
    for k, x in enumerate(lv):
        for f, _ in fpc_level_stats._fields_:
            setattr(levels[k], f, x[f])
    ck = fpc_checkpoint()
    ck.p = int(state["p"])
    ck.next_level = int(state["next_level"])
    for k, _ in _CK_ARRAYS:
        setattr(ck, k, arrs[k].ctypes.data if arrs[k].size else None)
    ck.n_levels = len(lv)
    ck.levels = ctypes.cast(levels, ctypes.c_void_p)
    return ck, (arrs, levels)


def fpc_checkpoint_of(res: dict) -> dict:
    """The level-boundary state of a fpc_skeleton result (views of its
    arrays), as fpc_checkpoint_of fills a fpc_checkpoint; fpc_skeleton(...,
    resume=) takes it."""
    out = {k: res[k] for k, _ in _CK_ARRAYS}
    out.update(p=res["p"], next_level=res["next_level"], levels=res["levels"])
    return out


def save_checkpoint(path: str, res: dict) -> None:
    """Writes the level-boundary state of a fpc_skeleton result (plain
    arrays, no pickled objects) for load_checkpoint."""
    lv = res["levels"]
    fi = [f for f, t in fpc_level_stats._fields_ if t is not ctypes.c_double]
    fd = [f for f, t in fpc_level_stats._fields_ if t is ctypes.c_double]
    si = np.array([[x[f] for f in fi] for x in lv], dtype=np.int64).reshape(len(lv), len(fi))
    sd = np.array([[x[f] for f in fd] for x in lv], dtype=np.float64).reshape(len(lv), len(fd))
    np.savez(path, p=np.int64(res["p"]), next_level=np.int64(res["next_level"]), level_int=si, level_double=sd,
             **{k: np.asarray(res[k]) for k, _ in _CK_ARRAYS})


def load_checkpoint(path: str) -> dict:
    """The state written by save_checkpoint, as a dict fpc_skeleton(...,
    resume=) takes."""
    with np.load(path, allow_pickle=False) as z:
        out = {k: z[k].copy() for k, _ in _CK_ARRAYS}
        out["p"] = int(z["p"])
        out["next_level"] = int(z["next_level"])
        fi = [f for f, t in fpc_level_stats._fields_ if t is not ctypes.c_double]
        fd = [f for f, t in fpc_level_stats._fields_ if t is ctypes.c_double]
        out["levels"] = [dict({f: int(a[c]) for c, f in enumerate(fi)}, **{f: float(b[c]) for c, f in enumerate(fd)})
                         for a, b in zip(z["level_int"], z["level_double"])]
    return out


def fpc_skeleton_batch(ctx: Context, instances, alpha: float = 0.01, max_level: int = -1,
                       precision: int = FPC_PREC_FP64, recheck_margin: float = 1e-3, max_tests: int = 0,
                       q_override: float = float("nan"), flags: int = 0, ill_cond_tau: float = 1e-4,
                       c32_method: int = FPC_CORR_BF16X6) -> list:
    """Skeletons of several instances in one call.  ``instances`` is a
    sequence of (X, rows): X a device tensor (x_rows x p, one dtype for
    all), rows None (the instance is X itself) or a device int32 tensor of
    row indices into X (a resample).  Returns one result dict per
    instance, as fpc_skeleton."""
    keep = []
    arr = (fpc_instance * len(instances))()
    dt = None
    for k, (X, rows) in enumerate(instances):
        X = X.contiguous()
        keep.append(X)
        if dt is None:
            dt = _dtype_code(X)
        elif _dtype_code(X) != dt:
            raise TypeError("every instance must have the same dtype")
        arr[k].p = X.shape[1]
        arr[k].X = _t_ptr(X).value
        arr[k].x_rows = X.shape[0]
        if rows is None:
            arr[k].n = X.shape[0]
            arr[k].rows = None
        else:
            rows = rows.contiguous()
            keep.append(rows)
            if str(rows.dtype) != "torch.int32":
                raise TypeError("rows must be int32")
            arr[k].n = rows.shape[0]
            arr[k].rows = _t_ptr(rows).value
    prm = fpc_params()
    prm.x_dtype = dt if dt is not None else FPC_F32
    prm.x_on_device = 1
    prm.alpha = float(alpha)
    prm.max_level = int(max_level)
    prm.precision = int(precision)
    prm.recheck_margin = float(recheck_margin)
    prm.schedule = FPC_REVERSE
    prm.order = FPC_ORDER_LEX
    prm.max_tests = int(max_tests)
    prm.q_override = float(q_override)
    prm.flags = int(flags)
    prm.ill_cond_tau = float(ill_cond_tau)
    prm.c32_method = int(c32_method)
    outs = (ctypes.POINTER(fpc_result) * max(len(instances), 1))()
    _check(_lib.fpc_skeleton_batch(ctx.handle, ctypes.byref(prm), len(instances), arr, outs), "fpc_skeleton_batch")
    owners = [_Owner(ctypes.cast(outs[k], ctypes.POINTER(fpc_result))) for k in range(len(instances))]
    return [_unpack(o.ptr, o) for o in owners]


class SepSets(Mapping):
    """Read-only {(i, j): sorted separating set} over the LIST-kind pairs.
    ``idx`` holds their pair indices in increasing order and ``off`` the
    offsets of their sets in ``nodes`` (the library stores the LIST sets in
    pair order, each as long as its level); the pair map is built lazily."""

    def __init__(self, p, idx, off, nodes):
        self._p, self._idx, self._off, self._nodes = p, idx, off, nodes
        self._map = None

    def _pairs(self):
        if self._map is None:
            p = self._p
            k = self._idx
            # inverse of k = i*p - i*(i+1)/2 + (j - i - 1)
            i = np.floor(((2 * p - 1) - np.sqrt((2 * p - 1) ** 2 - 8.0 * k)) / 2).astype(np.int64)
            i -= (i * p - i * (i + 1) // 2 > k)
            i += ((i + 1) * p - (i + 1) * (i + 2) // 2 <= k)
            j = k - (i * p - i * (i + 1) // 2) + i + 1
            self._map = {(int(a), int(b)): t for t, (a, b) in enumerate(zip(i.tolist(), j.tolist()))}
        return self._map

    def __getitem__(self, key):
        t = self._pairs()[key]
        return self._nodes[self._off[t]:self._off[t + 1]].tolist()

    def __iter__(self):
        return iter(self._pairs())

    def __len__(self):
        return len(self._idx)


class _Owner:
    """Holds one fpc_result and frees it once no array viewing its buffers
    is left (the arrays keep their owner alive)."""

    __slots__ = ("ptr",)

    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        lib = _lib
        if lib is not None and self.ptr:
            lib.fpc_result_free(self.ptr)
            self.ptr = None


def _view(field, ctype, dtype, n: int, owner: _Owner) -> np.ndarray:
    """numpy view of n elements of a result buffer, without a copy."""
    addr = ctypes.cast(field, ctypes.c_void_p).value
    if n <= 0 or not addr:
        return np.zeros(0, dtype)
    buf = (ctype * n).from_address(addr)
    buf._owner = owner
    return np.frombuffer(buf, dtype=dtype)


def _unpack(res, owner: _Owner | None = None) -> dict:
    """Result dict over the buffers of a POINTER(fpc_result); the buffers
    are freed when the last array taken from them is."""
    if owner is None:
        owner = _Owner(res)
    r = res.contents
    p = r.p
    P = p * (p - 1) // 2
    adj = _view(r.adj, ctypes.c_uint8, np.uint8, p * p, owner).reshape(p, p)
    lev = _view(r.sep_level, ctypes.c_int32, np.int32, P, owner)
    kind = _view(r.sep_kind, ctypes.c_int8, np.int8, P, owner)
    sep_off = _view(r.sep_off, ctypes.c_int64, np.int64, P + 1, owner)
    tot = int(sep_off[P])
    nodes = _view(r.sep_nodes, ctypes.c_int32, np.int32, tot, owner)
    idx = _view(r.list_pairs, ctypes.c_int64, np.int64, int(r.n_lists), owner)
    off = np.empty(len(idx) + 1, np.int64)
    off[:-1] = sep_off[idx]
    off[-1] = tot
    sepsets = SepSets(p, idx, off, nodes)
    levels = []
    for k in range(r.n_levels):
        s = r.levels[k]
        levels.append({f: getattr(s, f) for f, _ in fpc_level_stats._fields_})
    nlog = int(r.log_rows)
    log = None
    if nlog:
        log = dict(x=_view(r.log_x, ctypes.c_float, np.float32, nlog * 3, owner).reshape(nlog, 3),
                   y=_view(r.log_y, ctypes.c_uint8, np.uint8, nlog, owner),
                   group=_view(r.log_group, ctypes.c_int32, np.int32, nlog, owner),
                   level=_view(r.log_level, ctypes.c_int32, np.int32, nlog, owner))
    return dict(adj=adj, sep_level=lev, sep_kind=kind, sep_off=sep_off, sepsets=sepsets, sep_nodes=nodes,
                   levels=levels, log=log,
                   total_tests=int(r.total_tests), total_required=sum(x["tests_required"] for x in levels),
                   q=float(r.q), corr_ms=float(r.corr_ms),
                   first_level_ms=float(r.first_level_ms), total_ms=float(r.total_ms),
                   corr_max_abs_err=float(r.corr_max_abs_err), p=p, next_level=int(r.next_level))


def sepset_of(res: dict, i: int, j: int):
    """Recorded separating set of (i, j) from a fpc_skeleton result, or None."""
    if i > j:
        i, j = j, i
    p = res["p"]
    k = i * p - i * (i + 1) // 2 + (j - i - 1)
    kind = int(res["sep_kind"][k])
    if kind == FPC_SEP_NONE:
        return None
    if kind == FPC_SEP_ALL_BUT:
        return [v for v in range(p) if v not in (i, j)]
    return list(res["sepsets"][(i, j)])


def tests_per_second(res: dict) -> float:
    """Executed CI tests of the levels after the first / their kernel time."""
    lv = res["levels"][1:] if res["levels"] and res["levels"][0]["level"] == res["p"] - 2 else res["levels"]
    t = sum(x["kernel_ms"] for x in lv) / 1e3
    n = sum(x["tests_executed"] for x in lv)
    return n / t if t > 0 else math.nan
