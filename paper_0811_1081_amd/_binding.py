"""ctypes binding of ``libgspca.so`` (the C ABI declared in ``include/gspca.h``).

Argument marshalling only: PyTorch supplies device memory and the stream,
every step of the fit runs in the library's HIP kernels.  The binding refuses
to run when the library is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgspca.so")

# gspca_status
OK, NOT_CONVERGED, EINVAL, EWORKSPACE, EDEVICE, ENONFINITE, ENOMEM = 0, 1, -1, -2, -3, -4, -5
# gspca_dtype / gspca_algo / gspca_init / gspca_stop
F64, F32, BF16, FP8_E4M3 = 0, 1, 2, 3
STOP_SIGMA_REL, STOP_LOADING = 0, 1
GS, NIPALS = 0, 1
INIT_MAXNORM, INIT_COLUMN_K, INIT_GIVEN = 0, 1, 2

EXPORTS = (
    "gspca_default_options", "gspca_workspace_bytes", "gspca_fit_ex", "gspca_fit",
    "gspca_fit_f32", "gspca_status_string", "gspca_version", "gspca_quantized_bytes",
    "gspca_quantize", "gspca_batched_workspace_bytes", "gspca_batched_prepare",
    "gspca_batched_launch", "gspca_batched_tune",
    "gspca_noalloc_scratch_bytes", "gspca_fit_noalloc",
    # gspca_ws.h (learned warm start)
    "gspca_mlp_param_count", "gspca_mlp_workspace_bytes", "gspca_sketch",
    "gspca_sketch_workspace_bytes", "gspca_sketch_refine",
    "gspca_whiten_sketch",
    "gspca_mlp_sync", "gspca_mlp_forward", "gspca_mlp_loss_grad", "gspca_mlp_adam",
    "gspca_ws_predict",
    # gspca_block.h (block iteration)
    "gspca_block_workspace_bytes", "gspca_fit_block",
)

WS_RANK = 32  # GSPCA_WS_RANK (network input width)
WS_RMAX = 64  # GSPCA_WS_RMAX (widest sketch)


class Problem(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64),
                ("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("col_scale", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("init", ctypes.c_int32),
                ("implicit_deflation", ctypes.c_int32), ("stop", ctypes.c_int32),
                ("T0", ctypes.c_void_p),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("replay_iters", ctypes.c_void_p), ("replay_start_col", ctypes.c_void_p),
                ("profile", ctypes.c_void_p), ("reorth", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("pass_ms", ctypes.c_double), ("pass_launches", ctypes.c_int64),
                ("gemv_t_ms", ctypes.c_double), ("gemv_n_ms", ctypes.c_double),
                ("gemv_t_launches", ctypes.c_int64), ("gemv_n_launches", ctypes.c_int64),
                ("iterations", ctypes.c_int64), ("bytes_per_pass", ctypes.c_int64),
                ("single_pass", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchProblem(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("M", ctypes.c_int64),
                ("N", ctypes.c_int64), ("K", ctypes.c_int64), ("T", ctypes.c_void_p),
                ("P", ctypes.c_void_p), ("lambda_", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("iters", ctypes.c_void_p), ("start_col", ctypes.c_void_p),
                ("replay_iters", ctypes.c_void_p), ("replay_start_col", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("T0", ctypes.c_void_p)]


class BatchPlan(ctypes.Structure):
    _fields_ = [("opaque", ctypes.c_ubyte * 256)]


class Mlp(ctypes.Structure):
    _fields_ = [("d0", ctypes.c_int32), ("d1", ctypes.c_int32), ("d2", ctypes.c_int32),
                ("d3", ctypes.c_int32), ("theta", ctypes.c_void_p), ("theta_bf16", ctypes.c_void_p),
                ("grad", ctypes.c_void_p), ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p),
                ("step", ctypes.c_int32), ("pad", ctypes.c_int32)]


class BlockOptions(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("stop", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tol", ctypes.c_double),
                ("Omega", ctypes.c_void_p), ("Z0", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("T", ctypes.c_void_p), ("P", ctypes.c_void_p), ("lambda_", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p), ("iters", ctypes.c_void_p),
                ("start_col", ctypes.c_void_p)]


_lock = threading.Lock()
_lib = None


class LibraryMissing(RuntimeError):
    pass


def load() -> ctypes.CDLL:
    """Load libgspca.so (torch is imported first so that one HIP runtime is used)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                "libgspca.so is not built (%s); run `python -m paper_0811_1081_amd.build`" % LIB_PATH)
        import torch  # noqa: F401  (loads the HIP runtime the library links against)
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.gspca_default_options.restype = None
        L.gspca_default_options.argtypes = [ctypes.POINTER(Options)]
        L.gspca_workspace_bytes.restype = ctypes.c_size_t
        L.gspca_workspace_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options)]
        L.gspca_fit_ex.restype = ctypes.c_int
        L.gspca_fit_ex.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                   ctypes.POINTER(Result), vp, ctypes.c_size_t, vp]
        L.gspca_fit_noalloc.restype = ctypes.c_int
        L.gspca_fit_noalloc.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                        ctypes.POINTER(Result), vp]
        L.gspca_noalloc_scratch_bytes.restype = ctypes.c_size_t
        L.gspca_noalloc_scratch_bytes.argtypes = []
        L.gspca_fit.restype = ctypes.c_int
        L.gspca_fit.argtypes = [vp, i64, i64, i64, dbl, i32, vp, vp, vp, vp]
        L.gspca_fit_f32.restype = ctypes.c_int
        L.gspca_fit_f32.argtypes = [vp, i64, i64, i64, dbl, i32, vp, vp, vp, vp]
        L.gspca_status_string.restype = ctypes.c_char_p
        L.gspca_status_string.argtypes = [ctypes.c_int]
        L.gspca_version.restype = ctypes.c_int
        L.gspca_version.argtypes = []
        L.gspca_quantized_bytes.restype = ctypes.c_size_t
        L.gspca_quantized_bytes.argtypes = [i64, i64, i32]
        L.gspca_quantize.restype = ctypes.c_int
        L.gspca_quantize.argtypes = [vp, i64, i64, i64, i32, vp, vp, vp, ctypes.c_size_t, vp]
        L.gspca_batched_workspace_bytes.restype = ctypes.c_size_t
        L.gspca_batched_workspace_bytes.argtypes = [ctypes.POINTER(BatchProblem), i32]
        L.gspca_batched_prepare.restype = ctypes.c_int
        L.gspca_batched_prepare.argtypes = [ctypes.POINTER(BatchProblem), i32,
                                            ctypes.POINTER(Options), vp, ctypes.c_size_t,
                                            ctypes.POINTER(BatchPlan), vp]
        L.gspca_batched_launch.restype = ctypes.c_int
        L.gspca_batched_launch.argtypes = [ctypes.POINTER(BatchPlan), vp]
        L.gspca_batched_tune.restype = ctypes.c_int
        L.gspca_batched_tune.argtypes = [ctypes.POINTER(BatchPlan), vp]
        sz, flt, mlp = ctypes.c_size_t, ctypes.c_float, ctypes.POINTER(Mlp)
        for name, res, args in (
                ("gspca_mlp_param_count", i64, [i32, i32, i32, i32]),
                ("gspca_mlp_workspace_bytes", sz, [mlp, i64, i32, i64]),
                ("gspca_sketch_workspace_bytes", sz, [i64, i64, i32]),
                ("gspca_sketch_refine", ctypes.c_int,
                 [vp, i64, i64, i64, vp, i32, vp, vp, vp, sz, vp]),
                ("gspca_sketch", ctypes.c_int, [vp, i64, i64, i64, vp, i32, vp, vp]),
                ("gspca_whiten_sketch", ctypes.c_int, [vp, i64, i32, vp, vp, vp, vp, sz, vp]),
                ("gspca_mlp_sync", ctypes.c_int, [mlp, vp]),
                ("gspca_mlp_forward", ctypes.c_int, [mlp, vp, i64, vp, vp, sz, vp]),
                ("gspca_mlp_loss_grad", ctypes.c_int, [mlp, vp, vp, i32, i64, vp, vp, sz, vp]),
                ("gspca_mlp_adam", ctypes.c_int, [mlp, flt, flt, flt, flt, vp]),
                ("gspca_ws_predict", ctypes.c_int,
                 [mlp, vp, i64, i64, i64, vp, i32, i32, vp, vp, sz, vp]),
                ("gspca_block_workspace_bytes", sz, [i64, i64, i32]),
                ("gspca_fit_block", ctypes.c_int,
                 [vp, i64, i64, i64, i64, ctypes.POINTER(BlockOptions), vp, vp, vp, vp,
                  ctypes.POINTER(i32), vp, sz, vp])):
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return L


def status_string(st: int) -> str:
    return load().gspca_status_string(int(st)).decode()


class GspcaError(RuntimeError):
    def __init__(self, status: int):
        super().__init__("gspca: %s (%d)" % (status_string(status), status))
        self.status = status
