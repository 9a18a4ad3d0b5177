"""MI355X (gfx950) iterative PCA: GS-PCA and NIPALS-PCA on hand-written HIP kernels.

Python face of the C ABI in ``include/gspca.h``.  PyTorch tensors provide the
device memory and the stream; every step of a fit runs in ``libgspca.so``.

    import torch, paper_0811_1081_amd as gp
    out = gp.fit(X_cuda, K=16, tol=1e-10)      # X: (M, N) float32/float64 on cuda
    out["T"], out["P"], out["lambda"], out["iters"]

Method: Andrecut, arXiv:0811.1081, Sec. 2.2 (NIPALS-PCA) and Sec. 2.3 (GS-PCA).
"""
from __future__ import annotations

import ctypes

from . import _binding as _b
from ._binding import (Profile, EDEVICE, EINVAL, ENOMEM, ENONFINITE, EWORKSPACE, F32, F64, GS,  # noqa: F401
                       INIT_COLUMN_K, INIT_GIVEN, INIT_MAXNORM, NIPALS, NOT_CONVERGED, OK,
                       GspcaError, LibraryMissing, status_string)

__all__ = ["fit", "workspace_bytes", "column_major", "status_string", "GspcaError",
           "LibraryMissing", "load"]

_ALGOS = {"gs": GS, "nipals": NIPALS}
_INITS = {"maxnorm": INIT_MAXNORM, "column_k": INIT_COLUMN_K, "given": INIT_GIVEN}


def load():
    """Load the HIP library (raises LibraryMissing when it is not built)."""
    return _b.load()


def column_major(A):
    """Column-major (Fortran-ordered) copy of a 2-D tensor on the same device."""
    import torch
    M, N = A.shape
    out = torch.empty_strided((M, N), (1, M), dtype=A.dtype, device=A.device)
    out.copy_(A)
    return out


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("X must be float32 or float64, got %s" % t.dtype)


def _problem(X, K):
    if X.dim() != 2:
        raise ValueError("X must be 2-D")
    M, N = X.shape
    if X.stride(0) != 1 or X.stride(1) < max(M, 1):
        raise ValueError("X must be column-major (stride (1, ldx), ldx >= M); use column_major(X)")
    return _b.Problem(_dtype_code(X), X.data_ptr(), X.stride(1), M, N, int(K))


def _options(algo, init, tol, max_iter, T0=None, replay_iters=None, replay_start=None,
             implicit=False):
    o = _b.Options()
    o.algo = _ALGOS[algo]
    o.init = _INITS[init]
    o.implicit_deflation = 1 if implicit else 0
    o.T0 = T0.data_ptr() if T0 is not None else None
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.replay_iters = replay_iters.data_ptr() if replay_iters is not None else None
    o.replay_start_col = replay_start.data_ptr() if replay_start is not None else None
    return o


def workspace_bytes(X, K, algo="gs", init="maxnorm", tol=1e-7, max_iter=10000,
                    implicit=False) -> int:
    L = _b.load()
    pr = _problem(X, K)
    op = _options(algo, init, tol, max_iter, implicit=implicit)
    return int(L.gspca_workspace_bytes(pr, op))


def _workspace(nbytes, device):
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


def fit(X, K, tol=1e-7, max_iter=10000, algo="gs", init="maxnorm", T0=None,
        replay_iters=None, replay_start=None, workspace=None, stream=None, check=True,
        profile=None, implicit=False):
    """Fit K components of the column-major device matrix X (M x N).

    Returns a dict of device tensors: T (M x K), P (N x K) (column-major, dtype
    of X), lambda and sigma (float64, K), iters and start_col (int32, K), and
    the integer ``status``.  ``replay_iters`` / ``replay_start`` (int32 device
    tensors of length K) force each component's iteration count and start
    column.  ``implicit`` selects implicit deflation (X is never modified,
    GS-PCA only).  Raises GspcaError on a negative status when ``check``."""
    import torch
    L = _b.load()
    if not X.is_cuda:
        raise ValueError("X must be a device tensor")
    M, N = X.shape
    K = int(K)
    dev = X.device
    if T0 is not None and (T0.dtype != X.dtype or T0.device != dev or tuple(T0.shape) != (M, K)
                           or T0.stride(0) != 1 or T0.stride(1) != M):
        raise ValueError("T0 must be a column-major (M, K) tensor of X's dtype and device")
    for name, a in (("replay_iters", replay_iters), ("replay_start", replay_start)):
        if a is not None and (a.dtype != torch.int32 or a.device != dev or a.numel() != K
                              or not a.is_contiguous()):
            raise ValueError(name + " must be a contiguous int32 device tensor of length K")
    pr = _problem(X, K)
    op = _options(algo, init, tol, max_iter, T0, replay_iters, replay_start, implicit)
    if profile is not None:
        op.profile = ctypes.addressof(profile)
    T = torch.empty_strided((M, K), (1, M), dtype=X.dtype, device=dev)
    P = torch.empty_strided((N, K), (1, N), dtype=X.dtype, device=dev)
    lam = torch.empty(K, dtype=torch.float64, device=dev)
    sig = torch.empty(K, dtype=torch.float64, device=dev)
    iters = torch.empty(K, dtype=torch.int32, device=dev)
    start = torch.empty(K, dtype=torch.int32, device=dev)
    res = _b.Result(T.data_ptr(), P.data_ptr(), lam.data_ptr(), sig.data_ptr(),
                    iters.data_ptr(), start.data_ptr())
    nbytes = int(L.gspca_workspace_bytes(pr, op))
    if nbytes == 0:
        raise GspcaError(EINVAL)
    if workspace is None:
        _keep, wptr = _workspace(nbytes, dev)
    else:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise GspcaError(EWORKSPACE)
        wptr = workspace.data_ptr()
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    st = int(L.gspca_fit_ex(pr, op, res, wptr, nbytes, ctypes_stream(stream)))
    if check and st < 0:
        raise GspcaError(st)
    return {"T": T, "P": P, "lambda": lam, "sigma": sig, "iters": iters, "start_col": start,
            "status": st}


def ctypes_stream(stream):
    """Raw hipStream_t handle of a torch stream."""
    return stream.cuda_stream
