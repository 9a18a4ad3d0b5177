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
from ._binding import (BF16, EDEVICE, EINVAL, ENOMEM, ENONFINITE, EWORKSPACE, F32, F64,  # noqa: F401
                       FP8_E4M3, GS, INIT_COLUMN_K, INIT_GIVEN, INIT_MAXNORM, NIPALS,
                       NOT_CONVERGED, OK, STOP_LOADING, STOP_SIGMA_REL, GspcaError,
                       LibraryMissing, Profile, status_string)

__all__ = ["fit", "fit_block", "quantize", "Quantized", "Batch", "workspace_bytes", "column_major",
           "status_string", "GspcaError", "LibraryMissing", "Profile", "load"]

_ALGOS = {"gs": GS, "nipals": NIPALS}
_INITS = {"maxnorm": INIT_MAXNORM, "column_k": INIT_COLUMN_K, "given": INIT_GIVEN}
_STOPS = {"sigma": STOP_SIGMA_REL, "loading": STOP_LOADING}
_REORTHS = {"cgs": 0, "cgs2": 1, "mgs": 2}
_FMTS = {"bf16": BF16, "e4m3": FP8_E4M3}


class Quantized:
    """X stored as BF16 or FP8 (E4M3) codes in the library's row-panel layout
    with per-column FP32 scales (see gspca_quantize in include/gspca.h)."""

    def __init__(self, codes, scale, M, N, fmt):
        self.codes, self.scale, self.shape, self.fmt = codes, scale, (M, N), fmt
        self.device = codes.device
        self.dtype_code = _FMTS[fmt]


def quantize(X, fmt="bf16", stream=None) -> Quantized:
    """Quantise a column-major FP32 device matrix to BF16 or E4M3 codes."""
    import torch
    L = _b.load()
    if X.dtype != torch.float32 or not X.is_cuda or X.dim() != 2 or X.stride(0) != 1:
        raise ValueError("X must be a column-major float32 device matrix")
    M, N = X.shape
    code = _FMTS[fmt]
    nbytes = int(L.gspca_quantized_bytes(M, N, code))
    if nbytes == 0:
        raise GspcaError(EINVAL)
    Q = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
    scale = torch.empty(N, dtype=torch.float32, device=X.device)
    scratch = torch.empty(256, dtype=torch.uint8, device=X.device)
    if stream is None:
        stream = torch.cuda.current_stream(X.device)
    st = int(L.gspca_quantize(X.data_ptr(), M, N, X.stride(1), code, Q.data_ptr(),
                              scale.data_ptr(), scratch.data_ptr(), 256, ctypes_stream(stream)))
    if st != OK:
        raise GspcaError(st)
    return Quantized(Q, scale, M, N, fmt)


def load():
    """Load the HIP library (raises LibraryMissing when it is not built)."""
    return _b.load()


def column_major(A, align=1):
    """Column-major (Fortran-ordered) copy of a 2-D tensor on the same device,
    with the leading dimension rounded up to a multiple of `align` elements
    (padding rows are left unset and never read).  align=32 gives FP32
    columns that start on 128-byte boundaries: the batched kernel's row tiles
    then read whole cache lines (2048-problem batch: 104.5 -> 95.3 ms)."""
    import torch
    M, N = A.shape
    if align < 1:
        raise ValueError("align must be >= 1")
    ld = -(-M // align) * align
    out = torch.empty_strided((M, N), (1, ld), dtype=A.dtype, device=A.device)
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
    if isinstance(X, Quantized):
        M, N = X.shape
        return _b.Problem(X.dtype_code, X.codes.data_ptr(), M, M, N, int(K), X.scale.data_ptr())
    if X.dim() != 2:
        raise ValueError("X must be 2-D")
    M, N = X.shape
    if X.stride(0) != 1 or X.stride(1) < max(M, 1):
        raise ValueError("X must be column-major (stride (1, ldx), ldx >= M); use column_major(X)")
    return _b.Problem(_dtype_code(X), X.data_ptr(), X.stride(1), M, N, int(K), None)


def _options(algo, init, tol, max_iter, T0=None, replay_iters=None, replay_start=None,
             implicit=False, stop="sigma", reorth="cgs"):
    o = _b.Options()
    o.reorth = _REORTHS[reorth]
    o.algo = _ALGOS[algo]
    o.init = _INITS[init]
    o.implicit_deflation = 1 if implicit else 0
    o.stop = _STOPS[stop]
    o.T0 = T0.data_ptr() if T0 is not None else None
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.replay_iters = replay_iters.data_ptr() if replay_iters is not None else None
    o.replay_start_col = replay_start.data_ptr() if replay_start is not None else None
    return o


def workspace_bytes(X, K, algo="gs", init="maxnorm", tol=1e-7, max_iter=10000,
                    implicit=False, stop="sigma", reorth="cgs") -> int:
    L = _b.load()
    pr = _problem(X, K)
    op = _options(algo, init, tol, max_iter, implicit=implicit or isinstance(X, Quantized),
                  stop=stop, reorth=reorth)
    return int(L.gspca_workspace_bytes(pr, op))


def _workspace(nbytes, device):
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


def fit(X, K, tol=1e-7, max_iter=10000, algo="gs", init="maxnorm", T0=None,
        replay_iters=None, replay_start=None, workspace=None, stream=None, check=True,
        profile=None, implicit=False, stop="sigma", reorth="cgs", noalloc=False):
    """Fit K components of the column-major device matrix X (M x N).

    Returns a dict of device tensors: T (M x K), P (N x K) (column-major, dtype
    of X), lambda and sigma (float64, K), iters and start_col (int32, K), and
    the integer ``status``.  ``replay_iters`` / ``replay_start`` (int32 device
    tensors of length K) force each component's iteration count and start
    column.  ``implicit`` selects implicit deflation (X is never modified,
    GS-PCA only; always on for a Quantized X, whose outputs are float32).
    ``stop`` is "sigma" (the paper's relative test) or "loading" (the unit
    loading moved less than tol).  ``reorth`` is the form of GS-PCA's
    Gram-Schmidt steps: "cgs" (one classical pass, the paper's), "cgs2" (two
    passes) or "mgs" (modified); the last two need explicit deflation and
    F32/F64 data.  ``noalloc`` runs gspca_fit_noalloc: the library's fixed
    per-GPU scratch array is the workspace (no device allocation beyond the
    outputs; no replay, profile or ``workspace``).  Raises GspcaError on a
    negative status when ``check``."""
    import torch
    L = _b.load()
    quant = isinstance(X, Quantized)
    if not quant and not X.is_cuda:
        raise ValueError("X must be a device tensor")
    M, N = X.shape
    K = int(K)
    dev = X.device
    out_dtype = torch.float32 if quant else X.dtype
    implicit = implicit or quant
    if T0 is not None and (T0.dtype != out_dtype or T0.device != dev or tuple(T0.shape) != (M, K)
                           or T0.stride(0) != 1 or T0.stride(1) != M):
        raise ValueError("T0 must be a column-major (M, K) tensor of the output dtype and device")
    for name, a in (("replay_iters", replay_iters), ("replay_start", replay_start)):
        if a is not None and (a.dtype != torch.int32 or a.device != dev or a.numel() != K
                              or not a.is_contiguous()):
            raise ValueError(name + " must be a contiguous int32 device tensor of length K")
    pr = _problem(X, K)
    op = _options(algo, init, tol, max_iter, T0, replay_iters, replay_start, implicit, stop,
                  reorth)
    if profile is not None:
        op.profile = ctypes.addressof(profile)
    T = torch.empty_strided((M, K), (1, M), dtype=out_dtype, device=dev)
    P = torch.empty_strided((N, K), (1, N), dtype=out_dtype, device=dev)
    lam = torch.empty(K, dtype=torch.float64, device=dev)
    sig = torch.empty(K, dtype=torch.float64, device=dev)
    iters = torch.empty(K, dtype=torch.int32, device=dev)
    start = torch.empty(K, dtype=torch.int32, device=dev)
    res = _b.Result(T.data_ptr(), P.data_ptr(), lam.data_ptr(), sig.data_ptr(),
                    iters.data_ptr(), start.data_ptr())
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    if noalloc:
        if workspace is not None:
            raise ValueError("noalloc takes no workspace")
        with torch.cuda.device(dev):
            st = int(L.gspca_fit_noalloc(pr, op, res, ctypes_stream(stream)))
        if check and st < 0:
            raise GspcaError(st)
        return {"T": T, "P": P, "lambda": lam, "sigma": sig, "iters": iters,
                "start_col": start, "status": st}
    nbytes = int(L.gspca_workspace_bytes(pr, op))
    if nbytes == 0:
        raise GspcaError(EINVAL)
    if workspace is None:
        _keep, wptr = _workspace(nbytes, dev)
    else:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise GspcaError(EWORKSPACE)
        wptr = workspace.data_ptr()
    st = int(L.gspca_fit_ex(pr, op, res, wptr, nbytes, ctypes_stream(stream)))
    if check and st < 0:
        raise GspcaError(st)
    return {"T": T, "P": P, "lambda": lam, "sigma": sig, "iters": iters, "start_col": start,
            "status": st}


def fit_block(X, K, r=64, Omega=None, Z0=None, tol=1e-6, max_iter=50, stop="sigma",
              stream=None, check=True):
    """Block iteration with Rayleigh-Ritz for the K leading components of the
    column-major FP32 device matrix X (gspca_block.h; not in the paper).

    ``r`` (32 or 64) is the block width; the start block is X @ Omega (Omega
    N x r, row-major float32 device tensor) or the given M x r row-major Z0.
    ``stop``: "sigma" (relative change of the K leading estimates) or
    "loading" (the unit Ritz vectors moved less than tol).
    Returns T, P (column-major float32), lambda, sigma (float64), the
    iteration count and the status."""
    import torch
    L = _b.load()
    if not X.is_cuda or X.dtype != torch.float32 or X.stride(0) != 1:
        raise ValueError("X must be a column-major float32 device matrix")
    M, N = X.shape
    K, r = int(K), int(r)
    for name, a, shape in (("Omega", Omega, (N, r)), ("Z0", Z0, (M, r))):
        if a is not None and (a.dtype != torch.float32 or not a.is_cuda or
                              tuple(a.shape) != shape or not a.is_contiguous()):
            raise ValueError("%s must be a contiguous (row-major) float32 device tensor %s"
                             % (name, shape))
    if Omega is None and Z0 is None:
        raise ValueError("give Omega or Z0")
    op = _b.BlockOptions(r, int(max_iter), _STOPS[stop], 0, float(tol),
                         Omega.data_ptr() if Omega is not None else None,
                         Z0.data_ptr() if Z0 is not None else None)
    dev = X.device
    T = torch.empty_strided((M, K), (1, M), dtype=torch.float32, device=dev)
    P = torch.empty_strided((N, K), (1, N), dtype=torch.float32, device=dev)
    lam = torch.empty(K, dtype=torch.float64, device=dev)
    sig = torch.empty(K, dtype=torch.float64, device=dev)
    nbytes = int(L.gspca_block_workspace_bytes(M, N, r))
    if nbytes == 0:
        raise GspcaError(EINVAL)
    _keep, wptr = _workspace(nbytes, dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    its = ctypes.c_int32(0)
    st = int(L.gspca_fit_block(X.data_ptr(), X.stride(1), M, N, K, op, T.data_ptr(),
                               P.data_ptr(), lam.data_ptr(), sig.data_ptr(), ctypes.byref(its),
                               wptr, nbytes, ctypes_stream(stream)))
    if check and st < 0:
        raise GspcaError(st)
    return {"T": T, "P": P, "lambda": lam, "sigma": sig, "iters": int(its.value), "status": st}


def ctypes_stream(stream):
    """Raw hipStream_t handle of a torch stream."""
    return stream.cuda_stream


class Batch:
    """Many independent FP32 GS-PCA problems fitted in one persistent launch.

        b = Batch([X0, X1, ...], K=[8, 8, ...], tol=1e-6)   # column-major cuda float32
        b.launch(); torch.cuda.synchronize()                # or capture launch() in a graph
        b.T[i], b.P[i], b.lam[i], b.iters[i], b.status

    Outputs are preallocated device tensors; every launch refits all problems."""

    def __init__(self, Xs, K, tol=1e-6, max_iter=1000, init="maxnorm", stop="sigma",
                 replay_iters=None, replay_start=None, T0=None, stream=None):
        import torch
        L = _b.load()
        n = len(Xs)
        Ks = list(K) if hasattr(K, "__len__") else [int(K)] * n
        self.Xs = Xs
        dev = Xs[0].device
        self.T, self.P, self.lam, self.sigma, self.iters, self.start_col = [], [], [], [], [], []
        self.status = torch.zeros(n, dtype=torch.int32, device=dev)
        arr = (_b.BatchProblem * n)()
        self._keep = [replay_iters, replay_start, T0]
        if (init == "given") != (T0 is not None):
            raise ValueError("init='given' needs T0 (one column-major (M, K) float32 per problem)")
        for i, X in enumerate(Xs):
            if X.dtype != torch.float32 or X.stride(0) != 1 or not X.is_cuda:
                raise ValueError("batched problems must be column-major float32 device matrices")
            M, N = X.shape
            k = int(Ks[i])
            T = torch.empty_strided((M, k), (1, M), dtype=torch.float32, device=dev)
            P = torch.empty_strided((N, k), (1, N), dtype=torch.float32, device=dev)
            lam = torch.empty(k, dtype=torch.float64, device=dev)
            sig = torch.empty(k, dtype=torch.float64, device=dev)
            it = torch.empty(k, dtype=torch.int32, device=dev)
            sc = torch.empty(k, dtype=torch.int32, device=dev)
            self.T.append(T); self.P.append(P); self.lam.append(lam); self.sigma.append(sig)
            self.iters.append(it); self.start_col.append(sc)
            ri = replay_iters[i].data_ptr() if replay_iters is not None else None
            rs = replay_start[i].data_ptr() if replay_start is not None else None
            t0 = None
            if T0 is not None:
                g = T0[i]
                if (g.dtype != torch.float32 or tuple(g.shape) != (M, k) or g.stride() != (1, M)
                        or g.device != dev):
                    raise ValueError("T0[%d] must be a column-major (M, K) float32 device tensor" % i)
                t0 = g.data_ptr()
            arr[i] = _b.BatchProblem(X.data_ptr(), X.stride(1), M, N, k, T.data_ptr(),
                                     P.data_ptr(), lam.data_ptr(), sig.data_ptr(), it.data_ptr(),
                                     sc.data_ptr(), ri, rs, self.status.data_ptr() + 4 * i, t0)
        self._arr = arr
        nbytes = int(L.gspca_batched_workspace_bytes(arr, n))
        if nbytes == 0:
            raise GspcaError(EINVAL)
        self._ws, wptr = _workspace(nbytes, dev)
        op = _options("gs", init, tol, max_iter, implicit=True, stop=stop)
        self.plan = _b.BatchPlan()
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        st = int(L.gspca_batched_prepare(arr, n, op, wptr, nbytes, self.plan,
                                         ctypes_stream(stream)))
        if st != OK:
            raise GspcaError(st)

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.Xs[0].device)
        st = int(_b.load().gspca_batched_launch(self.plan, ctypes_stream(stream)))
        if st != OK:
            raise GspcaError(st)

    def tune(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.Xs[0].device)
        st = int(_b.load().gspca_batched_tune(self.plan, ctypes_stream(stream)))
        if st != OK:
            raise GspcaError(st)

    def shape(self):
        """(threads per workgroup, workgroups per compute unit) of the current plan."""
        raw = bytes(self.plan.opaque)
        import struct
        # PlanImpl: magic(8) items(8) order(8) queue(8) nprob(4) threads(4) occ(4)
        nprob, threads, occ = struct.unpack_from("<iii", raw, 32)
        return threads, occ
