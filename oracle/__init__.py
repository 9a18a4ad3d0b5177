"""FP64 CPU oracle for iterative PCA (NIPALS-PCA and GS-PCA) -- TEST INFRASTRUCTURE.

Only the test-suite, the package's ``smoke()`` check and the benchmark's
CPU-baseline leg may import this module.  The GPU library never does, and the
two share no code.  The arithmetic lives in plain C (``pca_oracle.c``,
``codec_oracle.c``); this module builds it with gcc on first use and marshals
numpy arrays to it.  See the header of ``pca_oracle.c`` for the paper passages
each routine follows (Andrecut, arXiv:0811.1081, Secs. 2.2-2.3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ("pca_oracle.c", "codec_oracle.c", "mlp_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]

ALGO_GS, ALGO_NIPALS = 0, 1
INIT_MAXNORM, INIT_COLUMN_K, INIT_GIVEN = 0, 1, 2
OK, NOT_CONVERGED, EINVAL, ENONFINITE = 0, 1, -1, -4
DBL_MIN = np.finfo(np.float64).tiny
FLT_MIN = float(np.finfo(np.float32).tiny)

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs)
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, *srcs, "-lm"], check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(LIB_PATH)
            i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
            vp = ctypes.c_void_p
            L.oracle_fit.restype = ctypes.c_int
            L.oracle_fit.argtypes = [ctypes.c_int, ctypes.c_int, vp, i64, i64, i64, i64, dbl, i32,
                                     ctypes.c_int, vp, vp, vp, dbl, ctypes.c_int, ctypes.c_int,
                                     vp, vp, vp, vp, vp, vp]
            L.oracle_gs_step.restype = ctypes.c_int
            L.oracle_gs_step.argtypes = [vp, i64, i64, vp, ctypes.c_int]
            L.oracle_score_step.restype = ctypes.c_int
            L.oracle_score_step.argtypes = [vp, i64, i64, i64, i64, vp, vp, vp, vp, vp, vp]
            L.oracle_jacobi_eig.restype = ctypes.c_int
            L.oracle_jacobi_eig.argtypes = [vp, i64, vp, vp]
            L.oracle_bf16_encode.restype = ctypes.c_uint16
            L.oracle_bf16_encode.argtypes = [ctypes.c_float]
            L.oracle_bf16_decode.restype = ctypes.c_float
            L.oracle_bf16_decode.argtypes = [ctypes.c_uint16]
            L.oracle_bf16_round.restype = None
            L.oracle_bf16_round.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
            L.oracle_e4m3_encode.restype = ctypes.c_uint8
            L.oracle_e4m3_encode.argtypes = [ctypes.c_float]
            L.oracle_e4m3_decode.restype = ctypes.c_double
            L.oracle_e4m3_decode.argtypes = [ctypes.c_uint8]
            L.oracle_quantize.restype = ctypes.c_int
            L.oracle_quantize.argtypes = [vp, i64, i64, i64, ctypes.c_int, vp, vp]
            L.oracle_dequantize.restype = ctypes.c_int
            L.oracle_dequantize.argtypes = [vp, vp, i64, i64, ctypes.c_int, vp]
            ci = ctypes.c_int
            L.oracle_mlp_forward.restype = None
            L.oracle_mlp_forward.argtypes = [vp, i64, ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, ci,
                                             ci, vp, vp, vp, vp]
            L.oracle_cos2_loss.restype = dbl
            L.oracle_cos2_loss.argtypes = [vp, vp, i64, ci, vp]
            L.oracle_mlp_backward.restype = None
            L.oracle_mlp_backward.argtypes = [vp, i64, ci, ci, ci, ci, vp, vp, vp, vp, vp, vp, ci,
                                              vp, vp, vp, vp, vp, vp, vp, vp]
            L.oracle_adam.restype = None
            L.oracle_adam.argtypes = [vp, vp, vp, vp, i64, dbl, dbl, dbl, dbl, ci]
            _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64_fortran(X):
    return np.asfortranarray(np.asarray(X, dtype=np.float64))


class Fit:
    """Result of one oracle fit: T (M x K), P (N x K), sigma, lam = sigma^2,
    iters, start_col, status, and R (residual) when requested."""

    def __init__(self, **kw):
        self.__dict__.update(kw)

    @property
    def V(self):
        """Normalised scores T / sigma (zero columns where sigma == 0)."""
        s = np.where(self.sigma > 0, self.sigma, 1.0)
        return self.T / s


def fit(X, K, tol=1e-10, max_iter=1000, algo="gs", implicit=False, init="maxnorm",
        T0=None, replay_iters=None, replay_start=None, tiny=DBL_MIN, want_R=False,
        stop="sigma", reorth="cgs") -> Fit:
    """Run NIPALS-PCA (algo='nipals') or GS-PCA (algo='gs') in FP64.

    ``stop`` is "sigma" (the relative test of the paper's programs) or
    "loading" (stop when the unit loading moved less than tol).  ``reorth``
    is the form of GS-PCA's two Gram-Schmidt steps: "cgs" (one classical
    pass, the paper's), "cgs2" (two classical passes) or "mgs" (modified).

    X is widened to float64 (an FP32 input is consumed exactly).  ``replay_iters``
    forces the number of iterations per component and ``replay_start`` the start
    column (entries < 0 fall back to ``init``)."""
    X = _f64_fortran(X)
    M, N = X.shape
    T = np.zeros((M, K), order="F")
    P = np.zeros((N, K), order="F")
    sigma = np.zeros(K)
    iters = np.zeros(K, dtype=np.int32)
    start = np.zeros(K, dtype=np.int32)
    R = np.zeros((M, N), order="F") if want_R else None
    algo_i = {"gs": ALGO_GS, "nipals": ALGO_NIPALS}[algo]
    init_i = {"maxnorm": INIT_MAXNORM, "column_k": INIT_COLUMN_K, "given": INIT_GIVEN}[init]
    T0a = _f64_fortran(T0) if T0 is not None else None
    ri = np.ascontiguousarray(replay_iters, dtype=np.int32) if replay_iters is not None else None
    rs = np.ascontiguousarray(replay_start, dtype=np.int32) if replay_start is not None else None
    st = lib().oracle_fit(algo_i, int(bool(implicit)), _ptr(X), M, N, M, K, float(tol),
                          int(max_iter), init_i, _ptr(T0a), _ptr(ri), _ptr(rs), float(tiny),
                          {"sigma": 0, "loading": 1}[stop], REORTH[reorth],
                          _ptr(T), _ptr(P), _ptr(sigma), _ptr(iters), _ptr(start), _ptr(R))
    return Fit(T=T, P=P, sigma=sigma, lam=sigma ** 2, iters=iters, start_col=start,
               status=st, R=R, algo=algo)


REORTH = {"cgs": 0, "cgs2": 1, "mgs": 2}


def gs_step(Q, x, reorth="cgs"):
    """One Gram-Schmidt step of x against the columns of Q in the chosen form
    (see ``fit``); returns the reduced vector."""
    Q = _f64_fortran(np.asarray(Q, dtype=np.float64).reshape(len(x), -1))
    xv = np.array(x, dtype=np.float64)
    st = lib().oracle_gs_step(_ptr(Q), Q.shape[0], Q.shape[1], _ptr(xv), REORTH[reorth])
    if st != OK:
        raise ValueError("oracle_gs_step failed: %d" % st)
    return xv


def score_step(X, k, V, sigma, P, p):
    """One GS-PCA score step on R_k = X - V diag(sigma) P^T (first k columns):
    returns (v, s) with s v = (I - V V^T) R_k p."""
    X = _f64_fortran(X)
    M, N = X.shape
    Vk = _f64_fortran(np.asarray(V)[:, :k]) if k > 0 else None
    Pk = _f64_fortran(np.asarray(P)[:, :k]) if k > 0 else None
    sk = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64)[:k]) if k > 0 else None
    pv = np.ascontiguousarray(p, dtype=np.float64)
    v = np.zeros(M)
    s = ctypes.c_double(0.0)
    st = lib().oracle_score_step(_ptr(X), M, N, M, k, _ptr(Vk), _ptr(sk), _ptr(Pk), _ptr(pv),
                                 _ptr(v), ctypes.byref(s))
    if st != OK:
        raise ValueError("oracle_score_step failed: %d" % st)
    return v, s.value


def jacobi_eig(A):
    """Eigen-decomposition of a symmetric matrix by cyclic Jacobi: (w desc, Q)."""
    A = _f64_fortran(A).copy(order="F")
    n = A.shape[0]
    w = np.zeros(n)
    Q = np.zeros((n, n), order="F")
    lib().oracle_jacobi_eig(_ptr(A), n, _ptr(w), _ptr(Q))
    return w, Q


def sketch_whiten(X, Omega, power=0):
    """Warm-start input rows (not in the paper): Y = X Omega, then the
    eigen-decomposition Y^T Y = Q diag(g) Q^T by cyclic Jacobi (g decreasing,
    each eigenvector's largest-magnitude entry made positive) and
    Z = sqrt(M) Y Q diag(g)^(-1/2); columns with g <= 0 are zero.  Each of the
    `power` refinement steps (one step of subspace iteration, Halko, Martinsson
    & Tropp 2011, Alg. 4.4) replaces Y by X (X^T Z / sqrt(M)) and whitens
    again.  FP64.  Returns (Y, Z, g) of the last step."""
    X = np.asarray(X, dtype=np.float64)
    Y = X @ np.asarray(Omega, dtype=np.float64)
    Z, g = whiten(Y)
    for _ in range(int(power)):
        Y = sketch_refine(X, Z)[1]
        Z, g = whiten(Y)
    return Y, Z, g


def sketch_refine(X, Z):
    """One refinement step on a whitened sketch Z (M x r): W = X^T Z / sqrt(M)
    (N x r) and Y = X W.  FP64.  Returns (W, Y)."""
    X = np.asarray(X, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    W = X.T @ Z / np.sqrt(X.shape[0])
    return W, X @ W


def whiten(Y):
    """The whitening half of sketch_whiten on a given sketch Y: (Z, g)."""
    Y = np.asarray(Y, dtype=np.float64)
    M = Y.shape[0]
    g, Q = jacobi_eig(Y.T @ Y)
    Q = np.array(Q)
    for c in range(Q.shape[1]):
        i = int(np.argmax(np.abs(Q[:, c])))
        if Q[i, c] < 0:
            Q[:, c] = -Q[:, c]
    scale = np.where(g > 0, np.sqrt(M) / np.sqrt(np.where(g > 0, g, 1.0)), 0.0)
    return (Y @ Q) * scale, g


def block_fit(X, K, Omega=None, Z0=None, tol=0.0, max_iter=10, stop="sigma"):
    """Block iteration with Rayleigh-Ritz (not in the paper; Halko, Martinsson
    & Tropp 2011, Alg. 4.4, orthonormalised by whitening), FP64, in the
    library's order of steps: V_0 from the whitened X Omega (or Z0); each
    iteration Y = X (X^T V), whitened (Ritz order; g the Ritz values of
    (X X^T)^2); stop when every s_i = g_i^(1/4), i < K, moved less than tol
    relatively, or (stop="loading") every unit Ritz vector v_i moved less
    than tol (|v_i - s v_i_prev|, s = +-1 aligning the signs); never for
    tol = 0.  Then w_i = X^T v_i, sigma_i = |w_i|,
    P = w / sigma, T = sigma v.  Returns (T, P, sigma, iterations, converged)."""
    X = np.asarray(X, dtype=np.float64)
    M = X.shape[0]
    if Z0 is not None:
        Z, g = whiten(Z0)
    else:
        Z, g = whiten(X @ np.asarray(Omega, dtype=np.float64))
    prev = np.zeros(K)
    it, conv = 0, False
    while it < max_iter:
        it += 1
        Zp = Z
        Z, g = whiten(sketch_refine(X, Z)[1])
        s = np.where(g[:K] > 0, g[:K], 0.0) ** 0.25
        if stop == "loading":
            c = np.abs(np.sum(Z[:, :K] * Zp[:, :K], axis=0)) / M
            passed = bool(np.all(np.sqrt(np.maximum(0.0, 2 - 2 * c)) < tol))
        else:
            passed = bool(np.all(np.abs(s - prev) < tol * s))
        prev = s
        if tol > 0 and passed:
            conv = True
            break
    V = Z[:, :K] / np.sqrt(M)
    W = X.T @ V
    sig = np.linalg.norm(W, axis=0)
    return V * sig, W / sig, sig, it, conv


def bf16_round(a):
    """Element-wise value of a stored as FP32 then bfloat16 (float64 array)."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    out = np.empty_like(a)
    lib().oracle_bf16_round(_ptr(a), _ptr(out), a.size)
    return out


def bf16_encode(x: float) -> int:
    return int(lib().oracle_bf16_encode(float(x)))


def bf16_decode(c: int) -> float:
    return float(lib().oracle_bf16_decode(int(c)))


def e4m3_encode(x: float) -> int:
    return int(lib().oracle_e4m3_encode(float(x)))


def e4m3_decode(c: int) -> float:
    return float(lib().oracle_e4m3_decode(int(c)))


FMT_BF16, FMT_E4M3 = 0, 1


def quantize(X, fmt):
    """Per-column-scaled codes of a binary32 matrix: (codes M x N, scales N)."""
    fmt_i = {"bf16": FMT_BF16, "e4m3": FMT_E4M3}[fmt] if isinstance(fmt, str) else int(fmt)
    X = np.asfortranarray(np.asarray(X, dtype=np.float32))
    M, N = X.shape
    codes = np.zeros((M, N), dtype=np.uint16 if fmt_i == FMT_BF16 else np.uint8, order="F")
    scale = np.zeros(N, dtype=np.float32)
    st = lib().oracle_quantize(_ptr(X), M, N, M, fmt_i, _ptr(codes), _ptr(scale))
    if st != 0:
        raise ValueError("oracle_quantize failed: %d" % st)
    return codes, scale


def dequantize(codes, scale, fmt, out=None):
    """x~ = decode(code) * s_j in FP64 (column-major); ``out`` may be a
    preallocated Fortran-ordered float64 (M, N) array to write into."""
    fmt_i = {"bf16": FMT_BF16, "e4m3": FMT_E4M3}[fmt] if isinstance(fmt, str) else int(fmt)
    codes = np.asfortranarray(codes)
    M, N = codes.shape
    if out is None:
        out = np.zeros((M, N), order="F")
    elif (out.shape != (M, N) or out.dtype != np.float64 or not out.flags["F_CONTIGUOUS"]):
        raise ValueError("out must be a Fortran-ordered float64 (M, N) array")
    sc = np.ascontiguousarray(scale, dtype=np.float32)
    lib().oracle_dequantize(_ptr(codes), _ptr(sc), M, N, fmt_i, _ptr(out))
    return out


# ---------------------------------------------------------------------------
# Warm-start network (see mlp_oracle.c): row-wise MLP d0 -> d1 -> d2 -> d3.

def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def mlp_forward(Z, params, round_bf16=False, skip=None):
    """params = (W1, b1, W2, b2, W3, b3) with W_l of shape (d_in, d_out).
    Returns (H1, H2, O); rows of Z are samples.  skip: an (M, d0) array whose
    first d3 columns are added to the output (the network's skip term; pass
    the unrounded inputs), or None."""
    W1, b1, W2, b2, W3, b3 = [_c64(x) for x in params]
    Z = _c64(Z)
    M, d0 = Z.shape
    d1, d2, d3 = W1.shape[1], W2.shape[1], W3.shape[1]
    H1 = np.zeros((M, d1)); H2 = np.zeros((M, d2)); O = np.zeros((M, d3))
    Zs = _c64(skip) if skip is not None else Z
    lib().oracle_mlp_forward(_ptr(Z), M, d0, d1, d2, d3, _ptr(W1), _ptr(b1), _ptr(W2), _ptr(b2),
                             _ptr(W3), _ptr(b3), int(bool(round_bf16)), int(skip is not None),
                             _ptr(Zs), _ptr(H1), _ptr(H2), _ptr(O))
    return H1, H2, O


def cos2_loss(O, V):
    """Sign-invariant loss sum_k 1 - cos^2(o_k, v_k) over columns; returns (L, dL/dO)."""
    O = _c64(O); V = _c64(V)
    M, K = O.shape
    dO = np.zeros((M, K))
    L = lib().oracle_cos2_loss(_ptr(O), _ptr(V), M, K, _ptr(dO))
    return L, dO


def mlp_backward(Z, params, H1, H2, dO, round_bf16=False, return_hidden=False):
    """Gradients (dW1, db1, dW2, db2, dW3, db3) of the loss whose dL/dO is dO;
    round_bf16 rounds the masked hidden gradients to bfloat16 where they are
    stored.  return_hidden: also return those hidden gradients (G1, G2)."""
    W1, b1, W2, b2, W3, b3 = [_c64(x) for x in params]
    Z = _c64(Z); H1 = _c64(H1); H2 = _c64(H2); dO = _c64(dO)
    M, d0 = Z.shape
    d1, d2, d3 = W1.shape[1], W2.shape[1], W3.shape[1]
    g = [np.zeros_like(W1), np.zeros(d1), np.zeros_like(W2), np.zeros(d2), np.zeros_like(W3),
         np.zeros(d3)]
    G1 = np.zeros((M, d1)); G2 = np.zeros((M, d2))
    lib().oracle_mlp_backward(_ptr(Z), M, d0, d1, d2, d3, _ptr(W1), _ptr(W2), _ptr(W3), _ptr(H1),
                              _ptr(H2), _ptr(dO), int(bool(round_bf16)), _ptr(g[0]), _ptr(g[1]),
                              _ptr(g[2]), _ptr(g[3]),
                              _ptr(g[4]), _ptr(g[5]), _ptr(G1), _ptr(G2))
    return (g, G1, G2) if return_hidden else g


def adam_step(w, g, m1, m2, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays w, m1, m2 with gradient g."""
    lib().oracle_adam(_ptr(w), _ptr(_c64(g)), _ptr(m1), _ptr(m2), w.size, lr, beta1, beta2, eps,
                      int(t))
