"""Seeded synthetic inputs for the iterative-PCA workloads.

This module only draws random matrices: it contains none of the PCA method's
arithmetic, and both the GPU library's tests and the CPU oracle consume what it
returns.  Every generator is a pure function of its integer seed tuple, drawn
from numpy's PCG64 in a fixed order, so a run on any machine reproduces the
same bytes.

Workloads (column-major / Fortran-ordered arrays, as the paper stores X,
Sec. 3):

* ``lowrank_gaussian``  X = A diag(s) B^T + noise*E, A, B, E i.i.d. N(0,1),
  s_i = 2^(-i/4); columns mean-centred.  (FP64 parity case, 512 x 128.)
* ``haar_spectrum``     X = U diag(s) V^T + noise*E with U, V Haar-random
  orthonormal (QR of a Gaussian with the sign of diag(R) fixed), s given;
  optionally column-centred.  Used for the collinear full-rank case
  (4096 x 512, s_i = 0.9^i), the large case (65536 x 8192, rank 64,
  s_i = 100 * 0.95^i), the batched instances and the warm-start instances.
* ``uniform_paper``     X uniform on [0, 1), rows centred: the data of the
  paper's Sec. 4 timing sweep.

Noise levels are standard deviations.
"""
from __future__ import annotations

import numpy as np

SEED_ROOT = 811


def rng_for(*key: int) -> np.random.Generator:
    """PCG64 generator for the seed tuple (811, *key)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, *key])))


def haar(rng: np.random.Generator, n: int, r: int) -> np.ndarray:
    """n x r matrix with orthonormal columns, Haar-distributed (QR of a Gaussian,
    columns sign-fixed so that diag(R) > 0)."""
    g = rng.standard_normal((n, r))
    q, rr = np.linalg.qr(g)
    d = np.sign(np.diag(rr))
    d[d == 0] = 1.0
    return q * d


def lowrank_gaussian(M: int = 512, N: int = 128, rank: int = 32, noise: float = 1e-3,
                     seed: tuple = (1, 0), centre: bool = True) -> np.ndarray:
    """FP64 X = A diag(2^(-i/4)) B^T + noise*E, columns centred (draw order A, B, E)."""
    rng = rng_for(*seed)
    A = rng.standard_normal((M, rank))
    B = rng.standard_normal((N, rank))
    E = rng.standard_normal((M, N))
    s = 2.0 ** (-np.arange(rank) / 4.0)
    X = (A * s) @ B.T + noise * E
    if centre:
        X -= X.mean(axis=0, keepdims=True)
    return np.asfortranarray(X)


def haar_spectrum(M: int, N: int, s: np.ndarray, noise: float, seed: tuple,
                  centre: bool = False, dtype=np.float64, block_cols: int = 256,
                  return_factors: bool = False):
    """X = U diag(s) V^T + noise*E with Haar U (M x r), V (N x r), r = len(s).

    Draw order: U, V, then the noise column block by column block
    (``block_cols`` columns at a time, each block drawn as a (cols, M) array so
    that it fills whole columns; float32 draws when dtype is float32 so that
    the large case stays cheap to generate).  The product is formed in float64
    and rounded once to ``dtype`` (round-to-nearest-even)."""
    s = np.asarray(s, dtype=np.float64)
    r = len(s)
    rng = rng_for(*seed)
    U = haar(rng, M, r)
    V = haar(rng, N, r)
    X = np.empty((M, N), dtype=dtype, order="F")
    Vs = V * s  # N x r
    ndt = np.float32 if dtype == np.float32 else np.float64
    for c0 in range(0, N, block_cols):
        c1 = min(N, c0 + block_cols)
        blk = Vs[c0:c1] @ U.T  # (cols, M): row j is column c0 + j of X
        if noise > 0:
            blk += noise * rng.standard_normal((c1 - c0, M), dtype=ndt)
        X[:, c0:c1] = blk.T
    if centre:
        mu = X.mean(axis=0, dtype=np.float64, keepdims=True)
        X -= mu.astype(dtype)
    if return_factors:
        return X, U, V
    return X


def uniform_paper(M: int, N: int, seed: tuple = (6, 0), centre_rows: bool = True) -> np.ndarray:
    """FP64 X uniform on [0, 1) (the data of the paper's timing sweep, Sec. 4),
    each row then centred -- its mean over the N entries subtracted -- as the
    paper's programs do to the data before the iteration (Eq. 1 and the
    listings centre rows although the prose speaks of columns; the generator
    takes the programs' reading and the fit itself never centres)."""
    rng = rng_for(*seed)
    X = rng.random((M, N))
    if centre_rows:
        X = X - X.mean(axis=1, keepdims=True)
    return np.asfortranarray(X)


# --------------------------------------------------------------------------
# The named workloads.


def case_small_f64() -> np.ndarray:
    """512 x 128 FP64, rank-32 signal 2^(-i/4) + 1e-3 noise, centred (K=16, tol 1e-10)."""
    return lowrank_gaussian(512, 128, 32, 1e-3, seed=(1, 0))


def case_collinear_f32(M: int = 4096, N: int = 512, seed_inst: int = 0) -> np.ndarray:
    """FP32 full-rank collinear data: s_i = 0.9^i, 1e-4 noise, centred (K=N, tol 1e-6)."""
    s = 0.9 ** np.arange(min(M, N))
    return haar_spectrum(M, N, s, 1e-4, seed=(2, seed_inst), centre=True, dtype=np.float32)


def case_large_f32(M: int = 65536, N: int = 8192, rank: int = 64,
                   seed_inst: int = 0, return_factors: bool = False):
    """FP32 rank-64 signal s_i = 100*0.95^i + 1e-2 noise, uncentred (K=32, tol 1e-6)."""
    s = 100.0 * 0.95 ** np.arange(rank)
    return haar_spectrum(M, N, s, 1e-2, seed=(3, seed_inst), centre=False,
                         dtype=np.float32, return_factors=return_factors)


def batched_shapes(count: int = 2048, seed: int = 0):
    """(M, N, K) of the uneven batched instances: M ~ U{64..4096}, N ~ U{16..512},
    K = min(8, N)."""
    rng = rng_for(4, 1_000_000 + seed)
    Ms = rng.integers(64, 4097, size=count)
    Ns = rng.integers(16, 513, size=count)
    return [(int(m), int(n), int(min(8, n))) for m, n in zip(Ms, Ns)]


def batched_instance(i: int, M: int, N: int) -> np.ndarray:
    """FP32 instance i of the batched workload: rank min(16, N), s_i = 0.8^i, 1e-3 noise."""
    r = min(16, N, M)
    s = 0.8 ** np.arange(r)
    return haar_spectrum(M, N, s, 1e-3, seed=(4, i), centre=False, dtype=np.float32)


def warmstart_instance(i: int, M: int = 2048, N: int = 256, return_factors: bool = False):
    """FP32 warm-start instance i: s_j = r^j with r ~ U[0.7, 0.95], full rank, no noise."""
    rng = rng_for(5, i)
    ratio = float(rng.uniform(0.7, 0.95))
    s = ratio ** np.arange(min(M, N))
    out = haar_spectrum(M, N, s, 0.0, seed=(5, 100_000 + i), centre=False,
                        dtype=np.float32, return_factors=return_factors)
    return (out, ratio) if not return_factors else (*out, ratio)


def sketch_matrix(N: int = 256, r: int = 32) -> np.ndarray:
    """Fixed Gaussian test matrix Omega (N x r, row-major) for the warm-start sketch X*Omega."""
    rng = rng_for(5, 999_999)
    return np.ascontiguousarray(rng.standard_normal((N, r)).astype(np.float32))


def map_threads(fn, items, workers: int = 8, log=None, every: int = 256):
    """[fn(x) for x in items] on a pool of threads of this process (numpy's
    QR, products and bulk random draws release the interpreter lock), with one
    BLAS thread per worker.  No child process is started, so the call is safe
    in a process that uses the GPU or runs under a profiler."""
    items = list(items)
    if workers <= 1 or len(items) < 4:
        return [fn(x) for x in items]
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    out = []
    with threadpool_limits(limits=1), ThreadPoolExecutor(max_workers=workers) as ex:
        for r in ex.map(fn, items):
            out.append(r)
            if log and len(out) % every == 0:
                log("generated %d / %d" % (len(out), len(items)))
    return out
