"""Pins of the oracle's block iteration with Rayleigh-Ritz (not in the
paper): convergence to the library SVD, the Ky Fan bound at every iteration,
exactness for rank <= r, and the equivalence of the two start forms."""
import numpy as np

from metrics import col_angles


def _gapped_case():
    from paper_0811_1081_amd import synth
    X = synth.haar_spectrum(500, 160, 0.85 ** np.arange(60), 1e-8, seed=(11, 3))
    return X.astype(np.float64), synth.sketch_matrix(160, 32).astype(np.float64)


def test_converges_to_library_svd(orc):
    X, Om = _gapped_case()
    K = 12
    T, P, s, it, conv = orc.block_fit(X, K, Omega=Om, tol=1e-13, max_iter=200)
    U, sv, Vt = np.linalg.svd(X, full_matrices=False)
    assert conv and it < 200
    assert np.abs(s / sv[:K] - 1).max() <= 1e-12
    assert col_angles(P, Vt[:K].T).max() <= 1e-8
    assert col_angles(T / s, U[:, :K]).max() <= 1e-8
    assert np.abs(T.T @ T - np.diag(s ** 2)).max() <= 1e-10 * s[0] ** 2


def test_ky_fan_bound_every_iteration(orc):
    """For any orthonormal v_0..v_(k-1), sum |X^T v_i|^2 <= sum_(i<k) sigma_i^2
    (Ky Fan); the block's outputs are such a set after every iteration, and
    the partial sums approach the bound from below."""
    X, Om = _gapped_case()
    sv = np.linalg.svd(X, compute_uv=False)
    K = 12
    prev = None
    for j in range(1, 5):
        T, P, s, it, _ = orc.block_fit(X, K, Omega=Om, tol=0.0, max_iter=j)
        assert it == j
        V = T / s
        assert np.abs(V.T @ V - np.eye(K)).max() <= 1e-12
        part = np.cumsum(s ** 2)
        assert np.all(part <= np.cumsum(sv[:K] ** 2) * (1 + 1e-12))
        if prev is not None:
            assert part[-1] >= prev * (1 - 1e-12)
        prev = part[-1]


def test_exact_for_rank_below_block(orc):
    # rank 20 <= r = 32: the first block already spans range(X)
    from paper_0811_1081_amd import synth
    rng = np.random.default_rng(9)
    M, N, rk = 300, 90, 20
    U = np.linalg.qr(rng.standard_normal((M, rk)))[0]
    V = np.linalg.qr(rng.standard_normal((N, rk)))[0]
    s0 = 0.97 ** np.arange(rk)
    X = (U * s0) @ V.T
    Om = synth.sketch_matrix(N, 32).astype(np.float64)
    T, P, s, it, _ = orc.block_fit(X, 10, Omega=Om, tol=0.0, max_iter=1)
    assert np.abs(s - s0[:10]).max() <= 1e-12
    assert col_angles(P, V[:, :10]).max() <= 1e-9


def test_given_start_equals_sketch_start(orc):
    X, Om = _gapped_case()
    a = orc.block_fit(X, 8, Omega=Om, tol=0.0, max_iter=3)
    b = orc.block_fit(X, 8, Z0=X @ Om, tol=0.0, max_iter=3)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[1], b[1])


def test_vector_change_stop(orc):
    """stop="loading": the iteration ends once every unit Ritz vector moved
    less than tol; the error left is then below tol times the contraction
    (sigma_(r+1) / sigma_K)^2 / (1 - that), far below tol for this gap."""
    X, Om = _gapped_case()
    K = 12
    T, P, s, it, conv = orc.block_fit(X, K, Omega=Om, tol=1e-6, max_iter=200, stop="loading")
    U, sv, Vt = np.linalg.svd(X, full_matrices=False)
    assert conv
    rho = (sv[32] / sv[K - 1]) ** 2
    assert col_angles(T / s, U[:, :K]).max() <= 1e-6 * rho / (1 - rho) * 4
    # one iteration fewer has not yet met the test
    T2, _, s2, _, _ = orc.block_fit(X, K, Omega=Om, tol=0.0, max_iter=it - 1)
    T3, _, s3, _, _ = orc.block_fit(X, K, Omega=Om, tol=0.0, max_iter=it - 2) if it > 2 else (T2, 0, s2, 0, 0)
    if it > 2:
        assert col_angles(T2 / s2, T3 / s3).max() >= 1e-6
