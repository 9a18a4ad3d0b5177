"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Method: Andrecut, arXiv:0811.1081, Sec. 2.2 (NIPALS-PCA) and Sec. 2.3
(GS-PCA).  The relative sigma test makes iteration counts sensitive to
rounding, so parity is checked on the same trajectory: the oracle replays the
GPU's per-component iteration counts and start columns.  Loadings and scores
are compared up to sign with the chordal angle 2 asin(|a - s b| / 2).

Tolerances (stated in the test, derived from the arithmetic):
  FP64 data: angle <= 1e-10, |sigma - sigma_o| <= 1e-12 sigma_0.
  FP32 data: angle <= 1e-5 for components whose relative gap to both
  neighbours is >= 2 % (FP32 rounding of R, ~6e-8 relative per element,
  amplified by 1/gap in the eigenvector), sigma within 1e-5 relative.
"""
import json
import os

import numpy as np
import pytest

from metrics import angle, col_angles, orth_err

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0811_1081_amd as gp
    gp.load()


def _gh():
    import gpu_helpers
    return gpu_helpers


def _replayed(orc, X, g, K, algo="gs", tiny=None, reorth="cgs"):
    kw = {} if tiny is None else {"tiny": tiny}
    return orc.fit(X, K, tol=0.0, max_iter=max(1, int(g["iters"].max())), algo=algo,
                   replay_iters=g["iters"], replay_start=g["start_col"], reorth=reorth, **kw)


def _gapped(sig, rel=0.02):
    s = np.asarray(sig, dtype=np.float64)
    ok = np.ones(len(s), dtype=bool)
    for k in range(len(s)):
        if k > 0 and s[k] > (1 - rel) * s[k - 1]:
            ok[k] = False
        if k + 1 < len(s) and s[k + 1] > (1 - rel) * s[k]:
            ok[k] = False
    return ok


# --------------------------------------------------------------------------
# FP64: the small low-rank case, both algorithms, element-by-element parity.

@pytest.mark.parametrize("algo", ["gs", "nipals"])
def test_small_f64_parity(orc, algo):
    from paper_0811_1081_amd import synth
    X = synth.case_small_f64()
    K = 16
    g = _gh().gpu_fit(X, K, tol=1e-10, max_iter=1000, algo=algo)
    assert g["status"] == 0
    o = _replayed(orc, X, g, K, algo)
    assert col_angles(g["P"], o.P).max() <= 1e-10
    assert col_angles(g["T"], o.T).max() <= 1e-10
    assert np.abs(g["sigma"] - o.sigma).max() <= 1e-12 * o.sigma[0]
    assert np.array_equal(g["lambda"], g["sigma"] ** 2)
    # same trajectory without replay: counts and start columns agree with the oracle
    free = orc.fit(X, K, tol=1e-10, max_iter=1000, algo=algo)
    assert np.array_equal(free.start_col, g["start_col"])
    assert np.abs(free.iters - g["iters"]).max() <= 1
    if algo == "gs":
        assert orth_err(g["P"]) <= 1e-13
        V = g["T"] / g["sigma"]
        assert orth_err(V) <= 1e-13


def test_golden_fixtures_on_gpu():
    g = json.load(open(os.path.join(GOLDEN, "rank1_3x2.json")))
    X = np.array(g["X_rows"])
    r = _gh().gpu_fit(X, 1, tol=g["tol"], max_iter=50)
    e = g["expect"]
    assert abs(r["sigma"][0] - 15.0) <= 1e-14 * 15
    assert angle(r["P"][:, 0], e["p"][0]) <= 1e-15
    assert list(r["iters"]) == e["iters"] and list(r["start_col"]) == e["start_col"]
    g = json.load(open(os.path.join(GOLDEN, "orthocols_4x3.json")))
    X = np.array(g["X_rows"])
    for mode in ("maxnorm", "column_k"):
        e = g["expect_" + mode]
        r = _gh().gpu_fit(X, 3, tol=g["tol"], max_iter=50, init=mode)
        np.testing.assert_allclose(r["sigma"], e["sigma"], rtol=1e-15, atol=0)
        for k, j in enumerate(e["p_index"]):
            assert angle(r["P"][:, k], np.eye(3)[:, j]) == 0.0
        assert list(r["iters"]) == e["iters"] and list(r["start_col"]) == e["start_col"]


# --------------------------------------------------------------------------
# FP32: ragged shapes spanning several tiles, wide and tall.

@pytest.mark.parametrize("shape", [(3001, 203), (517, 1029), (4099, 64), (64, 16)])
@pytest.mark.parametrize("algo", ["gs", "nipals"])
def test_f32_parity_ragged(orc, shape, algo):
    from paper_0811_1081_amd import synth
    M, N = shape
    r = min(M, N, 48)
    X = synth.haar_spectrum(M, N, 0.85 ** np.arange(r), 1e-4, seed=(9, M * 7 + N),
                            dtype=np.float32)
    K = min(12, r)
    g = _gh().gpu_fit(X, K, tol=1e-6, max_iter=1000, algo=algo)
    assert g["status"] == 0
    o = _replayed(orc, X, g, K, algo, tiny=orc.FLT_MIN)
    ok = _gapped(o.sigma)
    assert ok[:4].all()
    assert col_angles(g["P"], o.P)[ok].max() <= 1e-5
    assert col_angles(g["T"], o.T)[ok].max() <= 1e-5
    assert np.abs(g["sigma"] / o.sigma - 1).max() <= 1e-5
    if algo == "gs":
        assert orth_err(g["P"]) <= 1e-6
        assert orth_err(g["T"] / g["sigma"]) <= 1e-6


def test_f64_wide_and_tiny_shapes(orc):
    rng = np.random.default_rng(12)
    for (M, N, K) in [(1, 1, 1), (2, 1, 1), (1, 5, 1), (7, 3, 3), (40, 100, 10), (65, 9, 9)]:
        X = rng.standard_normal((M, N)) * (0.8 ** np.arange(N))
        g = _gh().gpu_fit(X, K, tol=1e-12, max_iter=3000)
        o = _replayed(orc, X, g, K)
        ok = _gapped(o.sigma, 0.05)
        if ok.any():
            assert col_angles(g["P"], o.P)[ok].max() <= 1e-9, (M, N, K)
        assert np.abs(g["sigma"] - o.sigma).max() <= 1e-11 * max(o.sigma[0], 1e-300), (M, N, K)


# --------------------------------------------------------------------------
# Implicit deflation (X never modified) and the two-pass path for wide X.

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape", [(3001, 203), (700, 1500)])
def test_implicit_deflation_parity(orc, dtype, shape):
    from paper_0811_1081_amd import synth
    M, N = shape
    X = synth.haar_spectrum(M, N, 0.85 ** np.arange(40), 1e-4, seed=(10, M + N), dtype=dtype)
    K = 12
    tol = 1e-10 if dtype == np.float64 else 1e-6
    g = _gh().gpu_fit(X, K, tol=tol, max_iter=2000, implicit=True)
    assert g["status"] == 0
    tiny = orc.DBL_MIN if dtype == np.float64 else orc.FLT_MIN
    o = orc.fit(X, K, tol=0.0, max_iter=int(g["iters"].max()), implicit=True,
                replay_iters=g["iters"], replay_start=g["start_col"], tiny=tiny)
    ok = _gapped(o.sigma)
    bound = 1e-10 if dtype == np.float64 else 1e-5
    assert col_angles(g["P"], o.P)[ok].max() <= bound
    assert col_angles(g["T"], o.T)[ok].max() <= bound
    assert np.abs(g["sigma"] / o.sigma - 1).max() <= (1e-12 if dtype == np.float64 else 1e-5)
    # the same start columns without replay (residual column norms formed implicitly)
    free = orc.fit(X, K, tol=tol, max_iter=2000, implicit=True, tiny=tiny)
    assert np.array_equal(free.start_col, g["start_col"])


# 16-byte aligned columns (matrix cores) and not; more than 64 components (two blocks)
@pytest.mark.parametrize("M,K", [(3000, 12), (3001, 12), (3000, 70)])
def test_given_start_implicit_f32_first_loadings(orc, M, K):
    """FP32, implicit deflation, given starts: the first loadings X^T t0 of
    all K given columns come from matrix-core passes before the first
    component (one per 64 columns, instead of one pass per component); a
    zero column falls back to the max-norm start (formed by a pass).
    Compared with the oracle on the same trajectory (replayed counts and
    start columns)."""
    from paper_0811_1081_amd import synth
    N = 203
    X = synth.haar_spectrum(M, N, 0.9 ** np.arange(100), 1e-4, seed=(12, M + N),
                            dtype=np.float32)
    rng = np.random.default_rng(M)
    a = orc.fit(X.astype(np.float64), K, tol=1e-3, max_iter=50, implicit=True)
    T0 = np.asfortranarray((a.T + 0.05 * rng.standard_normal(a.T.shape) * np.abs(a.T).max(axis=0))
                           .astype(np.float32))
    T0[:, 5] = 0.0  # falls back to the max-norm column
    g = _gh().gpu_fit(X, K, tol=1e-6, max_iter=2000, implicit=True, init="given",
                      T0=_gh().to_device(T0))
    assert g["status"] == 0
    assert g["start_col"][5] >= 0 and (np.delete(g["start_col"], 5) == -1).all()
    o = orc.fit(X, K, tol=0.0, max_iter=int(g["iters"].max()), implicit=True, init="given",
                T0=T0, replay_iters=g["iters"], replay_start=g["start_col"], tiny=orc.FLT_MIN)
    ok = _gapped(o.sigma)
    assert col_angles(g["P"], o.P)[ok].max() <= 1e-5
    assert col_angles(g["T"], o.T)[ok].max() <= 1e-5
    assert np.abs(g["sigma"] / o.sigma - 1).max() <= 1e-5


def test_implicit_rejected_for_nipals():
    import paper_0811_1081_amd as gp
    X = np.ones((50, 10))
    with pytest.raises(gp.GspcaError):
        _gh().gpu_fit(X, 2, algo="nipals", implicit=True)


@pytest.mark.parametrize("algo", ["gs", "nipals"])
def test_two_pass_path_wide(orc, algo):
    """N > 8192 runs the two-pass kernels (p <- R^T t and t <- R p separately)."""
    from paper_0811_1081_amd import synth
    M, N = 700, 8200
    X = synth.haar_spectrum(M, N, 0.8 ** np.arange(30), 1e-4, seed=(11, 0), dtype=np.float32)
    K = 6
    g = _gh().gpu_fit(X, K, tol=1e-6, algo=algo)
    o = _replayed(orc, X, g, K, algo, tiny=orc.FLT_MIN)
    assert col_angles(g["P"], o.P).max() <= 1e-5
    assert np.abs(g["sigma"] / o.sigma - 1).max() <= 1e-5


@pytest.mark.parametrize("algo", ["gs", "nipals"])
def test_paper_sweep_f64_parity(orc, algo):
    """The paper's timing data (Sec. 4: uniform entries, rows centred,
    N = M/2, K = 10, tol 1e-7, start column k) on the fused FP64 path, on the
    oracle's trajectory.  The spectrum is flat (gaps ~1 %), so the angle
    bound applies to components with a relative gap >= 1 %."""
    from paper_0811_1081_amd import synth
    X = synth.uniform_paper(500, 250, seed=(6, 500))
    K = 10
    g = _gh().gpu_fit(X, K, tol=1e-7, max_iter=10000, algo=algo, init="column_k")
    assert np.all(g["start_col"] == np.arange(K))
    o = _replayed(orc, X, g, K, algo)
    ok = _gapped(o.sigma, 0.01)
    assert ok.any()
    assert col_angles(g["P"], o.P)[ok].max() <= 1e-9
    assert np.abs(g["sigma"] - o.sigma).max() <= 1e-12 * o.sigma[0]


@pytest.mark.parametrize("algo", ["gs", "nipals"])
def test_two_pass_path_f64(orc, algo):
    """FP64 with N > 4096 runs the two-pass kernels (the large sizes of the
    paper's sweep, N = M/2 up to 7500, take this path)."""
    from paper_0811_1081_amd import synth
    X = synth.haar_spectrum(600, 4100, 0.8 ** np.arange(30), 1e-6, seed=(11, 1))
    K = 5
    g = _gh().gpu_fit(X, K, tol=1e-10, max_iter=3000, algo=algo)
    o = _replayed(orc, X, g, K, algo)
    assert col_angles(g["P"], o.P).max() <= 1e-10
    assert np.abs(g["sigma"] / o.sigma - 1).max() <= 1e-12


# --------------------------------------------------------------------------
# Re-orthogonalisation variants (two classical passes, modified Gram-Schmidt;
# not in the paper): two-pass path, against the oracle with the same form.

@pytest.mark.parametrize("reorth", ["cgs2", "mgs"])
def test_reorth_forms_parity_f64(orc, reorth):
    from paper_0811_1081_amd import synth
    X = synth.case_small_f64()
    K = 16
    g = _gh().gpu_fit(X, K, tol=1e-10, max_iter=1000, reorth=reorth)
    o = _replayed(orc, X, g, K, reorth=reorth)
    ok = _gapped(o.sigma)
    assert col_angles(g["P"], o.P)[ok].max() <= 1e-10
    assert np.abs(g["sigma"] - o.sigma).max() <= 1e-12 * o.sigma[0]
    assert orth_err(g["P"]) <= 1e-13


@pytest.mark.parametrize("reorth", ["cgs", "cgs2", "mgs"])
def test_reorth_forms_parity_f32_collinear(orc, reorth):
    """Full-rank collinear FP32 data (s_i = 0.9^i + noise): every form keeps
    the loadings and normalised scores orthonormal to FP32 rounding; the
    components with a clear gap match the FP64 oracle of the same form (the
    paper's single pass runs on the fused path, the variants on the two-pass
    path)."""
    from paper_0811_1081_amd import synth
    X = synth.case_collinear_f32(M=512, N=48)
    K = 24
    g = _gh().gpu_fit(_gh().to_device(X), K, tol=1e-6, max_iter=400, check=False,
                      reorth=reorth)
    o = _replayed(orc, X, g, K, tiny=orc.FLT_MIN, reorth=reorth)
    ok = _gapped(o.sigma)
    assert ok.any()
    assert col_angles(g["P"], o.P)[ok].max() <= 1e-5
    assert np.abs(g["sigma"] / o.sigma - 1).max() <= 1e-5
    assert orth_err(g["P"]) <= 1e-6
    V = g["T"] / g["sigma"]
    assert orth_err(V) <= 1e-6


def test_reorth_forms_rejected_where_unsupported():
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    X = _gh().to_device(synth.case_collinear_f32(M=256, N=32))
    with pytest.raises(gp.GspcaError):
        gp.fit(X, 4, implicit=True, reorth="cgs2")
    Q = gp.quantize(X, "bf16")
    with pytest.raises(gp.GspcaError):
        gp.fit(Q, 4, reorth="mgs")
    # NIPALS has no Gram-Schmidt step: the field is ignored
    a = gp.fit(X, 4, algo="nipals", reorth="mgs")
    b = gp.fit(X, 4, algo="nipals")
    assert bool((a["P"] == b["P"]).all())


# --------------------------------------------------------------------------
# Start-vector modes, replay, determinism.

def test_init_modes_and_given_start(orc):
    import torch
    from paper_0811_1081_amd import synth
    X = synth.case_small_f64()
    for mode in ("maxnorm", "column_k"):
        g = _gh().gpu_fit(X, 6, tol=1e-10, init=mode)
        o = orc.fit(X, 6, tol=1e-10, init=mode)
        assert np.array_equal(g["start_col"], o.start_col), mode
        assert col_angles(g["P"], o.P).max() <= 1e-8
    a = orc.fit(X, 4, tol=1e-10)
    T0 = np.asfortranarray(a.T.copy())
    T0[:, 2] = 0.0  # falls back to the max-norm column
    Td = _gh().to_device(T0)
    g = _gh().gpu_fit(X, 4, tol=1e-10, init="given", T0=Td)
    o = orc.fit(X, 4, tol=1e-10, init="given", T0=T0)
    assert list(g["start_col"]) == [-1, -1, o.start_col[2], -1]
    assert np.array_equal(g["start_col"], o.start_col)
    assert col_angles(g["P"], o.P).max() <= 1e-8
    del torch


def test_replay_forces_counts_and_columns(orc):
    from paper_0811_1081_amd import synth
    X = synth.case_small_f64()
    it = np.array([3, 1, 7, 2], dtype=np.int32)
    sc = np.array([5, -1, 0, 100], dtype=np.int32)
    import torch
    g = _gh().gpu_fit(X, 4, tol=1e-10, replay_iters=torch.from_numpy(it).cuda(),
                      replay_start=torch.from_numpy(sc).cuda())
    assert np.array_equal(g["iters"], it)
    assert g["start_col"][0] == 5 and g["start_col"][2] == 0 and g["start_col"][3] == 100
    o = orc.fit(X, 4, tol=1e-10, replay_iters=it, replay_start=sc)
    assert g["start_col"][1] == o.start_col[1]
    assert col_angles(g["P"], o.P).max() <= 1e-10
    assert np.abs(g["sigma"] - o.sigma).max() <= 1e-12 * o.sigma[0]


def test_bitwise_reproducible():
    from paper_0811_1081_amd import synth
    X = synth.case_collinear_f32(M=2000, N=300)
    a = _gh().gpu_fit(X, 20, tol=1e-6)
    b = _gh().gpu_fit(X, 20, tol=1e-6)
    for k in ("T", "P", "lambda", "iters", "start_col"):
        assert np.array_equal(a[k], b[k]), k


# --------------------------------------------------------------------------
# Degenerate and error paths.

def test_zero_matrix_degenerate(orc):
    X = np.zeros((70, 5))
    g = _gh().gpu_fit(X, 5, tol=1e-10)
    o = orc.fit(X, 5, tol=1e-10)
    assert g["status"] == 0
    assert np.all(g["sigma"] == 0) and np.all(g["T"] == 0) and np.all(g["iters"] == 0)
    assert np.array_equal(g["P"], o.P) and np.array_equal(g["P"], np.eye(5))


def test_rank_deficient_f64(orc):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((50, 3))
    B = rng.standard_normal((8, 3))
    X = A @ B.T
    g = _gh().gpu_fit(X, 6, tol=1e-12, max_iter=500)
    assert np.all(g["sigma"][3:] <= 1e-12 * g["sigma"][0])
    assert orth_err(g["P"]) <= 1e-10


def test_nonfinite_and_not_converged():
    import paper_0811_1081_amd as gp
    X = np.ones((100, 10))
    X[7, 3] = np.nan
    r = _gh().gpu_fit(X, 2, check=False)
    assert r["status"] == gp.ENONFINITE
    from paper_0811_1081_amd import synth
    X = synth.case_small_f64()
    r = _gh().gpu_fit(X, 3, tol=1e-12, max_iter=2)
    assert r["status"] == gp.NOT_CONVERGED
    assert np.all(r["iters"] == 2)
    assert orth_err(r["P"]) <= 1e-13


def test_convenience_entry_points(orc):
    import ctypes
    import torch
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    L = gp.load()
    X = synth.case_small_f64()
    Xd = _gh().to_device(X)
    M, N = X.shape
    K = 5
    T = torch.empty_strided((M, K), (1, M), dtype=torch.float64, device="cuda")
    P = torch.empty_strided((N, K), (1, N), dtype=torch.float64, device="cuda")
    lam = torch.empty(K, dtype=torch.float64, device="cuda")
    st = L.gspca_fit(Xd.data_ptr(), M, N, K, 1e-10, 1000, T.data_ptr(), P.data_ptr(),
                     lam.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    o = orc.fit(X, K, tol=1e-10)
    assert col_angles(P.cpu().numpy(), o.P).max() <= 1e-8
    X32 = X.astype(np.float32)
    Xd = _gh().to_device(X32)
    T = torch.empty_strided((M, K), (1, M), dtype=torch.float32, device="cuda")
    P = torch.empty_strided((N, K), (1, N), dtype=torch.float32, device="cuda")
    st = L.gspca_fit_f32(Xd.data_ptr(), M, N, K, 1e-6, 1000, T.data_ptr(), P.data_ptr(),
                         lam.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    assert np.abs(np.sqrt(lam.cpu().numpy()) / o.sigma - 1).max() <= 1e-5
