"""Pins of the oracle's Gram-Schmidt forms (the paper's single classical
pass, Sec. 2.3, and the re-orthogonalisation variants CGS2 and MGS, which
are not in the paper) against facts independent of the oracle's loops."""
import numpy as np

from metrics import col_angles


def _unit_columns(rng, n, k, mix):
    """n x k unit-norm columns, orthonormal for mix = 0, increasingly
    dependent as mix grows."""
    Q = np.linalg.qr(rng.standard_normal((n, k)))[0]
    A = Q + mix * Q[:, :1]
    return A / np.linalg.norm(A, axis=0)


def test_forms_on_orthonormal_columns_match_least_squares(orc):
    # with orthonormal columns all three remove the least-squares fit of x
    rng = np.random.default_rng(31)
    Q = _unit_columns(rng, 60, 12, 0.0)
    x = rng.standard_normal(60)
    coef, *_ = np.linalg.lstsq(Q, x, rcond=None)
    ref = x - Q @ coef
    for form in ("cgs", "cgs2", "mgs"):
        assert np.abs(orc.gs_step(Q, x, form) - ref).max() <= 1e-13, form


def test_forms_as_projector_products(orc):
    """On dependent unit columns the three forms differ: one classical pass is
    the single operator I - Q Q^T, two passes are its square, and the
    modified process is the ordered product of the rank-one projectors
    (I - q_(k-1) q_(k-1)^T) ... (I - q_0 q_0^T)."""
    rng = np.random.default_rng(32)
    n, k = 40, 6
    Q = _unit_columns(rng, n, k, 0.7)
    x = rng.standard_normal(n)
    I = np.eye(n)
    C = I - Q @ Q.T
    Pm = I.copy()
    for i in range(k):
        Pm = (I - np.outer(Q[:, i], Q[:, i])) @ Pm
    outs = {f: orc.gs_step(Q, x, f) for f in ("cgs", "cgs2", "mgs")}
    assert np.abs(outs["cgs"] - C @ x).max() <= 1e-12
    assert np.abs(outs["cgs2"] - C @ (C @ x)).max() <= 1e-12
    assert np.abs(outs["mgs"] - Pm @ x).max() <= 1e-12
    # and they are really different operators here
    assert np.abs(outs["mgs"] - outs["cgs"]).max() > 1e-2
    assert np.abs(outs["cgs2"] - outs["cgs"]).max() > 1e-2


def test_second_pass_restores_orthogonality(orc):
    """x almost inside span(Q): x = Q a + delta w, w a unit vector orthogonal
    to Q.  One classical pass leaves a component along Q of the order
    eps |a| / delta relative to what remains; the second pass removes it to
    rounding level (the classical "twice is enough")."""
    rng = np.random.default_rng(33)
    n, k = 200, 40
    Q = _unit_columns(rng, n, k, 0.0)
    w = rng.standard_normal(n)
    w -= Q @ (Q.T @ w)
    w -= Q @ (Q.T @ w)
    w /= np.linalg.norm(w)
    delta = 1e-10
    x = Q @ rng.standard_normal(k) + delta * w

    def leak(r):
        return np.linalg.norm(Q.T @ r) / np.linalg.norm(r)
    r1, r2 = orc.gs_step(Q, x, "cgs"), orc.gs_step(Q, x, "cgs2")
    assert leak(r1) >= 1e-9
    assert leak(r2) <= 1e-14
    assert abs(np.linalg.norm(r2) / delta - 1) <= 1e-4


def test_fits_agree_across_forms(orc):
    """With orthonormal earlier bases the three forms are the same map in
    exact arithmetic: the FP64 fits take the same iterations and agree to
    rounding."""
    from paper_0811_1081_amd import synth
    X = synth.case_small_f64()
    K = 16
    f = {r: orc.fit(X, K, tol=1e-10, max_iter=1000, reorth=r) for r in ("cgs", "cgs2", "mgs")}
    for r in ("cgs2", "mgs"):
        assert np.array_equal(f[r].iters, f["cgs"].iters), r
        assert np.abs(f[r].sigma / f["cgs"].sigma - 1).max() <= 1e-12, r
        assert col_angles(f[r].P, f["cgs"].P).max() <= 1e-10, r
    # NIPALS ignores the form (no Gram-Schmidt step)
    n1 = orc.fit(X, 4, tol=1e-10, max_iter=1000, algo="nipals")
    n2 = orc.fit(X, 4, tol=1e-10, max_iter=1000, algo="nipals", reorth="mgs")
    assert np.array_equal(n1.P, n2.P)
