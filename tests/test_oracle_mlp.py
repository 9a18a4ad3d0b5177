"""Pins of the oracle's warm-start network against central finite
differences, a hand-derived loss value and the definition of Adam."""
import numpy as np
import pytest


def _params(rng, dims):
    out = []
    for a, b in zip(dims[:-1], dims[1:]):
        out += [rng.standard_normal((a, b)) / np.sqrt(a), 0.1 * rng.standard_normal(b)]
    return out


def _loss(orc, Z, params, V):
    _, _, O = orc.mlp_forward(Z, params)
    return orc.cos2_loss(O, V)[0]


def test_cos2_loss_closed_form(orc):
    O = np.array([[1.0, 0.0], [0.0, 2.0], [0.0, 0.0]])
    V = np.array([[1.0, 1.0], [1.0, 1.0], [0.0, 0.0]])
    # column 0: cos^2 = (1)^2 / (1 * 2) = 1/2; column 1: (2)^2 / (4 * 2) = 1/2
    L, _ = orc.cos2_loss(O, V)
    assert abs(L - 1.0) <= 1e-15
    L2, dO = orc.cos2_loss(V, V)
    assert abs(L2) <= 1e-15 and np.abs(dO).max() <= 1e-15
    L3, _ = orc.cos2_loss(-3.0 * V, V)  # sign and scale invariant
    assert abs(L3) <= 1e-15


@pytest.mark.parametrize("seed", [0, 1])
def test_mlp_gradients_match_finite_differences(orc, seed):
    rng = np.random.default_rng(seed)
    dims = (6, 9, 7, 3)
    M = 11
    Z = rng.standard_normal((M, dims[0]))
    V = rng.standard_normal((M, dims[-1]))
    params = _params(rng, dims)
    H1, H2, O = orc.mlp_forward(Z, params)
    L, dO = orc.cos2_loss(O, V)
    grads = orc.mlp_backward(Z, params, H1, H2, dO)
    h = 1e-6
    for pi, (P, G) in enumerate(zip(params, grads)):
        num = np.zeros_like(P)
        it = np.nditer(P, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            old = P[idx]
            P[idx] = old + h
            lp = _loss(orc, Z, params, V)
            P[idx] = old - h
            lm = _loss(orc, Z, params, V)
            P[idx] = old
            num[idx] = (lp - lm) / (2 * h)
        rel = np.linalg.norm(num - G) / max(np.linalg.norm(G), 1e-12)
        assert rel <= 1e-6, (pi, rel)


def test_mlp_forward_matches_plain_numpy(orc):
    rng = np.random.default_rng(3)
    dims = (5, 8, 8, 2)
    Z = rng.standard_normal((13, 5))
    params = _params(rng, dims)
    W1, b1, W2, b2, W3, b3 = params
    h1 = np.maximum(Z @ W1 + b1, 0)
    h2 = np.maximum(h1 @ W2 + b2, 0)
    o = h2 @ W3 + b3
    H1, H2, O = orc.mlp_forward(Z, params)
    assert np.abs(O - o).max() <= 1e-12 and np.abs(H1 - h1).max() <= 1e-12


def test_mlp_bf16_rounding_points(orc):
    rng = np.random.default_rng(4)
    dims = (5, 8, 8, 2)
    Z = rng.standard_normal((13, 5))
    params = _params(rng, dims)
    H1, H2, _ = orc.mlp_forward(Z, params, round_bf16=True)
    for H in (H1, H2):
        r = np.array([orc.bf16_decode(orc.bf16_encode(float(x))) for x in H.ravel()]).reshape(H.shape)
        assert np.array_equal(H, r)


def test_adam_matches_definition(orc):
    rng = np.random.default_rng(5)
    w = rng.standard_normal(7)
    m1 = np.zeros(7); m2 = np.zeros(7)
    w0 = w.copy()
    g1 = rng.standard_normal(7)
    orc.adam_step(w, g1, m1, m2, lr=0.01, t=1)
    # first step: m_hat = g, v_hat = g^2 -> w -= lr * g / (|g| + eps)
    assert np.allclose(w, w0 - 0.01 * g1 / (np.abs(g1) + 1e-8), rtol=0, atol=1e-15)


def test_skip_term(orc):
    """The skip adds the first d3 inputs to the output and changes the
    parameter gradients only through dL/dO (finite differences)."""
    rng = np.random.default_rng(12)
    dims = (6, 9, 7, 3)
    M = 10
    Z = rng.standard_normal((M, dims[0]))
    V = rng.standard_normal((M, dims[-1]))
    params = _params(rng, dims)
    _, _, O0 = orc.mlp_forward(Z, params)
    H1, H2, O = orc.mlp_forward(Z, params, skip=Z)
    assert np.array_equal(O, O0 + Z[:, :3])
    L, dO = orc.cos2_loss(O, V)
    grads = orc.mlp_backward(Z, params, H1, H2, dO)
    h = 1e-6
    P = params[2]
    num = np.zeros_like(P)
    for idx in np.ndindex(P.shape):
        old = P[idx]
        P[idx] = old + h
        lp = orc.cos2_loss(orc.mlp_forward(Z, params, skip=Z)[2], V)[0]
        P[idx] = old - h
        lm = orc.cos2_loss(orc.mlp_forward(Z, params, skip=Z)[2], V)[0]
        P[idx] = old
        num[idx] = (lp - lm) / (2 * h)
    assert np.linalg.norm(num - grads[2]) <= 1e-6 * np.linalg.norm(grads[2])
