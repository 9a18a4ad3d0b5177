"""GPU tests of the learned warm start (gspca_ws.h) against the FP64 oracle:
sketch, whitening, the bf16 matrix-core network's forward pass, loss and
gradients at matched bf16 rounding points, Adam, the composed prediction, and
a three-arm comparison of the starts (max-norm column, the network's skip
path, the trained network) on held-out matrices.

Tolerances: per-tensor relative Frobenius error <= 2e-3 for bf16 products
with FP32 accumulation (a few bf16 units, 2^-8 each, on a minority of the
stored operands); the FP32 sketch within N u sum_j |x_j omega_j| (u = 2^-24).
"""
import numpy as np
import pytest

from metrics import col_angles

pytestmark = pytest.mark.gpu

DIMS = (32, 256, 256, 16)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0811_1081_amd as gp
    gp.load()


def _rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / max(
        np.linalg.norm(np.asarray(b, np.float64)), 1e-300)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _colmajor(a):
    import torch
    a = np.asarray(a, dtype=np.float32)
    M, N = a.shape
    t = torch.empty_strided((M, N), (1, M), dtype=torch.float32, device="cuda")
    t.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return t


def _oracle_params(orc, net):
    """Weights as the GPU uses them: bf16-rounded W, FP32 biases."""
    theta = net.theta.cpu().numpy().astype(np.float64)
    p = net.unpack(theta)
    return [orc.bf16_round(x) if i % 2 == 0 else x for i, x in enumerate(p)]


@pytest.mark.parametrize("M", [1000, 1001])  # 16-byte aligned columns, and not
def test_sketch_matches_oracle(orc, M):
    import torch
    from paper_0811_1081_amd import synth, warmstart as ws
    X = synth.warmstart_instance(1, M=M, N=200)[0]
    Om = synth.sketch_matrix(200, 32)
    Y = ws.sketch(_colmajor(X), _dev(Om))
    torch.cuda.synchronize()
    Yo = orc.sketch_whiten(X, Om)[0]
    # sequential FP32 accumulation over N terms: |error| <= N u sum_j |x_j omega_j|
    bound = 200 * 2.0 ** -24 * (np.abs(X.astype(np.float64)) @ np.abs(Om.astype(np.float64)))
    assert np.all(np.abs(Y.cpu().numpy() - Yo) <= bound + 1e-30)


@pytest.mark.parametrize("r", [32, 64])
def test_sketch_many_rows(r):
    """Y = X Omega at 65572 rows (the form for many rows: 256-row workgroups,
    36 rows in the last) and 150 columns (ragged 32-column chunks), against
    the FP64 product within the FP32 accumulation bound."""
    import torch
    from paper_0811_1081_amd import synth, warmstart as ws
    rng = np.random.default_rng(11 + r)
    M, N = 65572, 150
    X = rng.standard_normal((M, N)).astype(np.float32)
    Om = synth.sketch_matrix(N, r)
    Y = ws.sketch(_colmajor(X), _dev(Om))
    torch.cuda.synchronize()
    X64, O64 = X.astype(np.float64), Om.astype(np.float64)
    bound = N * 2.0 ** -24 * (np.abs(X64) @ np.abs(O64))
    assert np.all(np.abs(Y.cpu().numpy() - X64 @ O64) <= bound + 1e-30)


@pytest.mark.parametrize("r,M", [(32, 900), (64, 900), (64, 903)])  # aligned columns, and not
def test_refinement_step_matches_oracle(orc, r, M):
    import torch
    from paper_0811_1081_amd import synth, warmstart as ws
    X = synth.warmstart_instance(4, M=M, N=150)[0]  # 150 columns: ragged blocks
    Xd = _colmajor(X)
    Z = ws.whiten(ws.sketch(Xd, _dev(synth.sketch_matrix(150, r))))[0]
    W, Y = ws.sketch_refine(Xd, Z)
    torch.cuda.synchronize()
    Zh = Z.cpu().numpy().astype(np.float64)
    Wo, _ = orc.sketch_refine(X, Zh)  # the oracle's step on the GPU's own Z
    Xa = np.abs(X.astype(np.float64))
    M, N = X.shape
    # FP32 sums: M terms (per-lane runs and a butterfly) for W, N terms for Y
    assert np.all(np.abs(W.cpu().numpy() - Wo) <= M * 2.0 ** -24 * (Xa.T @ np.abs(Zh)) / np.sqrt(M))
    Wg = W.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(Y.cpu().numpy() - X.astype(np.float64) @ Wg)
                  <= N * 2.0 ** -24 * (Xa @ np.abs(Wg)) + 1e-30)


@pytest.mark.parametrize("r", [32, 64])
def test_whitening_matches_oracle(orc, r):
    import torch
    from paper_0811_1081_amd import synth, warmstart as ws
    X = synth.warmstart_instance(2, M=2049, N=256)[0]  # a ragged last tile of 64 rows
    Om = synth.sketch_matrix(256, r)
    Y = ws.sketch(_colmajor(X), _dev(Om))
    Z, g, flag = ws.whiten(Y)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy().astype(np.float64)
    Zo, go = orc.whiten(Yh)  # the same sketch, whitened by the oracle
    g = g.cpu().numpy()
    assert int(flag.item()) == 0
    assert np.abs(g - go).max() <= 1e-10 * go[0]
    Zg = Z.cpu().numpy().astype(np.float64)
    M = Zg.shape[0]
    # directions resolved in FP64 from the FP32 sketch: eigenvector errors grow
    # like eps * g_0 / (g_k * gap), so compare where g_k > 1e-8 g_0 with gaps
    ok = go > 1e-10 * go[0]
    gap = np.ones(r, dtype=bool)
    gap[:-1] &= (go[:-1] - go[1:]) > 1e-3 * go[:-1]
    gap[1:] &= (go[:-1] - go[1:]) > 1e-3 * go[:-1]
    sel = (go > 1e-8 * go[0]) & gap
    assert sel.sum() >= 16
    assert np.abs(Zg[:, sel] - Zo[:, sel]).max() <= 1e-4
    assert np.abs(Zg[:, ok].T @ Zg[:, ok] / M - np.eye(int(ok.sum()))).max() <= 1e-4


@pytest.mark.parametrize("r", [32, 64])
def test_whitening_equal_diagonal_pairs(r):
    """Y = Q diag(s) B with orthonormal Q (M x r), distinct known s and B a
    45-degree rotation of each index pair (2i, 2i + 1): Y^T Y = B^T diag(s^2) B
    has diagonal entries equal within each pair (up to the FP32 rounding of
    Y) and a non-zero off-diagonal entry in every pair block (the rotation's
    |t| = 1 limit), eigenvalues s^2 and eigenvectors the columns of B.  Checked against the library eigenvalues of the FP32
    Y's Gram matrix, the closed form s^2, and Z = +-sqrt(M) Q."""
    import torch
    from paper_0811_1081_amd import warmstart as ws
    rng = np.random.default_rng(5 + r)
    M = 1000
    Q, _ = np.linalg.qr(rng.standard_normal((M, r)))
    s = np.geomspace(10.0, 0.5, r)
    B = np.eye(r)
    h = np.sqrt(0.5)
    for i in range(0, r, 2):
        B[i:i + 2, i:i + 2] = [[h, h], [-h, h]]
    Y32 = ((Q * s) @ B).astype(np.float32)
    Z, g, flag = ws.whiten(_dev(Y32))
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    g = g.cpu().numpy()
    Y64 = Y32.astype(np.float64)
    lib = np.sort(np.linalg.eigvalsh(Y64.T @ Y64))[::-1]
    assert np.abs(g - lib).max() <= 1e-10 * lib[0]
    assert np.abs(g / s ** 2 - 1.0).max() <= 1e-5
    Zg = Z.cpu().numpy().astype(np.float64)
    cosines = np.abs(np.sum(Zg * Q, axis=0)) / np.sqrt(M)
    assert np.abs(cosines - 1.0).max() <= 1e-5
    assert np.abs(Zg.T @ Zg / M - np.eye(r)).max() <= 1e-5


@pytest.mark.parametrize("r", [32, 64])
def test_whitening_exact_equal_diagonals(r):
    """Integer columns y_2i = a_i e_2i + b_i e_2i+1, y_2i+1 = a_i e_2i - b_i e_2i+1
    (all sums exact): each pair block of Y^T Y is [[a^2 + b^2, a^2 - b^2],
    [a^2 - b^2, a^2 + b^2]] with exactly equal diagonal entries (d = 0, the
    rotation's t = 1 case), the other entries are exactly zero, the
    eigenvalues are 2 a_i^2 and 2 b_i^2 and the whitened columns are
    +-sqrt(M) e_2i and +-sqrt(M) e_2i+1."""
    import torch
    from paper_0811_1081_amd import warmstart as ws
    M, P = 1000, r // 2
    a = 40.0 + 2.0 * np.arange(P)  # even, 40 .. 40 + 2(P - 1)
    b = 1.0 + 2.0 * np.arange(P)   # odd: every value distinct
    Y = np.zeros((M, r), dtype=np.float32)
    for i in range(P):
        Y[2 * i, 2 * i], Y[2 * i + 1, 2 * i] = a[i], b[i]
        Y[2 * i, 2 * i + 1], Y[2 * i + 1, 2 * i + 1] = a[i], -b[i]
    Z, g, flag = ws.whiten(_dev(Y))
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    exact = np.sort(np.concatenate([2 * a ** 2, 2 * b ** 2]))[::-1]
    g = g.cpu().numpy()
    assert np.abs(g / exact - 1.0).max() <= 1e-13
    Zg = np.abs(Z.cpu().numpy().astype(np.float64)) / np.sqrt(M)
    # each whitened column is one unit vector: its row is 2i for eigenvalue
    # 2 a_i^2 and 2i + 1 for 2 b_i^2
    rows = [2 * int(np.where(a == np.sqrt(v / 2))[0][0]) if np.any(a == np.sqrt(v / 2))
            else 2 * int(np.where(b == np.sqrt(v / 2))[0][0]) + 1 for v in exact]
    expect = np.zeros((M, r))
    expect[rows, np.arange(r)] = 1.0
    assert np.abs(Zg - expect).max() <= 1e-6


def test_forward_matches_oracle(orc):
    import torch
    from paper_0811_1081_amd import warmstart as ws
    net = ws.WarmStartNet(K=DIMS[3], hidden=DIMS[1:3], seed=1, last_zero=False)
    rng = np.random.default_rng(7)
    rows = 3000  # 93.75 tiles of 32 rows: a ragged edge
    Z = rng.standard_normal((rows, 32)).astype(np.float32)
    # non-zero biases so that the bias path is exercised
    p = net.unpack(net.theta.cpu().numpy())
    for i in (1, 3, 5):
        p[i][:] = 0.1 * rng.standard_normal(p[i].shape)
    net.theta.copy_(torch.from_numpy(np.concatenate([x.ravel() for x in p]).astype(np.float32)))
    net.sync()
    O = net.forward(_dev(Z))
    torch.cuda.synchronize()
    params = _oracle_params(orc, net)
    H1, H2, Oo = orc.mlp_forward(orc.bf16_round(Z), params, round_bf16=True, skip=Z)
    assert _rel(O.cpu().numpy(), Oo) <= 2e-3
    # the bf16 copy is exactly the rounded master
    tb = (net.theta_bf16.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(tb.astype(np.float64), orc.bf16_round(net.theta.cpu().numpy()))


def _unit_scores(rng, ninst, Mi, K):
    V = np.zeros((ninst, K, Mi))  # per matrix: column-major Mi x K
    for b in range(ninst):
        q = np.linalg.qr(rng.standard_normal((Mi, K)))[0]
        V[b] = q.T
    return V


def test_loss_and_gradients_match_oracle(orc):
    import torch
    from paper_0811_1081_amd import warmstart as ws
    net = ws.WarmStartNet(K=DIMS[3], hidden=DIMS[1:3], seed=2, last_zero=False)
    rng = np.random.default_rng(8)
    ninst, Mi, K = 3, 700, DIMS[3]
    Z = rng.standard_normal((ninst * Mi, 32)).astype(np.float32)
    V = _unit_scores(rng, ninst, Mi, K).astype(np.float32)
    loss = net.loss_grad(_dev(Z), _dev(V.ravel()), ninst, Mi)
    torch.cuda.synchronize()
    g_gpu = net.unpack(net.grad.cpu().numpy())
    params = _oracle_params(orc, net)
    Zr = orc.bf16_round(Z)
    H1, H2, O = orc.mlp_forward(Zr, params, round_bf16=True, skip=Z)
    dO = np.zeros_like(O)
    L = 0.0
    for b in range(ninst):
        r = slice(b * Mi, (b + 1) * Mi)
        Lb, dOb = orc.cos2_loss(O[r], V[b].T.astype(np.float64))
        L += Lb / ninst
        dO[r] = dOb / ninst
    g_orc = orc.mlp_backward(Zr, params, H1, H2, orc.bf16_round(dO), round_bf16=True)
    assert abs(loss.item() - L) <= 1e-4 * L
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    for n, a, b in zip(names, g_gpu, g_orc):
        assert _rel(a, b) <= 2e-3, n


def test_adam_matches_oracle(orc):
    import torch
    from paper_0811_1081_amd import warmstart as ws
    net = ws.WarmStartNet(K=4, hidden=(32, 48), seed=3)
    rng = np.random.default_rng(9)
    w = net.theta.cpu().numpy().astype(np.float64)
    m1 = np.zeros_like(w)
    m2 = np.zeros_like(w)
    for t in (1, 2, 3):
        g = rng.standard_normal(w.size).astype(np.float32)
        net.grad.copy_(torch.from_numpy(g))
        net.adam(lr=1e-2)
        orc.adam_step(w, g.astype(np.float64), m1, m2, 1e-2, t)
    torch.cuda.synchronize()
    assert net.step == 3
    wg = net.theta.cpu().numpy()
    assert np.abs(wg - w).max() <= 1e-6 * (np.abs(w).max() + 1e-2)
    tb = (net.theta_bf16.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(tb.astype(np.float64), orc.bf16_round(wg))


def test_predict_composes_sketch_whiten_forward(orc):
    import torch
    from paper_0811_1081_amd import synth, warmstart as ws
    # a flat spectrum keeps every whitened direction well conditioned in FP32
    M, N = 1500, 128
    X = synth.haar_spectrum(M, N, np.linspace(1.0, 0.3, N), 0.0, seed=(15, 1), centre=False,
                            dtype=np.float32)
    net = ws.WarmStartNet(K=8, hidden=(64, 64), seed=4, last_zero=False)
    params = _oracle_params(orc, net)
    for r, power in ((32, 0), (32, 1), (64, 2)):
        Om = synth.sketch_matrix(N, r)
        T0 = net.predict(_colmajor(X), _dev(Om), power=power)
        torch.cuda.synchronize()
        _, Zo, _ = orc.sketch_whiten(X, Om, power=power)
        Zo = np.ascontiguousarray(Zo[:, :32])  # the network reads the first 32 directions
        _, _, Oo = orc.mlp_forward(orc.bf16_round(Zo), params, round_bf16=True, skip=Zo)
        assert T0.stride() == (1, M)
        assert _rel(T0.cpu().numpy(), Oo) <= 5e-3, (r, power)


def test_untrained_network_returns_the_sketch_directions():
    """With the last layer zero the output is the skip term: the first K
    whitened directions, exactly (FP32 copy)."""
    import torch
    from paper_0811_1081_amd import warmstart as ws
    net = ws.WarmStartNet(K=12, seed=6)
    Z = torch.randn(777, 32, device="cuda")
    O = net.forward(Z)
    torch.cuda.synchronize()
    assert torch.equal(O, Z[:, :12])


def test_errors_are_reported_on_host():
    import torch
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import warmstart as ws
    X = torch.zeros((10, 5), dtype=torch.float32, device="cuda").t().contiguous().t()
    with pytest.raises(ValueError):
        ws.sketch(X, torch.zeros((4, 32), device="cuda"))
    with pytest.raises(gp.GspcaError):
        ws.whiten(torch.zeros((10, 32), device="cuda"))  # M < 32
    net = ws.WarmStartNet(K=4, hidden=(32, 32), seed=0)
    with pytest.raises(gp.GspcaError):
        net.adam(lr=0.0)


def test_three_arms_trained_skip_maxnorm():
    """What the trained network gains, on held-out matrices of the warm-start
    family (s_j = r^j, r ~ U[0.7, 0.95], Haar factors; 512 x 128, K = 8):
    fits from the max-norm column, from the network's skip path alone (the
    untrained network: the first K whitened sketch directions) and from the
    trained network, the epoch chosen by the loss on held-out training
    matrices (epoch 0 = the untrained network).  Stated margins: the sketch
    start needs at most half the iterations of the max-norm start, and the
    trained network at most 2 % more than its skip path.  The trained
    network is not required to need fewer: for Haar factors the sketch's
    Ritz directions are already the best start a row-wise map of the sketch
    can give (at the workload's size, 15488 training matrices, no epoch
    lowers the held-out loss below the skip path's, so epoch 0 is chosen)."""
    import torch
    from paper_0811_1081_amd import synth, warmstart as ws
    M, N, K = 512, 128, 8
    Om = _dev(synth.sketch_matrix(N, 32))
    _, Ztr, Vtr, _ = ws.prepare(range(0, 48), M, N, K, Om, power=1)
    _, Zva, Vva, _ = ws.prepare(range(48, 56), M, N, K, Om, power=1)
    Xev, Zev, _, Vtrue = ws.prepare(range(16000, 16024), M, N, K, Om, power=1, keep_x=True)
    net = ws.WarmStartNet(K=K, hidden=(256, 256), seed=5)
    Zt, Vt = torch.cat(Ztr), torch.stack(Vtr)
    Zv, Vv = torch.cat(Zva), torch.stack(Vva).reshape(-1)
    best = net.loss_grad(Zv, Vv, 8, M).item()
    skip_loss, best_theta = best, net.theta.clone()
    per = 16
    for epoch in range(4):
        for j in range(0, 48, per):
            net.train_step(Zt[j * M:(j + per) * M], Vt[j:j + per].reshape(-1), per, M, lr=3e-4)
        v = net.loss_grad(Zv, Vv, 8, M).item()
        if v < best:
            best, best_theta = v, net.theta.clone()
    net.theta.copy_(best_theta)
    net.sync()
    assert best <= skip_loss
    r = ws.evaluate(net, Xev, Zev, Vtrue, K, Om, tol=1e-6)
    it = {k: v["iters_per_matrix_mean"] for k, v in r.items()}
    print("iterations per matrix:", it, "validation loss skip %.5f chosen %.5f"
          % (skip_loss, best))
    assert all(v["status_ok"] for v in r.values())
    assert it["skip_only"] <= 0.5 * it["maxnorm"], it
    assert it["trained"] <= 1.02 * it["skip_only"] + 1.0, it
    assert it["trained"] <= 0.5 * it["maxnorm"], it
    # at equal final error: the loading stop, errors against the generator's factors
    r = ws.evaluate(net, Xev, Zev, Vtrue, K, Om, tol=1e-4, stop="loading")
    it = {k: v["iters_per_matrix_mean"] for k, v in r.items()}
    e = {k: v["loading_error_median"] for k, v in r.items()}
    print("loading stop: iterations", it, "median loading error", e)
    assert it["skip_only"] <= 0.5 * it["maxnorm"], it
    assert it["trained"] <= 1.02 * it["skip_only"] + 1.0, it
    assert e["trained"] <= 2.0 * e["skip_only"] and e["skip_only"] <= 2.0 * e["maxnorm"], e
