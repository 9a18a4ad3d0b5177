"""GPU tests of the batched form: many independent GS-PCA problems (Sec. 2.3,
implicit deflation) in one persistent launch, hipGraph capture, autotuner.

Each sampled problem is checked against the FP64 oracle replaying the GPU's
iteration counts and start columns (FP32 bound 1e-5 on gapped components).
"""
import os

import numpy as np
import pytest

from metrics import col_angles, orth_err

pytestmark = pytest.mark.gpu


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


def _gapped(sig, rel=0.02):
    s = np.asarray(sig, dtype=np.float64)
    ok = np.ones(len(s), dtype=bool)
    for k in range(len(s)):
        if k > 0 and s[k] > (1 - rel) * s[k - 1]:
            ok[k] = False
        if k + 1 < len(s) and s[k + 1] > (1 - rel) * s[k]:
            ok[k] = False
    return ok


def _problems(count, seed, mmax=700, nmax=160):
    from paper_0811_1081_amd import synth
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        M = int(rng.integers(16, mmax))
        N = int(rng.integers(4, nmax))
        r = min(M, N, 12)
        X = synth.haar_spectrum(M, N, 0.75 ** np.arange(r), 1e-3, seed=(14, seed * 1000 + i),
                                dtype=np.float32)
        out.append((X, min(6, M, N)))
    return out


def _check(orc, X, K, T, P, sig, iters, start, directions=None):
    """Replay the GPU's trajectory in the oracle; angles of the gapped
    components among the first `directions` (all by default)."""
    o = orc.fit(X, K, tol=0.0, max_iter=max(1, int(iters.max())), implicit=True,
                replay_iters=iters, replay_start=start, tiny=orc.FLT_MIN)
    ok = _gapped(o.sigma)
    if directions is not None:
        ok[directions:] = False
    if ok.any():
        assert col_angles(P, o.P)[ok].max() <= 1e-5
        assert col_angles(T, o.T)[ok].max() <= 1e-5
    assert np.abs(sig - o.sigma).max() <= 1e-5 * o.sigma[0]
    assert orth_err(P) <= 1e-5


def test_batched_matches_oracle(orc):
    import torch
    import paper_0811_1081_amd as gp
    probs = _problems(40, seed=1)
    Xs = [_gh().to_device(X) for X, _ in probs]
    b = gp.Batch(Xs, [k for _, k in probs], tol=1e-6, max_iter=1000)
    b.launch()
    torch.cuda.synchronize()
    st = b.status.cpu().numpy()
    assert np.all(st == 0)
    for i, (X, K) in enumerate(probs):
        _check(orc, X, K, b.T[i].cpu().numpy(), b.P[i].cpu().numpy(), b.sigma[i].cpu().numpy(),
               b.iters[i].cpu().numpy(), b.start_col[i].cpu().numpy())
        free = orc.fit(X, K, tol=1e-6, max_iter=1000, implicit=True, tiny=orc.FLT_MIN)
        assert np.array_equal(free.start_col, b.start_col[i].cpu().numpy())
        assert np.array_equal(b.lam[i].cpu().numpy(), b.sigma[i].cpu().numpy() ** 2)


def test_batched_rank_deficient(orc):
    """Exactly low-rank matrices (rank 3, no noise) asked for 6 components:
    the components past the rank sit at the FP32 rounding floor, where the
    score's Gram-Schmidt products taken inside the pass cancel (|d| close to
    |t|) and the step is taken explicitly.  Parity with the FP64 oracle on
    the same trajectory for the three real components (directions) and for
    every sigma (the ones past the rank below 1e-5 sigma_0 on both sides;
    their directions are rounding noise, set by the arithmetic, and are not
    compared); loadings orthonormal."""
    import torch
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    shapes = [(300, 40), (200, 100), (700, 260), (90, 33), (1000, 512), (64, 16)]
    probs = []
    for i, (M, N) in enumerate(shapes):
        X = synth.haar_spectrum(M, N, np.array([1.0, 0.6, 0.3]), 0.0, seed=(14, 70_000 + i),
                                dtype=np.float32)
        probs.append((X, 6))
    Xs = [_gh().to_device(X) for X, _ in probs]
    b = gp.Batch(Xs, [k for _, k in probs], tol=1e-6, max_iter=300)
    b.launch()
    torch.cuda.synchronize()
    st = b.status.cpu().numpy()
    assert np.all((st == 0) | (st == 1))
    for i, (X, K) in enumerate(probs):
        sig = b.sigma[i].cpu().numpy()
        assert sig[3:].max() <= 1e-5 * sig[0]
        _check(orc, X, K, b.T[i].cpu().numpy(), b.P[i].cpu().numpy(), sig,
               b.iters[i].cpu().numpy(), b.start_col[i].cpu().numpy(), directions=3)


def test_batched_padded_leading_dimension():
    """Columns padded to a 128-byte multiple (and odd paddings), NaN in the
    padding rows: the kernel reads none of them, and the fit is bitwise the
    one of the unpadded matrices."""
    import torch
    import paper_0811_1081_amd as gp
    probs = _problems(12, seed=7, mmax=1500, nmax=300)
    Ks = [k for _, k in probs]
    dense = [_gh().to_device(X) for X, _ in probs]
    padded = []
    for i, (X, _) in enumerate(probs):
        M, N = X.shape
        ld = -(-M // 32) * 32 + (0 if i % 3 else 7)
        store = torch.full((N, ld), float("nan"), dtype=torch.float32, device="cuda")
        store[:, :M] = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
        Xp = store.t()[:M]
        assert Xp.stride() == (1, ld) and torch.equal(Xp, dense[i])
        padded.append(Xp)
    a = gp.Batch(dense, Ks, tol=1e-6, max_iter=1000)
    b = gp.Batch(padded, Ks, tol=1e-6, max_iter=1000)
    a.launch()
    b.launch()
    torch.cuda.synchronize()
    assert np.all(a.status.cpu().numpy() == 0) and np.all(b.status.cpu().numpy() == 0)
    for i in range(len(probs)):
        for x, y in ((a.T[i], b.T[i]), (a.P[i], b.P[i]), (a.sigma[i], b.sigma[i]),
                     (a.iters[i], b.iters[i]), (a.start_col[i], b.start_col[i])):
            assert torch.equal(x, y), i


def test_batched_equals_single_fit_trajectory(orc):
    """The batched kernel and the single-problem library path run the same
    method: with the same replayed counts their results agree."""
    import torch
    import paper_0811_1081_amd as gp
    probs = _problems(6, seed=2, mmax=2000, nmax=300)
    Xs = [_gh().to_device(X) for X, _ in probs]
    b = gp.Batch(Xs, [k for _, k in probs], tol=1e-6)
    b.launch()
    torch.cuda.synchronize()
    for i, (X, K) in enumerate(probs):
        g = gp.fit(Xs[i], K, implicit=True, tol=0.0, max_iter=int(b.iters[i].max()),
                   replay_iters=b.iters[i], replay_start=b.start_col[i])
        ok = _gapped(b.sigma[i].cpu().numpy())
        assert col_angles(g["P"].cpu().numpy(), b.P[i].cpu().numpy())[ok].max() <= 1e-5


def test_batched_replay_and_status():
    import torch
    import paper_0811_1081_amd as gp
    probs = _problems(5, seed=3)
    X_bad = np.ones((50, 10), dtype=np.float32)
    X_bad[3, 4] = np.nan
    Xs = [_gh().to_device(X) for X, _ in probs] + [_gh().to_device(X_bad)]
    Ks = [k for _, k in probs] + [2]
    its = [torch.full((k,), 3, dtype=torch.int32, device="cuda") for k in Ks]
    scs = [torch.full((k,), -1, dtype=torch.int32, device="cuda") for k in Ks]
    b = gp.Batch(Xs, Ks, tol=1e-6, replay_iters=its, replay_start=scs)
    b.launch()
    torch.cuda.synchronize()
    st = b.status.cpu().numpy()
    assert list(st[:-1]) == [0] * 5 and st[-1] == gp.ENONFINITE
    for i in range(5):
        assert np.all(b.iters[i].cpu().numpy() == 3)
    b2 = gp.Batch(Xs[:5], Ks[:5], tol=1e-12, max_iter=2)
    b2.launch()
    torch.cuda.synchronize()
    assert np.all(b2.status.cpu().numpy() == gp.NOT_CONVERGED)


def test_batched_graph_replays_match_eager():
    import torch
    import paper_0811_1081_amd as gp
    probs = _problems(24, seed=4)
    Xs = [_gh().to_device(X) for X, _ in probs]
    b = gp.Batch(Xs, [k for _, k in probs], tol=1e-6)
    b.launch()
    torch.cuda.synchronize()
    ref = [p.clone() for p in b.P]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.launch(stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for P in b.P:
            P.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for P, R in zip(b.P, ref):
            assert torch.equal(P, R), rep
        _ = torch.ones(10, device="cuda").sum().item()  # eager work between replays


def test_batched_autotune_and_cache(tmp_path):
    import torch
    import paper_0811_1081_amd as gp
    probs = _problems(30, seed=5)
    Xs = [_gh().to_device(X) for X, _ in probs]
    cache = tmp_path / "tune.jsonl"
    os.environ["GSPCA_TUNE_CACHE"] = str(cache)
    try:
        b = gp.Batch(Xs, [k for _, k in probs], tol=1e-6)
        b.tune()
        shape = b.shape()
        assert shape[0] in (256, 512, 1024) and 1 <= shape[1] <= 4
        lines = cache.read_text().strip().splitlines()
        assert len(lines) == 1 and '"threads":%d' % shape[0] in lines[0]
        b2 = gp.Batch(Xs, [k for _, k in probs], tol=1e-6)  # picks the cached shape
        assert b2.shape() == shape
        b2.launch()
        torch.cuda.synchronize()
        assert np.all(b2.status.cpu().numpy() == 0)
    finally:
        del os.environ["GSPCA_TUNE_CACHE"]


def test_batched_given_start(orc):
    """Warm-started batch: given vectors are used unless they fail the
    fallback rule (non-finite, or less than a tenth outside the earlier
    scores); results follow the oracle on the same start choice."""
    import torch
    import paper_0811_1081_amd as gp
    probs = _problems(8, seed=6, mmax=600, nmax=120)
    rng = np.random.default_rng(66)
    Xs, T0s, T0h = [], [], []
    for X, K in probs:
        ref = orc.fit(X, K, tol=1e-8, max_iter=2000, implicit=True, tiny=orc.FLT_MIN)
        V = ref.V
        M = X.shape[0]
        G = V + 0.3 * rng.standard_normal(V.shape) / np.sqrt(M)
        if K >= 3:
            w = rng.standard_normal(M)
            w -= V[:, :1] @ (V[:, :1].T @ w)
            G[:, 1] = V[:, 0] + 0.05 * w / np.linalg.norm(w)  # inside span(v0): falls back
            G[0, 2] = np.nan                                   # non-finite: falls back
        G = np.asfortranarray(G.astype(np.float32))
        T0h.append(G)
        T0s.append(gp.column_major(torch.from_numpy(np.ascontiguousarray(G)).cuda()))
        Xs.append(_gh().to_device(X))
    b = gp.Batch(Xs, [k for _, k in probs], tol=1e-6, max_iter=1000, init="given", T0=T0s)
    b.launch()
    torch.cuda.synchronize()
    assert np.all(b.status.cpu().numpy() == 0)
    for i, (X, K) in enumerate(probs):
        sc = b.start_col[i].cpu().numpy()
        free = orc.fit(X, K, tol=1e-6, max_iter=1000, implicit=True, tiny=orc.FLT_MIN,
                       init="given", T0=T0h[i].astype(np.float64))
        assert np.array_equal(sc, free.start_col), (i, sc, free.start_col)
        if K >= 3:
            assert sc[0] == -1 and sc[1] >= 0 and sc[2] >= 0
        its = b.iters[i].cpu().numpy()
        o = orc.fit(X, K, tol=0.0, max_iter=max(1, int(its.max())), implicit=True,
                    init="given", T0=T0h[i].astype(np.float64), replay_iters=its,
                    replay_start=sc, tiny=orc.FLT_MIN)
        ok = _gapped(o.sigma)
        if ok.any():
            assert col_angles(b.P[i].cpu().numpy(), o.P)[ok].max() <= 1e-5
    with pytest.raises(ValueError):
        gp.Batch(Xs, [k for _, k in probs], init="given")


@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_batched_single_pass_column_splits(orc, tmp_path, threads):
    """Every workgroup size on shapes at the edges of the single pass's column
    split (one column group, 32 and 64 columns per wave, groups past N, more
    than 64 columns per wave -> two reads) and of its row tiles (M below, at
    and past multiples of 64): parity with the FP64 oracle on the same
    trajectory."""
    import torch
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    shapes = [(5, 4), (63, 16), (64, 31), (65, 32), (200, 33), (130, 64), (300, 65),
              (129, 128), (700, 129), (257, 256), (1000, 257), (333, 300), (1100, 512),
              (520, 513), (300, 1024)]
    probs = []
    for i, (M, N) in enumerate(shapes):
        r = min(M, N, 12)
        X = synth.haar_spectrum(M, N, 0.75 ** np.arange(r), 1e-3, seed=(14, 50_000 + i),
                                dtype=np.float32)
        probs.append((X, min(4, M, N)))
    Xs = [_gh().to_device(X) for X, _ in probs]
    Ks = [k for _, k in probs]
    cache = tmp_path / "tune.jsonl"
    os.environ["GSPCA_TUNE_CACHE"] = str(cache)
    try:
        gp.Batch(Xs, Ks, tol=1e-6).tune()
        line = cache.read_text().strip().splitlines()[0]
        key = line.split('"key":"')[1].split('"')[0]
        cache.write_text('{"key":"%s","threads":%d,"occ":1,"ms":1.0}\n' % (key, threads))
        b = gp.Batch(Xs, Ks, tol=1e-6, max_iter=1000)
        assert b.shape() == (threads, 1)
        b.launch()
        torch.cuda.synchronize()
    finally:
        del os.environ["GSPCA_TUNE_CACHE"]
    assert np.all(b.status.cpu().numpy() == 0)
    for i, (X, K) in enumerate(probs):
        _check(orc, X, K, b.T[i].cpu().numpy(), b.P[i].cpu().numpy(), b.sigma[i].cpu().numpy(),
               b.iters[i].cpu().numpy(), b.start_col[i].cpu().numpy())
