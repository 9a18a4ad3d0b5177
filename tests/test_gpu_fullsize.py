"""GPU parity at the workload sizes and in the launch shapes the benchmark uses.

Method: Andrecut, arXiv:0811.1081, Sec. 2.3 (GS-PCA) and Sec. 2.2 (NIPALS-PCA),
through the C ABI.  Three kinds of check:

* Replayed trajectories at full width: the fused single pass with 8 and 16
  columns per thread (N = 3000 and N = 8192 in FP32, N = 4000 in FP64), with
  enough rows that every workgroup walks several interleaved row panels and
  the last panel is ragged; BF16 and FP8 codes at N = 8192 against the oracle
  run on the exactly dequantised matrix.  Element-by-element against the FP64
  oracle replaying the GPU's iteration counts and start columns.
* The full-rank collinear workload (4096 x 512, K = N = 512) and 64 instances
  of the 2048-problem batched workload in the benchmark's launch (tuned
  shape, hipGraph replay), against the oracle on the same trajectories.
* The 65536 x 8192 benchmark fit (K = 32, tol 1e-6; FP32 with explicit
  deflation, and BF16 / FP8 codes): at that size the oracle computes sampled
  outputs one by one -- the score step of Sec. 2.3 (t = R_k p, Gram-Schmidt
  against the earlier scores, sigma = |t|) from the GPU's own final loading
  and earlier components, which must reproduce the GPU's score and sigma
  (a relation that holds at every iteration, converged or not) -- plus the
  orthogonality of P and of the normalised scores.

Tolerances: FP64 angle <= 1e-10 and sigma within 1e-12 sigma_0; FP32 and codes
angle <= 1e-5 on components with a relative gap >= 2 % to both neighbours
(FP32 rounding of the residual, ~6e-8 per element, amplified by 1/gap) and
sigma within 1e-5 relative; the score step is one product with no gap
amplification (bound 1e-5 on the angle, 1e-6 relative on sigma).
"""
import numpy as np
import pytest

from metrics import col_angles, gapped, orth_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


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


def _say(msg):
    print("[fullsize] " + msg, flush=True)


def _replay(orc, X, g, K, algo="gs", implicit=False, tiny=None):
    kw = {} if tiny is None else {"tiny": tiny}
    return orc.fit(X, K, tol=0.0, max_iter=max(1, int(g["iters"].max())), algo=algo,
                   implicit=implicit, replay_iters=g["iters"], replay_start=g["start_col"], **kw)


def _check_replay(o, g, bound, sig_rel):
    ok = gapped(o.sigma)
    assert ok.any()
    assert col_angles(g["P"], o.P)[ok].max() <= bound
    assert col_angles(g["T"], o.T)[ok].max() <= bound
    assert np.abs(g["sigma"] / o.sigma - 1).max() <= sig_rel


# --------------------------------------------------------------------------
# Full-width fused pass: 16 and 8 columns per thread (512 threads), FP32.
# 16397 rows = 4100 panels of 4 rows: 16 per workgroup at 256 workgroups, the
# last one holding a single row.

_WIDE = {}


def _wide_matrix(N):
    if N not in _WIDE:
        from paper_0811_1081_amd import synth
        _WIDE.clear()
        _WIDE[N] = synth.haar_spectrum(16397, N, 10.0 * 0.55 ** np.arange(16), 1e-3,
                                       seed=(30, N), dtype=np.float32)
    return _WIDE[N]


@pytest.mark.parametrize("N,algo,implicit", [
    (8192, "gs", False), (8192, "gs", True), (8192, "nipals", False),
    (3000, "gs", False), (3000, "gs", True)])
def test_fused_f32_full_width(orc, N, algo, implicit):
    X = _wide_matrix(N)
    K = 3
    _say("fp32 16397x%d %s implicit=%s" % (N, algo, implicit))
    g = _gh().gpu_fit(X, K, tol=1e-6, max_iter=500, algo=algo, implicit=implicit)
    assert g["status"] == 0
    o = _replay(orc, X, g, K, algo, implicit, tiny=orc.FLT_MIN)
    _check_replay(o, g, 1e-5, 1e-5)
    free = orc.fit(X, K, tol=1e-6, max_iter=500, algo=algo, implicit=implicit, tiny=orc.FLT_MIN)
    assert np.array_equal(free.start_col, g["start_col"])
    if algo == "gs":
        assert orth_err(g["P"]) <= 1e-6
        assert orth_err(g["T"] / g["sigma"]) <= 1e-6


@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_quantized_full_width(orc, fmt):
    """Codes at N = 8192 (BF16: 8 rows per panel, FP8: 16; two workgroups per
    compute unit) against the oracle on the dequantised matrix X~."""
    import paper_0811_1081_amd as gp
    X = _wide_matrix(8192)
    K = 3
    _say("%s 16397x8192" % fmt)
    q = gp.quantize(_gh().to_device(X), fmt)
    g = _gh().gpu_fit(q, K, tol=1e-6, max_iter=500)
    assert g["status"] == 0
    codes, scale = orc.quantize(X, fmt)
    Xt = orc.dequantize(codes, scale, fmt)
    del codes
    o = _replay(orc, Xt, g, K, implicit=True, tiny=orc.FLT_MIN)
    _check_replay(o, g, 1e-5, 1e-5)
    assert orth_err(g["P"]) <= 1e-6


def test_fused_f64_eight_columns_per_thread(orc):
    """FP64 at N = 4000: 8 columns per thread, 2 rows per panel, 8195 rows =
    4098 panels (16 per workgroup, the last one ragged)."""
    from paper_0811_1081_amd import synth
    X = synth.haar_spectrum(8195, 4000, 10.0 * 0.55 ** np.arange(16), 1e-6, seed=(31, 0))
    K = 3
    _say("fp64 8195x4000")
    for implicit in (False, True):
        g = _gh().gpu_fit(X, K, tol=1e-10, max_iter=500, implicit=implicit)
        assert g["status"] == 0
        o = _replay(orc, X, g, K, implicit=implicit)
        assert col_angles(g["P"], o.P).max() <= 1e-10
        assert col_angles(g["T"], o.T).max() <= 1e-10
        assert np.abs(g["sigma"] - o.sigma).max() <= 1e-12 * o.sigma[0]


# --------------------------------------------------------------------------
# The full-rank collinear workload at its own size.

def test_collinear_full_rank_full_size(orc):
    """4096 x 512 FP32, K = N = 512, tol 1e-6, max_iter 1000 (the noise-level
    components run to the cap: NOT_CONVERGED is the expected status).  GS-PCA
    keeps both bases orthonormal to <= 1e-6; the squared sigmas add up to
    |X|_F^2 (each deflation removes exactly |t|^2); the leading 24
    components (signal well above the 1e-4 noise) match the oracle replaying
    the GPU's counts and start columns."""
    from paper_0811_1081_amd import synth
    X = synth.case_collinear_f32()
    K = 512
    _say("collinear 4096x512 K=512")
    g = _gh().gpu_fit(X, K, tol=1e-6, max_iter=1000, check=False)
    assert g["status"] in (0, 1)
    assert orth_err(g["P"]) <= 1e-6
    assert orth_err(g["T"] / np.where(g["sigma"] > 0, g["sigma"], 1.0)) <= 1e-6
    fro2 = float((X.astype(np.float64) ** 2).sum())
    assert abs(float(g["lambda"].sum()) / fro2 - 1.0) <= 1e-5
    K0 = 24
    sub = {k: (v[:, :K0] if k in ("T", "P") else v[:K0]) for k, v in g.items() if k != "status"}
    o = _replay(orc, X, sub, K0, tiny=orc.FLT_MIN)
    _check_replay(o, sub, 1e-5, 1e-5)


# --------------------------------------------------------------------------
# The batched workload: all 2048 problems in the benchmark's launch, 64 checked.

def _batched_sample(shapes):
    idx = set()
    order = np.argsort([-m * n for m, n, _ in shapes])
    idx.update(int(i) for i in order[:16])                                   # largest M N
    idx.update([i for i, (m, n, _) in enumerate(shapes) if m >= 4000][:16])
    idx.update([i for i, (m, n, _) in enumerate(shapes) if n >= 500][:16])
    rng = np.random.default_rng(4)
    for i in rng.permutation(len(shapes)):
        if len(idx) >= 64:
            break
        idx.add(int(i))
    return sorted(idx)[:64]


def test_batched_workload_sample(orc):
    import torch
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    shapes = synth.batched_shapes(2048)
    _say("batched: generating 2048 problems")
    host = synth.map_threads(lambda a: synth.batched_instance(*a),
                             [(i, m, n) for i, (m, n, _) in enumerate(shapes)], workers=16)
    sample = _batched_sample(shapes)
    keep = {i: host[i] for i in sample}
    Xs = [gp.column_major(torch.from_numpy(x).cuda()) for x in host]
    del host
    Ks = [k for _, _, k in shapes]
    b = gp.Batch(Xs, Ks, tol=1e-6, max_iter=1000)
    b.tune()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        b.launch(stream=s)
    graph.replay()
    torch.cuda.synchronize()
    st = b.status.cpu().numpy()
    assert np.all(st == 0)
    assert any(shapes[i][0] >= 4000 for i in sample) and any(shapes[i][1] >= 500 for i in sample)
    _say("batched: checking %d problems against the oracle" % len(sample))
    for i in sample:
        X, K = keep[i], Ks[i]
        it = b.iters[i].cpu().numpy()
        sc = b.start_col[i].cpu().numpy()
        o = orc.fit(X, K, tol=0.0, max_iter=max(1, int(it.max())), implicit=True,
                    replay_iters=it, replay_start=sc, tiny=orc.FLT_MIN)
        P, T, sig = b.P[i].cpu().numpy(), b.T[i].cpu().numpy(), b.sigma[i].cpu().numpy()
        ok = gapped(o.sigma)
        if ok.any():
            assert col_angles(P, o.P)[ok].max() <= 1e-5, (i, shapes[i])
            assert col_angles(T, o.T)[ok].max() <= 1e-5, (i, shapes[i])
        assert np.abs(sig - o.sigma).max() <= 1e-5 * o.sigma[0], (i, shapes[i])
        assert orth_err(P) <= 1e-5


# --------------------------------------------------------------------------
# The 65536 x 8192 benchmark fit: sampled score steps computed by the oracle.

_LARGE = {}


def _large():
    """The benchmark's input (FP32) and one FP64 buffer of its size that each
    test fills with the matrix the oracle reads (X, or the dequantised X~)."""
    if not _LARGE:
        from paper_0811_1081_amd import synth
        _say("large: generating 65536x8192")
        _LARGE["X"] = synth.case_large_f32()
        _LARGE["X64"] = np.empty(_LARGE["X"].shape, dtype=np.float64, order="F")
    return _LARGE["X"], _LARGE["X64"]


def _score_step_checks(orc, X64, g, ks):
    P = g["P"].astype(np.float64)
    sig = g["sigma"]
    V = g["T"].astype(np.float64) / sig
    for k in ks:
        v, s = orc.score_step(X64, k, V, sig, P, P[:, k])
        assert abs(s / sig[k] - 1.0) <= 1e-6, (k, s, sig[k])
        assert col_angles(V[:, k:k + 1], v[:, None])[0] <= 1e-5, k


@pytest.mark.parametrize("form", ["f32", "bf16", "e4m3"])
def test_large_workload_score_steps(orc, form):
    import torch
    import paper_0811_1081_amd as gp
    X, X64 = _large()
    K = 32
    Xd = _gh().to_device(X)
    _say("large %s: fit" % form)
    if form == "f32":
        g = _gh().gpu_fit(Xd, K, tol=1e-6, max_iter=1000)   # explicit deflation
        del Xd
        np.copyto(X64, X)                                    # exact widening
    else:
        q = gp.quantize(Xd, form)
        del Xd
        g = _gh().gpu_fit(q, K, tol=1e-6, max_iter=1000)
        del q
        codes, scale = orc.quantize(X, form)
        orc.dequantize(codes, scale, form, out=X64)
        del codes
    torch.cuda.empty_cache()
    assert g["status"] == 0
    assert orth_err(g["P"]) <= 1e-6
    assert orth_err(g["T"] / g["sigma"]) <= 1e-6
    assert np.all(np.diff(g["sigma"]) < 0)
    _say("large %s: oracle score steps" % form)
    _score_step_checks(orc, X64, g, [0, 1, 2, 15, 30, 31])
