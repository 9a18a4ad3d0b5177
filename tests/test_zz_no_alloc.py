"""gspca_fit_noalloc (the fit of gspca_fit_ex with the library's fixed per-GPU
scratch array as its workspace) against gspca_fit_ex on the same inputs.

Method: Andrecut, arXiv:0811.1081, Sec. 2.3 (GS-PCA) and Sec. 2.2 (NIPALS).
Both entry points run the same kernels in the same launch shapes on the same
data, and every reduction has a fixed order, so the outputs must agree bit
for bit; the oracle bar (sign-aligned angle <= 1e-5 for FP32, <= 1e-10 for
FP64) is implied.  Two calls in a row, the second on a smaller problem, show
that what the first call left in the shared array does not leak into the
second.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0811_1081_amd as gp
    gp.load()


def _dev(X):
    import torch
    import paper_0811_1081_amd as gp
    return gp.column_major(torch.from_numpy(X).to("cuda"))


def _same(a, b):
    import torch
    torch.cuda.synchronize()
    assert a["status"] == b["status"]
    for k in ("T", "P", "lambda", "sigma", "iters", "start_col"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("dtype,algo,implicit", [
    (np.float32, "gs", False), (np.float32, "gs", True), (np.float64, "gs", False),
    (np.float32, "nipals", False)])
def test_noalloc_matches_fit_ex_twice(dtype, algo, implicit):
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    tol = 1e-6 if dtype == np.float32 else 1e-10
    cases = [((3001, 203, 10), (40, 0)), ((517, 100, 6), (40, 1))]   # second one smaller
    for (M, N, K), seed in cases:
        X = synth.haar_spectrum(M, N, 0.85 ** np.arange(40), 1e-4, seed=seed, dtype=dtype)
        Xd = _dev(X)
        ref = gp.fit(Xd, K, tol=tol, max_iter=2000, algo=algo, implicit=implicit)
        out = gp.fit(Xd, K, tol=tol, max_iter=2000, algo=algo, implicit=implicit, noalloc=True)
        assert ref["status"] == 0
        _same(out, ref)


def test_noalloc_full_rank_collinear_fits_in_scratch():
    """The 4096 x 512 FP32 full-rank case (K = N = 512 needs ~12 MiB of
    workspace) fits the fixed array; a shorter run is compared here."""
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    L = gp.load()
    X = synth.case_collinear_f32()
    Xd = _dev(X)
    nb = gp.workspace_bytes(Xd, 512)
    assert 0 < nb <= int(L.gspca_noalloc_scratch_bytes())
    ref = gp.fit(Xd, 40, tol=1e-6, max_iter=300, check=False)
    out = gp.fit(Xd, 40, tol=1e-6, max_iter=300, check=False, noalloc=True)
    _same(out, ref)


def test_noalloc_refusals():
    import torch
    import paper_0811_1081_amd as gp
    L = gp.load()
    cap = int(L.gspca_noalloc_scratch_bytes())
    assert cap == 32 << 20
    # a problem whose workspace exceeds the array: EWORKSPACE, nothing run
    X = torch.zeros((4096, 4096), dtype=torch.float32, device="cuda").t()   # column-major
    assert gp.workspace_bytes(X, 4) > cap
    with pytest.raises(gp.GspcaError) as e:
        gp.fit(X, 4, noalloc=True)
    assert e.value.status == gp.EWORKSPACE
    # replay arrays and profiles are refused
    Y = torch.ones((64, 8), dtype=torch.float32, device="cuda").t().contiguous().t()
    it = torch.full((2,), 3, dtype=torch.int32, device="cuda")
    sc = torch.full((2,), -1, dtype=torch.int32, device="cuda")
    with pytest.raises(gp.GspcaError) as e:
        gp.fit(Y, 2, replay_iters=it, replay_start=sc, noalloc=True)
    assert e.value.status == gp.EINVAL
    with pytest.raises(gp.GspcaError) as e:
        gp.fit(Y, 2, profile=gp.Profile(), noalloc=True)
    assert e.value.status == gp.EINVAL
