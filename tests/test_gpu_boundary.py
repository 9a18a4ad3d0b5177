"""GPU: behaviour of the C ABI at its boundary under hipGraph capture.

The blocking entry points read their loop state back to the host, which a
captured stream cannot do: each must return GSPCA_EINVAL before enqueuing
anything, so that the capture stays valid and the rest of the captured work
replays.  After the capture the same calls succeed on an ordinary stream.
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


def _small():
    from paper_0811_1081_amd import synth
    return synth.lowrank_gaussian(300, 70, 8, 1e-3, seed=(7, 1))


def test_blocking_calls_refuse_capture():
    import torch
    import paper_0811_1081_amd as gp
    import gpu_helpers as gh
    X64 = _small()
    Xd = gh.to_device(X64)
    X32 = gh.to_device(X64, np.float32)
    K = 3
    nbytes = gp.workspace_bytes(Xd, K)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    y = torch.zeros(8, device="cuda")
    g = torch.cuda.CUDAGraph()
    seen = {}
    with torch.cuda.graph(g):
        out = gp.fit(Xd, K, workspace=ws, check=False)
        seen["fit_ex"] = out["status"]
        try:
            gp.quantize(X32, "bf16")
            seen["quantize"] = 0
        except gp.GspcaError as e:
            seen["quantize"] = e.status
        y.add_(1.0)  # the capture must still hold this
    assert seen["fit_ex"] == gp.EINVAL
    assert seen["quantize"] == gp.EINVAL
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert float(y[0]) == rep + 1.0
    # the same calls on an ordinary stream afterwards
    out = gp.fit(Xd, K, tol=1e-10, max_iter=1000)
    torch.cuda.synchronize()
    assert out["status"] == gp.OK
    q = gp.quantize(X32, "bf16")
    torch.cuda.synchronize()
    assert q.codes.numel() > 0


def test_convenience_and_block_refuse_capture():
    import ctypes
    import torch
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import _binding as b
    import gpu_helpers as gh
    L = b.load()
    X64 = _small()
    Xd = gh.to_device(X64)
    X32 = gh.to_device(X64, np.float32)
    M, N = X64.shape
    K = 3
    T = torch.empty(M * K, dtype=torch.float64, device="cuda")
    P = torch.empty(N * K, dtype=torch.float64, device="cuda")
    lam = torch.empty(K, dtype=torch.float64, device="cuda")
    Om = torch.randn(N, 32, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    y = torch.zeros(8, device="cuda")
    g = torch.cuda.CUDAGraph()
    codes = {}
    with torch.cuda.graph(g):
        s = torch.cuda.current_stream().cuda_stream
        codes["fit"] = int(L.gspca_fit(Xd.data_ptr(), M, N, K, ctypes.c_double(1e-10), 1000,
                                       T.data_ptr(), P.data_ptr(), lam.data_ptr(), s))
        try:
            gp.fit_block(X32, 4, r=32, Omega=Om)
            codes["block"] = 0
        except gp.GspcaError as e:
            codes["block"] = e.status
        y.add_(2.0)
    assert codes["fit"] == gp.EINVAL
    assert codes["block"] == gp.EINVAL
    g.replay()
    torch.cuda.synchronize()
    assert float(y[0]) == 2.0
    st = int(L.gspca_fit(Xd.data_ptr(), M, N, K, ctypes.c_double(1e-10), 1000, T.data_ptr(),
                         P.data_ptr(), lam.data_ptr(), torch.cuda.current_stream().cuda_stream))
    assert st == gp.OK
