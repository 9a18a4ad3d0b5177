"""Helpers for the GPU tests: move seeded numpy inputs to the device, run the
library through its C ABI, bring results back.  No PCA arithmetic here."""
from __future__ import annotations

import numpy as np


def to_device(X, dtype=None):
    import torch
    import paper_0811_1081_amd as gp
    t = torch.from_numpy(np.asarray(X, dtype=dtype) if dtype is not None else np.asarray(X))
    return gp.column_major(t.to("cuda"))


def gpu_fit(X, K, **kw):
    """Run the library on host array X; returns numpy copies of every output."""
    import torch
    import paper_0811_1081_amd as gp
    Xd = X if (hasattr(X, "is_cuda") or isinstance(X, gp.Quantized)) else to_device(X)
    out = gp.fit(Xd, K, **kw)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    return res


def replay_args(res):
    import torch
    it = torch.from_numpy(np.ascontiguousarray(res["iters"], dtype=np.int32)).cuda()
    sc = torch.from_numpy(np.ascontiguousarray(res["start_col"], dtype=np.int32)).cuda()
    return it, sc
