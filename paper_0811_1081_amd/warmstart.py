"""Learned warm start for GS-PCA (not in the paper; C ABI in ``include/gspca_ws.h``).

The paper starts each component from a residual column (Secs. 2.2-2.3).  Here
a row-wise network maps the whitened random sketch of X to K start vectors,
which ``fit(..., init="given", T0=...)`` consumes.  Every step -- sketch,
whitening, the bf16 matrix-core forward and backward passes, the loss and
Adam -- runs in ``libgspca.so``; this module only allocates tensors and passes
pointers.

    net = WarmStartNet(K=16, seed=0)
    T0 = net.predict(X, Omega)                    # X column-major float32 (M, N)
    out = gp.fit(X, 16, init="given", T0=T0)
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _binding as _b
from ._binding import OK, GspcaError

RANK = _b.WS_RANK


def _stream(stream, dev):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    return stream.cuda_stream


def _check(st):
    st = int(st)
    if st != OK:
        raise GspcaError(st)


def _aligned(nbytes, dev):
    import torch
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=dev)
    return buf, buf.data_ptr() + ((-buf.data_ptr()) % 256)


RANKS = (32, _b.WS_RMAX)  # sketch widths


def sketch(X, Omega, stream=None):
    """Y = X Omega (M x r, row-major float32).  X column-major float32 on the
    device, Omega (N x r) float32 on the device (row-major), r = 32 or 64."""
    import torch
    M, N = X.shape
    if X.dtype != torch.float32 or X.stride(0) != 1:
        raise ValueError("X must be column-major float32")
    Om = Omega.contiguous()
    r = Om.shape[1] if Om.dim() == 2 else -1
    if Om.dim() != 2 or Om.shape[0] != N or r not in RANKS or Om.dtype != torch.float32:
        raise ValueError("Omega must be (N, r) float32 with r in %s" % (RANKS,))
    Y = torch.empty((M, r), dtype=torch.float32, device=X.device)
    _check(_b.load().gspca_sketch(X.data_ptr(), X.stride(1), M, N, Om.data_ptr(), r,
                                  Y.data_ptr(), _stream(stream, X.device)))
    return Y


def sketch_refine(X, Z, stream=None):
    """One refinement step: (W, Y) with W = X^T Z / sqrt(M) (N x 32) and
    Y = X W (M x 32); whiten Y to finish it."""
    import torch
    M, N = X.shape
    if X.dtype != torch.float32 or X.stride(0) != 1:
        raise ValueError("X must be column-major float32")
    Z = Z.contiguous()
    r = Z.shape[1] if Z.dim() == 2 else -1
    if Z.dim() != 2 or Z.shape[0] != M or r not in RANKS or Z.dtype != torch.float32:
        raise ValueError("Z must be (M, r) float32 with r in %s" % (RANKS,))
    W = torch.empty((N, r), dtype=torch.float32, device=X.device)
    Y = torch.empty((M, r), dtype=torch.float32, device=X.device)
    nb = int(_b.load().gspca_sketch_workspace_bytes(M, N, r))
    buf, wp = _aligned(nb, X.device)
    _check(_b.load().gspca_sketch_refine(X.data_ptr(), X.stride(1), M, N, Z.data_ptr(), r,
                                         W.data_ptr(), Y.data_ptr(), wp, nb,
                                         _stream(stream, X.device)))
    return W, Y


def features(X, Omega, power=1, stream=None):
    """Whitened sketch after `power` refinement steps (the network's input)."""
    Z = whiten(sketch(X, Omega, stream), stream)[0]
    for _ in range(int(power)):
        Z = whiten(sketch_refine(X, Z, stream)[1], stream)[0]
    return Z


def whiten(Y, stream=None):
    """(Z, gamma, flag): Z = sqrt(M) Y Q diag(g)^(-1/2) (row-major M x r)."""
    import torch
    M, r = Y.shape
    Y = Y.contiguous()
    Z = torch.empty_like(Y)
    g = torch.empty(r, dtype=torch.float64, device=Y.device)
    flag = torch.zeros(1, dtype=torch.int32, device=Y.device)
    nb = int(_b.load().gspca_sketch_workspace_bytes(M, 1, r)) if M >= 1 and r in RANKS else 0
    buf, wp = _aligned(max(nb, 1), Y.device)
    _check(_b.load().gspca_whiten_sketch(Y.data_ptr(), M, r, Z.data_ptr(), g.data_ptr(),
                                         flag.data_ptr(), wp, nb, _stream(stream, Y.device)))
    return Z, g, flag


class WarmStartNet:
    """Row-wise network 32 -> d1 -> d2 -> K (K <= 32) with the skip term
    o = z[:K] + W3^T h2 + b3, FP32 master weights, bf16 copies and Adam state,
    all device tensors; parameters packed as W1 b1 W2 b2 W3 b3 with W_l
    row-major (d_in x d_out)."""

    def __init__(self, K, hidden=(256, 256), seed=0, device="cuda", last_zero=True):
        import torch
        self.dims = (RANK, int(hidden[0]), int(hidden[1]), int(K))
        L = _b.load()
        n = int(L.gspca_mlp_param_count(*self.dims))
        self.n = n
        self.device = torch.device(device)
        f32 = dict(dtype=torch.float32, device=self.device)
        self.theta = torch.from_numpy(self.init_params(self.dims, seed, last_zero)).to(self.device)
        self.theta_bf16 = torch.empty(n, dtype=torch.int16, device=self.device)
        self.grad = torch.zeros(n, **f32)
        self.adam_m = torch.zeros(n, **f32)
        self.adam_v = torch.zeros(n, **f32)
        self.net = _b.Mlp(*self.dims, self.theta.data_ptr(), self.theta_bf16.data_ptr(),
                          self.grad.data_ptr(), self.adam_m.data_ptr(), self.adam_v.data_ptr(), 0, 0)
        self._ws = None
        self._ws_ptr = 0
        self._ws_bytes = 0
        self.sync()

    @staticmethod
    def init_params(dims, seed, last_zero=True):
        """He-normal weights (std sqrt(2 / d_in)), zero biases, float32; the
        last layer zero (last_zero) so that the untrained network returns the
        sketch directions through its skip term."""
        rng = np.random.default_rng([811, 13, int(seed)])
        parts = []
        nl = len(dims) - 1
        for l, (a, b) in enumerate(zip(dims[:-1], dims[1:])):
            w = rng.standard_normal((a, b)) * np.sqrt(2.0 / a)
            if last_zero and l == nl - 1:
                w = np.zeros((a, b))
            parts.append(w.ravel())
            parts.append(np.zeros(b))
        return np.concatenate(parts).astype(np.float32)

    def unpack(self, flat):
        """Split a packed host vector into (W1, b1, W2, b2, W3, b3)."""
        out, o = [], 0
        for a, b in zip(self.dims[:-1], self.dims[1:]):
            out.append(flat[o:o + a * b].reshape(a, b)); o += a * b
            out.append(flat[o:o + b]); o += b
        return out

    @property
    def step(self):
        return int(self.net.step)

    def _workspace(self, rows, ninst, cols=0):
        need = int(_b.load().gspca_mlp_workspace_bytes(ctypes.byref(self.net), int(rows),
                                                        int(ninst), int(cols)))
        if need > self._ws_bytes:
            self._ws, self._ws_ptr = _aligned(need, self.device)
            self._ws_bytes = need
        return self._ws_ptr, self._ws_bytes

    def sync(self, stream=None):
        _check(_b.load().gspca_mlp_sync(ctypes.byref(self.net), _stream(stream, self.device)))

    def forward(self, Z, stream=None):
        """O (rows x K, column-major float32) for row-major float32 Z (rows x 32)."""
        import torch
        Z = Z.contiguous()
        rows = Z.shape[0]
        O = torch.empty_strided((rows, self.dims[3]), (1, rows), dtype=torch.float32,
                                device=self.device)
        p, nb = self._workspace(rows, 1)
        _check(_b.load().gspca_mlp_forward(ctypes.byref(self.net), Z.data_ptr(), rows,
                                           O.data_ptr(), p, nb, _stream(stream, self.device)))
        return O

    def loss_grad(self, Z, V, ninst, rows_per_inst, loss=None, stream=None):
        """Gradient of the mean loss over ninst matrices into self.grad; returns
        the loss as a device double tensor.  V: per matrix column-major
        (rows_per_inst x K) unit scores, stacked."""
        import torch
        if loss is None:
            loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        p, nb = self._workspace(int(ninst) * int(rows_per_inst), ninst)
        _check(_b.load().gspca_mlp_loss_grad(ctypes.byref(self.net), Z.data_ptr(), V.data_ptr(),
                                             int(ninst), int(rows_per_inst), loss.data_ptr(), p,
                                             nb, _stream(stream, self.device)))
        return loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(_b.load().gspca_mlp_adam(ctypes.byref(self.net), float(lr), float(beta1),
                                        float(beta2), float(eps), _stream(stream, self.device)))

    def train_step(self, Z, V, ninst, rows_per_inst, lr=1e-3, stream=None):
        loss = self.loss_grad(Z, V, ninst, rows_per_inst, stream=stream)
        self.adam(lr, stream=stream)
        return loss

    def predict(self, X, Omega, power=1, stream=None):
        """Start vectors T0 (M x K, column-major float32) for column-major float32 X
        (sketch of width Omega.shape[1], `power` refinement steps, network)."""
        import torch
        M, N = X.shape
        if X.dtype != torch.float32 or X.stride(0) != 1:
            raise ValueError("X must be column-major float32")
        Om = Omega.contiguous()
        r = Om.shape[1]
        if Om.dim() != 2 or Om.shape[0] != N or r not in RANKS:
            raise ValueError("Omega must be (N, r) float32 with r in %s" % (RANKS,))
        T0 = torch.empty_strided((M, self.dims[3]), (1, M), dtype=torch.float32,
                                 device=self.device)
        p, nb = self._workspace(M, 1, N)
        _check(_b.load().gspca_ws_predict(ctypes.byref(self.net), X.data_ptr(), X.stride(1), M, N,
                                          Om.data_ptr(), int(r), int(power), T0.data_ptr(), p, nb,
                                          _stream(stream, self.device)))
        return T0

    def state(self):
        """Host copy of the weights and Adam state (for np.savez)."""
        return {"dims": np.array(self.dims), "theta": self.theta.cpu().numpy(),
                "adam_m": self.adam_m.cpu().numpy(), "adam_v": self.adam_v.cpu().numpy(),
                "step": np.array(self.step)}

    def load_state(self, st):
        import torch
        if tuple(int(x) for x in st["dims"]) != self.dims:
            raise ValueError("dimension mismatch")
        for name in ("theta", "adam_m", "adam_v"):
            getattr(self, name).copy_(torch.from_numpy(np.asarray(st[name], dtype=np.float32)))
        self.net.step = int(st["step"])
        self.sync()


# ---------------------------------------------------------------------------
# Training and evaluation on synthetic matrices: s_j = r^j, r ~ U[0.7, 0.95],
# Haar factors, no noise (synth.warmstart_instance).  Targets are the unit
# scores of batched GS-PCA fits at a tight tolerance.

def _instance(args):
    from . import synth
    i, M, N = args
    X, U, V, ratio = synth.warmstart_instance(i, M=M, N=N, return_factors=True)
    return X, V[:, :64].astype(np.float32), ratio


def generate(indices, M, N, workers=8, log=None):
    """Host matrices for the given instance numbers, generated on threads of
    this process (no child processes, so it may run beside GPU work and under
    a profiler)."""
    from . import synth
    return synth.map_threads(_instance, [(int(i), M, N) for i in indices], workers, log=log)


def prepare(indices, M, N, K, Omega, tol=1e-7, max_iter=3000, chunk=512, power=1,
            keep_x=False, workers=8, log=None):
    """Device data for the instance numbers `indices`, made chunk by chunk
    (host matrices are generated, uploaded and dropped per chunk): the
    whitened sketch Z of each matrix, the unit scores V of its GS-PCA fit at
    a tight tolerance (column-major per matrix, K columns, the training
    targets), the generator's right factors (host, 64 columns) and, with
    keep_x, the matrices themselves on the device."""
    import torch
    from . import Batch, column_major
    indices = list(indices)
    Xs, Zs, Vs, Vtrue = [], [], [], []
    for lo in range(0, len(indices), chunk):
        host = generate(indices[lo:lo + chunk], M, N, workers)
        part = [column_major(torch.from_numpy(np.ascontiguousarray(x)).cuda())
                for x, _, _ in host]
        b = Batch(part, K, tol=tol, max_iter=max_iter)
        b.launch()
        for i, X in enumerate(part):
            Zs.append(features(X, Omega, power))
            Vs.append((b.T[i] / b.sigma[i].clamp_min(1e-30).float()).t().contiguous())
        Vtrue += [v for _, v, _ in host]
        if keep_x:
            Xs += part
        torch.cuda.synchronize()
        del b, part, host
        if log:
            log("prepared %d / %d" % (min(lo + chunk, len(indices)), len(indices)))
    return Xs, Zs, Vs, Vtrue


def evaluate(net, Xs, Zs, Vtrue, K, Omega, tol=1e-6, max_iter=3000, stop="sigma"):
    """Iterations of batched fits from three starts -- the max-norm column,
    the network's skip path alone (the first K whitened sketch directions,
    i.e. the untrained network) and the network -- and the final loading
    error (radians, sign-aligned) against the generator's factors."""
    import torch
    from . import Batch
    M = Xs[0].shape[0]
    starts = {"maxnorm": None,
              "skip_only": [(z[:, :K] / np.sqrt(M)).t().contiguous().t() for z in Zs],
              "trained": [net.forward(z)[:, :K] for z in Zs]}
    out = {}
    for name, T0 in starts.items():
        if T0 is not None:
            T0 = [t.contiguous().t().contiguous().t() if t.stride() != (1, M) else t for t in T0]
        b = Batch(Xs, K, tol=tol, max_iter=max_iter, stop=stop,
                  init="given" if T0 is not None else "maxnorm", T0=T0)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        b.launch()
        ev1.record()
        torch.cuda.synchronize()
        its = np.stack([x.cpu().numpy() for x in b.iters]).astype(np.float64)
        sc = np.stack([x.cpu().numpy() for x in b.start_col])
        err = []
        for i, P in enumerate(b.P):
            Pp = P.cpu().numpy().astype(np.float64)
            Vt = Vtrue[i][:, :K].astype(np.float64)
            s = np.sign(np.sum(Pp * Vt, axis=0))
            s[s == 0] = 1
            d = np.linalg.norm(Pp - Vt * s, axis=0)
            err.append(2 * np.arcsin(np.minimum(d / 2, 1.0)))
        err = np.array(err)
        out[name] = {
            "iters_per_matrix_mean": float(its.sum(1).mean()),
            "iters_per_matrix_median": float(np.median(its.sum(1))),
            "iters_per_component_mean": float(its.mean()),
            "loading_error_median": float(np.median(err)),
            "loading_error_max": float(err.max()),
            "fallback_rate": float(np.mean(sc >= 0)) if T0 is not None else None,
            "batch_ms": float(ev0.elapsed_time(ev1)),
            "status_ok": bool(np.all(b.status.cpu().numpy() == 0)),
        }
    return out


def main(argv=None):
    """Train on instances 0 .. train-1 (the last `val` of them held out for
    choosing the epoch), evaluate on instances 16000 .. 16000+eval-1."""
    import argparse
    import json
    import time

    import torch
    from . import synth
    ap = argparse.ArgumentParser(description="train and evaluate the learned warm start")
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--val", type=int, default=256,
                    help="training instances held out to choose the epoch (epoch 0 = the "
                         "untrained network, whose output is its skip path)")
    ap.add_argument("--eval", type=int, default=500)
    ap.add_argument("--M", type=int, default=2048)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--K", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=64, help="matrices per step")
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--power", type=int, default=1, help="sketch refinement steps")
    ap.add_argument("--save", default=None, help="write the chosen weights (.npz)")
    ap.add_argument("--out", default=None, help="write the summary JSON here too")
    a = ap.parse_args(argv)
    t0 = time.time()
    M, N, K = a.M, a.N, a.K
    ntr, nval, nev = a.train - a.val, a.val, a.eval

    def log(msg):
        print("%s (%.1fs)" % (msg, time.time() - t0), flush=True)

    Om = torch.from_numpy(synth.sketch_matrix(N, RANK)).cuda()
    _, Ztr, Vtr, _ = prepare(range(ntr), M, N, K, Om, power=a.power, workers=a.workers, log=log)
    _, Zva, Vva, _ = prepare(range(ntr, ntr + nval), M, N, K, Om, power=a.power,
                             workers=a.workers)
    Xev, Zev, _, Vtrue_ev = prepare(range(16000, 16000 + nev), M, N, K, Om, power=a.power,
                                    keep_x=True, workers=a.workers, log=log)
    log("targets and sketches ready")
    net = WarmStartNet(K=K, seed=0)
    Zall = torch.cat(Ztr)
    Vall = torch.stack(Vtr)
    del Ztr, Vtr
    Zva_all, Vva_all = torch.cat(Zva), torch.stack(Vva).reshape(-1)
    rng = np.random.default_rng([811, 14])

    def val_loss():
        return float(net.loss_grad(Zva_all, Vva_all, nval, M).item())

    losses, val = [], [val_loss()]
    best, best_ep, best_theta = val[0], 0, net.theta.clone()
    log("epoch 0 (untrained: skip path) validation loss %.5f" % val[0])
    for ep in range(1, a.epochs + 1):
        perm = rng.permutation(ntr)
        el = []
        for lo in range(0, ntr - a.batch + 1, a.batch):
            idx = torch.from_numpy(perm[lo:lo + a.batch]).cuda()
            zz = Zall.view(ntr, M, RANK)[idx].reshape(-1, RANK)
            vv = Vall[idx].reshape(-1)
            el.append(net.train_step(zz, vv, a.batch, M, lr=a.lr))
        losses.append(float(torch.stack(el).mean().item()))
        val.append(val_loss())
        if val[-1] < best:
            best, best_ep, best_theta = val[-1], ep, net.theta.clone()
        log("epoch %d train loss %.5f validation loss %.5f" % (ep, losses[-1], val[-1]))
    net.theta.copy_(best_theta)
    net.sync()
    res = {"M": M, "N": N, "K": K, "train": ntr, "val": nval, "eval": nev, "epochs": a.epochs,
           "lr": a.lr, "power": a.power, "train_loss": losses, "val_loss": val,
           "chosen_epoch": best_ep, "tol": a.tol}
    res["sigma_stop"] = evaluate(net, Xev, Zev, Vtrue_ev, K, Om, tol=a.tol)
    res["loading_stop"] = evaluate(net, Xev, Zev, Vtrue_ev, K, Om, tol=1e-4, stop="loading")
    res["seconds"] = time.time() - t0
    line = json.dumps(res)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    if a.save:
        np.savez(a.save, dims=np.array(net.dims), theta=net.theta.cpu().numpy(),
                 chosen_epoch=np.array(best_ep), power=np.array(a.power))


def load_trained(path, device="cuda"):
    """A WarmStartNet with the weights written by ``main(--save)``."""
    st = np.load(path, allow_pickle=False)
    dims = tuple(int(x) for x in st["dims"])
    net = WarmStartNet(K=dims[3], hidden=(dims[1], dims[2]), seed=0, device=device)
    import torch
    net.theta.copy_(torch.from_numpy(np.asarray(st["theta"], dtype=np.float32)))
    net.sync()
    return net


if __name__ == "__main__":
    main()
