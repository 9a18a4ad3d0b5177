#!/usr/bin/env python3
"""Benchmark: GS-PCA fits of the large FP32 workload on one MI355X.

One step = one complete fit (R <- X copy, K = 32 components, every iteration
of Sec. 2.3 of Andrecut, arXiv:0811.1081, deflations, finishing) of a
65536 x 8192 FP32 matrix with a rank-64 spectrum 100 * 0.95^i plus N(0, 1e-2)
noise, tol 1e-6, max_iter 1000, through the C ABI, inputs resident in HBM.

Prints one JSON line with whole-job throughput (components/s), the roofline
of the dominant streaming kernel (HIP-event timed inside the timed region),
the FP64 CPU oracle timed on a bounded sample of the same workload, and (FP32
runs) the BF16 + warm-start form against plain FP32 at the same loading
accuracy ("precision_form").
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GS-PCA components/s + HBM GB/s vs peak; BF16+warm-start vs FP32 at 1e-5 err"
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD published peak


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def host_info():
    """Host CPU of this run: logical CPUs, the ones this process may use, model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable": usable, "model": model}


def cpu_baseline(X, mean_iters, n_short=1, n_long=6, max_threads=16):
    """FP64 oracle on the full input, timed two ways (a baseline, not the
    target).  One core (after one untimed call): one component with n_short
    and n_long replayed iterations (explicit deflation, as the GPU fit); the
    per-iteration and fixed costs are extrapolated to the GPU's mean
    iterations per component.
    All cores: the same oracle, unmodified, on T threads at once (the C
    library releases the interpreter lock), each thread fitting one component
    of the shared FP64 matrix with 1 and 3 replayed iterations (implicit form,
    which reads X in place -- identical arithmetic for a first component); the
    aggregate rate is T components per extrapolated per-component time."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    X64 = np.asfortranarray(X, dtype=np.float64)
    oracle.fit(X64, 1, tol=0.0, max_iter=1, replay_iters=np.array([1], dtype=np.int32),
               tiny=oracle.FLT_MIN)  # first call: library load and first-touch costs
    times = []
    for n in (n_short, n_long):
        t0 = time.perf_counter()
        oracle.fit(X64, 1, tol=0.0, max_iter=n, replay_iters=np.array([n], dtype=np.int32),
                   tiny=oracle.FLT_MIN)
        times.append(time.perf_counter() - t0)
    per_iter = max((times[1] - times[0]) / (n_long - n_short), 1e-9)
    fixed = max(times[0] - per_iter * n_short, 0.0)
    per_comp = fixed + per_iter * mean_iters
    one = {
        "value": 1.0 / per_comp, "unit": "components/s", "cores": 1, "kind": "oracle",
        "sample": ("FP64 oracle GS-PCA on the full %dx%d input, 1 component with %d and %d "
                   "replayed iterations (%.1f s and %.1f s); per-component cost = fixed %.2f s "
                   "+ %.2f s/iteration x %.1f mean GPU iterations"
                   % (X.shape[0], X.shape[1], n_short, n_long, times[0], times[1], fixed,
                      per_iter, mean_iters)),
    }
    host = host_info()
    nt = max(1, min(max_threads, host["usable"]))

    def one_fit(n):
        oracle.fit(X64, 1, tol=0.0, max_iter=n, replay_iters=np.array([n], dtype=np.int32),
                   implicit=True, tiny=oracle.FLT_MIN)

    walls = []
    with ThreadPoolExecutor(max_workers=nt) as ex:
        for n in (1, 3):
            t0 = time.perf_counter()
            list(ex.map(one_fit, [n] * nt))
            walls.append(time.perf_counter() - t0)
    pi_all = max((walls[1] - walls[0]) / 2.0, 1e-9)
    fx_all = max(walls[0] - pi_all, 0.0)
    agg = nt / (fx_all + pi_all * mean_iters)
    log("oracle baseline: one core %.4f, %d threads %.4f components/s"
        % (one["value"], nt, agg))
    return {
        "value": agg, "unit": "components/s", "cores": nt, "kind": "oracle",
        "sample": ("FP64 oracle, %d threads at once on the full %dx%d input, each one "
                   "component with 1 and 3 replayed iterations (%.1f s and %.1f s wall); "
                   "aggregate = %d / (fixed %.2f s + %.2f s/iteration x %.1f mean GPU "
                   "iterations); a baseline, not the target"
                   % (nt, X.shape[0], X.shape[1], walls[0], walls[1], nt, fx_all, pi_all,
                      mean_iters)),
        "host": host,
        "one_core": one,
    }


def loading_angles(P, R):
    """Sign-aligned chordal angles between the columns of P and R (radians)."""
    import torch
    P = P.double()
    R = R.double()
    s = torch.sign((P * R).sum(0))
    s[s == 0] = 1
    d = (P - R * s).norm(dim=0)
    return 2 * torch.asin(torch.clamp(d / 2, max=1.0))


def reference_loadings(Xd, P0, K, steps=12, extra=32):
    """Loadings of X to FP64 accuracy, independent of the library: subspace
    iteration on the Gram matrix X^T X (FP64, torch/rocBLAS) from P0 plus
    `extra` random columns, then a Rayleigh-Ritz step.  With the large
    workload's spectrum the error falls by (sigma_65 / sigma_32)^2 ~ 0.03 per
    step."""
    import torch
    X64 = Xd.double()
    G = X64.T @ X64
    del X64
    gen = torch.Generator(device=Xd.device).manual_seed(811)
    Q = torch.cat([P0.double(), torch.randn(G.shape[0], extra, dtype=torch.float64,
                                            device=Xd.device, generator=gen)], 1)
    for _ in range(steps):
        Q, _ = torch.linalg.qr(G @ Q)
    w, U = torch.linalg.eigh(Q.T @ G @ Q)
    idx = torch.argsort(w, descending=True)[:K]
    return Q @ U[:, idx]


def precision_form(gp, Xd, K, tol_loading, max_iter, log, low_tol=1e-5, refine_implicit=True):
    """Reduced-precision forms against plain FP32 at the same loading
    accuracy.  Every form ends with the same loading stop (|p_j - s p_(j-1)|
    < tol_loading) on the FP32 matrix, and every result is compared with the
    FP64 reference loadings.
      plain:      FP32 fit, max-norm starts.
      bf16:       BF16 codes (one quantisation pass), BF16 fit (implicit
                  deflation) with the loading stop at low_tol -- about where
                  the BF16 representation error stops further progress --
                  then FP32 refinement from the BF16 scores (implicit
                  deflation: X is read-only, no per-component rewrite).
      bf16_warm:  the same with warm starts for the BF16 fit: a sketch of
                  width 64 (oversampled for K = 32), two refinement steps,
                  whitened, through the untrained network -- i.e. its skip
                  path alone, the Ritz directions of the sketch (the trained
                  network of the 2048 x 256, K = 16 workload does not apply
                  to K = 32 and does not improve on its skip path there).
      warm_fp32:  the warm start followed directly by the FP32 fit.
      e4m3:       as bf16 with FP8 E4M3 codes (loading stop 3 x low_tol: the
                  FP8 representation error is larger).
      block_fp32: not GS-PCA: the block iteration with Rayleigh-Ritz
                  (gspca_fit_block) from the same sketch, all K at once.
      block_warm_fp32: the block iteration's scores as the given starts of
                  the FP32 GS-PCA fit (which then ends at its own loading
                  stop, usually after two iterations per component).
    Times are HIP-event totals with the input resident in HBM."""
    import torch
    from paper_0811_1081_amd import synth, warmstart as ws
    M, N = Xd.shape

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        out = fn()
        b.record()
        torch.cuda.synchronize()
        return out, a.elapsed_time(b)

    plain, ms_plain = timed(lambda: gp.fit(Xd, K, tol=tol_loading, max_iter=max_iter,
                                           stop="loading", check=False))
    Pref = reference_loadings(Xd, plain["P"], K)
    log("precision form: plain FP32 %.1f ms" % ms_plain)
    Om = torch.from_numpy(synth.sketch_matrix(N, 64)).cuda()
    net = ws.WarmStartNet(K=K, seed=0)  # last layer zero: the skip path (Ritz start)
    net.predict(Xd, Om, power=2)        # workspace allocation outside the timing
    codes = {}
    for fmt in ("bf16", "e4m3"):
        codes[fmt] = timed(lambda: gp.quantize(Xd, fmt))
    out = {"loading_stop_tol": tol_loading, "bf16_loading_tol": low_tol,
           "plain_fp32": {"ms": ms_plain, "iters_mean": float(plain["iters"].double().mean()),
                          "max_loading_err": float(loading_angles(plain["P"], Pref).max()),
                          "status": int(plain["status"])}}
    for name, fmt, warm, ltol in (("bf16", "bf16", False, low_tol),
                                  ("bf16_warm", "bf16", True, low_tol),
                                  ("e4m3", "e4m3", False, 3 * low_tol),
                                  ("warm_fp32", None, True, None)):
        Q, ms_q = codes[fmt] if fmt else (None, 0.0)
        T0, ms_ws = (timed(lambda: net.predict(Xd, Om, power=2)) if warm else (None, 0.0))
        kw = {"init": "given", "T0": T0} if warm else {}
        if Q is not None:
            low, ms_low = timed(lambda: gp.fit(Q, K, tol=ltol, max_iter=max_iter, stop="loading",
                                               check=False, **kw))
            start = low["T"]
        else:
            low, ms_low, start = None, 0.0, T0
        fin, ms_fin = timed(lambda: gp.fit(Xd, K, tol=tol_loading, max_iter=max_iter,
                                           init="given", T0=start, stop="loading",
                                           check=False, implicit=refine_implicit))
        total = ms_q + ms_ws + ms_low + ms_fin
        out[name] = {"ms": total, "speedup_vs_plain": ms_plain / total, "low_loading_tol": ltol,
                     "start": ("sketch Ritz directions (network skip path, untrained)" if warm
                               else "max-norm column"),
                     "quantize_ms": ms_q,
                     "warm_start_ms": ms_ws, "bf16_fit_ms": ms_low, "fp32_refine_ms": ms_fin,
                     "bf16_iters_mean": float(low["iters"].double().mean()) if low else None,
                     "refine_iters_mean": float(fin["iters"].double().mean()),
                     "bf16_max_loading_err": (float(loading_angles(low["P"], Pref).max())
                                              if low else None),
                     "start_max_loading_err": (float(loading_angles(
                         gp.column_major(torch.nn.functional.normalize(
                             Xd.T @ T0, dim=0)), Pref).max()) if warm else None),
                     "max_loading_err": float(loading_angles(fin["P"], Pref).max()),
                     "status": int(fin["status"])}
        log("precision form: %s %.1f ms" % (name, total))
    # beyond the paper: the block iteration with Rayleigh-Ritz on the FP32
    # matrix from the same width-64 sketch, stopped when the unit Ritz vectors
    # move less than 5e-5 (the error left is ~30x smaller at this gap)
    gp.fit_block(Xd, K, r=64, Omega=Om, tol=5e-5, max_iter=100, stop="loading")  # warm-up
    blk, ms_blk = timed(lambda: gp.fit_block(Xd, K, r=64, Omega=Om, tol=5e-5, max_iter=100,
                                             stop="loading", check=False))
    out["block_fp32"] = {"ms": ms_blk, "speedup_vs_plain": ms_plain / ms_blk,
                         "iterations": blk["iters"], "vector_change_tol": 5e-5,
                         "max_loading_err": float(loading_angles(blk["P"], Pref).max()),
                         "status": int(blk["status"])}
    log("precision form: block_fp32 %.1f ms, %d iterations" % (ms_blk, blk["iters"]))
    fin, ms_fin = timed(lambda: gp.fit(Xd, K, tol=tol_loading, max_iter=max_iter, init="given",
                                       T0=blk["T"], stop="loading", check=False,
                                       implicit=refine_implicit))
    total = ms_blk + ms_fin
    out["block_warm_fp32"] = {"ms": total, "speedup_vs_plain": ms_plain / total,
                              "block_ms": ms_blk, "fp32_refine_ms": ms_fin,
                              "refine_iters_mean": float(fin["iters"].double().mean()),
                              "max_loading_err": float(loading_angles(fin["P"], Pref).max()),
                              "status": int(fin["status"])}
    log("precision form: block_warm_fp32 %.1f ms (GS-PCA %.1f ms, %.2f iterations per "
        "component)" % (total, ms_fin, out["block_warm_fp32"]["refine_iters_mean"]))
    return out


def measured_traffic(kernel, form, M, N):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (profiles/traffic.json), or None when that record is for another
    configuration or the kernel's sources (SHA-256 of each file listed under
    "kernel_sources") have changed since it was measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get("%s %s %dx%d" % (kernel, form, M, N))
        if rec is None:
            return None
        for src, digest in rec["kernel_sources"].items():
            with open(os.path.join(ROOT, src), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != digest:
                    return None
        return float(rec["bytes"])
    except (OSError, ValueError, KeyError, AttributeError):
        return None


def _batched_instance(args):
    from paper_0811_1081_amd import synth
    i, M, N = args
    return synth.batched_instance(i, M, N)


def generate_batched(shapes, workers=8):
    """Host matrices of the batched workload, generated on threads of this
    process (no child processes: safe under rocprofv3)."""
    from paper_0811_1081_amd import synth
    return synth.map_threads(_batched_instance,
                             [(i, m, n) for i, (m, n, _) in enumerate(shapes)], workers)


def bench_batched(args):
    """The batched form: 2048 uneven FP32 problems (M ~ U{64..4096},
    N ~ U{16..512}, rank min(16, N), s_i = 0.8^i, 1e-3 noise, K = min(8, N)),
    tol 1e-6, fitted by one persistent launch replayed from a hipGraph, with
    the autotuned launch shape.  One step = one replay (every problem refit)."""
    import numpy as np
    from paper_0811_1081_amd import synth
    shapes = synth.batched_shapes(args.batch_count)
    log("generating %d batched problems" % len(shapes))
    t0 = time.perf_counter()
    host = generate_batched(shapes)
    log("generated in %.1f s" % (time.perf_counter() - t0))
    import torch
    import paper_0811_1081_amd as gp
    gp.load()
    # columns on 128-byte boundaries (leading dimension a multiple of 32)
    Xs = [gp.column_major(torch.from_numpy(x).cuda(), align=32) for x in host]
    del host
    Ks = [k for _, _, k in shapes]
    b = gp.Batch(Xs, Ks, tol=args.tol, max_iter=args.max_iter)
    b.tune()
    threads, occ = b.shape()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.launch(stream=s)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        g.replay()
    ev1.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    st = b.status.cpu().numpy()
    its = [x.cpu().numpy() for x in b.iters]
    comps = sum(Ks)
    mn = np.array([m * n for m, n, _ in shapes], dtype=np.float64)
    it_sum = np.array([int(x.sum()) for x in its], dtype=np.float64)
    compulsory = float(mn.sum() * 4)              # every matrix read from HBM once
    # reads of each matrix: its column norms, per component the first loading
    # (q = X^T t0) and one read per iteration (t and q from one pass; two when
    # a problem has more than 64 columns per wave), and W's column X^T v for
    # every component but the last
    nwaves = threads // 64
    per_iter = np.array([1.0 if n <= 64 * nwaves else 2.0 for _, n, _ in shapes])
    kk = np.array([k for _, _, k in shapes], dtype=np.float64)
    reads = 1.0 + kk + per_iter * it_sum + (kk - 1.0)
    streamed = float((mn * 4 * reads).sum())
    res = {
        "metric": "batched GS-PCA components/s (2048 uneven problems, one persistent launch)",
        "value": comps * args.steps / elapsed, "unit": "components/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched_f32_%d_problems" % len(shapes), "problems": len(shapes),
                   "sum_MN": int(mn.sum()), "K_total": comps, "tol": args.tol,
                   "max_iter": args.max_iter, "threads": threads, "workgroups_per_cu": occ},
        "roofline": {"bound": "hbm", "kernel": "k_batched", "achieved": streamed / ms / 1e6,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": streamed / ms / 1e6 / HBM_PEAK_GBPS, "traffic": None,
                     "bytes_per_launch": streamed, "avg_launch_us": ms * 1e3,
                     "compulsory_bytes": compulsory,
                     "note": "algorithmic bytes: each problem's matrix is read once per "
                             "iteration (t = X p and q = X^T t from one pass), once per "
                             "component for its first loading and for W, and once for the "
                             "column norms; part of the re-reads are served by L2/MALL"},
        "cache_stream_GBps": streamed / ms / 1e6,
        "iters_mean": float(it_sum.sum() / comps),
        "status_ok": int((st == 0).sum()), "status_not_converged": int((st == 1).sum()),
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        import oracle
        log("timing the FP64 oracle on a bounded sample of the batch")
        dt = 0.0
        done = 0
        for i, (m, n, k) in enumerate(shapes):
            X = synth.batched_instance(i, m, n)
            t0 = time.perf_counter()
            oracle.fit(X, k, tol=args.tol, max_iter=args.max_iter, implicit=True,
                       tiny=oracle.FLT_MIN)
            dt += time.perf_counter() - t0
            done += k
            if dt > 15.0:
                break
        res["cpu_baseline"] = {"value": done / dt, "unit": "components/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "FP64 oracle on the first %d problems of the batch "
                                         "(%d components, %.1f s of fitting)" % (i + 1, done, dt)}
    print(json.dumps(res), flush=True)


def _events_ms(fn, reps):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a.record()
        out = fn()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return out, times[len(times) // 2]


def bench_small(args):
    """512 x 128 FP64 (rank-32 signal 2^(-i/4) + 1e-3 noise, centred columns),
    K = 16, tol 1e-10: GS-PCA and NIPALS, median of 5 fits, parity against
    the FP64 oracle on the same trajectory (replayed counts and columns)."""
    import numpy as np
    import torch
    import oracle
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    gp.load()
    X = synth.case_small_f64()
    Xd = gp.column_major(torch.from_numpy(X).cuda())
    K, tol = 16, 1e-10
    res = {"metric": "GS-PCA / NIPALS components/s, FP64 512x128 (cache-resident)",
           "unit": "components/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "small_f64_512x128_K16", "M": 512, "N": 128, "K": K,
                      "tol": tol, "max_iter": 1000}}
    for algo in ("gs", "nipals"):
        out, ms = _events_ms(lambda: gp.fit(Xd, K, tol=tol, max_iter=1000, algo=algo), 5)
        its = out["iters"].cpu().numpy()
        sc = out["start_col"].cpu().numpy()
        o = oracle.fit(X, K, tol=0.0, max_iter=int(its.max()), algo=algo, replay_iters=its,
                       replay_start=sc)
        P = out["P"].cpu().numpy()
        s = np.sign(np.sum(P * o.P, axis=0))
        ang = 2 * np.arcsin(np.minimum(np.linalg.norm(P - o.P * s, axis=0) / 2, 1.0))
        PtP = P.T @ P
        res[algo] = {"ms_per_fit": ms, "components_per_s": K / ms * 1e3,
                     "iters_mean": float(its.mean()), "max_loading_angle_vs_oracle": float(ang.max()),
                     "orth_P": float(np.abs(PtP - np.eye(K)).max())}
    res["value"] = res["gs"]["components_per_s"]
    res["ms_per_step"] = res["gs"]["ms_per_fit"]
    res["steps"], res["warmup"] = 5, 1
    res["roofline"] = None
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        oracle.fit(X, K, tol=tol, max_iter=1000)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": K / dt, "unit": "components/s", "cores": 1,
                               "kind": "oracle", "sample": "one full FP64 oracle fit (%.2f s)" % dt}
    print(json.dumps(res), flush=True)


def bench_paper_sweep(args):
    """The paper's own timing sweep (Sec. 4, Fig. 1): X uniform on [0, 1) with
    rows centred, N = M/2, K = 10, tol 1e-7, max_iter 10000, start column k,
    explicit deflation, FP64, GS-PCA and NIPALS-PCA.  Each size is timed with
    the matrix resident on the device and, as the paper's programs did, with
    the host-to-device copy of X and the copy back of T and P inside the
    timing.  The one-core FP64 oracle is timed on the smaller sizes."""
    import numpy as np
    import torch
    import oracle
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    gp.load()
    K, tol, max_iter = 10, 1e-7, 10000
    sizes = [int(x) for x in args.sweep_sizes.split(",")]
    rows = []
    for M in sizes:
        N = M // 2
        X = synth.uniform_paper(M, N, seed=(6, M))
        Xh = torch.from_numpy(X).pin_memory()  # column-major (Fortran) view
        Xd = torch.empty_strided((M, N), (1, M), dtype=torch.float64, device="cuda")
        Xd.copy_(Xh)
        Th = torch.empty((K, M), dtype=torch.float64).pin_memory()
        Ph = torch.empty((K, N), dtype=torch.float64).pin_memory()
        reps = 3 if M * N <= 32e6 else 2
        row = {"M": M, "N": N}
        for algo in ("gs", "nipals"):
            def run():
                return gp.fit(Xd, K, tol=tol, max_iter=max_iter, algo=algo, init="column_k",
                              check=False)

            def run_h2d():
                Xd.copy_(Xh, non_blocking=True)
                out = run()
                Th.copy_(out["T"].t(), non_blocking=True)
                Ph.copy_(out["P"].t(), non_blocking=True)
                return out
            out, ms = _events_ms(run, reps)
            _, ms_h2d = _events_ms(run_h2d, reps)
            its = out["iters"].cpu().numpy()
            P = out["P"].double()
            sig = out["sigma"].double()
            V = out["T"].double() / torch.where(sig > 0, sig, torch.ones_like(sig))
            eye = torch.eye(K, dtype=torch.float64, device="cuda")
            row[algo] = {"ms": ms, "ms_with_transfer": ms_h2d, "status": int(out["status"]),
                         "iters_total": int(its.sum()), "us_per_iteration": ms * 1e3 / its.sum(),
                         "orth_P": float((P.T @ P - eye).abs().max()),
                         "orth_V": float((V.T @ V - eye).abs().max())}
            if not args.no_cpu_baseline and M <= args.sweep_cpu_max:
                t0 = time.perf_counter()
                o = oracle.fit(X, K, tol=tol, max_iter=max_iter, algo=algo, init="column_k")
                dt = time.perf_counter() - t0
                row[algo]["cpu_oracle_ms"] = dt * 1e3
                row[algo]["cpu_oracle_iters_total"] = int(o.iters.sum())
                row[algo]["cpu_over_gpu_with_transfer"] = dt * 1e3 / ms_h2d
            if M == sizes[0] and M <= args.sweep_cpu_max:
                # parity on the same trajectory (replayed counts and columns);
                # the oracle only runs on the sizes it is timed on
                o = oracle.fit(X, K, tol=0.0, max_iter=int(its.max()), algo=algo,
                               replay_iters=its, replay_start=out["start_col"].cpu().numpy())
                Pg = out["P"].cpu().numpy()
                sgn = np.sign(np.sum(Pg * o.P, axis=0))
                ang = 2 * np.arcsin(np.minimum(np.linalg.norm(Pg - o.P * sgn, axis=0) / 2, 1.0))
                row[algo]["max_loading_angle_vs_oracle"] = float(ang.max())
            log("sweep M=%d %s: %.2f ms (%.2f with transfer), %d iterations" % (
                M, algo, ms, ms_h2d, int(its.sum())))
        row["gs_over_nipals"] = row["gs"]["ms"] / row["nipals"]["ms"] - 1.0
        row["gs_over_nipals_per_iteration"] = (row["gs"]["us_per_iteration"] /
                                               row["nipals"]["us_per_iteration"] - 1.0)
        rows.append(row)
        del Xd, Xh
        torch.cuda.empty_cache()
    big = rows[-1]
    res = {"metric": "GS-PCA ms per fit, the paper's FP64 sweep (uniform, N = M/2, K = 10)",
           "value": big["gs"]["ms"], "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": big["gs"]["ms"], "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "paper_sweep_f64_uniform_rowcentred", "sizes": sizes, "K": K,
                      "tol": tol, "max_iter": max_iter, "init": "column_k"},
           "roofline": None, "cpu_baseline": None, "sweep": rows}
    cpu_rows = [r for r in rows if "cpu_oracle_ms" in r["gs"]]
    if cpu_rows:
        r = cpu_rows[-1]
        res["cpu_baseline"] = {"value": r["gs"]["cpu_oracle_ms"], "unit": "ms", "cores": 1,
                               "kind": "oracle",
                               "sample": "full FP64 oracle GS-PCA fit at M=%d, N=%d" % (r["M"], r["N"])}
    print(json.dumps(res), flush=True)


def bench_orthogonality(args):
    """Loss of orthogonality against the component index (the paper's claim
    about NIPALS, Secs. 2.2-2.3, with the re-orthogonalisation variants as
    the comparison): 4096 x 512 FP32 full-rank collinear data (s_i = 0.9^i,
    1e-4 noise, centred), tol 1e-6, max_iter 1000, NIPALS and GS-PCA with one
    classical pass (the paper's), two passes and modified Gram-Schmidt;
    max |P_k^T P_k - I| and max |V_k^T V_k - I| over the first k components."""
    import numpy as np
    import torch
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    gp.load()
    X = synth.case_collinear_f32()
    Xd = gp.column_major(torch.from_numpy(X).cuda())
    M, N = X.shape
    K = args.ortho_k
    ks = [k for k in (8, 16, 32, 64, 128, 256, 512) if k <= K]
    forms = [("nipals", "cgs"), ("gs", "cgs"), ("gs", "cgs2"), ("gs", "mgs")]
    out = {}
    for algo, reorth in forms:
        name = algo if algo == "nipals" else "gs_" + reorth
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = gp.fit(Xd, K, tol=1e-6, max_iter=1000, algo=algo, reorth=reorth, check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        P = r["P"].double()
        sig = r["sigma"].double()
        V = r["T"].double() / torch.where(sig > 0, sig, torch.ones_like(sig))
        GP, GV = P.T @ P, V.T @ V
        eye = torch.eye(K, dtype=torch.float64, device="cuda")
        its = r["iters"].cpu().numpy()
        out[name] = {"s_per_fit": dt, "status": int(r["status"]), "iters_total": int(its.sum()),
                     "orth_P": {str(k): float((GP[:k, :k] - eye[:k, :k]).abs().max()) for k in ks},
                     "orth_V": {str(k): float((GV[:k, :k] - eye[:k, :k]).abs().max()) for k in ks}}
        log("orthogonality %s: %.2f s, |V^T V - I| at K: %.2e" % (name, dt,
                                                                 out[name]["orth_V"][str(ks[-1])]))
    res = {"metric": "max |V_K^T V_K - I| of GS-PCA (one classical pass), FP32 4096x512 full rank",
           "value": out["gs_cgs"]["orth_V"][str(ks[-1])], "unit": "abs", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": out["gs_cgs"]["s_per_fit"] * 1e3,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "orthogonality_f32_4096x512", "M": M, "N": N, "K": K,
                      "tol": 1e-6, "max_iter": 1000},
           "roofline": None, "cpu_baseline": None, "forms": out}
    print(json.dumps(res), flush=True)


def bench_collinear(args):
    """4096 x 512 FP32 full rank (s_i = 0.9^i + 1e-4 noise, centred), K = N =
    512, tol 1e-6, max_iter 1000: GS-PCA vs NIPALS orthogonality and
    throughput (cache-resident: the matrix is 8 MiB)."""
    import numpy as np
    import torch
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth
    gp.load()
    X = synth.case_collinear_f32()
    Xd = gp.column_major(torch.from_numpy(X).cuda())
    M, N = X.shape
    K = N
    fro2 = float(np.sum(X.astype(np.float64) ** 2))
    res = {"metric": "GS-PCA components/s and orthogonality, FP32 4096x512 full rank",
           "unit": "components/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "collinear_f32_4096x512_K512", "M": M, "N": N, "K": K,
                      "tol": 1e-6, "max_iter": 1000}}
    for algo in ("gs", "nipals"):
        t0 = time.perf_counter()
        out = gp.fit(Xd, K, tol=1e-6, max_iter=1000, algo=algo, check=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        P = out["P"].double()
        sig = out["sigma"].double()
        V = out["T"].double() / torch.where(sig > 0, sig, torch.ones_like(sig))
        eye = torch.eye(K, dtype=torch.float64, device="cuda")
        its = out["iters"].cpu().numpy()
        res[algo] = {"s_per_fit": dt, "components_per_s": K / dt, "status": int(out["status"]),
                     "iters_mean": float(its.mean()), "iters_max": int(its.max()),
                     "orth_P": float((P.T @ P - eye).abs().max()),
                     "orth_V": float((V.T @ V - eye).abs().max()),
                     "sum_lambda_over_fro2": float(out["lambda"].sum()) / fro2}
        log("collinear %s: %.2f s, orth_P %.2e orth_V %.2e" % (algo, dt, res[algo]["orth_P"],
                                                            res[algo]["orth_V"]))
    res["value"] = res["gs"]["components_per_s"]
    res["ms_per_step"] = res["gs"]["s_per_fit"] * 1e3
    res["steps"], res["warmup"] = 1, 0
    res["roofline"] = None
    res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--M", type=int, default=65536)
    ap.add_argument("--N", type=int, default=8192)
    ap.add_argument("--K", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--implicit", action="store_true", help="implicit deflation (X read-only)")
    ap.add_argument("--form", default="f32", choices=["f32", "bf16", "e4m3"],
                    help="storage of X streamed by the iteration (bf16/e4m3: quantised codes, "
                         "implicit deflation)")
    ap.add_argument("--no-precision-form", action="store_true",
                    help="skip the BF16 + warm-start vs FP32 comparison at equal loading error")
    ap.add_argument("--loading-tol", type=float, default=5e-7,
                    help="loading stop of that comparison")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one device-to-device copy of 1 GiB first (calibrates HBM byte "
                         "counters of a profiler run against a kernel of known traffic)")
    ap.add_argument("--workload", default="large",
                    choices=["large", "batched", "small", "collinear", "paper_sweep",
                             "orthogonality"],
                    help="large: the 65536 x 8192 fit (default); batched: 2048 uneven "
                         "problems; small: 512 x 128 FP64; collinear: 4096 x 512 FP32, K = N; "
                         "paper_sweep: the paper's FP64 timing sweep (uniform, N = M/2, K = 10); "
                         "orthogonality: NIPALS vs the Gram-Schmidt forms on the collinear case")
    ap.add_argument("--ortho-k", type=int, default=128,
                    help="components of the orthogonality study")
    ap.add_argument("--batch-count", type=int, default=2048)
    ap.add_argument("--sweep-sizes", default="500,1000,2000,4000,8000,15000",
                    help="row counts M of the paper sweep (N = M/2)")
    ap.add_argument("--sweep-cpu-max", type=int, default=2000,
                    help="largest M of the paper sweep at which the oracle is timed")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "small":
        bench_small(args)
        return
    if args.workload == "collinear":
        bench_collinear(args)
        return
    if args.workload == "paper_sweep":
        bench_paper_sweep(args)
        return
    if args.workload == "orthogonality":
        bench_orthogonality(args)
        return

    import numpy as np
    import torch
    import paper_0811_1081_amd as gp
    from paper_0811_1081_amd import synth

    gp.load()
    M, N, K = args.M, args.N, args.K
    log("generating %dx%d FP32 input" % (M, N))
    t0 = time.perf_counter()
    X = synth.case_large_f32(M, N)
    log("generated in %.1f s" % (time.perf_counter() - t0))
    Xd = gp.column_major(torch.from_numpy(X).to("cuda"))
    Xfit = Xd
    if args.form != "f32":
        Xfit = gp.quantize(Xd, args.form)
        args.implicit = True
    ws_bytes = gp.workspace_bytes(Xfit, K, implicit=args.implicit)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
    ws_view = ws[(-ws.data_ptr()) % 256:]
    torch.cuda.synchronize()
    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b

    def step(profile=None):
        return gp.fit(Xfit, K, tol=args.tol, max_iter=args.max_iter, workspace=ws_view,
                      profile=profile, implicit=args.implicit)

    for i in range(args.warmup):
        out = step()
        torch.cuda.synchronize()
        log("warmup %d: status %d, iters %s" % (i, out["status"], out["iters"].cpu().tolist()))

    prof = gp.Profile()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for i in range(args.steps):
        outs.append(step(prof))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = outs[-1]
    iters = out["iters"].cpu().numpy()
    log("timed %d steps in %.3f s; status %d; iters %s" % (args.steps, elapsed, out["status"],
                                                            iters.tolist()))

    comps = K * args.steps
    value = comps / elapsed
    # roofline of the dominant streaming kernel: algorithmic bytes = one read of the data
    if prof.single_pass:
        dom, ms, n_l = "k_pass", prof.pass_ms, prof.pass_launches
        passes_per_iter = 1.0
    else:
        dom = "gemv_t" if prof.gemv_t_ms >= prof.gemv_n_ms else "gemv_n"
        ms = prof.gemv_t_ms if dom == "gemv_t" else prof.gemv_n_ms
        n_l = prof.gemv_t_launches if dom == "gemv_t" else prof.gemv_n_launches
        passes_per_iter = 2.0
    avg_s = ms / max(n_l, 1) / 1e3
    bytes_per_launch = float(prof.bytes_per_pass)
    achieved = bytes_per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    total_iters = int(prof.iterations)
    fit_gbps = passes_per_iter * total_iters * bytes_per_launch / elapsed / 1e9
    fit_alg_gbps = total_iters * bytes_per_launch / elapsed / 1e9

    P = out["P"].double()
    V = (out["T"].double() / out["sigma"]).double()
    eye = torch.eye(K, dtype=torch.float64, device="cuda")
    orth_p = float((P.T @ P - eye).abs().max())
    orth_v = float((V.T @ V - eye).abs().max())

    form = "%s_%s_%s" % ({"f32": "plain_fp32", "bf16": "bf16_codes",
                          "e4m3": "fp8_e4m3_codes"}[args.form],
                         "implicit" if args.implicit else "explicit",
                         "single_pass" if prof.single_pass else "two_pass")
    res = {
        "metric": METRIC, "value": value, "unit": "components/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16", "e4m3": "fp8_e4m3"}[args.form],
        "data": "synthetic",
        "config": {"workload": "large_f32_lowrank_%dx%d_K%d" % (M, N, K), "M": M, "N": N,
                   "K": K, "tol": args.tol, "max_iter": args.max_iter, "algo": "gs",
                   "form": form},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(dom, form, M, N),
                     "avg_launch_us": avg_s * 1e6, "bytes_per_launch": bytes_per_launch,
                     "launches_timed": int(n_l)},
        "iters_mean": float(iters.mean()),
        "iterations_timed": total_iters,
        "fit_stream_GBps": fit_gbps,
        "fit_algorithmic_GBps": fit_alg_gbps,
        "orth_P": orth_p, "orth_V": orth_v,
        "cpu_baseline": None,
    }
    if args.form == "f32" and not args.no_precision_form:
        del ws, ws_view, outs, out
        torch.cuda.empty_cache()
        res["precision_form"] = precision_form(gp, Xd, K, args.loading_tol, 3000, log)
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(X, float(iters.mean()))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
