"""Benchmark of the fast Slepian projection on one MI355X.

One step = one slepian_project call over the whole batch: B x by the FFT
product plus the low-rank transition correction, every kernel of the path.
Default workload: N = 65536, W = 1/8, eps = 1e-6, 256 signals of 64 random
tones plus white noise at 20 dB SNR (synthetic stand-in for the paper's random
vectors; Section 4.1 uses W = 1/4, 1/16, 1/64 and N up to 2^20).

Prints one JSON line.  `value` is GSamples/s = N * batch * steps / elapsed
seconds of the timed region (inputs already resident in HBM, HIP events on the
library's stream, torch.cuda.synchronize() on both sides).  The CPU leg times
the FP64 oracle on 32 of the signals; the GPU outputs for those signals must
match the oracle's to 1e-5 relative l2 error (checked before timing; the
script exits non-zero otherwise).  The many-plans workload is timed too.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GSamples/s projected at 1e-5 rel. err, batched mixed vs plain FP32; % HBM/MFMA roof"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (N, W, eps, batch, signal config)
    "paper-scale N=65536 W=1/8 eps=1e-6 b=256": (65536, 1.0 / 8, 1e-6, 256, 2),
    "small N=1024 W=1/16 eps=1e-6 b=8": (1024, 1.0 / 16, 1e-6, 8, 1),
    "precision N=262144 W=0.05 eps=1e-4 b=1024": (262144, 0.05, 1e-4, 1024, 3),
}
DEFAULT = "paper-scale N=65536 W=1/8 eps=1e-6 b=256"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _finite(v):
    """The JSON line with NaN and infinities replaced by null (strict JSON)."""
    import math
    if isinstance(v, float):
        return v if math.isfinite(v) else None
    if isinstance(v, dict):
        return {k: _finite(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_finite(x) for x in v]
    return v


def kernel_bytes(name: str, N: int, b: int, L: int, r: int, pairs_per_launch: int, col_log2: int = 0,
                 fwd_chunks: bool = False):
    """Algorithmic HBM bytes of one launch of each kernel of the path: what the
    method must move (FP32 signal in/out 4 B/sample, complex64 intermediates
    8 B/point, spectrum 4 B/point once, U 4 B/entry once)."""
    P = pairs_per_launch
    if name == "row_conv":
        return P * 16.0 * L + 4.0 * L
    if name == "col_fwd":
        return P * (8.0 * N + 8.0 * L)
    if name.startswith("col_fwd_corr"):
        # x in, Z out, U read once, one partial of C per 16 columns written
        chunks = L // (2 ** col_log2) // 16 if col_log2 else 0
        return P * (8.0 * N + 8.0 * L) + 4.0 * N * r + 4.0 * r * b * chunks
    if name == "col_inv":
        return P * (8.0 * L + 8.0 * N)
    if name.startswith("col_inv_corr"):
        # Z in, y out, U and d (.) C read once
        return P * (8.0 * L + 8.0 * N) + 4.0 * N * r + 4.0 * r * b
    if name.startswith("corr_partial"):
        return 4.0 * N * b + 4.0 * N * r
    if name == "corr_apply":
        return 8.0 * N * b + 4.0 * N * r
    if name in ("conv_single", "conv_single_corr"):
        return P * 8.0 * N + 4.0 * L + 4.0 * N * r
    if name == "corr_reduce":
        # chunk partials read once (one per 256 samples, or one per 16
        # columns when pass A forms them), d (.) C written once
        chunks = L // (2 ** col_log2) // 16 if fwd_chunks else (N + 255) // 256
        return 4.0 * b * r * (chunks + 1)
    return None


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary
    (profiles/traffic_<kernel>.md or traffic_<kernel>_<tag>.md) taken on this
    workload with the current kernel sources; else None."""
    import glob
    try:
        from paper_1611_04950_amd.build import source_digest
        digest = source_digest()
    except Exception:
        return None
    paths = [os.path.join(ROOT, "profiles", f"traffic_{kernel}.md")] + \
        sorted(glob.glob(os.path.join(ROOT, "profiles", f"traffic_{kernel}_*.md")))
    for path in paths:
        if not os.path.exists(path):
            continue
        vals = {}
        for line in open(path):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip()
        if vals.get("source_digest") == digest and vals.get("workload") == workload:
            try:
                return float(vals["hbm_bytes_per_launch"])
            except (KeyError, ValueError):
                return None
    return None


def copy_bandwidth(dev, mib=256, reps=10):
    """Achieved bandwidth of a plain device copy (read + write bytes / time);
    also the reference kernel for scaling FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.randn(n, device=dev)
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"copy_MiB": mib, "copy_ms": round(ms, 4), "copy_GBs": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)}


def cpu_baseline(N, W, eps, x_sample, min_seconds):
    """The oracle's FP64 fast projection timed on this host (1 thread), on a
    sample of the workload's signals.  Returns the timing record, the
    oracle's outputs for the sample, against which the GPU's outputs for the
    same signals are checked, the sample's exact projection, and the same
    timing record and outputs of the oracle's fast factorization (compress,
    then recover) on that sample."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import slepian_oracle as o
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        tp = o.transition_plan(N, W, eps, 1 - eps)
        setup = time.perf_counter() - t0
        xs = x_sample.T.astype(np.float64)
        reps = 0
        t0 = time.perf_counter()
        while True:
            ref = o.project_fast(N, W, eps, xs, tp=tp)
            reps += 1
            el = time.perf_counter() - t0
            if el >= min_seconds:
                break
    samples = reps * xs.shape[0] * xs.shape[1]
    # the exact projection S_K S_K^T x of the sample, for which the oracle's
    # fast projection at eps = 1e-13 stands in (Corollary 2 puts it within
    # 1e-13 ||x||); outside the timed loop
    with threadpool_limits(limits=1):
        exact = o.project_fast(N, W, 1e-13, xs)
    # the oracle's fast factorization (Section 1.3): compression T2^T x and
    # recovery T1 c of the same sample, timed the same way after its setup
    from oracle import factorization as fz
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        fac = fz.fast_factorization(N, W, eps)
        fsetup = time.perf_counter() - t0
        freps = 0
        t0 = time.perf_counter()
        while True:
            fref = fz.recover(fac, fz.compress(fac, xs))
            freps += 1
            fel = time.perf_counter() - t0
            if fel >= min_seconds / 2:
                break
    fcpu = {"value": freps * xs.shape[0] * xs.shape[1] / fel / 1e6, "unit": "MSamples/s (compress + recover)",
            "cores": 1, "kind": "oracle",
            "sample": f"{xs.shape[1]} signals of the workload, compressed and recovered {freps} times ({fel:.1f} s); "
                      f"oracle setup {fsetup:.1f} s not included", "setup_s": fsetup}
    # the same fast projection with every host core (FFT workers and BLAS threads)
    import scipy.fft as sfft
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    with threadpool_limits(limits=ncores), sfft.set_workers(ncores):
        mreps = 0
        t0 = time.perf_counter()
        while True:
            o.project_fast(N, W, eps, xs, tp=tp)
            mreps += 1
            mel = time.perf_counter() - t0
            if mel >= min_seconds / 2:
                break
    multi = {"value": mreps * xs.shape[0] * xs.shape[1] / mel / 1e6, "unit": "MSamples/s", "cores": ncores,
             "kind": "oracle", "sample": f"{xs.shape[1]} signals of the workload, projected {mreps} times ({mel:.1f} s) "
                                         f"with {ncores} FFT workers and BLAS threads"}
    return {"value": samples / el / 1e6, "unit": "MSamples/s", "cores": 1, "kind": "oracle",
            "sample": f"{xs.shape[1]} signals of the workload, projected {reps} times ({el:.1f} s); "
                      f"oracle setup (transition vectors) {setup:.1f} s not included",
            "setup_s": setup, "all_cores": multi, "host": host_info()}, ref.T, exact.T, fcpu, fref.T


def host_info():
    """nproc and the CPU model of the host the oracle ran on."""
    import platform
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count(),
            "cpu_model": model or platform.processor(), "machine": platform.machine()}


def exact_vs_fast(sizes=(1024, 2048, 4096), W=1.0 / 16, eps=1e-6, b=8):
    """Section 4.1's comparison on the CPU oracle (all host cores): the exact
    projection S_K S_K^T x (precompute: dense eigendecomposition of B; apply:
    two products with the N x K basis) against the fast projection B x +
    U diag(d) U^T x (precompute: transition vectors; apply: FFT product plus
    the rank-r correction), per signal, at W = 1/16, eps = 1e-6."""
    import numpy as np
    import scipy.fft as sfft
    from threadpoolctl import threadpool_limits

    from oracle import slepian_oracle as o
    out = []
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    rng = np.random.default_rng(4100)
    with threadpool_limits(limits=ncores), sfft.set_workers(ncores):
        for N in sizes:
            x = rng.standard_normal((N, b))
            K = o.choose_K(N, W)
            t0 = time.perf_counter()
            _, S = o.dense_eig(N, W)
            SK = np.ascontiguousarray(S[:, :K])
            t_pre_exact = time.perf_counter() - t0
            t0 = time.perf_counter()
            reps = 0
            while reps < 3 or time.perf_counter() - t0 < 0.2:
                ye = SK @ (SK.T @ x)
                reps += 1
            t_exact = (time.perf_counter() - t0) / reps / b
            t0 = time.perf_counter()
            tp = o.transition_plan(N, W, eps, 1 - eps)
            t_pre_fast = time.perf_counter() - t0
            t0 = time.perf_counter()
            reps = 0
            while reps < 3 or time.perf_counter() - t0 < 0.2:
                yf = o.project_fast(N, W, eps, x, tp=tp)
                reps += 1
            t_fast = (time.perf_counter() - t0) / reps / b
            dist = float((np.linalg.norm(yf - ye, axis=0) / np.linalg.norm(x, axis=0)).max())
            out.append({"N": N, "K": K, "exact_apply_us_per_signal": round(t_exact * 1e6, 2),
                        "fast_apply_us_per_signal": round(t_fast * 1e6, 2),
                        "exact_precompute_s": round(t_pre_exact, 3), "fast_precompute_s": round(t_pre_fast, 3),
                        "fast_vs_exact_rel_to_x": dist})
    return {"W": W, "eps": eps, "signals": b, "cores": ncores, "sizes": out}


def traced_roofline(call, steps, N, b, info, workload):
    """Per-kernel average launch durations over `steps` traced calls (HIP
    events around each launch, on the launch's stream), each kernel's
    algorithmic and (when the committed counter summary matches the current
    sources) measured HBM GB/s, and the roofline record of the kernel with
    the largest share of the step."""
    from paper_1611_04950_amd import slepian as S
    import torch
    S.slepian_trace_enable(True)
    S.slepian_trace_read(reset=True)
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    stats = S.slepian_trace_read(reset=True)
    S.slepian_trace_enable(False)
    kernels = {}
    total = sum(v["total_ms"] for v in stats.values())
    for name, st in stats.items():
        kernels[name] = {"avg_us": st["total_ms"] / st["launches"] * 1e3, "launches_per_step": st["launches"] / steps,
                         "share": st["total_ms"] / total}
    pairs = (b + 1) // 2
    dom = max(stats, key=lambda k: stats[k]["total_ms"])
    for name in kernels:
        ppl = pairs / kernels[name]["launches_per_step"] if not name.startswith("corr") else pairs
        kb = kernel_bytes(name, N, b, info["L"], info["r"], ppl, info["col_log2"],
                          any(k.startswith("col_fwd_corr") for k in stats))
        kernels[name]["alg_bytes"] = kb
        kernels[name]["alg_GBs"] = None if kb is None else kb / (kernels[name]["avg_us"] * 1e-6) / 1e9
        t = read_traffic(name, workload)
        if t is not None:
            kernels[name]["hbm_bytes"] = t
            kernels[name]["hbm_GBs"] = t / (kernels[name]["avg_us"] * 1e-6) / 1e9
    nbytes = kernels[dom]["alg_bytes"]
    achieved = nbytes / (kernels[dom]["avg_us"] * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": read_traffic(dom, workload), "kernel": dom,
                "alg_bytes_per_launch": nbytes, "avg_launch_us": round(kernels[dom]["avg_us"], 3)}
    return kernels, roofline


def plain_fp32_per_signal(plan, x, N, W, eps, info, dev, ms_batched, work):
    """The plain FP32 per-signal path the batched path is compared with: one
    signal at a time, no pair packing, no fusion, no graph: a complex FP32
    FFT of the zero-padded signal (torch.fft, i.e. the ROCm FFT library), the
    spectrum multiply, the inverse FFT and truncation, then the correction as
    two FP32 matrix-vector products (torch.mv) with the plan's transition
    vectors.  Its output is checked against the library's.  Also the
    library's own path called with one signal per call."""
    import math

    import torch

    from paper_1611_04950_amd import slepian as S
    L, K = info["L"], info["K"]
    # kernel spectrum: DFT of the circulant embedding of B's first column (FP64, kept FP32)
    k = torch.arange(1, N, dtype=torch.float64, device=dev)
    col = torch.zeros(L, dtype=torch.float64, device=dev)
    col[0] = 2 * W
    col[1:N] = torch.sin(2 * math.pi * W * k) / (math.pi * k)
    col[L - N + 1:] = torch.flip(col[1:N], dims=[0])
    chat = torch.fft.fft(col).real.to(torch.float32)
    # transition vectors and projection weights (Lemma 4)
    l0, lam, V = S.slepian_plan_eigenpairs(plan)
    ells = torch.arange(l0, l0 + lam.numel())
    sel = (lam > eps) & (lam < 1 - eps)
    d = torch.where(ells < K, 1 - lam, -lam)[sel]
    U = V[sel.to(V.device)].T.contiguous().to(torch.float32)          # N x r
    d32 = d.to(torch.float32).to(dev)

    def one(xs):
        z = torch.zeros(L, dtype=torch.complex64, device=dev)
        z[:N] = xs
        yv = torch.fft.ifft(torch.fft.fft(z) * chat)[:N].real
        return yv + torch.mv(U, d32 * torch.mv(U.T, xs))

    b = x.shape[0]
    yp = torch.empty_like(x)
    for s in range(min(b, 4)):
        yp[s] = one(x[s])
    torch.cuda.synchronize()
    yl = S.slepian_project(plan, x[:4], precision=S.SLEPIAN_FP32)
    torch.cuda.synchronize()
    agree = float((torch.linalg.vector_norm((yp[:4] - yl).double(), dim=1) /
                   torch.linalg.vector_norm(yl.double(), dim=1)).max())
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for s in range(b):
        yp[s] = one(x[s])
    e1.record(stream)
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1)
    # the library's own batched path, called with one signal per call
    ys = torch.empty_like(x)
    for s in range(min(b, 8)):
        S.slepian_project(plan, x[s:s + 1], ys[s:s + 1], work=work)
    torch.cuda.synchronize()
    e0.record(stream)
    for s in range(b):
        S.slepian_project(plan, x[s:s + 1], ys[s:s + 1], work=work)
    e1.record(stream)
    torch.cuda.synchronize()
    lms = e0.elapsed_time(e1)
    return {"value": round(N * b / (pms * 1e-3) / 1e9, 3), "unit": "GSamples/s", "ms_per_step": round(pms, 4),
            "speedup_batched": round(pms / ms_batched, 2),
            "impl": "per signal: complex FP32 FFT (torch.fft) of the zero-padded signal, spectrum multiply, inverse "
                    "FFT, FP32 U^T x and U (d C) by torch.mv; no pair packing, fusion or graph",
            "max_rel_diff_vs_library": agree,
            "library_one_signal_per_call": {"value": round(N * b / (lms * 1e-3) / 1e9, 3), "ms_per_step": round(lms, 4),
                                            "speedup_batched": round(lms / ms_batched, 2)}}


def bench_batching(args, dev):
    """The many-plans workload: 512 plans (N log-uniform over 2^10..2^17, W
    uniform in [0.01, 0.25], eps in {1e-3, 1e-6}, 4..64 Gaussian signals each)
    projected by one grouped call (one HIP graph), in the correction
    arithmetic of --precision; bitwise equality with the single-plan calls
    (whose parity the test suite checks on the same plans) is checked before
    timing."""
    import torch

    from paper_1611_04950_amd import slepian as S
    from paper_1611_04950_amd import synth

    specs = synth.batching_plans(512)
    log("bench: batching workload, creating 512 plans")
    t0 = time.perf_counter()
    prec = S.SLEPIAN_MIXED if args.precision == "mixed" else S.SLEPIAN_FP32
    # tuned among the variants the grouped launches take, for each plan's batch
    plans = S.slepian_plan_batch([(n, w, e) for n, w, e, _ in specs], precision=prec, tune=2 * args.tune,
                                 tune_batch=[bb for *_, bb in specs])
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    xs = [synth.gaussian(n, bb, 4000 * 1000 + 100 * i, device=dev) for i, (n, _, _, bb) in enumerate(specs)]
    ys = [torch.empty_like(xx) for xx in xs]
    total = sum(n * bb for n, _, _, bb in specs)
    G = S.slepian_group_create(plans, [bb for *_, bb in specs])
    S.slepian_group_project(G, xs, ys)  # first call tunes the launch shapes and captures the graph
    torch.cuda.synchronize()
    # the grouped call must reproduce the single-plan calls bit for bit (whose
    # parity with the oracle the test suite checks on these same plans)
    same = all(torch.equal(yy, S.slepian_project(p, xx)) for p, xx, yy in zip(plans, xs, ys))
    torch.cuda.synchronize()
    log(f"bench: batching, group == single-plan calls: {same}")
    if not same:
        log("bench: batching check failed")
        sys.exit(1)
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    steps = max(3, args.steps // 2)
    for _ in range(2):
        S.slepian_group_project(G, xs, ys)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        S.slepian_group_project(G, xs, ys)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # the same plans one call each, for comparison
    e0.record(stream)
    for p, xx, yy in zip(plans, xs, ys):
        S.slepian_project(p, xx, yy)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_each = e0.elapsed_time(e1)
    S.slepian_trace_enable(True)
    S.slepian_trace_read(reset=True)
    S.slepian_group_project(G, xs, ys)
    torch.cuda.synchronize()
    st = S.slepian_trace_read(reset=True)
    S.slepian_trace_enable(False)
    value = total / (ms * 1e-3) / 1e9
    gi = G.info
    rows = {}
    for p in plans:
        k = f"rows_2^{p.info['row_log2']}"
        rows[k] = rows.get(k, 0) + 1
    log(f"bench: batching {ms:.3f} ms per grouped call, {value:.2f} GSamples/s; plan by plan {ms_each:.3f} ms; "
        f"{gi['grouped']} plans grouped, {gi['other']} one by one; {rows}")
    return {"workload": "512 plans, N log-uniform 2^10..2^17, W U[0.01,0.25], eps {1e-3,1e-6}, 4-64 signals",
            "precision": args.precision,
            "value": round(value, 3), "unit": "GSamples/s", "ms_per_call": round(ms, 4), "steps": steps,
            "samples": total, "plan_by_plan_ms": round(ms_each, 4),
            "speedup_vs_plan_by_plan": round(ms_each / ms, 2), "plans_setup_s": round(setup, 2),
            "matches_single_plan_calls": same, "group_info": gi, "plan_rows": rows,
            "kernels_traced_ms": {k: round(v["total_ms"], 4) for k, v in st.items()}}


def _time_calls(fn, steps, warmup, dev):
    import torch
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_precision(args, dev):
    """N = 262144, W = 0.05, eps = 1e-4, 1024 signals of 64 tones at 20 dB:
    the mixed-precision projection (BF16 hi/lo correction) and the FP32 one.
    Parity of sampled signals with the oracle at this size is a GPU test."""
    import torch

    from paper_1611_04950_amd import slepian as S
    from paper_1611_04950_amd import synth
    N, W, eps, b, cfg = WORKLOADS["precision N=262144 W=0.05 eps=1e-4 b=1024"]
    log("bench: precision workload")
    t0 = time.perf_counter()
    plan = S.slepian_plan(N, W, eps, precision=S.SLEPIAN_MIXED if args.precision == "mixed" else S.SLEPIAN_FP32,
                          tune=args.tune, tune_batch=b)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    x = synth.config_signals(cfg, N, b, W, device=dev)
    y = torch.empty_like(x)
    out = {"workload": "precision N=262144 W=0.05 eps=1e-4 b=1024", "plan_setup_s": round(setup, 3),
           "r": plan.info["r"], "L": plan.info["L"],
           "launch": {k: plan.info[k] for k in ("row_log2", "col_log2", "cic_shape", "cic_maxlog1", "tuned")}}
    wsz = S.slepian_workspace_size(plan, S.SLEPIAN_OP_PROJECT, b)
    work = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)
    for name, p in (("mixed", S.SLEPIAN_MIXED), ("fp32", S.SLEPIAN_FP32), ("bf16_raw", S.SLEPIAN_BF16_RAW)):
        ms = _time_calls(lambda: S.slepian_project(plan, x, y, work=work, precision=p), max(3, args.steps // 4), 2,
                         dev)
        out[name] = {"ms_per_call": round(ms, 4), "value": round(N * b / (ms * 1e-3) / 1e9, 3), "unit": "GSamples/s"}
    prec = S.SLEPIAN_MIXED if args.precision == "mixed" else S.SLEPIAN_FP32
    kernels, roof = traced_roofline(lambda: S.slepian_project(plan, x, y, work=work, precision=prec),
                                    max(3, args.steps // 4), N, b, plan.info, out["workload"])
    out["roofline"] = roof
    out["kernels"] = {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                      for k, v in kernels.items()}
    out["compulsory_byte_efficiency"] = round(out[args.precision]["value"] * 1e9 * 8 / (HBM_PEAK_GBS * 1e9), 4)
    log(f"bench: precision workload mixed {out['mixed']['value']} GSamples/s, fp32 {out['fp32']['value']}; "
        f"dominant kernel {roof['kernel']} at {roof['frac']:.3f} of 8 TB/s")
    del x, y, work
    return out


def bench_fourier_extension(args, dev):
    """The Fourier-extension experiment at its largest size (Section 4.2):
    M = 2560 (N = 5121, W = 1/3, T = 1.5), the right-hand side by a
    2^24-point quadrature, solved with the fast pseudoinverse (eps = 1e-5,
    rank K = #{lambda >= 1e-4}) and the fast Tikhonov operator (alpha =
    1e-8); relative RMS errors of the extensions and of the truncated Fourier
    series with as many terms.  The comparison with the exact operators runs
    in the GPU tests at smaller M (a dense eigendecomposition at N = 5121 is
    left out here)."""
    import numpy as np
    import torch

    from paper_1611_04950_amd import fourier_ext as fe
    from paper_1611_04950_amd import slepian as S
    from paper_1611_04950_amd import synth
    M, T, eps, thr, alpha = 2560, 1.5, 1e-5, 1e-4, 1e-8
    N, W = 2 * M + 1, 1.0 / (2 * T)
    log("bench: Fourier-extension workload")
    fp = synth.fe_function()
    Q = synth.fe_grid(M)
    yh = synth.fe_coefficients(fp, M, T, Q, device=dev)
    t0 = time.perf_counter()
    Pp = fe.truncated_plan(M, T, eps, thr)
    torch.cuda.synchronize()
    setup_p = time.perf_counter() - t0
    t0 = time.perf_counter()
    Pt = S.slepian_plan(N, W, eps, alpha=alpha)
    torch.cuda.synchronize()
    setup_t = time.perf_counter() - t0
    y = torch.tensor(np.stack([yh.real, yh.imag]), dtype=torch.float32, device=dev)
    xs = torch.empty(y.shape, dtype=torch.float64, device=dev)
    ms_p = _time_calls(lambda: S.slepian_lsq(Pp, y, mode=S.SLEPIAN_PINV, tol=0.0, max_iter=0, x=xs), 20, 3, dev)
    ms_t = _time_calls(lambda: S.slepian_lsq(Pt, y, mode=S.SLEPIAN_TIKHONOV, alpha=alpha, tol=0.0, max_iter=0,
                                             x=xs), 20, 3, dev)
    gp = fe.solve(Pp, yh, S.SLEPIAN_PINV, device=dev)
    gt = fe.solve(Pt, yh, S.SLEPIAN_TIKHONOV, alpha=alpha, device=dev)
    e_fs = synth.fe_rel_rms(fp, synth.fe_coefficients(fp, M, 1.0, Q, device=dev), 1.0, Q, device=dev)
    e_p = synth.fe_rel_rms(fp, gp, T, Q, device=dev)
    e_t = synth.fe_rel_rms(fp, gt, T, Q, device=dev)
    log(f"bench: Fourier extension M={M}: series {e_fs:.3e}, fast pinv {e_p:.3e} ({ms_p:.3f} ms), "
        f"fast Tikhonov {e_t:.3e} ({ms_t:.3f} ms)")
    return {"workload": f"Fourier extension M={M} (N={N}, W=1/3, T=1.5), quadrature 2^{Q.bit_length() - 1}",
            "K": Pp.info["K"], "r_pinv": Pp.info["r"], "r_tik": Pt.info["r_tik"],
            "plan_setup_s": {"pinv": round(setup_p, 3), "tikhonov": round(setup_t, 3)},
            "ms_per_solve": {"pinv": round(ms_p, 4), "tikhonov": round(ms_t, 4)},
            "rel_rms_error": {"fourier_series": e_fs, "extension_fast_pinv": e_p,
                              "extension_fast_tikhonov": e_t},
            "series_over_extension": round(e_fs / e_p, 1)}


def bench_eigen_gap(args, dev):
    """Figure 1's study from the GPU plans: #{eps < lambda < 1 - eps} for
    W = 1/4, N = 2^4 .. 2^16, and for N = 2^16, W = 2^-14 .. 2^-2, with eps
    in {1e-3, 1e-6, 1e-9, 1e-12}, beside the asymptotic count
    (2/pi^2) log N log(1/eps - 1) (Section 1.2) and Corollary 1's bound."""
    import torch

    from paper_1611_04950_amd import slepian as S
    log("bench: eigenvalue-gap study")
    t0 = time.perf_counter()
    epss = (1e-3, 1e-6, 1e-9, 1e-12)

    def count(N, W, eps):
        return int(S.slepian_plan(N, W, eps).info["r"])

    vs_n = {f"{e:g}": [count(1 << lg, 0.25, e) for lg in range(4, 17)] for e in epss}
    vs_w = {f"{e:g}": [count(1 << 16, 2.0 ** -k, e) for k in range(14, 1, -1)] for e in epss}
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    asym = {f"{e:g}": [round(2.0 / math.pi ** 2 * math.log(1 << lg) * math.log(1.0 / e - 1.0), 1)
                       for lg in range(4, 17)] for e in epss}
    cor1 = {f"{e:g}": round((8.0 / math.pi ** 2 * math.log(8 * (1 << 16)) + 12.0) * math.log(15.0 / e), 1)
            for e in epss}
    log(f"bench: eigenvalue gap, {2 * 13 * len(epss)} plans in {el:.1f} s; N = 2^16, W = 1/4: "
        + ", ".join(f"eps {k}: {v[-1]}" for k, v in vs_n.items()))
    return {"workload": "eigenvalue gap: W=1/4, N=2^4..2^16; N=2^16, W=2^-14..2^-2; eps 1e-3..1e-12",
            "log2_N": list(range(4, 17)), "count_vs_N": vs_n, "asymptotic_vs_N": asym,
            "log2_W": list(range(-14, -1)), "count_vs_W_at_N_2_16": vs_w,
            "corollary1_bound_at_N_2_16": cor1, "plans": 2 * 13 * len(epss), "seconds": round(el, 2)}


def bench_multiband(args, dev):
    """Multiband (modulated Slepian) dictionary (Section 1.4, application i):
    N = 2^20, W = 1/256, eps = 1e-6, eight bands centred at (2k + 1)/32,
    k = 0..7, 16 real signals, in the bench's correction precision.  The
    projection onto the dictionary's span (conjugate gradients on the band
    sum, steps reported), and the band sum itself from the prepared band set
    (one FFT product with the band-sum kernel and one modulated correction
    of rank 2 x 8 r) against the band-by-band call (demodulation, the plan's
    projection of 2 x 8 x 16 real rows, remodulation), which computes the
    same band sum."""
    import torch

    from paper_1611_04950_amd import slepian as S
    from paper_1611_04950_amd import synth
    N, W, eps, b = 1 << 20, 1.0 / 256, 1e-6, 16
    freqs = [(2 * k + 1) / 32 for k in range(8)]
    log("bench: multiband workload")
    plan = S.slepian_plan(N, W, eps, precision=S.SLEPIAN_MIXED if args.precision == "mixed" else S.SLEPIAN_FP32)
    t0 = time.perf_counter()
    bands = S.slepian_bands_create(plan, freqs)
    setup = time.perf_counter() - t0
    x = synth.gaussian(N, b, 4242, device=dev)
    y = torch.empty_like(x)
    work = torch.empty(S.slepian_bands_workspace_size(bands, b), dtype=torch.uint8, device=dev)
    ms = _time_calls(lambda: S.slepian_project_bands(bands, x, y, work=work), 20, 3, dev)
    S.slepian_trace_enable(True)
    S.slepian_trace_read(reset=True)
    S.slepian_project_bands(bands, x, y, work=work)
    torch.cuda.synchronize()
    st = S.slepian_trace_read(reset=True)
    S.slepian_trace_enable(False)
    del work
    # the projection onto the dictionary's span (CG on the band sum)
    work = torch.empty(S.slepian_bands_span_workspace_size(bands, b), dtype=torch.uint8, device=dev)
    ys = torch.empty_like(x)
    _, steps = S.slepian_project_bands_span(bands, x, ys, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        _, steps = S.slepian_project_bands_span(bands, x, ys, work=work)
    torch.cuda.synchronize()
    ms_span = (time.perf_counter() - t0) / reps * 1e3
    gap = ((torch.linalg.vector_norm((y - ys).double(), dim=1) / torch.linalg.vector_norm(ys.double(), dim=1))
           .max().item())
    log(f"bench: multiband span projection {ms_span:.3f} ms per call ({max(steps)} CG steps), "
        f"band sum differs from it by {gap:.2e}")
    del work, ys
    nb = len(freqs) * b
    work = torch.empty(S.slepian_workspace_size(plan, S.SLEPIAN_OP_MULTIBAND, nb), dtype=torch.uint8, device=dev)
    y2 = torch.empty_like(x)
    ms_band = _time_calls(lambda: S.slepian_project_multiband(plan, freqs, x, y2, work=work), 5, 1, dev)
    torch.cuda.synchronize()
    diff = ((torch.linalg.vector_norm((y - y2).double(), dim=1) / torch.linalg.vector_norm(y2.double(), dim=1))
            .max().item())
    del work, y2
    log(f"bench: multiband N=2^20, {len(freqs)} bands x {b} signals: prepared {ms:.3f} ms per call, "
        f"band by band {ms_band:.3f} ms (max rel diff {diff:.1e})")
    return {"workload": f"multiband dictionary N=2^20, W=1/256, eps=1e-6, bands (2k+1)/32 k=0..7, {b} signals",
            "precision": args.precision, "K": plan.info["K"], "r": plan.info["r"], "bands": freqs, "signals": b,
            "span_projection": {"ms_per_call": round(ms_span, 3), "cg_steps": steps,
                                "input_GSamples_per_s": round(N * b / (ms_span * 1e-3) / 1e9, 3),
                                "band_sum_rel_distance": gap,
                                "timing": "wall clock per synchronous call, one D2H check per step"},
            "band_sum_ms_per_call": round(ms, 4), "band_sum_input_GSamples_per_s": round(N * b / (ms * 1e-3) / 1e9, 3),
            "band_set_setup_s": round(setup, 3),
            "band_by_band_ms_per_call": round(ms_band, 4), "speedup_vs_band_by_band": round(ms_band / ms, 2),
            "max_rel_diff_vs_band_by_band": diff,
            "kernels_traced_ms": {k: round(v["total_ms"], 4) for k, v in st.items()}}


def bench_factorization(args, dev, check=None):
    """Fast factorization S_K S_K^T ~= T1 T2^T (Section 1.3, Theorem 1) at the
    paper-scale size N = 65536, W = 1/8, eps = 1e-6, 256 signals: compression
    T2^T x (length-N DFT bins through the FFT passes plus [L2 U]^T x on the
    matrix cores) and recovery T1 c, in the bench's correction precision,
    with L1, L2 from Theorem 1's construction (the reported figures) and,
    beside it, from the eigenpairs of B - F F^* (key "eig_factor").
    Also reports the distance of the round trip from the plan's fast
    projection (both within eps of S_K S_K^T, so at most 3 eps apart) and,
    given the CPU leg's `check`, the round trip of its signal sample against
    the oracle's (per-signal relative error, gated at 1e-5) with the oracle's
    timing beside it."""
    from paper_1611_04950_amd import slepian as S
    out = _bench_factorization(args, dev, S.SLEPIAN_FACTOR_THEOREM1, check)
    out["eig_factor"] = _bench_factorization(args, dev, S.SLEPIAN_FACTOR_EIG, None)
    return out


def _bench_factorization(args, dev, method, check):
    import torch

    from paper_1611_04950_amd import slepian as S
    from paper_1611_04950_amd import synth
    N, W, eps, b = 65536, 1.0 / 8, 1e-6, 256
    name = "theorem1" if method == S.SLEPIAN_FACTOR_THEOREM1 else "eig"
    log(f"bench: factorization workload ({name} factor)")
    plan = S.slepian_plan(N, W, eps, precision=S.SLEPIAN_MIXED if args.precision == "mixed" else S.SLEPIAN_FP32)
    t0 = time.perf_counter()
    F = S.slepian_factor_create(plan, method)
    setup = time.perf_counter() - t0
    x = synth.gaussian(N, b, 6200, device=dev)
    kp = F.info["kprime"]
    c = torch.empty((b, kp), dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    work = torch.empty(S.slepian_factor_workspace_size(F, b), dtype=torch.uint8, device=dev)
    ms_c = _time_calls(lambda: S.slepian_factor_compress(F, x, c, work=work), 20, 3, dev)
    ms_r = _time_calls(lambda: S.slepian_factor_recover(F, c, y, work=work), 20, 3, dev)
    # per-launch averages over ten traced calls of each direction (HIP events
    # around each launch), against each kernel's algorithmic bytes: x and y
    # once (4 B per sample), the even frequency rows of the pair intermediate
    # once (8 B per complex value, L/2 per pair), the kept bins once (8 B,
    # kf per pair), [V U] once (4 B per entry; BF16 hi + lo in the fused pass)
    S.slepian_trace_enable(True)
    S.slepian_trace_read(reset=True)
    for _ in range(10):
        S.slepian_factor_compress(F, x, c, work=work)
    torch.cuda.synchronize()
    st_c = S.slepian_trace_read(reset=True)
    for _ in range(10):
        S.slepian_factor_recover(F, c, y, work=work)
    torch.cuda.synchronize()
    st_r = S.slepian_trace_read(reset=True)
    S.slepian_trace_enable(False)
    L, P, kf, rt = 2 * N, b // 2, F.info["kf"], F.info["r1"] + F.info["r"]
    rp = (rt + 31) // 32 * 32
    even_rows = P * (L // 2) * 8.0
    alg = {"col_fwd_even": 4.0 * N * b + even_rows, "dft_bins_row": even_rows + P * kf * 8.0,
           "corr_partial_bf16x3": 4.0 * N * b + 4.0 * N * rt, "corr_partial": 4.0 * N * b + 4.0 * N * rt,
           "dft_from_bins_row": P * kf * 8.0 + even_rows,
           "col_inv_even_corr_bf16x3": even_rows + 4.0 * N * b + 4.0 * N * rp + 4.0 * rt * b,
           "col_inv_even_corr": even_rows + 4.0 * N * b + 4.0 * N * rp + 4.0 * rt * b}

    def roof(st):
        out = {}
        for k, v in st.items():
            us = 1000.0 * v["total_ms"] / max(v["launches"], 1)
            e = {"avg_us": round(us, 2)}
            if k in alg:
                gbs = alg[k] / (us * 1e-6) / 1e9
                e.update({"alg_bytes": alg[k], "alg_GBs": round(gbs, 1), "frac_of_8TBs": round(gbs / 8000.0, 3)})
            out[k] = e
        dom = max(out, key=lambda k: out[k]["avg_us"])
        return out, dom
    p = S.slepian_project(plan, x)
    torch.cuda.synchronize()
    dist = ((torch.linalg.vector_norm((y - p).double(), dim=1) / torch.linalg.vector_norm(x.double(), dim=1))
            .max().item())
    kc, dc = roof(st_c)
    kr, dr = roof(st_r)
    vs_oracle = None
    if check is not None:
        import numpy as np
        ys = S.slepian_factor_recover(F, S.slepian_factor_compress(F, check["sample"]))
        torch.cuda.synchronize()
        ys = ys.double().cpu().numpy()
        ref = check["ref"]
        vs_oracle = float((np.linalg.norm(ys - ref, axis=1) / np.linalg.norm(ref, axis=1)).max())
        if not vs_oracle <= 1e-5:
            log(f"bench: factorization parity gate failed ({vs_oracle:.2e})")
            sys.exit(1)
    log(f"bench: factorization ({name}) N={N}, K'={kp} (kf {F.info['kf']}, r1 {F.info['r1']}, r {F.info['r']}): "
        f"compress {ms_c:.3f} ms, recover {ms_r:.3f} ms, setup {setup:.2f} s, |T1T2^T x - P~x|/|x| <= {dist:.1e}")
    return {"workload": f"fast factorization N={N}, W=1/8, eps=1e-6, {b} signals", "factor": name,
            "theorem1_pieces": {"r_h": F.info["r_h"], "r_a": F.info["r_a"], "r_b": F.info["r_b"]}
            if name == "theorem1" else None,
            "precision": args.precision, "K": plan.info["K"], "kf": F.info["kf"], "r1": F.info["r1"],
            "r": F.info["r"], "kprime": kp, "setup_subspace": F.info["subspace"], "setup_s": round(setup, 3),
            "compress_ms": round(ms_c, 4), "recover_ms": round(ms_r, 4),
            "compress_GSamples_per_s": round(N * b / (ms_c * 1e-3) / 1e9, 3),
            "recover_GSamples_per_s": round(N * b / (ms_r * 1e-3) / 1e9, 3),
            "max_dist_to_fast_projection_rel_to_x": dist,
            "parity_max_rel_err_vs_oracle": vs_oracle,
            "cpu_oracle": None if check is None else check["cpu"],
            "compress_kernels": kc, "compress_dominant": dc, "recover_kernels": kr, "recover_dominant": dr}


def bench_coeffs(args, dev):
    """Slepian coefficients c = S_K^T x (Section 1.3, the compression to K
    numbers) at the paper-scale size N = 65536, W = 1/8 (K = 16384), 256
    signals: a hand-written matrix-core GEMM (coeffs.hip), FP32 for an FP32
    plan and three BF16 products of hi/lo halves for a mixed plan.  The first
    call computes all K Slepian vectors; the timed calls reuse them."""
    import torch

    from paper_1611_04950_amd import slepian as S
    from paper_1611_04950_amd import synth
    N, W, eps, b = 65536, 1.0 / 8, 1e-6, 256
    log("bench: coefficients workload")
    x = synth.gaussian(N, b, 6100, device=dev)
    out = {"workload": f"slepian_coeffs N={N}, W=1/8, K=16384, {b} signals",
           "flops_per_call": 2.0 * 16384 * b * N}
    for name, prec, peak in (("fp32", S.SLEPIAN_FP32, 157.3), ("mixed", S.SLEPIAN_MIXED, 2500.0)):
        P = S.slepian_plan(N, W, eps, precision=prec)
        K = P.info["K"]
        t0 = time.perf_counter()
        c = S.slepian_coeffs(P, x)
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        ms = _time_calls(lambda: S.slepian_coeffs(P, x, c), 5, 1, dev)
        tf = 2.0 * K * b * N / (ms * 1e-3) / 1e12
        mfma = tf * (3 if prec != S.SLEPIAN_FP32 else 1)
        out[name] = {"ms_per_call": round(ms, 3), "TFLOP_s": round(tf, 1), "first_call_s": round(first, 2),
                     "matrix_TFLOP_s": round(mfma, 1), "frac_of_peak": round(mfma / peak, 3),
                     "peak_TFLOP_s": peak}
        log(f"bench: coefficients {name}: {ms:.3f} ms per call, {tf:.1f} TFLOP/s "
            f"({mfma:.0f} TFLOP/s on the matrix cores, {100 * mfma / peak:.1f}% of peak)")
        del P, c
        torch.cuda.empty_cache()
    return out


def bench_lsq(args, dev):
    """N = 2^20, W = 0.02, eps = 1e-6, 64 signals of 200 tones at 10 dB:
    Tikhonov (alpha = 1e-3) solve refined to a 1e-10 FP64 normal-equation
    residual.  The residual is the library's own FP64 check; the CPU
    recomputation and the comparison with the oracle's solve are GPU tests."""
    import torch

    from paper_1611_04950_amd import slepian as S
    from paper_1611_04950_amd import synth
    N, W, eps, b, alpha = 1 << 20, 0.02, 1e-6, 64, 1e-3
    log("bench: least-squares workload")
    t0 = time.perf_counter()
    plan = S.slepian_plan(N, W, eps, alpha=alpha)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    yv = synth.config_signals(5, N, b, W, device=dev)
    xs = torch.empty(yv.shape, dtype=torch.float64, device=dev)
    wsz = S.slepian_workspace_size(plan, S.SLEPIAN_OP_LSQ, b)
    work = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)
    rep = {}

    def solve():
        _, r = S.slepian_lsq(plan, yv, mode=S.SLEPIAN_TIKHONOV, alpha=alpha, tol=1e-10, max_iter=30, x=xs,
                             work=work)
        rep.update(r)

    t0 = time.perf_counter()
    solve()
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        solve()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    fast_ms = _time_calls(lambda: S.slepian_lsq(plan, yv, mode=S.SLEPIAN_TIKHONOV, alpha=alpha, tol=0.0,
                                                max_iter=0, x=xs, work=work), 3, 1, dev)
    log(f"bench: least squares {ms:.2f} ms per refined solve ({rep.get('iterations')} sweeps, "
        f"residual {rep.get('rel_residual'):.2e})")
    return {"workload": "least squares N=2^20 W=0.02 eps=1e-6 b=64 alpha=1e-3 tol=1e-10",
            "plan_setup_s": round(setup, 3), "r": plan.info["r"], "r_tik": plan.info["r_tik"],
            "ms_per_refined_solve": round(ms, 3), "first_call_ms": round(first * 1e3, 3),
            "refinement_sweeps": rep.get("iterations"), "rel_residual": rep.get("rel_residual"),
            "rel_residual_unrefined": rep.get("rel_residual_first"),
            "ms_fast_operator_only": round(fast_ms, 3),
            "value": round(N * b / (ms * 1e-3) / 1e9, 3), "unit": "GSamples/s solved (wall clock, synchronising)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # 200 untimed steps (~30 ms of work) before the timed ones
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-signal FP32 comparison")
    ap.add_argument("--tune", type=int, default=1, help="1: tune the plans' launch variants at creation")
    ap.add_argument("--exact-vs-fast", type=int, default=1,
                    help="1: time the oracle's exact and fast projections at N = 1024..4096 (CPU)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only time a plain 256 MiB device-to-device copy (HBM calibration)")
    ap.add_argument("--precision", choices=["mixed", "fp32"], default="mixed",
                    help="correction arithmetic of the timed batched path (the FFT product is FP32 in both)")
    ap.add_argument("--no-batching", action="store_true",
                    help="skip the many-plans workload (512 plans through one grouped call)")
    ap.add_argument("--extra", default="all",
                    help="comma-separated extra workloads to run (precision, lsq, fourier, eigengap, multiband, "
                         "coeffs, factorization), or all")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the precision (N=2^18, 1024 signals) and least-squares (N=2^20) workloads")
    args = ap.parse_args()

    if args.copy_only:
        import torch
        print(json.dumps(copy_bandwidth(torch.device("cuda:0"))), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the workload's "
              f"signals are independent and would shard across GPUs without communication.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1611_04950_amd import slepian as S
    from paper_1611_04950_amd import synth

    N, W, eps, b, cfg = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    log(f"bench: plan N={N} W={W} eps={eps}")
    t0 = time.perf_counter()
    # launch variants tuned at creation for this batch size, in the timed precision
    prec0 = S.SLEPIAN_MIXED if args.precision == "mixed" else S.SLEPIAN_FP32
    plan = S.slepian_plan(N, W, eps, precision=prec0, tune=args.tune, tune_batch=b)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = plan.info
    log(f"bench: plan ready in {setup_s:.2f} s: K={info['K']} L={info['L']} r={info['r']}; rows 2^{info['row_log2']}, "
        f"L1 2^{info['col_log2']}, pass C shape {info['cic_shape']}, fused up to 2^{info['cic_maxlog1']}")

    x = synth.config_signals(cfg, N, b, W, device=dev)
    y = torch.empty_like(x)
    wsz = S.slepian_workspace_size(plan, S.SLEPIAN_OP_PROJECT, b)
    work = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    # The GPU outputs for a sample of the signals in every precision, kept on
    # the host: the CPU oracle leg gates them after the timed region, so the
    # seconds of CPU work do not leave the GPU idle (and its clocks down)
    # right before the timed steps.
    prec = S.SLEPIAN_MIXED if args.precision == "mixed" else S.SLEPIAN_FP32
    ns = min(b, 32)
    gpu_out = {}
    if not args.no_cpu:
        for p in (S.SLEPIAN_FP32, S.SLEPIAN_BF16_RAW, prec):
            S.slepian_project(plan, x, y, work=work, precision=p)
            torch.cuda.synchronize()
            gpu_out[p] = y[:ns].double().cpu().numpy()
        x_sample = x[:ns].double().cpu().numpy()

    # The other workloads run before the headline is timed: the GPU then
    # comes to the headline's warm-up steps busy, at its sustained clocks,
    # so the timed steps measure the same throughput whatever the warm-up
    # count (the factorization leg, which the CPU leg's oracle outputs
    # check, runs after it).
    extras = set() if args.no_extra else (
        {"precision", "lsq", "fourier", "eigengap", "multiband", "coeffs", "factorization"} if args.extra == "all"
        else set(args.extra.split(",")))
    coeffs = bench_coeffs(args, dev) if "coeffs" in extras else None
    egap = bench_eigen_gap(args, dev) if "eigengap" in extras else None
    fext = bench_fourier_extension(args, dev) if "fourier" in extras else None
    mband = bench_multiband(args, dev) if "multiband" in extras else None
    lsq = bench_lsq(args, dev) if "lsq" in extras else None
    batching = None if args.no_batching else bench_batching(args, dev)
    # last, the workload closest to the headline's (FFT passes, no matrix-core GEMM)
    precision = bench_precision(args, dev) if "precision" in extras else None

    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def timed(p, steps):
        for _ in range(args.warmup):
            S.slepian_project(plan, x, y, work=work, precision=p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            S.slepian_project(plan, x, y, work=work, precision=p)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps, (time.perf_counter() - t0) / steps * 1e3

    # the other precision's figure, over at least 100 steps; then the
    # headline: exactly `warmup` untimed and `steps` timed steps
    other = S.SLEPIAN_FP32 if prec == S.SLEPIAN_MIXED else S.SLEPIAN_MIXED
    steps_other = max(args.steps, 100)
    ms_other, _ = timed(other, steps_other)
    ms_per_step, wall_ms = timed(prec, args.steps)
    value = N * b / (ms_per_step * 1e-3) / 1e9
    log(f"bench: {ms_per_step:.4f} ms/step (wall {wall_ms:.4f}), {value:.2f} GSamples/s; "
        f"other precision {ms_other:.4f} ms/step")

    # per-kernel durations with HIP events around each launch (traced pass)
    kernels, roofline = traced_roofline(lambda: S.slepian_project(plan, x, y, work=work, precision=prec),
                                        args.steps, N, b, info, args.workload)

    # The CPU leg: the FP64 oracle timed on the sample; its outputs gate the
    # GPU results kept above (both precisions) before anything is reported.
    cpu = None
    err = err_sel = None
    extra_err = None
    fac_check = None
    if not args.no_cpu:
        log(f"bench: timing the CPU oracle on {ns} signals")
        cpu, ref, exact, fcpu, fref = cpu_baseline(N, W, eps, x_sample, args.cpu_seconds)
        fac_check = {"sample": x[:ns].contiguous(), "ref": fref, "cpu": fcpu}

        def rel(ys, r):
            return float((np.linalg.norm(ys - r, axis=1) / np.linalg.norm(r, axis=1)).max())

        err, err_sel = rel(gpu_out[S.SLEPIAN_FP32], ref), rel(gpu_out[prec], ref)
        log(f"bench: max rel err vs oracle on signals 0..{ns - 1}: fp32 {err:.3e}, {args.precision} {err_sel:.3e}")
        if not (err <= 1e-5 and err_sel <= 1e-5):
            log("bench: parity gate failed; no throughput reported")
            sys.exit(1)
        # the BF16 correction without its lo terms, and the distance of the
        # selected precision's result from the exact projection
        err_raw = rel(gpu_out[S.SLEPIAN_BF16_RAW], ref)
        xn = np.linalg.norm(x_sample, axis=1)
        err_exact = float((np.linalg.norm(gpu_out[prec] - exact, axis=1) / xn).max())
        log(f"bench: bf16 without lo terms {err_raw:.3e} vs the oracle; {args.precision} vs the exact projection "
            f"{err_exact:.3e} of ||x|| (Corollary 2 bound eps = {eps:g})")
        extra_err = {"bf16_raw_vs_oracle": err_raw, "vs_exact_projection_rel_to_x": err_exact,
                     "corollary2_bound_rel_to_x": eps}
    plain = None
    if not args.no_plain:
        plain = plain_fp32_per_signal(plan, x, N, W, eps, info, dev, ms_per_step, work)

    factor = bench_factorization(args, dev, fac_check) if "factorization" in extras else None
    if factor and coeffs:
        factor["speedup_compress_vs_dense_coeffs"] = round(coeffs[args.precision]["ms_per_call"] / factor["compress_ms"], 1)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GSamples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32+bf16x3" if args.precision == "mixed" else "fp32",
        "precision": ("FP32 FFT product; correction on matrix cores, BF16 hi/lo operands, FP32 accumulation"
                      if args.precision == "mixed" else "FP32 FFT product; FP32 matrix-core correction"),
        "fp32_batched": {"value": round(N * b / (ms_other * 1e-3) / 1e9, 3) if prec == S.SLEPIAN_MIXED else None,
                         "ms_per_step": round(ms_other, 5) if prec == S.SLEPIAN_MIXED else None,
                         "steps": steps_other, "warmup": args.warmup},
        "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "W": W, "eps": eps, "batch": b, "K": info["K"],
                   "L": info["L"], "r": info["r"],
                   "launch": {k: info[k] for k in ("row_log2", "col_log2", "cic_shape", "cic_maxlog1", "tuned",
                                                   "tune_us")}},
        "parity_max_rel_err": err_sel,
        "parity_max_rel_err_fp32": err,
        "errors": extra_err,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain_fp32_per_signal": plain,
        "compulsory_byte_efficiency": round(value * 1e9 * 8 / (HBM_PEAK_GBS * 1e9), 4),
        "plan_setup_s": round(setup_s, 3),
        "hbm_copy": copy_bandwidth(dev),
        "device": {"name": torch.cuda.get_device_name(dev),
                   "cu": torch.cuda.get_device_properties(dev).multi_processor_count},
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()},
        "batching": batching,
        "precision_workload": precision,
        "least_squares_workload": lsq,
        "fourier_extension_workload": fext,
        "eigenvalue_gap_study": egap,
        "multiband_workload": mband,
        "coefficients_workload": coeffs,
        "factorization_workload": factor,
    }
    if not args.no_cpu and args.exact_vs_fast:
        log("bench: exact vs fast projection on the CPU oracle")
        out["cpu_exact_vs_fast"] = exact_vs_fast()
    print(json.dumps(_finite(out)), flush=True)


if __name__ == "__main__":
    main()
