"""Benchmark: LS forward+backward cell updates per second (N^2 L / s) on one
MI355X, FP32-scaled sweep, with the plain FP64 path measured beside it.

Workload of the timed step: N = 10,000 mosaic haplotypes of 200 founders,
L = 100,000 variants, mu = 1e-4, rho from Exp(mean 1e-3) spacings; a
backward sweep that keeps beta at 100 evenly spaced targets, a forward sweep
that turns alpha and beta into posteriors and half distances at those
targets, and the symmetrisation into 100 full N x N FP32 distance matrices
(40 GB resident in HBM). Inputs are generated before the timed region and are
resident on the device.

Outside the timed region the same line reports: the FP64 step; the FP32
posterior error against FP64 over every recipient and target; the FP64 CPU
oracle's rate (all host cores and one core) and the FP32 error against it on
the oracle's sample; the gradient workload (N = 2,000, L = 50,000: PAC and its
gradient for all recipients, error against the oracle on 256 recipients); the
large workload (N = 100,000, L = 10,000: five resident 100k x 100k FP32
distance matrices from recipient windows, error against the oracle on 64
recipients); the precision study (N = 50,000: FP32 and FP16-stored vectors
against the oracle); and the average linkage of the step's 100 distance
matrices.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X vector peaks (dense, no sparsity): FP32 157.3 TFLOP/s,
# FP64 78.6 TFLOP/s, an FMA counting as two flops.
FP32_PEAK = 157.3e12
FP64_PEAK = 78.6e12
# Algorithmic flops per cell and direction: FMA (2) + MUL + ADD; the emission
# select is not a flop.
FLOPS_PER_CELL = 4
# Issue ceiling of the VALU in lane-instructions/s: 256 CUs x 4 SIMDs x 32
# lanes x 2.4 GHz, i.e. two wave64 instructions per SIMD every four cycles
# (the sweep's VALU counters show more than one per four cycles). The
# masked-emission sweep needs 3 lane-instructions per cell: FMA, the
# EXEC-masked multiply (one instruction per 64 cells whatever the mask) and
# the column-sum ADD.
ISSUE_PEAK = 256 * 4 * 32 * 2.4e9
ISSUE_OPS_PER_CELL = 3
HBM_PEAK = 8.0e12
SWEEP_CHUNK = 2048  # variants per sweep launch (the library splits longer sweeps)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_bwd_fp32_c2_traffic.txt")
SWEEP_SOURCES = ["ls_sweep.h", "ls_device.h", "ls_internal.h", "ls_sweep_f32_bwd.hip"]


def sweep_source_hash():
    """SHA-1 over the sources of the FP32 backward sweep kernel."""
    import hashlib
    h = hashlib.sha1()
    for name in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2212_11403_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(shape):
    """HBM bytes per launch of the backward sweep from the committed counter
    summary, or None if it is absent or was taken on other kernel sources or
    another kernel shape."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha1") != sweep_source_hash():
            return None
        if kv.get("shape") != f"{shape[0]}x{shape[1]}":
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration():
    """A plain elementwise copy over 2 GiB buffers, for scaling the FETCH_SIZE
    and WRITE_SIZE counters (profiled under rocprofv3 --pmc)."""
    import torch
    n = 1 << 29  # 2 GiB per buffer, well above the 256 MB last-level cache
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)  # elementwise kernel: reads and writes 2 GiB
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n}),
          flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Timer:
    """HIP events on the stream the library launches on (torch's current
    stream, handed to every call)."""

    def __init__(self, torch):
        self.torch = torch
        self.e = [torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]

    def __enter__(self):
        self.e[0].record(self.torch.cuda.current_stream())
        return self

    def __exit__(self, *a):
        self.e[1].record(self.torch.cuda.current_stream())

    def ms(self):
        self.e[1].synchronize()
        return self.e[0].elapsed_time(self.e[1])


def oracle_rate(oracle, x, nthreads, count, seed):
    """The oracle (FP64 C) on `count` seeded recipients over the full
    workload: forward, backward and posteriors at every target."""
    from lsinputs import seeded_recipients
    N, L = x["N"], x["L"]
    sample = seeded_recipients(N, count, seed=seed)
    t0 = time.perf_counter()
    ref = oracle.run_pass(x["H"], N, L, x["rho"], x["mu"], sample, x["targets"], want=("P",),
                          nthreads=nthreads)
    dt = time.perf_counter() - t0
    return len(sample) * float(N) * L / dt, dt, sample, ref


def c2_accuracy_all(ls, torch, model, targets, N, window=50):
    """Max abs posterior error of the FP32 sweep against the FP64 sweep over
    every recipient and target (decoded in windows of targets, compared on
    the device)."""
    err = 0.0
    ll_err = 0.0
    for lo in range(0, len(targets), window):
        tg = targets[lo:lo + window]
        p32 = ls.decode(model, tg, "fp32", want=("P",))
        ll32 = p32["fwd"].log_scale.clone()
        p32 = p32["P"]
        out64 = ls.decode(model, tg, "fp64", want=("P",))
        p64 = out64["P"]
        for k in range(len(tg)):
            err = max(err, float((p32[k].double() - p64[k]).abs().max().item()))
        ll64 = out64["fwd"].log_scale
        ll_err = max(ll_err, float(((ll32 - ll64).abs() / ll64.abs()).max().item()))
        del p32, p64, out64
        torch.cuda.empty_cache()
    return err, ll_err


def cluster_matrices(ls, torch, D, check):
    """Average pairwise linkage (section 6) of the step's T distance matrices,
    resident on the device (one workgroup per matrix, side by side), timed
    with HIP events; with `check`, matrix 0's merges and leaf order against
    the oracle's."""
    T, N = int(D.shape[0]), int(D.shape[1])
    D0 = D[0].cpu().numpy() if check else None
    torch.cuda.synchronize()
    with Timer(torch) as t:
        Z, order = ls.average_linkage(D)
    ms = t.ms()
    out = {"matrices": T, "N": N, "ms": ms, "ms_per_matrix": ms / T,
           "method": "average pairwise linkage, FP32, merges equal to the plain algorithm's"}
    if check:
        import oracle
        t0 = time.perf_counter()
        Zr, orr = oracle.average_linkage(D0)
        out["oracle_seconds_one_matrix"] = time.perf_counter() - t0
        out["matrix0_equals_oracle"] = bool(np.array_equal(Z[0].cpu().numpy(), Zr) and
                                            np.array_equal(order[0].cpu().numpy(), orr))
    return out


def gradient_workload(ls, torch, oracle, nthreads, reps=3):
    """PAC and its gradient for every recipient of the gradient workload
    (N = 2,000, L = 50,000), FP32 and FP64, timed with HIP events; error of
    both against the oracle's exact score on 256 seeded recipients."""
    from lsinputs import make_inputs, seeded_recipients
    x = make_inputs("c4")
    N, L, rho, mu = x["N"], x["L"], x["rho"], x["mu"]
    m = ls.Model(x["H"], N, rho, mu)
    out = {"workload": f"N={N}, L={L}, gradient w.r.t. {L - 1} rho_l and mu, all {N} recipients"}
    for prec in ("fp32", "fp64"):
        ls.loglik_grad(m, None, prec, grad=True)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            with Timer(torch) as t:
                ls.loglik_grad(m, None, prec, grad=True)
            ts.append(t.ms())
        with Timer(torch) as t:
            ls.loglik_grad(m, None, prec, grad=False)
        out[f"{prec}_gradient_ms"] = float(np.mean(ts))
        out[f"{prec}_loglik_only_ms"] = t.ms()
    rec = seeded_recipients(N, 256, seed=404)
    t0 = time.perf_counter()
    ref = oracle.run_gradient(x["H"], N, L, rho, mu, rec, nthreads=nthreads)
    out["oracle_seconds_256"] = time.perf_counter() - t0
    gr = ref["grad_rho"].sum(axis=0)
    gm = ref["grad_mu"].sum()
    ll = ref["loglik"].sum()
    for prec in ("fp32", "fp64"):
        g = ls.loglik_grad(m, rec, prec, grad=True)
        grg = g["grad_rho"].cpu().numpy()
        out[f"{prec}_grad_rho_rel_err_vs_oracle"] = float(np.abs(grg - gr).max() / np.abs(gr).max())
        out[f"{prec}_grad_mu_rel_err_vs_oracle"] = float(abs(g["grad_mu"].item() - gm) / abs(gm))
        out[f"{prec}_pac_rel_err_vs_oracle"] = float(abs(g["pac"].item() - ll) / abs(ll))
    out["oracle_sample"] = "256 seeded recipients, exact score (full forward table per recipient)"
    # the autograd path: PACLoglik forward (checkpoints) + backward (adjoint)
    from paper_2212_11403_amd import PACLoglik
    Hd = m.H
    r = torch.tensor(rho, dtype=torch.float64, device="cuda", requires_grad=True)
    u = torch.tensor(mu, dtype=torch.float64, device="cuda", requires_grad=True)
    ts = []
    for k in range(reps + 1):
        r.grad = u.grad = None
        with Timer(torch) as t:
            PACLoglik.apply(r, u, Hd, N, "fp32").backward()
        if k:
            ts.append(t.ms())
    out["fp32_autograd_forward_backward_ms"] = float(np.mean(ts))
    # central differences of the FP64 PAC (all recipients) on 64 seeded
    # components with rho_l >= 1e-4, step 1e-4 rho_l; norm-wise error of the
    # analytic gradients over those components. The PAC sums 2,000 x 50,000
    # FP64 log terms, so it carries rounding of about 1e-12 relative; a step
    # of 1e-6 rho_l turns that into a 1e-4 error of the difference, while at
    # 1e-4 rho_l both that and the truncation error are near 1e-9.
    rng = np.random.default_rng(505)
    idx = np.sort(rng.choice(np.flatnonzero(rho >= 1e-4), 64, replace=False))
    g64 = ls.loglik_grad(m, None, "fp64", grad=True)["grad_rho"].cpu().numpy()[idx]
    g32 = ls.loglik_grad(m, None, "fp32", grad=True)["grad_rho"].cpu().numpy()[idx]
    fd = np.empty(len(idx))
    mf = ls.Model(x["H"], N, rho, mu)
    for n, l in enumerate(idx):
        h = 1e-4 * rho[l]
        vals = []
        for sgn in (1.0, -1.0):
            rr = rho.copy()
            rr[l] += sgn * h
            mf.update(rr, mu)
            vals.append(ls.loglik_grad(mf, None, "fp64", grad=False)["pac"].item())
        fd[n] = (vals[0] - vals[1]) / (2 * h)
    scale = np.abs(fd).max()
    out["fd_components"] = int(len(idx))
    out["fp64_grad_rho_vs_central_differences"] = float(np.abs(g64 - fd).max() / scale)
    out["fp32_grad_rho_vs_central_differences"] = float(np.abs(g32 - fd).max() / scale)
    return out


def precision_workload(ls, torch, oracle, nthreads, count=64, timed_recipients=2560):
    """The precision study (N = 50,000, L = 20,000, rare-variant mosaic, 20
    targets): FP32, FP16-stored and FP64 vectors against the FP64 oracle on
    `count` seeded recipients (posteriors at every target, log-likelihoods),
    and the forward+backward cell rate of each on `timed_recipients`
    recipients."""
    from lsinputs import make_inputs, seeded_recipients
    t0 = time.time()
    x = make_inputs("c3")
    N, L, targets = x["N"], x["L"], x["targets"]
    log(f"inputs c3: N={N} L={L} ({time.time() - t0:.1f}s)")
    m = ls.Model(x["H"], N, x["rho"], x["mu"])
    rec = seeded_recipients(N, count, seed=3030)
    t0 = time.perf_counter()
    ref = oracle.run_pass(x["H"], N, L, x["rho"], x["mu"], rec, targets, want=("P",),
                          nthreads=nthreads)
    out = {"workload": f"N={N}, L={L}, {len(targets)} targets, rare-variant mosaic of "
                       f"{x['cfg']['K']} founders",
           "oracle_sample": f"{len(rec)} seeded recipients, all donors, all variants, all targets",
           "oracle_seconds": time.perf_counter() - t0}
    trec = np.arange(min(timed_recipients, N), dtype=np.int32)
    for prec in ("fp32", "f16", "fp64"):
        r = ls.decode(m, targets, prec, recipients=rec, want=("P",))
        P = r["P"].double().cpu().numpy()
        ll = r["fwd"].log_scale.cpu().numpy()
        out[f"{prec}_max_posterior_err_vs_oracle"] = float(np.abs(P - ref["P"]).max())
        out[f"{prec}_max_rel_loglik_err_vs_oracle"] = float(
            np.max(np.abs(ll - ref["llf"]) / np.abs(ref["llf"])))
        del r, P
        ms = 0.0
        for d in (1, 0):
            tab = ls.Table(m, d, prec, trec)
            torch.cuda.synchronize()
            with Timer(torch) as t:
                if d == 1:
                    ls.backward(tab, m, 0)
                else:
                    ls.forward(tab, m, L - 1)
            ms += t.ms()
            del tab
        out[f"{prec}_fwd_bwd_cells_per_s"] = len(trec) * float(N) * L / (ms / 1e3)
        out[f"{prec}_shape"] = list(ls.kernel_shape(N, prec))
    torch.cuda.empty_cache()
    return out


def large_workload(ls, torch, oracle, nthreads, window=12_500, check=64):
    """All 100,000 recipients of the large workload (L = 10,000, 5 targets)
    in windows, each writing its rows of the half distances into five
    resident 100k x 100k FP32 matrices, then the in-place symmetrisation.
    One timed pass; FP32 posterior and log-likelihood error against the
    oracle on `check` seeded recipients."""
    from lsinputs import make_inputs, seeded_recipients
    t0 = time.time()
    x = make_inputs("c5")
    N, L, targets = x["N"], x["L"], x["targets"]
    T = len(targets)
    log(f"inputs c5: N={N} L={L} T={T} ({time.time() - t0:.1f}s)")
    m = ls.Model(x["H"], N, x["rho"], x["mu"])
    # the window: what fits beside the matrices (its snapshots and two tables
    # take (T + 2) N FP32 values per recipient), at most `window`
    free, _ = torch.cuda.mem_get_info()
    d_bytes = T * N * N * 4
    fit = int((free - d_bytes - (8 << 30)) // ((T + 2) * N * 4))
    window = min(window, fit)
    if window < 256:
        return {"error": f"not enough device memory for {T} resident {N}x{N} matrices "
                         f"({free / 2**30:.0f} GiB free)"}
    D = torch.empty((T, N, N), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with Timer(torch) as t:
        res = ls.distance_matrices(m, targets, "fp32", window=window, D=D)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = t.ms()
    cells = float(N) * N * L
    out = {"workload": f"N={N} haplotypes, L={L} variants, mosaic of {x['cfg']['K']} founders, "
                       f"T={T} targets, {T} resident {N}x{N} FP32 distance matrices",
           "value": cells / (ms / 1e3), "unit": "cells/s", "seconds": ms / 1e3,
           "wall_seconds": wall, "window": window, "shape": list(ls.kernel_shape(N, "fp32"))}
    # D symmetric with a zero diagonal on sampled entries
    rng = np.random.default_rng(5)
    a = torch.as_tensor(rng.integers(0, N, 4096), device="cuda")
    b = torch.as_tensor(rng.integers(0, N, 4096), device="cuda")
    out["sym_check"] = bool(torch.equal(D[:, a, b], D[:, b, a]) and
                           bool((D[:, a, a] == 0).all().item()))
    ll = res["loglik"].cpu().numpy()
    del res, D
    torch.cuda.empty_cache()
    rec = seeded_recipients(N, check, seed=555)
    t0 = time.perf_counter()
    ref = oracle.run_pass(x["H"], N, L, x["rho"], x["mu"], rec, targets, want=("P",),
                          nthreads=nthreads)
    out["oracle_seconds"] = time.perf_counter() - t0
    p = ls.decode(m, targets, "fp32", recipients=rec, want=("P",))["P"].double().cpu().numpy()
    out["max_posterior_err_vs_oracle"] = float(np.abs(p - ref["P"]).max())
    out["max_rel_loglik_err_vs_oracle"] = float(np.max(np.abs(ll[rec] - ref["llf"]) /
                                                       np.abs(ref["llf"])))
    out["oracle_sample"] = f"{len(rec)} seeded recipients, all donors, all variants"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the all-recipient FP32 vs FP64 comparison")
    ap.add_argument("--no-gradient", action="store_true", help="skip the gradient workload")
    ap.add_argument("--no-large", action="store_true", help="skip the large workload")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32 / FP16-stored precision workload")
    ap.add_argument("--no-clustering", action="store_true",
                    help="skip the average linkage of the step's distance matrices")
    ap.add_argument("--profile", action="store_true",
                    help="the timed steps only (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1 "
                                   "(recipient sharding across GPUs is a design note only)"}))
        sys.exit(2)
    if args.profile:
        args.no_cpu_baseline = args.no_fp64 = args.no_accuracy = True
        args.no_gradient = args.no_large = args.no_clustering = args.no_precision = True

    import torch

    import paper_2212_11403_amd as ls
    from lsinputs import get_config, make_inputs

    cfg = get_config(args.config)
    t0 = time.time()
    x = make_inputs(cfg)
    N, L, targets = x["N"], x["L"], x["targets"]
    T = len(targets)
    log(f"inputs {args.config}: N={N} L={L} T={T} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    model = ls.Model(x["H"], N, x["rho"], x["mu"])
    torch.cuda.synchronize()

    def run_step(prec, bufs, ev=None):
        fwd = ls.Table(model, 0, prec)
        bck = ls.Table(model, 1, prec)
        if ev:
            ev[0].record(stream)
        ls.backward(bck, model, 0, targets, bufs["bsnap"])
        if ev:
            ev[1].record(stream)
        ls.forward(fwd, model, L - 1, targets, bufs["bsnap"], None, bufs["E"])
        if ev:
            ev[2].record(stream)
        ls.distance_symmetrise(bufs["E"], bufs["E"], prec)
        if ev:
            ev[3].record(stream)
        return fwd, bck

    def timed(prec, steps, warmup, after=None):
        dt = ls.io_dtype(prec)
        bufs = dict(bsnap=torch.empty((T, N, N), dtype=dt, device=dev),
                    E=torch.empty((T, N, N), dtype=dt, device=dev))
        for _ in range(warmup):
            run_step(prec, bufs)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        tabs = None
        for k in range(steps):
            tabs = run_step(prec, bufs, evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        bwd_ms = np.mean([e[0].elapsed_time(e[1]) for e in evs])
        fwd_ms = np.mean([e[1].elapsed_time(e[2]) for e in evs])
        sym_ms = np.mean([e[2].elapsed_time(e[3]) for e in evs])
        status = ls.status_check(tabs[0])
        ll = tabs[0].log_scale.cpu().numpy()
        extra = after(bufs["E"]) if after else None
        del bufs
        torch.cuda.empty_cache()
        return dict(wall=wall, ms_per_step=1e3 * wall / steps, bwd_ms=bwd_ms, fwd_ms=fwd_ms,
                    sym_ms=sym_ms, status=status, loglik=ll, extra=extra)

    shape = ls.kernel_shape(N, "fp32")
    log(f"fp32 shape {shape}, fp64 shape {ls.kernel_shape(N, 'fp64')}")
    after = None
    if not args.no_clustering:
        def after(D):
            return cluster_matrices(ls, torch, D, check=not args.no_cpu_baseline)
    r32 = timed("fp32", args.steps, args.warmup, after)
    cells = float(N) * N * L
    value = cells / (r32["ms_per_step"] / 1e3)
    log(f"fp32: {r32['ms_per_step']:.1f} ms/step (bwd {r32['bwd_ms']:.1f}, fwd+post "
        f"{r32['fwd_ms']:.1f}, sym {r32['sym_ms']:.1f}) -> {value:.3e} cells/s")

    # roofline of the dominant kernel: the backward sweep, launched once per
    # SWEEP_CHUNK variants; per-launch figures are averages over the sweep
    launches = -(-(L - 1) // SWEEP_CHUNK)
    launch_s = r32["bwd_ms"] / 1e3 / launches
    cells_launch = cells / launches
    flops = FLOPS_PER_CELL * cells_launch / launch_s
    lane_ops = ISSUE_OPS_PER_CELL * cells_launch / launch_s
    rows_bytes = SWEEP_CHUNK * N / 8.0                 # one bit per donor and variant
    snap_bytes = T / launches * float(N) * N * 4       # beta snapshots, FP32
    roofline = {"bound": "alu", "achieved": flops / 1e12, "peak": FP32_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": flops / FP32_PEAK,
                "traffic": measured_traffic(shape),
                "kernel": f"sweep_kernel<PrecF32,{shape[0]},1> (backward)",
                "flops_per_cell": FLOPS_PER_CELL, "launches_per_sweep": launches,
                "cells_per_launch": cells_launch, "launch_ms": launch_s * 1e3,
                "algorithmic_bytes_per_launch": rows_bytes + snap_bytes,
                "issue": {"achieved_lane_ops_per_s": lane_ops, "peak_lane_ops_per_s": ISSUE_PEAK,
                          "frac": lane_ops / ISSUE_PEAK, "ops_per_cell": ISSUE_OPS_PER_CELL}}
    line = {
        "metric": "LS fwd+bwd cell updates/s (N^2 L / s), FP32-scaled sweep",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded mosaic haplotypes)",
        "config": {"workload": f"{args.config}: N={N} haplotypes, L={L} variants, mosaic of "
                               f"{cfg['K']} founders, T={T} targets, full N x N FP32 distances",
                   "N": N, "L": L, "targets": T, "slots_per_wave": shape[0],
                   "waves_per_recipient": shape[1]},
        "roofline": roofline,
        "cpu_baseline": None,
        "fp32_breakdown_ms": {"backward_sweep": r32["bwd_ms"], "forward_sweep_and_posterior":
                              r32["fwd_ms"], "symmetrise": r32["sym_ms"]},
        "nonfinite_status": int(r32["status"]),
    }
    if r32["extra"] is not None:
        line["clustering"] = r32["extra"]
        log(f"clustering: {r32['extra']}")

    r64 = None
    if not args.no_fp64:
        r64 = timed("fp64", args.fp64_steps, 0)
        log(f"fp64: {r64['ms_per_step']:.1f} ms/step (bwd {r64['bwd_ms']:.1f}, fwd+post "
            f"{r64['fwd_ms']:.1f})")
        f64_flops = FLOPS_PER_CELL * cells / (r64["bwd_ms"] / 1e3)
        line["fp64"] = {"value": cells / (r64["ms_per_step"] / 1e3), "ms_per_step":
                        r64["ms_per_step"], "backward_sweep_ms": r64["bwd_ms"],
                        "forward_sweep_and_posterior_ms": r64["fwd_ms"],
                        "shape": list(ls.kernel_shape(N, "fp64")),
                        "backward_flops_frac": f64_flops / FP64_PEAK}
        ll32, ll64 = r32["loglik"], r64["loglik"]
        line["max_rel_loglik_err_fp32_vs_fp64"] = float(np.max(np.abs(ll32 - ll64) / np.abs(ll64)))
    if not args.no_fp64 and not args.no_accuracy:
        t0 = time.time()
        e, _ = c2_accuracy_all(ls, torch, model, targets, N)
        line["max_posterior_err_fp32_vs_fp64"] = e
        line["accuracy_scope"] = f"all {N} recipients x {T} targets ({N * N * T:.1e} posteriors)"
        log(f"fp32 vs fp64 over all recipients: {e:.3e} ({time.time() - t0:.1f}s)")

    oracle = None
    nthreads = 1
    if not (args.no_cpu_baseline and args.no_gradient and args.no_large and args.no_precision):
        import oracle
        nthreads = oracle.default_threads()
    if not args.no_cpu_baseline:
        rate, dt_cpu, sample, ref = oracle_rate(oracle, x, nthreads, 3 * nthreads, 2212)
        rate1, dt1, _, _ = oracle_rate(oracle, x, 1, 2, 2213)
        line["cpu_baseline"] = {
            "value": rate, "unit": "cells/s", "cores": int(nthreads), "kind": "oracle",
            "sample": f"{len(sample)} seeded recipients x all {N} donors x all {L} variants, "
                      f"forward+backward+posteriors at {T} targets, FP64 C, {dt_cpu:.1f} s",
            "one_core": {"value": rate1, "cores": 1,
                         "sample": f"2 seeded recipients, same work, {dt1:.1f} s"}}
        p_s = ls.decode(model, targets, "fp32", recipients=sample, want=("P",))["P"]
        line["max_posterior_err_fp32_vs_oracle"] = float(
            np.abs(p_s.double().cpu().numpy() - ref["P"]).max())
        del p_s, ref
        log(f"oracle: {rate:.3e} cells/s on {nthreads} threads ({dt_cpu:.1f}s), "
            f"{rate1:.3e} on one ({dt1:.1f}s)")
    del model
    torch.cuda.empty_cache()

    if not args.no_gradient:
        t0 = time.time()
        line["gradient_workload"] = gradient_workload(ls, torch, oracle, nthreads)
        log(f"gradient workload: {line['gradient_workload']} ({time.time() - t0:.1f}s)")
        torch.cuda.empty_cache()
    if not args.no_precision:
        t0 = time.time()
        line["precision_workload"] = precision_workload(ls, torch, oracle, nthreads)
        log(f"precision workload: {line['precision_workload']} ({time.time() - t0:.1f}s)")
    if not args.no_large:
        t0 = time.time()
        line["large_workload"] = large_workload(ls, torch, oracle, nthreads)
        log(f"large workload: {line['large_workload']} ({time.time() - t0:.1f}s)")
        torch.cuda.empty_cache()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
