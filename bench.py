"""Benchmark: LS forward+backward cell updates per second (N^2 L / s) on one
MI355X, FP32-scaled sweep, with the plain FP64 path measured beside it.

Workload (one "step" = the whole hot path over one batch): N = 10,000
mosaic haplotypes of 200 founders, L = 100,000 variants, mu = 1e-4, rho from
Exp(mean 1e-3) spacings; a backward sweep that keeps beta at 100 evenly
spaced targets, a forward sweep that turns alpha and beta into posteriors
and half distances at those targets, and the symmetrisation into 100 full
N x N FP32 distance matrices (40 GB resident in HBM). Inputs are generated
before the timed region and are resident on the device.

Prints one JSON line (see the README of this repository for the fields).
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

# FP32 vector peak in lane-operations/s: 157.3 TFLOP/s counts an FMA as two
# flops, i.e. 78.6e12 FP32 lane-operations/s = 256 CUs x 4 SIMDs x 32 lanes x
# 2.4 GHz (each SIMD issues two wave64 FP32 instructions per four cycles,
# which the SQ_ACTIVE_INST_VALU2 counter shows happening in this kernel).
VALU_PEAK = 256 * 4 * 32 * 2.4e9
# FP64 vector peak: 78.6 TFLOP/s, i.e. 39.3e12 FP64 FMA lane-operations/s.
VALU_PEAK_F64 = 256 * 4 * 16 * 2.4e9
OPS_PER_CELL = 4                  # emission select, FMA, MUL, ADD per cell per direction
SWEEP_CHUNK = 2048                # variants per sweep launch (the library splits longer sweeps)
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
    """A plain 1 GiB device-to-device copy, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (profiled under rocprofv3 --pmc)."""
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


def stream_probe():
    """Practical HBM rates of plain streaming kernels (torch elementwise ops
    over 4 GiB, event-timed), the yardstick for the HBM-bound kernels."""
    import torch
    n = 1 << 30
    x = torch.rand(n, device="cuda")
    y = torch.empty_like(x)

    def rate(f, nbytes, reps=5):
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return nbytes / (e0.elapsed_time(e1) / reps / 1e3) / 1e12

    out = {"unit": "TB/s",
           "read_write_in_place": rate(lambda: x.mul_(1.0000001), 8 * n),
           "read_write": rate(lambda: torch.mul(x, 1.0000001, out=y), 8 * n),
           "write_only": rate(lambda: y.fill_(0.5), 4 * n)}
    print(json.dumps(out), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--err-recipients", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--stream-probe", action="store_true",
                    help="print the HBM rates of plain streaming kernels and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.stream_probe:
        stream_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1 "
                                   "(recipient sharding across GPUs is a design note only)"}))
        sys.exit(2)

    import torch

    import paper_2212_11403_amd as ls
    from lsinputs import get_config, make_inputs, seeded_recipients

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

    def timed(prec, steps, warmup):
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
        del bufs
        torch.cuda.empty_cache()
        return dict(wall=wall, ms_per_step=1e3 * wall / steps, bwd_ms=bwd_ms, fwd_ms=fwd_ms,
                    sym_ms=sym_ms, status=status, loglik=ll)

    log(f"fp32 shape {ls.kernel_shape(N, 'fp32')}, fp64 shape {ls.kernel_shape(N, 'fp64')}")
    r32 = timed("fp32", args.steps, args.warmup)
    cells = float(N) * N * L
    value = cells / (r32["ms_per_step"] / 1e3)
    log(f"fp32: {r32['ms_per_step']:.1f} ms/step (bwd {r32['bwd_ms']:.1f}, fwd+post "
        f"{r32['fwd_ms']:.1f}, sym {r32['sym_ms']:.1f}) -> {value:.3e} cells/s")
    r64 = None
    if not args.no_fp64:
        r64 = timed("fp64", args.fp64_steps, 0)
        log(f"fp64: {r64['ms_per_step']:.1f} ms/step (bwd {r64['bwd_ms']:.1f}, fwd+post "
            f"{r64['fwd_ms']:.1f})")

    # posterior error of the FP32 sweep against FP64 (GPU) and against the
    # FP64 oracle, on seeded recipients (outside the timed region)
    rec = seeded_recipients(N, max(args.err_recipients, 1), seed=2212)
    p32 = None
    if args.err_recipients > 0:
        p32 = ls.decode(model, targets, "fp32", recipients=rec, want=("P",))["P"]
    err = {}
    if p32 is not None and not args.no_fp64:
        out64 = ls.decode(model, targets, "fp64", recipients=rec, want=("P",))
        p64 = out64["P"]
        err["max_posterior_err_fp32_vs_fp64"] = float((p32.double() - p64).abs().max().item())
        ll32 = r32["loglik"]
        ll64 = r64["loglik"]
        err["max_rel_loglik_err_fp32_vs_fp64"] = float(np.max(np.abs(ll32 - ll64) / np.abs(ll64)))
        del out64, p64

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nthreads = oracle.default_threads()
        # about 10-20 s of oracle work on the host's cores
        sample = seeded_recipients(N, 3 * nthreads, seed=2212)
        t0 = time.perf_counter()
        ref = oracle.run_pass(x["H"], N, L, x["rho"], x["mu"], sample, targets, want=("P",),
                              nthreads=nthreads)
        dt_cpu = time.perf_counter() - t0
        cpu_rate = len(sample) * float(N) * L / dt_cpu
        cpu = {"value": cpu_rate, "unit": "cells/s", "cores": int(nthreads), "kind": "oracle",
               "sample": f"{len(sample)} seeded recipients x all {N} donors x all {L} variants, "
                         f"forward+backward+posteriors at {T} targets, FP64 C, {dt_cpu:.1f} s"}
        if p32 is not None:
            p_s = ls.decode(model, targets, "fp32", recipients=sample, want=("P",))["P"]
            err["max_posterior_err_fp32_vs_oracle"] = float(
                np.abs(p_s.double().cpu().numpy() - ref["P"]).max())
            del p_s
        log(f"oracle: {cpu_rate:.3e} cells/s on {nthreads} threads ({dt_cpu:.1f}s)")
    del p32

    # roofline of the dominant kernel: the backward sweep, launched once per
    # SWEEP_CHUNK variants; per-launch figures are averages over the sweep
    shape = ls.kernel_shape(N, "fp32")
    launches = -(-(L - 1) // SWEEP_CHUNK)
    bwd_s = r32["bwd_ms"] / 1e3
    achieved = OPS_PER_CELL * cells / bwd_s
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                "unit": "TOP/s", "frac": achieved / VALU_PEAK,
                "traffic": measured_traffic(shape),
                "kernel": f"sweep_kernel<PrecF32,{shape[0]},1> (backward)",
                "ops_per_cell": OPS_PER_CELL, "launches_per_sweep": launches,
                "cells_per_launch": cells / launches,
                "launch_ms": r32["bwd_ms"] / launches}
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
        "cpu_baseline": cpu,
        "fp32_breakdown_ms": {"backward_sweep": r32["bwd_ms"], "forward_sweep_and_posterior":
                              r32["fwd_ms"], "symmetrise": r32["sym_ms"]},
        "nonfinite_status": int(r32["status"]),
    }
    if r64 is not None:
        a64 = OPS_PER_CELL * cells / (r64["bwd_ms"] / 1e3)
        line["fp64"] = {"value": cells / (r64["ms_per_step"] / 1e3), "ms_per_step":
                        r64["ms_per_step"], "backward_sweep_ms": r64["bwd_ms"],
                        "forward_sweep_and_posterior_ms": r64["fwd_ms"],
                        "shape": list(ls.kernel_shape(N, "fp64")),
                        "backward_alu_frac": a64 / VALU_PEAK_F64}
    line.update(err)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
