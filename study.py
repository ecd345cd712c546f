"""Measurements on the workloads other than the benchmark's (one JSON line each).

    python study.py c4   gradient of the PAC log-likelihood (N = 2,000,
                         L = 50,000): time per gradient in FP32 and FP64,
                         VALU and HBM rooflines of the pass, FP32 and FP64
                         adjoint vs the FP64 oracle score over all recipients
                         and vs central differences of the FP64 GPU PAC at 64
                         seeded rho_l
    python study.py c3   precision study (N = 50,000, L = 20,000, rare-variant
                         mosaic, 20 targets): FP32 and FP16-stored posteriors
                         and log-likelihoods vs the FP64 oracle on seeded
                         recipients, and the decode time of all recipients
    python study.py c2   FP32 against FP64 on the benchmark workload (N = 10,000,
                         L = 100,000, 100 targets) over all recipients and
                         targets: posterior and distance errors; both GPU
                         paths against the oracle on 256 seeded recipients
    python study.py c5   the share of one GPU of the large workload
                         (N = 100,000, L = 10,000, 5 targets): recipients
                         [0, 12,500) against all 100,000 donors, FP32 decode
                         time, E-write bandwidth, posterior error vs the oracle
    python study.py c2var  the benchmark workload's decode step (N = 10,000,
                         L = 100,000, 100 targets, all recipients, FP32) with a
                         scalar mu, a per-variant mu (log-uniform within a
                         decade of the workload's mu) and a skewed prior
                         matrix Pi: decode time of each and its posteriors
                         and log-likelihoods vs the oracle on seeded
                         recipients
    python study.py c4var  the gradient workload (N = 2,000, L = 50,000) with a
                         scalar mu, a per-variant mu (log-uniform within a
                         decade of the workload's mu) and a skewed prior
                         matrix: time per gradient in FP32 and FP64, and the
                         gradient vs the oracle score on seeded recipients
    python study.py emu  (CPU only) numpy emulation of the FP32 forward sweep
                         against the same recursion in FP64, with the column
                         sum taken in the kernel's order, with Kahan lane sums
                         and an FP64 tree, or exactly rounded; the emissions
                         plain or divided by 1-mu; c = A/S rounded to nearest
                         or through a reciprocal with a one-sided 1-ulp error.
                         Reports the log-likelihood error and the error of the
                         renormalised vectors for each variant.

Inputs are the seeded synthetic workloads of `lsinputs`; the oracle runs on
the host's cores.
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

VALU_PEAK = 256 * 4 * 32 * 2.4e9      # FP32 lane-operations/s (157.3 TFLOP/s / 2)
VALU_PEAK_F64 = 256 * 4 * 16 * 2.4e9  # FP64 lane-operations/s (78.6 TFLOP/s / 2)
HBM_PEAK = 8.0e12                     # bytes/s


def log(msg):
    print(f"[study] {msg}", file=sys.stderr, flush=True)


def events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _chunks(rec, size):
    for lo in range(0, len(rec), size):
        yield rec[lo:lo + size]


def _oracle_pass(oracle, x, rec, targets, want, label, chunk=64):
    """The oracle's pass over `rec` in chunks, with a progress line each."""
    parts = []
    t0 = time.perf_counter()
    for sub in _chunks(rec, chunk):
        parts.append(oracle.run_pass(x["H"], x["N"], x["L"], x["rho"], x["mu"], sub, targets,
                                     want=want))
        done = sum(len(p["llf"]) for p in parts)
        log(f"{label} oracle: {done}/{len(rec)} recipients ({time.perf_counter() - t0:.0f} s)")
    out = {k: np.concatenate([p[k] for p in parts], axis=1 if parts[0][k].ndim >= 2 else 0)
           for k in parts[0]}
    return out, time.perf_counter() - t0


def study_c4(args):
    import torch

    import oracle
    import paper_2212_11403_amd as ls
    from lsinputs import make_inputs, seeded_recipients

    x = make_inputs("c4")
    N, L, rho, mu = x["N"], x["L"], x["rho"], x["mu"]
    model = ls.Model(x["H"], N, rho, mu)
    out = {"study": "c4 gradient", "N": N, "L": L, "recipients": N}
    res = {}
    for prec in ("fp32", "fp64"):
        ls.loglik_grad(model, None, prec, grad=True)  # warm-up
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record()
        g = ls.loglik_grad(model, None, prec, grad=True)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        e0.record()
        ls.loglik_grad(model, None, prec, grad=False)
        e1.record()
        torch.cuda.synchronize()
        ms_ll = e0.elapsed_time(e1)
        res[prec] = g
        cells = float(N) * N * L
        seg = int(np.ceil(np.sqrt(L)))
        esz = 4 if prec == "fp32" else 8
        # forward with checkpoints (4 ops/cell), per segment a forward
        # recompute (4) and the adjoint pass (8: select, fma, mul, add for
        # the backward vector; fma, add, select, fma for d, Sa and M; plus
        # fma and mul on the half of the variants whose alpha it derives)
        ops = 17.0 * cells
        # alpha at every second variant written by the recompute and read by
        # the adjoint, plus checkpoints written once and read once
        hbm = 1.0 * cells * esz + 2.0 * (L / seg) * N * N * esz
        peak = VALU_PEAK if prec == "fp32" else VALU_PEAK_F64
        out[prec] = {"gradient_ms": ms, "loglik_only_ms": ms_ll,
                     "cells_per_s": cells / (ms / 1e3),
                     "valu_frac": ops / (ms / 1e3) / peak,
                     "hbm_frac": hbm / (ms / 1e3) / HBM_PEAK,
                     "pac": float(g["pac"].item())}
        log(f"{prec}: gradient {ms:.1f} ms, log-likelihood only {ms_ll:.1f} ms")
    # the recombination map (eq. rho) and its chain rule to (s, gamma) over
    # the L - 1 intervals: map distances that give this rho at s = gamma = 1
    cM = torch.tensor(-100.0 * np.log1p(-rho), dtype=torch.float64, device="cuda")
    gr_dev = res["fp32"]["grad_rho"].contiguous()
    ls.calc_rho(cM, 1.0, 1.0)
    ls.rho_map_grad(cM, 1.0, 1.0, gr_dev)
    torch.cuda.synchronize()
    e0, e1 = events()
    e0.record()
    for _ in range(10):
        ls.calc_rho(cM, 1.3, 0.9)
        ls.rho_map_grad(cM, 1.3, 0.9, gr_dev)
    e1.record()
    torch.cuda.synchronize()
    out["rho_map_and_chain_rule_ms"] = e0.elapsed_time(e1) / 10
    g32, g64 = res["fp32"], res["fp64"]
    gr32 = g32["grad_rho"].cpu().numpy()
    gr64 = g64["grad_rho"].cpu().numpy()
    out["fp32_vs_fp64_grad_rho_normwise"] = float(np.abs(gr32 - gr64).max() / np.abs(gr64).max())
    out["fp32_vs_fp64_grad_mu_rel"] = float(abs(g32["grad_mu"].item() - g64["grad_mu"].item())
                                           / abs(g64["grad_mu"].item()))
    # the oracle's exact score over the recipients (all of them by default),
    # summed chunk by chunk (it holds an L x N FP64 table per thread)
    rec = (np.arange(N, dtype=np.int32) if args.recipients >= N
           else seeded_recipients(N, args.recipients, seed=404))
    t0 = time.perf_counter()
    ll_ref, rg, gm_ref, done = 0.0, np.zeros(L - 1), 0.0, 0
    for sub in _chunks(rec, 250):
        ref = oracle.run_gradient(x["H"], N, L, rho, mu, sub)
        ll_ref += ref["loglik"].sum()
        rg += ref["grad_rho"].sum(axis=0)
        gm_ref += ref["grad_mu"].sum()
        done += len(sub)
        log(f"c4 oracle: {done}/{len(rec)} recipients ({time.perf_counter() - t0:.0f} s)")
    dt = time.perf_counter() - t0
    gsub = ls.loglik_grad(model, rec, "fp32", grad=True)
    gsub64 = ls.loglik_grad(model, rec, "fp64", grad=True)
    for name, gg in (("fp32", gsub), ("fp64", gsub64)):
        out[f"{name}_vs_oracle_grad_rho_normwise"] = float(
            np.abs(gg["grad_rho"].cpu().numpy() - rg).max() / np.abs(rg).max())
        out[f"{name}_vs_oracle_grad_mu_rel"] = float(abs(gg["grad_mu"].item() - gm_ref)
                                                     / abs(gm_ref))
        out[f"{name}_vs_oracle_pac_rel"] = float(abs(gg["pac"].item() - ll_ref) / abs(ll_ref))
    out["oracle_recipients"] = len(rec)
    out["oracle_seconds"] = dt
    # central differences of the FP64 GPU PAC (all recipients), h = 1e-6 rho_l
    rng = np.random.default_rng(7)
    picks = rng.choice(np.nonzero(rho >= 1e-4)[0], args.fd, replace=False)
    worst = 0.0
    gmax = np.abs(gr32).max()
    for l in picks:
        h = 1e-6 * rho[l]
        rp, rm = rho.copy(), rho.copy()
        rp[l] += h
        rm[l] -= h
        fp = ls.loglik_grad(ls.Model(x["H"], N, rp, mu), None, "fp64", grad=False)["pac"].item()
        fm = ls.loglik_grad(ls.Model(x["H"], N, rm, mu), None, "fp64", grad=False)["pac"].item()
        fd = (fp - fm) / (2 * h)
        worst = max(worst, abs(fd - gr32[l]) / gmax)
    out["fp32_vs_fd_normwise_max"] = worst
    out["fd_components"] = int(len(picks))
    print(json.dumps(out), flush=True)


def _decode_errors(ls, model, x, rec, targets, prec, ref):
    r = ls.decode(model, targets, prec, recipients=rec, want=("P", "E"))
    P = r["P"].double().cpu().numpy()
    E = r["E"].double().cpu().numpy()
    ll = r["fwd"].log_scale.cpu().numpy()
    both = (ref["P"] >= 1e-4)
    return {"max_abs_posterior_err": float(np.abs(P - ref["P"]).max()),
            "max_rel_loglik_err": float(np.max(np.abs(ll - ref["llf"]) / np.abs(ref["llf"]))),
            "max_abs_half_distance_err_p_ge_1e-4": float(np.abs(E - ref["E"])[both].max()),
            "nonfinite": int(ls.status_check(r["fwd"]))}


def study_c3(args):
    import torch

    import oracle
    import paper_2212_11403_amd as ls
    from lsinputs import make_inputs, seeded_recipients

    x = make_inputs("c3")
    N, L, targets = x["N"], x["L"], x["targets"]
    model = ls.Model(x["H"], N, x["rho"], x["mu"])
    rec = seeded_recipients(N, args.recipients, seed=3)
    ref, dt = _oracle_pass(oracle, x, rec, targets, ("P", "E"), "c3")
    out = {"study": "c3 precision", "N": N, "L": L, "targets": len(targets),
           "oracle_recipients": len(rec), "oracle_seconds": dt}
    for prec in ("fp32", "f16"):
        out[prec] = _decode_errors(ls, model, x, rec, targets, prec, ref)
        out[prec]["shape"] = list(ls.kernel_shape(N, prec))
        # decode of all recipients (posteriors not kept: the forward stages
        # alpha into E and writes half distances), in windows that fit HBM
        win = args.window
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for lo in range(0, N, win):
            sub = np.arange(lo, min(N, lo + win), dtype=np.int32)
            ls.decode(model, targets, prec, recipients=sub, want=("E",))
        torch.cuda.synchronize()
        sec = time.perf_counter() - t1
        out[prec]["decode_all_seconds"] = sec
        out[prec]["cells_per_s"] = float(N) * N * L / sec
        log(f"{prec}: {out[prec]}")
    print(json.dumps(out), flush=True)


def study_c5(args):
    import torch

    import oracle
    import paper_2212_11403_amd as ls
    from lsinputs import make_inputs, seeded_recipients

    x = make_inputs("c5")
    N, L, targets = x["N"], x["L"], x["targets"]
    T = len(targets)
    model = ls.Model(x["H"], N, x["rho"], x["mu"])
    share = np.arange(0, N // 8, dtype=np.int32)
    R = len(share)
    out = {"study": "c5 one-GPU share", "N": N, "L": L, "targets": T, "recipients": R,
           "shape": list(ls.kernel_shape(N, "fp32"))}
    fwd = ls.Table(model, 0, "fp32", share)
    bck = ls.Table(model, 1, "fp32", share)
    bsnap = torch.empty((T, R, N), dtype=torch.float32, device="cuda")
    E = torch.empty((T, R, N), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    ls.backward(bck, model, 0, targets, bsnap)
    ev[1].record(stream)
    ls.forward(fwd, model, L - 1, targets, bsnap, None, E)
    ev[2].record(stream)
    torch.cuda.synchronize()
    bwd_ms, fwd_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    cells = float(R) * N * L
    out["backward_ms"] = bwd_ms
    out["forward_and_posterior_ms"] = fwd_ms
    out["cells_per_s"] = cells / ((bwd_ms + fwd_ms) / 1e3)
    out["backward_valu_frac"] = 4 * cells / (bwd_ms / 1e3) / VALU_PEAK
    # a forward sweep without targets: the difference is the staging of
    # alpha at the targets and the posterior/half-distance rows (alpha and
    # beta read twice each, E written once: 20 B per entry)
    fwd2 = ls.Table(model, 0, "fp32", share)
    ev[0].record(stream)
    ls.forward(fwd2, model, L - 1)
    ev[1].record(stream)
    torch.cuda.synchronize()
    plain_ms = ev[0].elapsed_time(ev[1])
    out["forward_without_targets_ms"] = plain_ms
    out["target_outputs_ms"] = fwd_ms - plain_ms
    out["target_outputs_GBps"] = 20.0 * T * R * N / ((fwd_ms - plain_ms) / 1e3) / 1e9
    status = ls.status_check(fwd)
    out["nonfinite"] = int(status)
    rec = seeded_recipients(R, args.recipients, seed=5)
    ref, out["oracle_seconds"] = _oracle_pass(oracle, x, rec, targets, ("P",), "c5", chunk=32)
    out["oracle_recipients"] = len(rec)
    r = ls.decode(model, targets, "fp32", recipients=rec, want=("P",))
    out["max_abs_posterior_err_vs_oracle"] = float(
        np.abs(r["P"].double().cpu().numpy() - ref["P"]).max())
    print(json.dumps(out), flush=True)


def study_c2(args):
    import torch

    import paper_2212_11403_amd as ls
    from lsinputs import make_inputs

    x = make_inputs("c2")
    N, L, targets = x["N"], x["L"], x["targets"]
    model = ls.Model(x["H"], N, x["rho"], x["mu"])
    eps = 2.0 ** -52
    floor_half = -0.5 * np.log(eps)
    worst_p = worst_d = 0.0
    floor_diff = 0
    considered = 0
    win = args.targets_per_window
    t0 = time.perf_counter()
    for lo in range(0, len(targets), win):
        tw = targets[lo:lo + win]
        r64 = ls.decode(model, tw, "fp64", want=("P",))
        P64 = r64["P"]
        del r64
        r32 = ls.decode(model, tw, "fp32", want=("P",))
        P32 = r32["P"]
        del r32
        for k in range(len(tw)):
            a = P64[k]
            b = P32[k].double()
            worst_p = max(worst_p, float((a - b).abs().max().item()))
            # distances d_ji = -(log max(p_ji, eps) + log max(p_ij, eps)) / 2
            ea = -0.5 * torch.log(torch.clamp(a, min=eps))
            eb = -0.5 * torch.log(torch.clamp(b, min=eps))
            da = ea + ea.T
            db = eb + eb.T
            keep = (a >= 1e-4) & (a.T >= 1e-4)
            if bool(keep.any()):
                worst_d = max(worst_d, float((da - db).abs()[keep].max().item()))
            considered += int(keep.sum().item())
            fa = (a < eps)
            fb = (b < eps)
            floor_diff += int((fa != fb).sum().item())
            del a, b, ea, eb, da, db, keep, fa, fb
        del P64, P32
        torch.cuda.empty_cache()
        log(f"targets {lo}..{lo + len(tw) - 1}: worst posterior error so far {worst_p:.3e}")
    out = {"study": "c2 fp32 vs fp64, all recipients", "N": N, "L": L, "targets": len(targets),
           "max_abs_posterior_err": worst_p,
           "max_abs_distance_err_where_both_p_ge_1e-4": worst_d,
           "distance_entries_compared": considered,
           "eps_floor_decisions_differing": floor_diff,
           "half_distance_floor": floor_half,
           "seconds": time.perf_counter() - t0}
    if args.recipients:
        # both GPU paths against the oracle on seeded recipients, all targets
        import oracle
        from lsinputs import seeded_recipients
        rec = seeded_recipients(N, args.recipients, seed=2212)
        ref, dt = _oracle_pass(oracle, x, rec, targets, ("P",), "c2", chunk=32)
        out["oracle_recipients"] = len(rec)
        out["oracle_seconds"] = dt
        for prec in ("fp64", "fp32"):
            r = ls.decode(model, targets, prec, recipients=rec, want=("P",))
            P = r["P"].double().cpu().numpy()
            ll = r["fwd"].log_scale.cpu().numpy()
            del r
            err = np.abs(P - ref["P"])
            out[f"{prec}_vs_oracle_max_abs_posterior_err"] = float(err.max())
            if prec == "fp64":
                out["fp64_vs_oracle_max_rel_posterior_err"] = float(
                    np.max(err / np.maximum(np.abs(ref["P"]), 1e-300)))
            out[f"{prec}_vs_oracle_max_rel_loglik_err"] = float(
                np.max(np.abs(ll - ref["llf"]) / np.abs(ref["llf"])))
            del P, err
            log(f"c2 {prec} vs oracle: {out[f'{prec}_vs_oracle_max_abs_posterior_err']:.3e}")
    print(json.dumps(out), flush=True)


class _Fp32Forward:
    """FP32 forward recursion of the copying model (eq. fwd0, fwd1) over R
    recipients, vectorised over donors, with the rounding of each operation
    made explicit so that the variants of the study differ in one place.

    The donor column of a recipient is laid out as the sweep kernel holds it:
    `nslot` slots per lane, 64 lanes per wave, `nwaves` waves (zero padded).
    """

    def __init__(self, h, rho, mu, rec, nslot, nwaves):
        self.h, self.rho, self.mu, self.rec = h, rho, mu, rec
        self.nslot, self.nwaves = nslot, nwaves
        L, N = h.shape
        assert 64 * nslot * nwaves >= N

    def colsum(self, v, how):
        f32 = np.float32
        if how == "exact":
            return v.astype(np.float64).sum(axis=1).astype(f32)
        R, N = v.shape
        P = 64 * self.nslot * self.nwaves
        x = np.zeros((R, P), f32)
        x[:, :N] = v
        x = x.reshape(R, self.nwaves, self.nslot, 64)
        if how == "kahan":
            acc = x[:, :, 0].copy()
            comp = np.zeros_like(acc)
            for s in range(1, self.nslot):
                y = (x[:, :, s] - comp).astype(f32)
                t = (acc + y).astype(f32)
                comp = ((t - acc).astype(f32) - y).astype(f32)
                acc = t
            lanes = acc.astype(np.float64) - comp.astype(np.float64)
            return lanes.sum(axis=(1, 2)).astype(f32)
        # kernel order: even and odd slots in two chains per lane, the chains
        # added, a pairwise tree over the 64 lanes, then the waves in order
        a0, a1 = x[:, :, 0].copy(), x[:, :, 1].copy()
        for s in range(2, self.nslot):
            if s & 1:
                a1 = (a1 + x[:, :, s]).astype(f32)
            else:
                a0 = (a0 + x[:, :, s]).astype(f32)
        t = (a0 + a1).astype(f32)
        while t.shape[-1] > 1:
            t = (t[..., 0::2] + t[..., 1::2]).astype(f32)
        t = t[..., 0]
        acc = t[:, 0].copy()
        for w in range(1, self.nwaves):
            acc = (acc + t[:, w]).astype(f32)
        return acc

    def run(self, prec, summation="kernel", emission="plain", recip="nearest", every=500):
        h, rho, mu, rec = self.h, self.rho, self.mu, self.rec
        L, N = h.shape
        R = len(rec)
        f64 = prec == "fp64"
        ft = np.float64 if f64 else np.float32
        keep = np.ones((R, N), ft)
        keep[np.arange(R), rec] = 0
        omu = (1.0 - 2.0 * mu) + mu
        if emission == "unit" and not f64:
            th_m, th_x, log_unit = np.float32(1.0), np.float32(mu / omu), np.log(omu)
        else:
            th_m, th_x, log_unit = ft(omu), ft(mu), 0.0
        ll = np.zeros(R)
        snaps = []
        v = None
        for l in range(L):
            same = h[l][None, :] == h[l][rec][:, None]
            th = np.where(same, th_m, th_x).astype(ft)
            if l == 0:
                v = (th * (keep * ft(1.0 / (N - 1)))).astype(ft)
            else:
                if f64:
                    S = v.sum(axis=1)
                    c = (1.0 - rho[l - 1]) / S
                    pre = c[:, None] * v + (rho[l - 1] / (N - 1)) * keep
                else:
                    S = self.colsum(v, summation)
                    A = np.float32(1.0 - rho[l - 1])
                    if recip == "nearest":
                        c = (A / S).astype(np.float32)
                    else:
                        exact = 1.0 / S.astype(np.float64)
                        r = exact.astype(np.float32)
                        toward = np.float32(0.0) if recip == "low" else np.float32(np.inf)
                        off = (r.astype(np.float64) > exact) if recip == "low" else \
                              (r.astype(np.float64) < exact)
                        r = np.where(off, np.nextafter(r, toward), r)
                        c = (A * r).astype(np.float32)
                    b = np.float32(rho[l - 1] / (N - 1))
                    # c v + b with one rounding (a fused multiply-add)
                    pre = (c[:, None].astype(np.float64) * v + float(b) * keep).astype(np.float32)
                ll += np.log(np.asarray(S, np.float64)) + log_unit
                v = (th * pre).astype(ft)
            if l % every == every - 1:
                w = v.astype(np.float64)
                snaps.append(w / w.sum(axis=1, keepdims=True))
        ll += np.log(v.astype(np.float64).sum(axis=1)) + log_unit
        return ll, snaps


def study_emu(args):
    from lsinputs.mosaic import MosaicSpec, mosaic_haplotypes, rho_from_spacings, spacings

    N, L, R = args.emu_n, args.emu_l, args.recipients
    spec = MosaicSpec(n_haps=N, n_variants=L, n_founders=200, switch=1e-3, flip=1e-4, seed=5)
    _, h = mosaic_haplotypes(spec, unpacked=True)
    rho = rho_from_spacings(spacings(L - 1, 1e-3, 7))
    mu = 1e-4
    rec = np.arange(R) * (N // R)
    nslot = 40
    nwaves = -(-N // (64 * nslot))
    em = _Fp32Forward(np.asarray(h, np.uint8), rho, mu, rec, nslot, nwaves)
    t0 = time.perf_counter()
    ll64, ref = em.run("fp64")
    variants = [
        ("kernel", "plain", "low"), ("kernel", "plain", "high"),
        ("kernel", "plain", "nearest"), ("kahan", "plain", "nearest"),
        ("exact", "plain", "nearest"), ("kernel", "unit", "nearest"),
        ("exact", "unit", "nearest"),
    ]
    rows = []
    for summation, emission, recip in variants:
        ll, snaps = em.run("fp32", summation, emission, recip)
        d = np.concatenate([np.abs(a - b).ravel() for a, b in zip(snaps, ref)])
        w = np.concatenate([b.ravel() for b in ref])
        big = w >= 1e-3
        lle = np.abs(ll - ll64) / np.abs(ll64)
        rows.append({"sum": summation, "emission": emission, "reciprocal": recip,
                     "loglik_rel_err_max": float(lle.max()),
                     "loglik_rel_err_mean": float(lle.mean()),
                     "vector_max_abs_err": float(d.max()),
                     "vector_rel_rms_err_where_ge_1e-3": float(np.sqrt(np.mean((d[big] / w[big]) ** 2)))})
        log(f"{summation}/{emission}/{recip}: loglik {lle.mean():.2e} (mean rel), "
            f"vector rel-rms {rows[-1]['vector_rel_rms_err_where_ge_1e-3']:.2e}")
    out = {"study": "FP32 forward sweep emulation", "N": N, "L": L, "recipients": R,
           "layout": f"{nslot} slots x 64 lanes x {nwaves} waves", "mean_loglik": float(ll64.mean()),
           "variants": rows, "seconds": time.perf_counter() - t0}
    print(json.dumps(out), flush=True)


def study_c2var(args):
    import torch

    import oracle
    import paper_2212_11403_amd as ls
    from lsinputs import make_inputs, seeded_recipients

    x = make_inputs("c2")
    N, L, targets = x["N"], x["L"], x["targets"]
    rng = np.random.default_rng(2212)
    mu_vec = x["mu"] * 10.0 ** rng.uniform(-1.0, 1.0, L)
    W = rng.random((N, N)) ** 3
    np.fill_diagonal(W, 0.0)
    Pi = W / W.sum(axis=0, keepdims=True)
    del W
    rec = seeded_recipients(N, args.recipients, seed=22)
    out = {"study": "c2 variants (FP32 decode)", "N": N, "L": L, "targets": len(targets),
           "oracle_recipients": len(rec)}
    variants = [("scalar_mu", x["mu"], None), ("vector_mu", mu_vec, None),
                ("prior_matrix", x["mu"], Pi)]
    for name, mu, prior in variants:
        model = ls.Model(x["H"], N, x["rho"], mu, prior=prior)
        ls.decode(model, targets[:1], "fp32", want=("E",))  # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = ls.decode(model, targets, "fp32", want=("E",))
        torch.cuda.synchronize()
        sec = time.perf_counter() - t1
        del r
        res = {"decode_seconds": sec, "cells_per_s": float(N) * N * L / sec}
        t0 = time.perf_counter()
        ref = oracle.run_pass(x["H"], N, L, x["rho"], mu, rec, targets, want=("P",), prior=prior)
        res["oracle_seconds"] = time.perf_counter() - t0
        g = ls.decode(model, targets, "fp32", recipients=rec, want=("P",))
        res["max_posterior_err_vs_oracle"] = float(np.abs(g["P"].double().cpu().numpy()
                                                          - ref["P"]).max())
        ll = g["fwd"].log_scale.cpu().numpy()
        res["max_rel_loglik_err_vs_oracle"] = float(np.max(np.abs(ll - ref["llf"])
                                                           / np.abs(ref["llf"])))
        out[name] = res
        log(f"{name}: {res}")
        del model, g
        torch.cuda.empty_cache()
    out["vector_mu_time_ratio"] = out["vector_mu"]["decode_seconds"] / out["scalar_mu"]["decode_seconds"]
    out["prior_time_ratio"] = out["prior_matrix"]["decode_seconds"] / out["scalar_mu"]["decode_seconds"]
    print(json.dumps(out), flush=True)


def study_c4var(args):
    import torch

    import oracle
    import paper_2212_11403_amd as ls
    from lsinputs import make_inputs, seeded_recipients

    x = make_inputs("c4")
    N, L = x["N"], x["L"]
    rng = np.random.default_rng(4)
    mu_vec = x["mu"] * 10.0 ** rng.uniform(-1.0, 1.0, L)
    W = rng.random((N, N)) ** 3
    np.fill_diagonal(W, 0.0)
    Pi = W / W.sum(axis=0, keepdims=True)
    rec = seeded_recipients(N, args.recipients, seed=44)
    out = {"study": "c4 gradient with a per-variant mu and with a prior matrix", "N": N, "L": L,
           "oracle_recipients": len(rec)}
    for name, mu, prior in (("scalar_mu", x["mu"], None), ("vector_mu", mu_vec, None),
                            ("prior_matrix", x["mu"], Pi)):
        model = ls.Model(x["H"], N, x["rho"], mu, prior=prior)
        t0 = time.perf_counter()
        ref = oracle.run_gradient(x["H"], N, L, x["rho"], mu, rec, prior=prior)
        res = {"oracle_seconds": time.perf_counter() - t0}
        for prec in ("fp32", "fp64"):
            ls.loglik_grad(model, None, prec, grad=True)  # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                ls.loglik_grad(model, None, prec, grad=True)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t1) / reps * 1e3
            g = ls.loglik_grad(model, rec, prec, grad=True)
            gr = g["grad_rho"].cpu().numpy()
            rr = ref["grad_rho"].sum(axis=0)
            gm = g["grad_mu"].cpu().numpy()
            rm = ref["grad_mu_l"].sum(axis=0) if "grad_mu_l" in ref else ref["grad_mu"].sum()
            res[prec] = {"ms_per_gradient": ms,
                         "rho_err_normwise": float(np.abs(gr - rr).max() / np.abs(rr).max()),
                         "mu_err_normwise": float(np.max(np.abs(gm - rm)) / np.max(np.abs(rm))),
                         "pac_rel_err": float(abs(g["pac"].item() - ref["loglik"].sum())
                                              / abs(ref["loglik"].sum()))}
        out[name] = res
        log(f"{name}: {res}")
    out["vector_mu_time_ratio_fp32"] = (out["vector_mu"]["fp32"]["ms_per_gradient"]
                                        / out["scalar_mu"]["fp32"]["ms_per_gradient"])
    out["vector_mu_time_ratio_fp64"] = (out["vector_mu"]["fp64"]["ms_per_gradient"]
                                        / out["scalar_mu"]["fp64"]["ms_per_gradient"])
    for prec in ("fp32", "fp64"):
        out[f"prior_time_ratio_{prec}"] = (out["prior_matrix"][prec]["ms_per_gradient"]
                                           / out["scalar_mu"][prec]["ms_per_gradient"])
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c2", "c3", "c4", "c5", "c2var", "c4var", "emu"])
    ap.add_argument("--recipients", type=int, default=None,
                    help="seeded recipients checked against the oracle")
    ap.add_argument("--fd", type=int, default=64, help="finite-difference components (c4)")
    ap.add_argument("--window", type=int, default=12_500, help="recipients per decode (c3)")
    ap.add_argument("--targets-per-window", type=int, default=20, help="targets per decode (c2)")
    ap.add_argument("--emu-n", type=int, default=5000, help="haplotypes (emu)")
    ap.add_argument("--emu-l", type=int, default=10_000, help="variants (emu)")
    args = ap.parse_args()
    if args.which == "emu":
        args.recipients = args.recipients or 32
        study_emu(args)
        return
    import paper_2212_11403_amd as ls
    ls.load()
    # default oracle samples: c2 and c3 256 seeded recipients, c4 all of
    # them, c5 64 of the GPU's share
    if args.which == "c2":
        args.recipients = 256 if args.recipients is None else args.recipients
        study_c2(args)
    elif args.which == "c4":
        args.recipients = args.recipients or 2000
        study_c4(args)
    elif args.which == "c4var":
        args.recipients = args.recipients or 32
        study_c4var(args)
    elif args.which == "c2var":
        args.recipients = args.recipients or 16
        study_c2var(args)
    elif args.which == "c3":
        args.recipients = args.recipients or 256
        study_c3(args)
    else:
        args.recipients = args.recipients or 64
        study_c5(args)


if __name__ == "__main__":
    main()
