"""The larger workloads at full size, checked on seeded recipients.

The GPU runs the full N and L with the kernel shape the benchmark uses (the
shape depends only on N and the precision); the oracle computes the sampled
recipients one by one."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from lsinputs import make_inputs, seeded_recipients

from _gpu import (F32_LOGLIK_RTOL, F32_POST_ATOL, F64_ATOL_LOG, F64_ATOL_PROB,
                  check_reduced, f64_rtol, need_gpu, rel_close)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    need_gpu()
    import paper_2212_11403_amd as m
    m.load()
    return m


def _np(t):
    return t.double().cpu().numpy()


def _check(ls, name, precs, nrec, seed):
    x = make_inputs(name)
    N, L = x["N"], x["L"]
    rec = seeded_recipients(N, nrec, seed)
    targets = x["targets"]
    ref = oracle.run_pass(x["H"], N, L, x["rho"], x["mu"], rec, targets, want=("P", "E"))
    m = ls.Model(x["H"], N, x["rho"], x["mu"])
    errs = {}
    for prec in precs:
        r = ls.decode(m, targets, prec, recipients=rec, want=("P", "E"))
        P, E = _np(r["P"]), _np(r["E"])
        ll = _np(r["fwd"].log_scale)
        errs[prec] = (np.abs(P - ref["P"]).max(), np.max(np.abs(ll - ref["llf"]) / np.abs(ref["llf"])))
        print(f"{name} {prec} shape {ls.kernel_shape(N, prec)}: max abs posterior err "
              f"{errs[prec][0]:.3e}, max rel loglik err {errs[prec][1]:.3e}")
        if prec == "fp64":
            tol = f64_rtol(N)
            rel_close(P, ref["P"], tol, F64_ATOL_PROB)
            rel_close(E, ref["E"], tol, max(F64_ATOL_LOG, tol))
            rel_close(ll, ref["llf"], tol, F64_ATOL_LOG)
        else:
            check_reduced(prec, P, ref["P"], "prob")
            check_reduced(prec, ll, ref["llf"], "log")
    return errs


def test_c2_fp64_and_fp32_sampled(ls):
    """N = 10,000, L = 100,000, 100 targets."""
    _check(ls, "c2", ("fp64", "fp32"), 12, seed=2)


def test_c3_precision_study_sampled(ls):
    """N = 50,000, L = 20,000, rare-variant mosaic: FP64, FP32 and
    FP16-stored vectors (rounded to half at every variant) against the FP64
    oracle. FP64 runs 100-slot groups of 8 waves, two waves per SIMD."""
    assert ls.kernel_shape(50_000, "fp64") == (100, 8)
    _check(ls, "c3", ("fp64", "fp32", "f16"), 12, seed=3)


def test_c3_precision_study_256(ls):
    """The precision study at its stated sample: 256 seeded recipients of the
    N = 50,000 workload, posteriors at all 20 targets and log-likelihoods,
    FP64, FP32 and FP16-stored vectors against the FP64 oracle."""
    errs = _check(ls, "c3", ("fp64", "fp32", "f16"), 256, seed=256)
    print(f"c3, 256 recipients: FP64 {errs['fp64']}, FP32 {errs['fp32']}, "
          f"FP16-stored {errs['f16']}")


def test_c5_fp32_sampled(ls):
    """N = 100,000, L = 10,000, 5 targets."""
    _check(ls, "c5", ("fp32",), 8, seed=5)


def test_fp64_runs_are_bitwise_identical(ls):
    x = make_inputs("c1")
    m = ls.Model(x["H"], x["N"], x["rho"], x["mu"])
    a = ls.decode(m, x["targets"], "fp64", want=("P",))
    b = ls.decode(m, x["targets"], "fp64", want=("P",))
    assert np.array_equal(_np(a["P"]), _np(b["P"]))
    assert np.array_equal(_np(a["fwd"].log_scale), _np(b["fwd"].log_scale))
