"""Helpers for the GPU tests: device availability and tolerances."""

from __future__ import annotations

import os

import numpy as np
import pytest

# FP64 path vs the FP64 oracle: relative 1e-12 per entry (plus a floor far
# below any value the recursions produce). Quantities in the log domain
# (half distances, log scales) carry the relative error of the probability
# they come from as an absolute error, so they get an absolute 1e-12 floor.
F64_RTOL = 1e-12
F64_ATOL_PROB = 1e-300
F64_ATOL_LOG = 1e-12


def f64_rtol(N):
    """FP64 tolerance for N donors: the oracle adds each column sum (and
    each posterior normaliser) one donor after another, so its relative
    error is bounded by (N - 1) u (u = 2^-53), which every normalised entry
    inherits; the path's own per-step rounding (a few u per entry) stays
    below 1e-12 at the sizes tested. The larger of the two; it exceeds
    1e-12 from N = 9,008 up (5.6e-12 at N = 50,000)."""
    return max(F64_RTOL, (N - 1) * 2.0 ** -53)
# FP32 sweep: max abs posterior error.
F32_POST_ATOL = 1e-5
# FP32 sweep: relative error of a log-likelihood (FP64 sum of log column
# sums). With c = A/S rounded to nearest and the match emission exactly 1,
# the per-step errors have no common sign and the observed error is 1e-7 to
# 3e-7 at L = 10,000 to 100,000; a biased reciprocal or a rounded 1-mu gives
# 2e-6 to 6e-6 there.
F32_LOGLIK_RTOL = 1e-6
# FP16-stored vectors (rounded to half, unit roundoff u = 2^-11, after
# every update): an entry's relative error settles near u / sqrt(rho) per
# the renormalised recursion, a few 1e-3 to 1e-2 at the workloads' rho;
# the bound on posteriors is set from the arithmetic, the measured
# maximum is printed by each test. The log-likelihood adds the log of each
# step's column sum of rounded entries: a relative error of at most u per
# step (all of the mass on one donor), with no common sign, so a random
# walk of standard deviation up to u sqrt(L / 3), about 0.01 at L = 2,000
# (an emulation of the half-stored forward on the CPU gives the same
# figures). Against |log P|, which grows like L, that is 1e-4 to 4e-4 on
# the test workloads (L = 12 to 20,000); the bound leaves room for the
# shortest sequences, where |log P| is smallest.
F16_POST_ATOL = 5e-2
F16_LOGLIK_RTOL = 1e-3


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_close(got, ref, rtol, atol):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    nan_g, nan_r = np.isnan(got), np.isnan(ref)
    assert np.array_equal(nan_g, nan_r), "NaN pattern differs"
    ok = ~nan_r
    err = np.abs(got[ok] - ref[ok])
    lim = rtol * np.abs(ref[ok]) + atol
    bad = err > lim
    if bad.any():
        idx = np.argmax(err - lim)
        raise AssertionError(f"{bad.sum()} entries out of tolerance; worst got={got[ok][idx]!r} "
                             f"ref={ref[ok][idx]!r} err={err[idx]:.3e} lim={lim[idx]:.3e}")


class forced_shape:
    """Context manager: make the library use a given (slots, waves) shape."""

    def __init__(self, nslot, nwaves):
        self.v = f"{nslot},{nwaves}"

    def __enter__(self):
        self.old = os.environ.get("LS_FORCE_SHAPE")
        os.environ["LS_FORCE_SHAPE"] = self.v

    def __exit__(self, *a):
        if self.old is None:
            os.environ.pop("LS_FORCE_SHAPE", None)
        else:
            os.environ["LS_FORCE_SHAPE"] = self.old


def check_reduced(prec, got, ref, what):
    """FP32 or FP16-stored results against the FP64 oracle: posteriors by
    the max absolute error, log-likelihoods by the max relative error."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if what == "log":
        err = np.max(np.abs(got - ref) / np.abs(ref))
        lim = F16_LOGLIK_RTOL if prec == "f16" else F32_LOGLIK_RTOL
    else:
        err = np.abs(got - ref).max()
        lim = F16_POST_ATOL if prec == "f16" else F32_POST_ATOL
    print(f"{prec} {what}: max error {err:.3e} (bound {lim:.0e})")
    assert err <= lim, (prec, what, err, lim)
    return err
