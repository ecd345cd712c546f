"""The zero-total rule of eq. postprob and the eps floor of eq. distmat on
the GPU, against the FP64 oracle, through the C ABI (libls.so).

The oracle's side of both is pinned in tests/test_oracle_pins.py (exact
enumeration); here the HIP path must reproduce it: p_ji = eps for every
donor of a recipient whose sum_j alpha_j beta_j is 0 at a target, half
distances -log(eps)/2 there, and floored half distances where the exact
posterior is below eps."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from lsinputs import pack_haplotypes

from _gpu import (F16_POST_ATOL, F32_POST_ATOL, F64_ATOL_LOG, F64_ATOL_PROB, F64_RTOL, need_gpu,
                  rel_close)
from _pins import EPS64, tiny_posterior_case, zero_sum_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    need_gpu()
    import paper_2212_11403_amd as m
    m.load()
    return m


def _np(t):
    return t.double().cpu().numpy()


def _check(prec, P, E, ref):
    if prec == "fp64":
        rel_close(P, ref["P"], F64_RTOL, F64_ATOL_PROB)
        rel_close(E, ref["E"], F64_RTOL, F64_ATOL_LOG)
    else:
        assert np.array_equal(np.isnan(P), np.isnan(ref["P"]))
        ok = ~np.isnan(ref["P"])
        post = F16_POST_ATOL if prec == "f16" else F32_POST_ATOL
        assert np.abs(P[ok] - ref["P"][ok]).max() <= post
        if prec == "fp32":
            rel_close(E, ref["E"], 1e-6, 1e-6)
        else:
            # half storage: E follows the posterior it comes from (0 on the
            # diagonal, where the oracle's is 0 too)
            want = np.where(ref["E"] == 0.0, 0.0, -0.5 * np.log(np.maximum(P, EPS64)))
            rel_close(E, want, 1e-5, 1e-6)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "f16"])
def test_zero_total_small(ls, prec):
    """The hand-built case of the oracle pin: mu = 0, rho_t = 0, supports of
    alpha^t and beta^t disjoint."""
    h, rho, mu, i, t = zero_sum_case()
    L, N = h.shape
    H = pack_haplotypes(h)
    rf = np.array([float(r) for r in rho])
    rec = np.array([i], np.int32)
    tg = np.array([t], np.int32)
    ref = oracle.run_pass(H, N, L, rf, float(mu), rec, tg, want=("P", "E"))
    m = ls.Model(H, N, rf, float(mu))
    r = ls.decode(m, tg, prec, recipients=rec, want=("P", "E"))
    P, E = _np(r["P"]), _np(r["E"])
    print(f"{prec}: P = {P[0, 0]}, E = {E[0, 0]}")
    donors = np.arange(N) != i
    assert np.all(P[0, 0, donors] == EPS64) and P[0, 0, i] == 0.0
    _check(prec, P, E, ref)
    # the sweeps run on past the target into a total underflow (appendix
    # A.3), which the status words report
    assert ls.status_check(r["fwd"]) == ls.LS_WARN_NONFINITE


@pytest.mark.parametrize("prec", ["fp64", "fp32", "f16"])
def test_zero_total_among_many(ls, prec):
    """N = 300 with a mutation probability per variant that is 0 at t and
    t+1 only, rho_t = 0, and recipient 0 the only haplotype carrying allele
    1 at both: every other haplotype mismatches it at t or at t+1, so its
    total is 0 at t while every other recipient has a positive total. All
    recipients against the oracle at t and at two other targets."""
    rng = np.random.default_rng(77)
    N, L, t = 300, 40, 20
    h = (rng.random((L, N)) < 0.4).astype(np.uint8)
    pat = rng.integers(0, 3, size=N)  # 0: (1,0), 1: (0,1), 2: (0,0) at (t, t+1)
    h[t] = (pat == 0)
    h[t + 1] = (pat == 1)
    h[t, 0] = h[t + 1, 0] = 1
    h[t, 1], h[t + 1, 1] = 1, 0
    h[t, 2], h[t + 1, 2] = 0, 1
    mu = np.full(L, 1e-3)
    mu[t] = mu[t + 1] = 0.0
    rho = rng.uniform(1e-3, 0.05, L - 1)
    rho[t] = 0.0
    H = pack_haplotypes(h)
    rec = np.arange(N, dtype=np.int32)
    tg = np.array([5, t, 33], np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, tg, want=("P", "E"))
    m = ls.Model(H, N, rho, mu)
    r = ls.decode(m, tg, prec, want=("P", "E"))
    P, E = _np(r["P"]), _np(r["E"])
    assert np.all(P[1, 0, 1:] == EPS64)
    assert np.all(ref["P"][1, 0, 1:] == EPS64)
    _check(prec, P, E, ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_eps_floor_on_tiny_posteriors(ls, prec):
    """Half distances where the posterior is below eps are -log(eps)/2 (the
    oracle pin's case with mu = 2^-40)."""
    h, rho, mu = tiny_posterior_case()
    L, N = h.shape
    H = pack_haplotypes(h)
    rf = np.array([float(r) for r in rho])
    rec = np.arange(N, dtype=np.int32)
    tg = np.arange(L, dtype=np.int32)
    ref = oracle.run_pass(H, N, L, rf, float(mu), rec, tg, want=("P", "E"))
    assert (ref["P"][ref["P"] > 0] < EPS64).sum() >= 4
    m = ls.Model(H, N, rf, float(mu))
    r = ls.decode(m, tg, prec, want=("P", "E"))
    P, E = _np(r["P"]), _np(r["E"])
    if prec == "fp64":
        _check(prec, P, E, ref)
    else:
        # FP32 posteriors near 2^-40 carry FP32's relative error; the floor
        # itself must match wherever the oracle's posterior is below eps
        # (entries within 1% of eps are left out: FP32 rounding of the
        # posterior could put them on either side; none is that close here)
        floored = (ref["P"] < 0.99 * EPS64) & (ref["P"] > 0)
        assert floored.sum() >= 8
        np.testing.assert_allclose(E[floored], 26.0 * np.log(2.0), rtol=1e-6)
        assert np.abs(P - ref["P"]).max() <= F32_POST_ATOL
