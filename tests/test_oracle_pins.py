"""Pins for the FP64 oracle: each test checks it against something other than
itself -- exact enumeration, closed forms, invariants of the model, an
independent log-domain implementation, or values printed in the paper.
CPU only."""

from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from lsinputs import (evenly_spaced_targets, make_inputs, pack_haplotypes, packed_bytes,
                      rho_from_spacings, unpack_haplotypes)

from _pins import (EPS64, enumerate_exact, floor_checks, logdomain_fb, raw_forward,
                   rho0_closed_form, rho0_closed_form_grad, rho1_closed_form, rho_map_checks,
                   tiny_posterior_case, zero_sum_case)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")


def _rand_h(L, N, seed, p=0.5):
    rng = np.random.default_rng(seed)
    return (rng.random((L, N)) < p).astype(np.uint8)


def _run(h01, rho, mu, recips, targets, want=("A", "B", "P", "E", "logF", "logG")):
    L, N = h01.shape
    return oracle.run_pass(pack_haplotypes(h01), N, L, np.asarray(rho, float), mu, recips,
                           targets, want=want, nthreads=2)


# --------------------------------------------------------------------------
# exact enumeration over every copying path (exact rationals)

ENUM_CASES = [
    # (L, N, seed, mu, rho numerators over 32)
    (5, 4, 1, Fraction(1, 16), [3, 17, 1, 29]),
    (6, 5, 2, Fraction(3, 32), [5, 0, 31, 12, 32]),   # includes rho = 0 and rho = 1
    (4, 3, 3, Fraction(1, 4), [9, 2, 20]),
    (7, 3, 4, Fraction(1, 32), [1, 2, 3, 4, 5, 6]),
]


@pytest.mark.parametrize("L,N,seed,mu,rnum", ENUM_CASES)
def test_oracle_matches_exact_enumeration(L, N, seed, mu, rnum):
    h01 = _rand_h(L, N, seed)
    rho = [Fraction(k, 32) for k in rnum]
    recips = np.arange(N, dtype=np.int32)
    targets = np.arange(L, dtype=np.int32)
    res = _run(h01, [float(r) for r in rho], float(mu), recips, targets)
    grad = oracle.run_gradient(pack_haplotypes(h01), N, L, np.array([float(r) for r in rho]),
                               float(mu), recips, nthreads=2)
    for i in range(N):
        ex = enumerate_exact(h01.tolist(), rho, mu, i)
        logP = np.log(float(ex["P"]))
        assert abs(res["llf"][i] - logP) <= 1e-13 * abs(logP) + 1e-14
        assert abs(res["llb"][i] - logP) <= 1e-13 * abs(logP) + 1e-14
        assert abs(grad["loglik"][i] - logP) <= 1e-13 * abs(logP) + 1e-14
        post = np.array([[float(x) for x in row] for row in ex["post"]])
        got = res["P"][:, i, :]
        np.testing.assert_allclose(got, post, rtol=1e-12, atol=1e-15)
        assert np.all(got[:, i] == 0.0)
        dr = np.array([float(x) for x in ex["dlogP_drho"]])
        np.testing.assert_allclose(grad["grad_rho"][i], dr, rtol=1e-10, atol=1e-12)
        assert abs(grad["grad_mu"][i] - float(ex["dlogP_dmu"])) <= 1e-10 * abs(float(ex["dlogP_dmu"])) + 1e-10


@pytest.mark.parametrize("L,N,seed,mnum,rnum", [
    (5, 4, 6, [1, 3, 2, 8, 1], [3, 17, 1, 29]),
    (6, 3, 7, [4, 1, 1, 16, 2, 5], [5, 0, 31, 12, 32]),
])
def test_oracle_per_variant_mu_matches_enumeration(L, N, seed, mnum, rnum):
    """A mutation probability per variant (the paper's mu may be a vector of
    length L, section 3.4): posteriors and likelihoods by enumeration."""
    h01 = _rand_h(L, N, seed)
    rho = [Fraction(k, 32) for k in rnum]
    mu = [Fraction(k, 32) for k in mnum]
    res = _run(h01, [float(r) for r in rho], np.array([float(m) for m in mu]),
               np.arange(N, dtype=np.int32), np.arange(L, dtype=np.int32))
    for i in range(N):
        ex = enumerate_exact(h01.tolist(), rho, mu, i)
        logP = np.log(float(ex["P"]))
        assert abs(res["llf"][i] - logP) <= 1e-13 * abs(logP) + 1e-14
        assert abs(res["llb"][i] - logP) <= 1e-13 * abs(logP) + 1e-14
        post = np.array([[float(x) for x in row] for row in ex["post"]])
        np.testing.assert_allclose(res["P"][:, i, :], post, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("L,N,seed,mnum,rnum", [
    (5, 4, 6, [1, 3, 2, 8, 1], [3, 17, 1, 29]),
    (6, 3, 7, [4, 1, 1, 16, 2, 5], [5, 0, 31, 12, 32]),
    (4, 5, 8, [2, 20, 1, 5], [7, 2, 11]),
])
def test_oracle_per_variant_mu_gradient_matches_enumeration(L, N, seed, mnum, rnum):
    """d log P / d rho_l and d log P / d mu^l for every variant, by exact
    differentiation of the enumerated likelihood."""
    h01 = _rand_h(L, N, seed)
    rho = [Fraction(k, 32) for k in rnum]
    mu = [Fraction(k, 32) for k in mnum]
    g = oracle.run_gradient(pack_haplotypes(h01), N, L, np.array([float(r) for r in rho]),
                            np.array([float(m) for m in mu]), np.arange(N, dtype=np.int32))
    for i in range(N):
        ex = enumerate_exact(h01.tolist(), rho, mu, i)
        logP = np.log(float(ex["P"]))
        assert abs(g["loglik"][i] - logP) <= 1e-13 * abs(logP) + 1e-14
        dr = np.array([float(x) for x in ex["dlogP_drho"]])
        np.testing.assert_allclose(g["grad_rho"][i], dr, rtol=1e-10, atol=1e-12)
        dm = np.array([float(x) for x in ex["dlogP_dmu_l"]])
        np.testing.assert_allclose(g["grad_mu_l"][i], dm, rtol=1e-10, atol=1e-10)
        assert abs(g["grad_mu"][i] - dm.sum()) <= 1e-10 * np.abs(dm).sum() + 1e-10


def test_oracle_constant_mu_vector_gradient_equals_scalar():
    """A constant vector gives the scalar model's gradient bit for bit (the
    terms are added in the same order), and the per-variant terms add up to
    it."""
    L, N = 30, 8
    h01 = _rand_h(L, N, 14)
    rho = rho_from_spacings(np.random.default_rng(14).exponential(0.05, L - 1))
    rec = np.arange(N, dtype=np.int32)
    a = oracle.run_gradient(pack_haplotypes(h01), N, L, rho, 0.02, rec)
    b = oracle.run_gradient(pack_haplotypes(h01), N, L, rho, np.full(L, 0.02), rec)
    for k in ("loglik", "grad_rho", "grad_mu"):
        assert np.array_equal(a[k], b[k]), k
    np.testing.assert_allclose(b["grad_mu_l"].sum(axis=1), b["grad_mu"], rtol=1e-12)


def test_oracle_constant_mu_vector_equals_scalar():
    L, N = 40, 9
    h01 = _rand_h(L, N, 12)
    rho = rho_from_spacings(np.random.default_rng(12).exponential(0.05, L - 1))
    rec, tg = np.arange(N, dtype=np.int32), np.array([3, 20, 39], np.int32)
    a = _run(h01, rho, 0.03, rec, tg)
    b = _run(h01, rho, np.full(L, 0.03), rec, tg)
    for k in ("P", "E", "llf", "llb", "logF", "logG"):
        assert np.array_equal(a[k], b[k]), k


def test_distance_definition_on_enumerated_posteriors():
    """eq. distmat applied to exact posteriors equals the oracle's D."""
    L, N = 5, 4
    h01 = _rand_h(L, N, 9)
    mu = Fraction(1, 8)
    rho = [Fraction(k, 32) for k in (4, 9, 1, 30)]
    t = 2
    exact = np.zeros((N, N))
    for i in range(N):
        ex = enumerate_exact(h01.tolist(), rho, mu, i)
        exact[i] = [float(x) for x in ex["post"][t]]
    eps = 2.0 ** -52
    Dref = np.zeros((N, N))
    for a in range(N):
        for b in range(N):
            if a != b:
                Dref[a, b] = -(np.log(max(exact[a, b], eps)) + np.log(max(exact[b, a], eps))) / 2
    D = oracle.distances(pack_haplotypes(h01), N, L, np.array([float(r) for r in rho]),
                         float(mu), np.array([t], np.int32))[0]
    np.testing.assert_allclose(D, Dref, rtol=1e-12, atol=1e-14)
    assert np.all(np.diag(D) == 0.0)
    np.testing.assert_array_equal(D, D.T)


# --------------------------------------------------------------------------
# closed forms

def test_rho_zero_closed_form():
    L, N, mu = 60, 25, 0.02
    h01 = _rand_h(L, N, 5, p=0.3)
    rho = np.zeros(L - 1)
    recips = np.array([0, 7, 24], np.int32)
    targets = np.array([0, 31, L - 1], np.int32)
    res = _run(h01, rho, mu, recips, targets)
    grad = oracle.run_gradient(pack_haplotypes(h01), N, L, rho, mu, recips, nthreads=2)
    for r, i in enumerate(recips):
        logP, post = rho0_closed_form(h01, mu, i)
        assert abs(res["llf"][r] - logP) <= 1e-12 * abs(logP)
        assert abs(res["llb"][r] - logP) <= 1e-12 * abs(logP)
        for k in range(len(targets)):
            np.testing.assert_allclose(res["P"][k, r], post, rtol=1e-11, atol=1e-300)
        g0 = rho0_closed_form_grad(h01, mu, i)
        np.testing.assert_allclose(grad["grad_rho"][r], g0, rtol=1e-10, atol=1e-12)


def test_rho_one_closed_form():
    L, N, mu = 40, 17, 0.05
    h01 = _rand_h(L, N, 6)
    rho = np.ones(L - 1)
    recips = np.array([3, 16], np.int32)
    targets = np.arange(L, dtype=np.int32)
    res = _run(h01, rho, mu, recips, targets)
    for r, i in enumerate(recips):
        logP, post = rho1_closed_form(h01, mu, i)
        assert abs(res["llf"][r] - logP) <= 1e-12 * abs(logP)
        np.testing.assert_allclose(res["P"][:, r, :], post, rtol=1e-12, atol=1e-300)


def test_two_haplotypes_closed_form():
    L, mu = 300, 0.01
    h01 = _rand_h(L, 2, 7, p=0.5)
    rng = np.random.default_rng(8)
    rho = rng.random(L - 1)
    recips = np.array([0, 1], np.int32)
    res = _run(h01, rho, mu, recips, np.array([0, 150, L - 1], np.int32))
    grad = oracle.run_gradient(pack_haplotypes(h01), 2, L, rho, mu, recips, nthreads=2)
    m = int((h01[:, 0] != h01[:, 1]).sum())
    logP = m * np.log(mu) + (L - m) * np.log1p(-mu)
    for r in range(2):
        assert abs(res["llf"][r] - logP) <= 1e-12 * abs(logP)
        assert abs(res["llb"][r] - logP) <= 1e-12 * abs(logP)
        other = 1 - r
        assert np.all(res["P"][:, r, other] == 1.0)
        assert np.all(res["P"][:, r, r] == 0.0)
        assert np.all(grad["grad_rho"][r] == 0.0)
        assert abs(grad["grad_mu"][r] - (m / mu - (L - m) / (1 - mu))) <= 1e-9 * abs(m / mu)
    D = oracle.distances(pack_haplotypes(h01), 2, L, rho, mu, np.array([5], np.int32))[0]
    assert np.all(D == 0.0)


# --------------------------------------------------------------------------
# invariants at a realistic size (the small plain-FP64 workload)

@pytest.fixture(scope="module")
def c1():
    return make_inputs("c1", unpacked=True)


@pytest.fixture(scope="module")
def c1_all(c1):
    x = c1
    rec = np.arange(x["N"], dtype=np.int32)
    targets = np.arange(0, x["L"], 97, dtype=np.int32)
    res = oracle.run_pass(x["H"], x["N"], x["L"], x["rho"], x["mu"], rec, targets,
                          want=("A", "B", "P", "E", "logF", "logG"))
    return targets, res


def test_c1_posteriors_sum_to_one_and_loglik_agree(c1, c1_all):
    targets, res = c1_all
    s = res["P"].sum(axis=2)
    assert np.max(np.abs(s - 1.0)) < 1e-13
    assert np.all(res["P"] >= 0.0) and np.all(res["P"] <= 1.0)
    ll = res["llf"]
    assert np.max(np.abs(res["llb"] - ll) / np.abs(ll)) < 1e-13
    assert np.all(res["status"] == 0)


def test_c1_scale_invariance_at_every_target(c1, c1_all):
    """log sum_j alpha^l beta^l + log F^{l-1} + log G^l = log P for every l
    (from P = sum_j alpha~^l beta~^l and the definitions of F and G)."""
    targets, res = c1_all
    A, B = res["A"], res["B"]
    S = A.sum(axis=2)
    logFm1 = res["logF"] - np.log(S)
    lhs = np.log((A * B).sum(axis=2)) + logFm1 + res["logG"]
    rel = np.abs(lhs - res["llf"][None, :]) / np.abs(res["llf"][None, :])
    assert rel.max() < 1e-13


def test_c1_bounds(c1, c1_all):
    """alpha <= 1 and rho_l <= beta^l <= 1 + 1/min(pi) (appendix A.3)."""
    targets, res = c1_all
    x = c1
    assert res["A"].max() <= 1.0
    N = x["N"]
    B = res["B"]
    for k, t in enumerate(targets):
        if t < x["L"] - 1:
            off = ~np.eye(N, dtype=bool)
            assert B[k][off].min() >= x["rho"][t] * (1 - 1e-15)
    assert B.max() <= 1.0 + (N - 1)


def test_c1_distances_symmetric_and_bounded(c1, c1_all):
    targets, res = c1_all
    E = res["E"][0]
    D = oracle.symmetrise(E)
    np.testing.assert_array_equal(D, D.T)
    assert np.all(np.diag(D) == 0.0)
    assert D.min() >= 0.0 and D.max() <= -np.log(2.0 ** -52) + 1e-12


def test_c1_logdomain_cross_check(c1):
    x = c1
    h01 = x["h01"]
    for i in (0, 77, 199):
        logP, post = logdomain_fb(h01, x["rho"], x["mu"], i)
        targets = np.array([0, 500, 1999], np.int32)
        res = oracle.run_pass(x["H"], x["N"], x["L"], x["rho"], x["mu"], np.array([i], np.int32),
                              targets, want=("P",))
        assert abs(res["llf"][0] - logP) <= 1e-11 * abs(logP)
        np.testing.assert_allclose(res["P"][:, 0, :], post[targets], rtol=1e-9, atol=1e-15)


def test_raw_recursion_equals_scaled_times_F():
    """alpha~^l = F^{l-1} alpha^l (appendix A.1) while the raw form is finite."""
    L, N, mu = 30, 12, 0.01
    h01 = _rand_h(L, N, 12)
    rho = rho_from_spacings(np.random.default_rng(3).exponential(0.05, L - 1))
    raw = raw_forward(h01, rho, mu, 4)
    res = _run(h01, rho, mu, np.array([4], np.int32), np.arange(L, dtype=np.int32))
    A = res["A"][:, 0, :]
    logFm1 = res["logF"][:, 0] - np.log(A.sum(axis=1))
    np.testing.assert_allclose(A * np.exp(logFm1)[:, None], raw, rtol=1e-12, atol=0)


def test_oracle_gradient_matches_finite_differences(c1):
    x = c1
    N, L = 40, 400
    h01 = x["h01"][:L, :N]
    H = pack_haplotypes(h01)
    rho = x["rho"][: L - 1].copy()
    mu = x["mu"]
    rec = np.arange(N, dtype=np.int32)
    g = oracle.run_gradient(H, N, L, rho, mu, rec)
    G = g["grad_rho"].sum(axis=0)
    def pac(r, m):
        return oracle.run_pass(H, N, L, r, m, rec, want=())["llf"].sum()
    for l in (0, 17, 200, L - 2):
        h = 1e-6 * max(rho[l], 1e-3)
        rp, rm = rho.copy(), rho.copy()
        rp[l] += h
        rm[l] -= h
        fd = (pac(rp, mu) - pac(rm, mu)) / (2 * h)
        assert abs(fd - G[l]) <= 1e-5 * max(abs(G[l]), 1.0)
    h = 1e-7
    fd = (pac(rho, mu + h) - pac(rho, mu - h)) / (2 * h)
    assert abs(fd - g["grad_mu"].sum()) <= 1e-5 * abs(fd)


def test_total_underflow_gives_nan_columns_with_zero_diagonal():
    """mu = 0 and a variant where the recipient carries an allele no donor
    has: every emission is 0, the forward sum is 0 and the column becomes NaN
    (appendix A.3); the diagonal stays 0."""
    L, N = 8, 6
    h01 = _rand_h(L, N, 21)
    h01[3, :] = 0
    h01[3, 2] = 1
    rho = np.full(L - 1, 0.1)
    res = _run(h01, rho, 0.0, np.array([2, 4], np.int32), np.array([5], np.int32))
    assert res["status"][0] & 1
    P = res["P"][0, 0]
    assert P[2] == 0.0 and np.all(np.isnan(np.delete(P, 2)))
    assert np.isnan(res["llf"][0])
    # recipient 4 is unaffected apart from the same mismatch pattern at l = 3
    # (donor 2 mismatches, the others match), so its column stays finite
    assert res["status"][1] == 0 and np.all(np.isfinite(res["P"][0, 1]))


# --------------------------------------------------------------------------
# values printed in the paper

def test_paper_cache_size():
    g = json.load(open(GOLDEN))["cache_size"]
    assert packed_bytes(g["n_haps"], g["n_variants"]) == g["bytes"]


def test_paper_uniform_prior():
    g = json.load(open(GOLDEN))["uniform_prior"]
    # R prints 15 significant digits
    assert f"{1.0 / (g['n_haps'] - 1):.15g}" == g["printed"]


def test_paper_calc_rho_values():
    g = json.load(open(GOLDEN))["calc_rho"]
    for m, printed in g["pairs"]:
        got = rho_from_spacings(np.array([float(m)]))[0]
        # printed to 15 digits from a map difference that is itself rounded;
        # 1 - exp(-m) differs from m by m/2 relative (~1e-8), far above this
        assert abs(got - float(printed)) <= 1e-13 * float(printed)


def test_oracle_recombination_map():
    """The oracle's CalcRho (eq. rho) and its chain rule to (s, gamma)."""
    g = json.load(open(GOLDEN))["calc_rho"]
    assert rho_map_checks(oracle.calc_rho, oracle.rho_map_grad, g["pairs"])


def test_oracle_epsilon_matches_paper():
    g = json.load(open(GOLDEN))["epsilon"]
    assert abs(oracle.EPS - g["approx"]) < 5e-19
    assert EPS64 == 2.0 ** -52 and abs(EPS64 - g["approx"]) < 5e-19


def test_zero_total_posterior_rule():
    """eq. postprob, section 2.2: where sum_j alpha_j beta_j = 0 every donor
    gets p_ji = eps, and eq. distmat then gives -log(eps)/2 = 26 log 2. The
    case is built so that alpha^t and beta^t are finite and non-zero with
    disjoint supports (zero_sum_case); exact enumeration confirms that every
    copying path has probability 0."""
    h, rho, mu, i, t = zero_sum_case()
    L, N = h.shape
    ex = enumerate_exact(h.tolist(), rho, mu, i)
    assert ex["P"] == 0
    res = _run(h, [float(r) for r in rho], float(mu), np.array([i], np.int32),
               np.array([t], np.int32), want=("A", "B", "P", "E"))
    a, b = res["A"][0, 0], res["B"][0, 0]
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
    assert a.sum() > 0 and b.sum() > 0 and np.dot(a, b) == 0.0
    donors = np.arange(N) != i
    assert np.all(res["P"][0, 0, donors] == EPS64) and res["P"][0, 0, i] == 0.0
    np.testing.assert_allclose(res["E"][0, 0, donors], 26.0 * np.log(2.0), rtol=1e-15)
    assert res["E"][0, 0, i] == 0.0


def test_epsilon_floor_on_tiny_posteriors():
    """eq. distmat floors p at eps = 2^-52 before the log: against the exact
    posteriors of a case with entries below 2^-52 and between 2^-52 and
    2^-23, and with the zero-total case above (floor_checks)."""
    def run(h01, rho, mu, rec, tg):
        return _run(h01, rho, mu, rec, tg, want=("P", "E"))
    assert floor_checks(run)


def test_packing_round_trip_and_bit_order():
    h01 = _rand_h(13, 70, 30)
    W = pack_haplotypes(h01)
    assert W.shape == (13, 8)
    assert np.array_equal(unpack_haplotypes(W, 70), h01)
    l, j = 5, 37
    assert ((W[l, j // 32] >> (j % 32)) & 1) == h01[l, j]
    assert np.all(W[:, 3:] == 0)


def test_targets_are_evenly_spaced():
    t = evenly_spaced_targets(2000, 10)
    assert list(t) == [100, 300, 500, 700, 900, 1100, 1300, 1500, 1700, 1900]


# ---------------------------------------------------------------------------
# non-uniform prior copying matrix Pi (section 2.1; column i belongs to
# recipient i, Pi_ii = 0, columns sum to 1)

def _rand_prior(N, seed):
    """Rational left stochastic N x N matrix with a zero diagonal."""
    W = np.random.default_rng(seed).integers(1, 10, size=(N, N))
    Pi = [[Fraction(0)] * N for _ in range(N)]
    for i in range(N):
        tot = sum(int(W[j, i]) for j in range(N) if j != i)
        for j in range(N):
            if j != i:
                Pi[j][i] = Fraction(int(W[j, i]), tot)
    return Pi


@pytest.mark.parametrize("L,N,seed,mnum,rnum", [
    (5, 4, 21, 4, [3, 17, 1, 29]),
    (4, 5, 22, [2, 9, 1, 5], [7, 2, 11]),
    (6, 3, 23, 6, [5, 0, 31, 12, 32]),
])
def test_oracle_prior_matrix_matches_enumeration(L, N, seed, mnum, rnum):
    """Posteriors, both log-likelihoods and the gradient (rho, and mu as a
    scalar or per variant) under a random prior matrix, by enumeration."""
    h01 = _rand_h(L, N, seed)
    Pi = _rand_prior(N, seed)
    Pf = np.array([[float(x) for x in row] for row in Pi])
    rho = [Fraction(k, 32) for k in rnum]
    mu = [Fraction(k, 32) for k in mnum] if isinstance(mnum, list) else Fraction(mnum, 32)
    mu_arg = np.array([float(m) for m in mu]) if isinstance(mu, list) else float(mu)
    rf = np.array([float(r) for r in rho])
    H = pack_haplotypes(h01)
    rec = np.arange(N, dtype=np.int32)
    res = oracle.run_pass(H, N, L, rf, mu_arg, rec, np.arange(L, dtype=np.int32), want=("P",),
                          prior=Pf)
    g = oracle.run_gradient(H, N, L, rf, mu_arg, rec, prior=Pf)
    for i in range(N):
        ex = enumerate_exact(h01.tolist(), rho, mu, i, prior=Pi)
        logP = np.log(float(ex["P"]))
        for v in (res["llf"][i], res["llb"][i], g["loglik"][i]):
            assert abs(v - logP) <= 1e-13 * abs(logP) + 1e-14
        post = np.array([[float(x) for x in row] for row in ex["post"]])
        np.testing.assert_allclose(res["P"][:, i, :], post, rtol=1e-12, atol=1e-15)
        dr = np.array([float(x) for x in ex["dlogP_drho"]])
        np.testing.assert_allclose(g["grad_rho"][i], dr, rtol=1e-10, atol=1e-12)
        assert abs(g["grad_mu"][i] - float(ex["dlogP_dmu"])) <= 1e-10 * abs(float(ex["dlogP_dmu"])) + 1e-10
        if isinstance(mu, list):
            dm = np.array([float(x) for x in ex["dlogP_dmu_l"]])
            np.testing.assert_allclose(g["grad_mu_l"][i], dm, rtol=1e-10, atol=1e-10)


def test_oracle_uniform_prior_matrix_equals_default():
    L, N = 30, 9
    h01 = _rand_h(L, N, 31)
    rho = rho_from_spacings(np.random.default_rng(31).exponential(0.05, L - 1))
    Pf = np.full((N, N), 1.0 / (N - 1))
    np.fill_diagonal(Pf, 0.0)
    H, rec, tg = pack_haplotypes(h01), np.arange(N, dtype=np.int32), np.array([2, 17], np.int32)
    a = oracle.run_pass(H, N, L, rho, 0.02, rec, tg, want=("P", "B", "logF", "logG"))
    b = oracle.run_pass(H, N, L, rho, 0.02, rec, tg, want=("P", "B", "logF", "logG"), prior=Pf)
    for k in ("P", "B", "logF", "logG", "llf", "llb"):
        assert np.array_equal(a[k], b[k]), k
    ga = oracle.run_gradient(H, N, L, rho, 0.02, rec)
    gb = oracle.run_gradient(H, N, L, rho, 0.02, rec, prior=Pf)
    for k in ("loglik", "grad_rho", "grad_mu"):
        assert np.array_equal(ga[k], gb[k]), k


def test_oracle_prior_matrix_full_recombination_closed_form():
    """With rho = 1 between every pair of variants the copied donor is
    redrawn from the prior at each variant, independently: p^l_j =
    Pi_ji theta^l_j / sum_k Pi_ki theta^l_k and P = prod_l sum_k Pi_ki
    theta^l_k."""
    L, N, mu = 12, 40, 0.07
    rng = np.random.default_rng(41)
    h01 = (rng.random((L, N)) < 0.4).astype(np.uint8)
    W = rng.random((N, N)) ** 3
    np.fill_diagonal(W, 0.0)
    Pf = W / W.sum(axis=0, keepdims=True)
    rec = np.array([0, 5, 39], np.int32)
    res = oracle.run_pass(pack_haplotypes(h01), N, L, np.ones(L - 1), mu, rec,
                          np.arange(L, dtype=np.int32), want=("P",), prior=Pf)
    for r, i in enumerate(rec):
        ll = 0.0
        for l in range(L):
            th = np.where(h01[l] == h01[l, i], 1.0 - mu, mu)
            w = Pf[:, i] * th
            np.testing.assert_allclose(res["P"][l, r], w / w.sum(), rtol=1e-12, atol=1e-300)
            ll += np.log(w.sum())
        assert abs(res["llf"][r] - ll) <= 1e-12 * abs(ll)
        assert abs(res["llb"][r] - ll) <= 1e-12 * abs(ll)
