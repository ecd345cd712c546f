"""Independent references the oracle is pinned to.

Nothing here reuses the oracle's recursions. Each helper computes a quantity
from its mathematical definition in the paper (section 2.1: the LS HMM with
emission eq. emission, transition eq. transition, uniform prior with zero
self-copying):

* ``enumerate_exact`` sums over every hidden path in exact rational
  arithmetic, so the likelihood, posterior marginals and derivatives are exact.
* ``logdomain_fb`` is the textbook forward-backward over the full transition
  matrix with log-sum-exp, in FP64 (no scale factors at all).
* ``raw_forward`` is the unscaled recursion (eq. raw_forward), valid while it
  does not underflow.
* closed forms for rho = 0 (no recombination), rho = 1 (independent sites)
  and N = 2 (a single donor).
"""

from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def _theta_exact(h, l, j, i, mu):
    return mu if h[l][j] != h[l][i] else 1 - mu


def enumerate_exact(h, rho, mu, i, prior=None):
    """Exact P(h_i | h_-i), posterior marginals p[l][j] and the derivatives
    d log P / d rho_l (length L-1) and d log P / d mu, by summing over all
    (N-1)^L copying paths. ``h`` is an L x N nested list of 0/1; ``rho`` a list
    of L-1 Fractions; ``mu`` a Fraction, or a list of L Fractions (one per
    variant), in which case ``dlogP_dmu_l`` holds the derivative with respect
    to each. ``prior``: an N x N nested list of Fractions, prior[j][i] the
    prior probability that recipient i copies donor j (its diagonal is not
    used), or None for the uniform prior."""
    L, N = len(h), len(h[0])
    mus = list(mu) if isinstance(mu, (list, tuple)) else [mu] * L
    donors = [j for j in range(N) if j != i]
    pi_of = [Fraction(1, N - 1) if prior is None else prior[j][i] for j in range(N)]
    P = Fraction(0)
    marg = [[Fraction(0)] * N for _ in range(L)]
    dP_drho = [Fraction(0)] * (L - 1)
    dP_dmu = [Fraction(0)] * L
    for path in itertools.product(donors, repeat=L):
        em = [_theta_exact(h, l, path[l], i, mus[l]) for l in range(L)]
        tr = [rho[l] * pi_of[path[l + 1]] + (1 - rho[l]) * (1 if path[l] == path[l + 1] else 0)
              for l in range(L - 1)]
        start = pi_of[path[0]]
        prob = start
        for e in em:
            prob *= e
        for t in tr:
            prob *= t
        P += prob
        for l in range(L):
            marg[l][path[l]] += prob
        # d prob / d rho_l: replace T_l by its derivative pi_k - 1{j=k}
        for l in range(L - 1):
            d = pi_of[path[l + 1]] - (1 if path[l] == path[l + 1] else 0)
            rest = start
            for e in em:
                rest *= e
            for m, t in enumerate(tr):
                if m != l:
                    rest *= t
            dP_drho[l] += rest * d
        # d prob / d mu: product rule over the emissions, d theta/d mu = +-1
        for l in range(L):
            d = 1 if h[l][path[l]] != h[l][i] else -1
            rest = start
            for m, e in enumerate(em):
                if m != l:
                    rest *= e
            for t in tr:
                rest *= t
            dP_dmu[l] += rest * d
    if P == 0:
        # every path has probability 0: the posterior is undefined
        return dict(P=P, post=None)
    post = [[marg[l][j] / P for j in range(N)] for l in range(L)]
    return dict(P=P, post=post, dlogP_drho=[d / P for d in dP_drho],
                dlogP_dmu=sum(dP_dmu) / P, dlogP_dmu_l=[d / P for d in dP_dmu])


def _logsumexp(a, axis=None):
    m = np.max(a, axis=axis, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    s = np.log(np.sum(np.exp(a - m), axis=axis, keepdims=True)) + m
    return np.squeeze(s, axis=axis) if axis is not None else float(s.ravel()[0])


def logdomain_fb(h01, rho, mu, i):
    """Textbook log-domain forward-backward for recipient i over the full
    (N-1) x (N-1) transition matrix. Returns (log P, posterior [L][N])."""
    h01 = np.asarray(h01)
    L, N = h01.shape
    donors = np.array([j for j in range(N) if j != i])
    D = donors.size
    logpi = -np.log(N - 1)
    mis = h01[:, donors] != h01[:, [i]]
    logth = np.where(mis, np.log(mu), np.log1p(-mu))
    la = np.empty((L, D))
    la[0] = logpi + logth[0]
    for l in range(1, L):
        T = np.full((D, D), rho[l - 1] / (N - 1)) + np.eye(D) * (1 - rho[l - 1])
        with np.errstate(divide="ignore"):
            logT = np.log(T)
        la[l] = logth[l] + _logsumexp(la[l - 1][:, None] + logT, axis=0)
    lb = np.zeros((L, D))
    for l in range(L - 2, -1, -1):
        T = np.full((D, D), rho[l] / (N - 1)) + np.eye(D) * (1 - rho[l])
        with np.errstate(divide="ignore"):
            logT = np.log(T)
        lb[l] = _logsumexp(logT + (logth[l + 1] + lb[l + 1])[None, :], axis=1)
    logP = _logsumexp(la[-1])
    post = np.zeros((L, N))
    post[:, donors] = np.exp(la + lb - logP)
    return logP, post


def raw_forward(h01, rho, mu, i):
    """Unscaled forward probabilities alpha~ (eq. raw_forward), [L][N]."""
    h01 = np.asarray(h01)
    L, N = h01.shape
    pi = np.full(N, 1.0 / (N - 1))
    pi[i] = 0.0
    th = np.where(h01 != h01[:, [i]], mu, 1.0 - mu)
    a = np.empty((L, N))
    a[0] = th[0] * pi
    for l in range(1, L):
        F = a[l - 1].sum()
        a[l] = th[l] * ((1 - rho[l - 1]) * a[l - 1] + rho[l - 1] * F * pi)
    return a


def rho0_closed_form(h01, mu, i):
    """rho == 0: the copied donor never changes. Returns (log P, posterior
    [N], the same at every variant)."""
    h01 = np.asarray(h01)
    L, N = h01.shape
    m = (h01 != h01[:, [i]]).sum(axis=0).astype(float)
    logw = m * np.log(mu) + (L - m) * np.log1p(-mu) - np.log(N - 1)
    logw[i] = -np.inf
    logP = _logsumexp(logw)
    return logP, np.exp(logw - logP)


def rho0_closed_form_grad(h01, mu, i):
    """d log P / d rho_l at rho == 0, l = 0..L-2:
    [(sum_j pi A_j)(sum_k pi B_k) - sum_j pi A_j B_j] / sum_j pi A_j B_j with
    A_j = prod_{l' <= l} theta_j, B_j = prod_{l' > l} theta_j (log domain)."""
    h01 = np.asarray(h01)
    L, N = h01.shape
    donors = [j for j in range(N) if j != i]
    logth = np.where(h01[:, donors] != h01[:, [i]], np.log(mu), np.log1p(-mu))
    cum = np.cumsum(logth, axis=0)
    total = cum[-1]
    lpi = -np.log(N - 1)
    out = np.empty(L - 1)
    for l in range(L - 1):
        logA = cum[l]
        logB = total - cum[l]
        sa = _logsumexp(lpi + logA)
        sb = _logsumexp(lpi + logB)
        sab = _logsumexp(lpi + logA + logB)
        out[l] = np.exp(sa + sb - sab) - 1.0
    return out


def rho1_closed_form(h01, mu, i):
    """rho == 1: variants are independent. Returns (log P, posterior [L][N])."""
    h01 = np.asarray(h01)
    L, N = h01.shape
    th = np.where(h01 != h01[:, [i]], mu, 1.0 - mu)
    th[:, i] = 0.0
    w = th / (N - 1)
    s = w.sum(axis=1)
    return float(np.log(s).sum()), w / s[:, None]


def rho_map_checks(calc_rho, rho_map_grad, printed_pairs) -> bool:
    """Checks of the recombination map (eq. rho) and its chain rule that do
    not reuse the code under test: the paper's printed CalcRho values (with
    s = gamma = 1, reading the centimorgan argument as m = cM / 100 Morgans),
    the gamma = 1 closed form 1 - exp(-s m) at distances where it has no
    cancellation, the limits s = 0, m = 0 and m large, and central
    differences of f(s, gamma) = sum_l g_l rho_l(s, gamma)."""
    ok = True
    for m, printed in printed_pairs:
        got = calc_rho(np.array([100.0 * float(m)]), 1.0, 1.0)[0]
        ok &= abs(got - float(printed)) <= 1e-13 * float(printed)
    cM = np.array([0.5, 3.0, 10.0, 40.0, 150.0])
    ok &= bool(np.allclose(calc_rho(cM, 0.7, 1.0), 1.0 - np.exp(-0.7 * cM / 100.0),
                           rtol=1e-14, atol=0.0))
    ok &= bool(np.all(calc_rho(cM, 0.0, 1.3) == 0.0))
    ok &= calc_rho(np.array([0.0]), 2.0, 0.5)[0] == 0.0
    ok &= calc_rho(np.array([1e6]), 1.0, 1.0)[0] == 1.0
    rng = np.random.default_rng(5)
    cM = rng.exponential(2.0, 40)
    cM[::7] = 0.0
    g = rng.normal(size=40)
    s, ga = 1.7, 0.8
    gs, gg = rho_map_grad(cM, s, ga, g)

    def f(s_, g_):
        return float(np.dot(g, calc_rho(cM, s_, g_)))

    hs, hg = 1e-6 * s, 1e-6 * ga
    fds = (f(s + hs, ga) - f(s - hs, ga)) / (2 * hs)
    fdg = (f(s, ga + hg) - f(s, ga - hg)) / (2 * hg)
    ok &= abs(gs - fds) <= 1e-7 * abs(fds)
    ok &= abs(gg - fdg) <= 1e-7 * abs(fdg)
    return bool(ok)


# ---------------------------------------------------------------------------
# The floor and the zero-total rule of the posterior (section 2.2, eq.
# postprob) and of the distance (section 2.1, eq. distmat). The constant is
# double precision machine epsilon, taken from numpy's description of the
# type (the paper prints it as about 2.22e-16), not from the code under test.

EPS64 = float(np.finfo(np.float64).eps)


def zero_sum_case():
    """A recipient whose forward and backward vectors at target t are finite
    and non-zero but have disjoint support, so sum_j alpha_j beta_j = 0.

    mu = 0 (an emission is 0 on every mismatch) and rho_t = 0 (no switch
    between t and t+1). Recipient 0 carries allele 1 at t and at t+1; donors
    1 and 2 match it at t and not at t+1, donor 3 the reverse; at every other
    variant all four haplotypes carry allele 0. alpha^t lives on donors 1 and
    2 only (donor 3 mismatches at t) and beta^t on donor 3 only (with
    rho_t = 0, beta^t_j is proportional to theta^{t+1}_j beta^{t+1}_j), so
    every copying path has probability 0.

    Returns (h01 [L][N], rho as Fractions [L-1], mu, recipient, target)."""
    L, N, t = 5, 4, 2
    h = np.zeros((L, N), dtype=np.uint8)
    h[t, [0, 1, 2]] = 1
    h[t + 1, [0, 3]] = 1
    rho = [Fraction(1, 4), Fraction(1, 2), Fraction(0), Fraction(1, 8)]
    return h, rho, Fraction(0), 0, t


def tiny_posterior_case():
    """Exact posteriors spanning many orders of magnitude: mu = 2^-40, so
    that a donor mismatching the recipient where it is copied has a
    posterior near mu times the switch probabilities around it. Some exact
    posteriors fall below 2^-52 and many between 2^-52 and single
    precision's epsilon 2^-23. Returns (h01, rho Fractions, mu Fraction)."""
    h = np.array([[0, 1, 0, 0],
                  [0, 0, 0, 0],
                  [1, 0, 0, 1],
                  [0, 0, 1, 0],
                  [1, 0, 0, 1],
                  [1, 0, 0, 1]], dtype=np.uint8)
    rho = [Fraction(k, 256) for k in (17, 27, 37, 2, 3)]
    return h, rho, Fraction(1, 2 ** 40)


def floor_checks(run_pass) -> bool:
    """The zero-total rule and the eps floor, against exact enumeration.

    ``run_pass(h01, rho_float, mu_float, recipients, targets)`` returns the
    oracle's dict with P and E. Checks: (1) in zero_sum_case the exact
    likelihood is 0 (so eq. postprob has no value) and the pass gives
    p_ji = eps for every donor, p_ii = 0, and half distances -log(eps)/2 =
    26 log 2; (2) in tiny_posterior_case the half distances equal
    -log(max(p, eps))/2 of the exact posteriors, with entries on both sides
    of the floor and some between eps and single precision's epsilon."""
    ok = True
    h, rho, mu, i, t = zero_sum_case()
    ex = enumerate_exact(h.tolist(), rho, mu, i)
    ok &= ex["P"] == 0 and ex["post"] is None
    res = run_pass(h, np.array([float(r) for r in rho]), float(mu), np.array([i], np.int32),
                   np.array([t], np.int32))
    P, E = res["P"][0, 0], res["E"][0, 0]
    donors = np.arange(h.shape[1]) != i
    ok &= bool(np.all(P[donors] == EPS64)) and P[i] == 0.0
    half = 26.0 * np.log(2.0)  # -log(2^-52) / 2
    ok &= bool(np.all(np.abs(E[donors] - half) <= 1e-14 * half)) and E[i] == 0.0

    h, rho, mu = tiny_posterior_case()
    L, N = h.shape
    rec = np.arange(N, dtype=np.int32)
    tg = np.arange(L, dtype=np.int32)
    res = run_pass(h, np.array([float(r) for r in rho]), float(mu), rec, tg)
    below = between = 0
    for i in range(N):
        ex = enumerate_exact(h.tolist(), rho, mu, i)
        post = np.array([[float(x) for x in row] for row in ex["post"]])
        # the floor decides on the exact posterior; entries within one
        # rounding of eps would be ambiguous, and none is that close here
        Eref = np.empty((L, N))
        for l in range(L):
            for j in range(N):
                if j == i:
                    Eref[l, j] = 0.0
                    continue
                q = ex["post"][l][j]
                ok &= abs(float(q) / EPS64 - 1.0) > 1e-6
                Eref[l, j] = -np.log(float(q) if q > Fraction(EPS64) else EPS64) / 2
                below += q < Fraction(EPS64)
                between += Fraction(EPS64) < q < Fraction(2.0 ** -23)
        ok &= bool(np.allclose(res["P"][:, i, :], post, rtol=1e-11, atol=1e-300))
        ok &= bool(np.allclose(res["E"][:, i, :], Eref, rtol=1e-12, atol=1e-13))
    ok &= below >= 4 and between >= 10
    return bool(ok)
