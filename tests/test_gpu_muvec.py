"""Per-variant mutation probability mu^l (section 3.4: mu may be a vector of
length L): the GPU decode and log-likelihood against the FP64 oracle, through
the C ABI (libls.so)."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from lsinputs import pack_haplotypes, rho_from_spacings

from _gpu import (F32_LOGLIK_RTOL, F32_POST_ATOL, F64_ATOL_LOG, F64_ATOL_PROB, F64_RTOL,
                  check_reduced,
                  forced_shape, need_gpu, rel_close)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    need_gpu()
    import paper_2212_11403_amd as m
    m.load()
    return m


def _np(t):
    return t.double().cpu().numpy()


def _case(N, L, seed):
    """Mosaic haplotypes and a mu that varies over four decades, with some
    variants above 1/2 (the mismatch emission is then the larger one) and one
    at exactly 0."""
    rng = np.random.default_rng(seed)
    K = max(2, min(8, N // 3))
    F = (rng.random((L, K)) < 0.4).astype(np.uint8)
    which = rng.integers(0, K, size=(L, N))
    sw = rng.random((L, N)) < 0.05
    base = rng.integers(0, K, size=N)
    idx = np.where(np.cumsum(sw, axis=0) == 0, base[None, :], which)
    h = F[np.arange(L)[:, None], idx]
    h = (h ^ (rng.random((L, N)) < 0.01)).astype(np.uint8)
    rho = rho_from_spacings(rng.exponential(0.05, L - 1))
    mu = 10.0 ** rng.uniform(-5, -1, L)
    hi = rng.random(L) < 0.1
    mu[hi] = rng.uniform(0.5, 0.8, hi.sum())
    # mu = 0 at a variant where no allele is carried by a single haplotype,
    # so every recipient keeps a matching donor there
    ones = h.sum(axis=1)
    ok = np.flatnonzero((ones != 1) & (ones != N - 1))
    if ok.size:
        mu[ok[np.argmin(np.abs(ok - L // 2))]] = 0.0
    return pack_haplotypes(h), rho, mu


def _check(prec, got, ref, what):
    if prec == "fp64":
        tol = F64_ATOL_LOG if what == "log" else F64_ATOL_PROB
        rel_close(got, ref, F64_RTOL, tol)
    else:
        check_reduced(prec, got, ref, what)


CASES = [(65, 40), (700, 30), (1031, 12), (200, 5000)]


@pytest.mark.parametrize("N,L", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "f16"])
def test_vector_mu_decode_matches_oracle(ls, N, L, prec):
    """Posteriors, half distances, beta snapshots and both log scales; L =
    5000 spans several sweep launches per direction. FP16-stored vectors
    against the FP16 bounds."""
    H, rho, mu = _case(N, L, seed=N + 13 * L)
    targets = np.unique(np.array([0, L // 3, L // 2, L - 1], np.int32))
    rec = np.arange(N, dtype=np.int32) if N <= 300 else np.array([0, 1, 63, 64, N - 1], np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, targets, want=("P", "E", "B", "logG"))
    m = ls.Model(H, N, rho, mu)
    r = ls.decode(m, targets, prec, recipients=rec, want=("P", "E"))
    assert ls.status_check(r["fwd"]) == ls.LS_OK
    _check(prec, _np(r["P"]), ref["P"], "prob")
    _check(prec, _np(r["fwd"].log_scale), ref["llf"], "log")
    _check(prec, _np(r["bck"].log_scale), ref["logG"][0], "log")
    if prec == "fp64":
        rel_close(_np(r["E"]), ref["E"], F64_RTOL, F64_ATOL_LOG)
        rel_close(_np(r["bsnap"]), ref["B"], F64_RTOL, F64_ATOL_PROB)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_constant_vector_equals_scalar(ls, prec):
    """A vector holding the same mu at every variant gives the scalar
    model's results. In FP32 arithmetic the vectors are the same bits (the
    divided emission pairs and the coefficient tables are the same numbers)
    and the log scales agree to rounding (the backward sums the log divisors
    from a prefix table instead of one per step). The FP64 sweep divides a
    scalar mu's pair by its larger member and keeps per-variant pairs as
    they are, so there everything agrees to rounding."""
    N, L = 300, 3000
    H, rho, _ = _case(N, L, seed=3)
    mu = 0.003
    ms = ls.Model(H, N, rho, mu)
    mv = ls.Model(H, N, rho, np.full(L, mu))
    targets = [0, 5, 1500, L - 1]
    a = ls.decode(ms, targets, prec, want=("P",))
    b = ls.decode(mv, targets, prec, want=("P",))
    same = np.array_equal if prec == "fp32" else (
        lambda x, y: np.allclose(x, y, rtol=1e-13, atol=1e-300))
    assert same(_np(a["P"]), _np(b["P"]))
    assert same(_np(a["bsnap"]), _np(b["bsnap"]))
    for k in ("fwd", "bck"):
        assert same(_np(a[k].state), _np(b[k].state))
        assert np.allclose(_np(a[k].log_scale), _np(b[k].log_scale), rtol=1e-12, atol=0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vector_mu_tables_in_steps_equal_direct(ls, prec):
    """Tables moved a few variants at a time (each call resumes from the
    stored table) equal one direct move: the vectors bit for bit, the log
    scales to rounding."""
    N, L = 150, 60
    H, rho, mu = _case(N, L, seed=21)
    m = ls.Model(H, N, rho, mu)
    a = ls.Table(m, 0, prec)
    ls.forward(a, m, 47)
    b = ls.Table(m, 0, prec)
    for t in (0, 1, 9, 10, 30, 47):
        ls.forward(b, m, t)
    assert np.array_equal(_np(a.state), _np(b.state))
    assert np.allclose(_np(a.log_scale), _np(b.log_scale), rtol=1e-13, atol=1e-12)
    c = ls.Table(m, 1, prec)
    ls.backward(c, m, 4)
    d = ls.Table(m, 1, prec)
    for t in (L - 1, L - 2, 40, 39, 11, 4):
        ls.backward(d, m, t)
    assert np.array_equal(_np(c.state), _np(d.state))
    assert np.allclose(_np(c.log_scale), _np(d.log_scale), rtol=1e-13, atol=1e-12)
    # and the forward table against the oracle at variant 47
    ref = oracle.run_pass(H, N, L, rho, mu, np.arange(N), np.array([47], np.int32),
                          want=("A", "logF"))
    _check(prec, _np(b.log_scale), ref["logF"][0], "log")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "f16"])
def test_vector_mu_loglik(ls, prec):
    """The log-likelihood entry point (no gradient) takes a vector mu."""
    N, L = 400, 800
    H, rho, mu = _case(N, L, seed=8)
    rec = np.array([0, 7, 200, 399], np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, (), want=())
    m = ls.Model(H, N, rho, mu)
    out = ls.loglik_grad(m, recipients=rec, prec=prec, grad=False)
    _check(prec, _np(out["loglik"]), ref["llf"], "log")
    _check(prec, _np(out["pac"]), np.array([ref["llf"].sum()]), "log")


def test_vector_mu_unsupported_and_invalid(ls):
    N, L = 70, 10
    H, rho, mu = _case(N, L, seed=4)
    m = ls.Model(H, N, rho, mu)
    with pytest.raises(ls.LsError) as e:
        ls.loglik_grad(m, prec="f16", grad=True)  # as with a scalar mu
    assert e.value.code == 4  # LS_ERR_UNSUPPORTED
    with pytest.raises(ValueError):
        ls.Model(H, N, rho, mu[:-1])
    for bad in (1.5, -1e-3, np.nan):
        v = mu.copy()
        v[3] = bad
        with pytest.raises(ls.LsError) as e:
            ls.Model(H, N, rho, v)
        assert e.value.code == 1  # LS_ERR_ARG
    # models that differ only in mu_vec do not share tables
    v = mu.copy()
    v[2] *= 0.5
    m2 = ls.Model(H, N, rho, v)
    t = ls.Table(m, 0, "fp32")
    ls.forward(t, m, 3)
    with pytest.raises(ls.LsError) as e:
        ls.forward(t, m2, 5)
    assert e.value.code == 3  # LS_ERR_STATE


# ---------------------------------------------------------------------------
# gradient with respect to each mu^l (and rho) with a per-variant mu

def _grad_case(N, L, seed):
    """As _case, with mu^l > 0 everywhere (d/d mu^l has a 1/mu^l term)."""
    H, rho, mu = _case(N, L, seed)
    mu[mu == 0.0] = 1e-3
    return H, rho, mu


def _check_grad(ls, H, N, L, rho, mu, rec, prec):
    ref = oracle.run_gradient(H, N, L, rho, mu, rec)
    out = ls.loglik_grad(ls.Model(H, N, rho, mu), rec, prec, grad=True)
    ll = ref["loglik"].sum()
    tol_ll = 1e-12 if prec == "fp64" else F32_LOGLIK_RTOL
    assert abs(float(out["pac"].item()) - ll) <= tol_ll * abs(ll)
    if L > 1:
        g = out["grad_rho"].cpu().numpy()
        scale = max(np.abs(ref["grad_rho"]).sum(axis=0).max(), 1.0)
        assert np.abs(g - ref["grad_rho"].sum(axis=0)).max() <= (1e-10 if prec == "fp64" else 1e-6) * scale
    # d/d mu^l sums one term M/mu - (1-M)/(1-mu) per recipient; its rounding
    # scales with the two parts, M/mu + (1-M)/(1-mu), before they cancel
    # (M, the mismatch share of the posterior, recovered from the term)
    gml = ref["grad_mu_l"]
    M = (gml + 1.0 / (1.0 - mu)) / (1.0 / mu + 1.0 / (1.0 - mu))
    parts = (M / mu + (1.0 - M) / (1.0 - mu)).sum(axis=0)
    got = out["grad_mu"].cpu().numpy()
    assert got.shape == (L,)
    err = np.abs(got - gml.sum(axis=0)) / parts
    print(f"{prec} N={N} L={L}: max error of d/d mu^l relative to its parts {err.max():.2e}")
    # observed: up to 2e-14 (FP64) and 3e-7 (FP32)
    assert err.max() <= (1e-12 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("N,L", [(2, 50), (40, 300), (130, 200), (40, 1), (40, 2), (40, 7),
                                 (40, 10)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vector_mu_gradient_vs_oracle(ls, N, L, prec):
    """All recipients; L = 1, 2, 7 and 10 give one-variant and two-variant
    segments and segments that end at the last variant."""
    H, rho, mu = _grad_case(N, L, seed=3 * N + L)
    _check_grad(ls, H, N, L, rho, mu, np.arange(N, dtype=np.int32), prec)


@pytest.mark.parametrize("prec,N,ns,nw", [("fp32", 10000, 16, 13), ("fp64", 4000, 8, 13)])
def test_vector_mu_gradient_wide_groups(ls, prec, N, ns, nw):
    L = 61
    H, rho, mu = _grad_case(N, L, seed=N + 1)
    rec = np.array([0, 63, N // 2, N - 1], np.int32)
    with forced_shape(ns, nw):
        _check_grad(ls, H, N, L, rho, mu, rec, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vector_mu_gradient_constant_vector(ls, prec):
    """A constant vector: the rho gradient equals the scalar model's (bit for
    bit in FP32 arithmetic, to rounding in FP64, where only the scalar pair
    is divided by its larger member), the per-variant mu terms add up to the
    scalar d/d mu, and log P is the same with and without the gradient."""
    N, L = 200, 400
    H, rho, _ = _grad_case(N, L, seed=17)
    ms = ls.Model(H, N, rho, 0.004)
    mv = ls.Model(H, N, rho, np.full(L, 0.004))
    a = ls.loglik_grad(ms, None, prec, grad=True)
    b = ls.loglik_grad(mv, None, prec, grad=True)
    c = ls.loglik_grad(mv, None, prec, grad=False)
    ga, gb = a["grad_rho"].cpu().numpy(), b["grad_rho"].cpu().numpy()
    if prec == "fp32":
        assert np.array_equal(ga, gb)
    else:
        assert np.allclose(ga, gb, rtol=1e-12, atol=1e-12 * np.abs(gb).max())
    assert np.array_equal(b["loglik"].cpu().numpy(), c["loglik"].cpu().numpy())
    gs, gv = float(a["grad_mu"].item()), float(b["grad_mu"].sum().item())
    assert abs(gs - gv) <= 1e-12 * float(b["grad_mu"].abs().sum().item())
    x, y = float(a["pac"].item()), float(b["pac"].item())
    assert abs(x - y) <= 1e-12 * abs(x)


def test_vector_mu_autograd(ls):
    import torch
    N, L = 60, 80
    H, rho, mu = _grad_case(N, L, seed=5)
    r = torch.tensor(rho, dtype=torch.float64, device="cuda", requires_grad=True)
    m = torch.tensor(mu, dtype=torch.float64, device="cuda", requires_grad=True)
    pac = ls.PACLoglik.apply(r, m, H, N, "fp64")
    pac.backward()
    ref = oracle.run_gradient(H, N, L, rho, mu, np.arange(N, dtype=np.int32))
    rel_close(m.grad.cpu().numpy(), ref["grad_mu_l"].sum(axis=0), 1e-9, 1e-9)
    rel_close(r.grad.cpu().numpy(), ref["grad_rho"].sum(axis=0), 1e-9, 1e-9)
