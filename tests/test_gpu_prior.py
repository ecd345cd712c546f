"""Non-uniform prior copying matrix Pi (section 2.1, eq. transition with
Pi_ki in place of 1/(N-1)): the GPU decode and log-likelihood against the
FP64 oracle, through the C ABI (libls.so)."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from lsinputs import pack_haplotypes, rho_from_spacings

from _gpu import (F32_LOGLIK_RTOL, F32_POST_ATOL, F64_ATOL_LOG, F64_ATOL_PROB, F64_RTOL,
                  check_reduced,
                  need_gpu, rel_close)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    need_gpu()
    import paper_2212_11403_amd as m
    m.load()
    return m


def _np(t):
    return t.double().cpu().numpy()


def _case(N, L, seed, mu=0.01):
    """Mosaic haplotypes and a skewed prior: each recipient favours a few
    donors (weights u^3), columns normalised off the diagonal."""
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
    W = rng.random((N, N)) ** 3
    np.fill_diagonal(W, 0.0)
    Pi = W / W.sum(axis=0, keepdims=True)
    return pack_haplotypes(h), rho, mu, Pi


def _check(prec, got, ref, what):
    if prec == "fp64":
        rel_close(got, ref, F64_RTOL, F64_ATOL_LOG if what == "log" else F64_ATOL_PROB)
    else:
        check_reduced(prec, got, ref, what)


CASES = [(65, 40), (700, 30), (1031, 12), (200, 3000), (8000, 10)]


@pytest.mark.parametrize("N,L", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_prior_decode_matches_oracle(ls, N, L, prec):
    """Posteriors, half distances, beta snapshots and both log scales;
    L = 3000 spans two sweep launches per direction, N = 8000 takes the
    widest groups the prior column leaves room for."""
    H, rho, mu, Pi = _case(N, L, seed=N + 7 * L)
    targets = np.unique(np.array([0, L // 3, L - 1], np.int32))
    rec = np.arange(N, dtype=np.int32) if N <= 300 else np.array([0, 1, 63, 64, N - 1], np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, targets, want=("P", "E", "B", "logG"), prior=Pi)
    m = ls.Model(H, N, rho, mu, prior=Pi)
    r = ls.decode(m, targets, prec, recipients=rec, want=("P", "E"))
    assert ls.status_check(r["fwd"]) == ls.LS_OK
    _check(prec, _np(r["P"]), ref["P"], "prob")
    _check(prec, _np(r["fwd"].log_scale), ref["llf"], "log")
    _check(prec, _np(r["bck"].log_scale), ref["logG"][0], "log")
    if prec == "fp64":
        rel_close(_np(r["E"]), ref["E"], F64_RTOL, F64_ATOL_LOG)
        rel_close(_np(r["bsnap"]), ref["B"], F64_RTOL, F64_ATOL_PROB)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uniform_prior_matrix_equals_default(ls, prec):
    """The uniform matrix is the default model (the kernel may take another
    group shape for it, so results agree to rounding)."""
    N, L = 300, 500
    H, rho, mu, _ = _case(N, L, seed=2)
    Pi = np.full((N, N), 1.0 / (N - 1))
    np.fill_diagonal(Pi, 0.0)
    targets = [0, 250, L - 1]
    a = ls.decode(ls.Model(H, N, rho, mu), targets, prec, want=("P",))
    b = ls.decode(ls.Model(H, N, rho, mu, prior=Pi), targets, prec, want=("P",))
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert np.abs(_np(a["P"]) - _np(b["P"])).max() <= tol
    for k in ("fwd", "bck"):
        x, y = _np(a[k].log_scale), _np(b[k].log_scale)
        assert np.max(np.abs(x - y) / np.abs(x)) <= (1e-13 if prec == "fp64" else 1e-7)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_prior_tables_in_steps_equal_direct(ls, prec):
    N, L = 150, 60
    H, rho, mu, Pi = _case(N, L, seed=21)
    m = ls.Model(H, N, rho, mu, prior=Pi)
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
    ref = oracle.run_pass(H, N, L, rho, mu, np.arange(N), np.array([4, 47], np.int32),
                          want=("B", "logF", "logG"), prior=Pi)
    _check(prec, _np(b.log_scale), ref["logF"][1], "log")
    _check(prec, _np(d.log_scale), ref["logG"][0], "log")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_prior_loglik(ls, prec):
    N, L = 400, 600
    H, rho, mu, Pi = _case(N, L, seed=8)
    rec = np.array([0, 7, 200, 399], np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, (), want=(), prior=Pi)
    out = ls.loglik_grad(ls.Model(H, N, rho, mu, prior=Pi), recipients=rec, prec=prec, grad=False)
    _check(prec, _np(out["loglik"]), ref["llf"], "log")


@pytest.mark.parametrize("N,L", [(65, 40), (1031, 12), (200, 3000)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "f16"])
def test_prior_with_vector_mu_matches_oracle(ls, N, L, prec):
    """A prior matrix together with a per-variant mu (mu over four decades,
    some above 1/2); FP16 storage also with the prior alone."""
    H, rho, _, Pi = _case(N, L, seed=N + 11 * L)
    rng = np.random.default_rng(N + L)
    mu = 10.0 ** rng.uniform(-5, -1, L)
    mu[rng.random(L) < 0.1] = 0.6
    targets = np.unique(np.array([0, L // 2, L - 1], np.int32))
    rec = np.arange(N, dtype=np.int32) if N <= 300 else np.array([0, 64, N - 1], np.int32)
    for m_arg in ((mu, 0.01) if prec == "f16" else (mu,)):
        ref = oracle.run_pass(H, N, L, rho, m_arg, rec, targets, want=("P", "logG"), prior=Pi)
        m = ls.Model(H, N, rho, m_arg, prior=Pi)
        r = ls.decode(m, targets, prec, recipients=rec, want=("P",))
        assert ls.status_check(r["fwd"]) == ls.LS_OK
        _check(prec, _np(r["P"]), ref["P"], "prob")
        _check(prec, _np(r["fwd"].log_scale), ref["llf"], "log")
        if prec != "f16":
            # FP16-stored backward tables with a prior hold a positive multiple
            # of beta (normalised by the plain column sum), not log G^0
            _check(prec, _np(r["bck"].log_scale), ref["logG"][0], "log")


def test_prior_invalid(ls):
    N, L = 70, 10
    H, rho, mu, Pi = _case(N, L, seed=4)
    m = ls.Model(H, N, rho, mu, prior=Pi)
    with pytest.raises(ls.LsError) as e:
        ls.loglik_grad(m, prec="f16", grad=True)  # as without a prior
    assert e.value.code == 4  # LS_ERR_UNSUPPORTED
    with pytest.raises(ValueError):
        ls.Model(H, N, rho, mu, prior=Pi[:-1])
    bad = Pi.copy()
    bad[:, 5] *= 0.9          # a column that does not sum to 1
    with pytest.raises(ls.LsError) as e:
        ls.Model(H, N, rho, mu, prior=bad)
    assert e.value.code == 1  # LS_ERR_ARG
    bad = Pi.copy()
    bad[3, 7] = -bad[3, 7]    # a negative entry
    with pytest.raises(ls.LsError) as e:
        ls.Model(H, N, rho, mu, prior=bad)
    assert e.value.code == 1
    # models that differ only in the prior do not share tables
    P2 = Pi.copy()
    P2[[1, 2], 0] = P2[[2, 1], 0]
    m2 = ls.Model(H, N, rho, mu, prior=P2)
    t = ls.Table(m, 0, "fp32")
    ls.forward(t, m, 3)
    with pytest.raises(ls.LsError) as e:
        ls.forward(t, m2, 5)
    assert e.value.code == 3  # LS_ERR_STATE


PRIOR_SHAPES = [  # (precision, N, slots, waves): multi-wave layouts and special slots
    ("fp64", 700, 4, 3), ("fp64", 1031, 4, 5), ("fp64", 333, 1, 6), ("fp64", 4160, 16, 5),
    ("fp32", 700, 3, 4), ("fp32", 1031, 12, 2), ("fp32", 4160, 12, 6),
]


@pytest.mark.parametrize("prec,N,ns,nw", PRIOR_SHAPES)
def test_prior_forced_shapes(ls, prec, N, ns, nw):
    """Group shapes chosen by hand (each must fit the doubled per-slot
    registers of the prior column): every lane of every slot class holds
    the right prior entry."""
    from _gpu import forced_shape
    L = 9
    H, rho, mu, Pi = _case(N, L, seed=N + 3 * ns + nw)
    targets = np.array([0, 2, 5], np.int32)  # the backward table ends at variant 0
    rec = np.array(sorted({0, 1, 63, 64, N // 2, N - 2, N - 1}), dtype=np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, targets, want=("P", "B", "logG"), prior=Pi)
    m = ls.Model(H, N, rho, mu, prior=Pi)
    with forced_shape(ns, nw):
        r = ls.decode(m, targets, prec, recipients=rec, want=("P",))
    _check(prec, _np(r["P"]), ref["P"], "prob")
    _check(prec, _np(r["fwd"].log_scale), ref["llf"], "log")
    _check(prec, _np(r["bck"].log_scale), ref["logG"][0], "log")
    if prec == "fp64":
        rel_close(_np(r["bsnap"]), ref["B"], F64_RTOL, F64_ATOL_PROB)


# ---------------------------------------------------------------------------
# gradient under a prior matrix

def _check_grad(ls, H, N, L, rho, mu, Pi, rec, prec):
    ref = oracle.run_gradient(H, N, L, rho, mu, rec, prior=Pi)
    m = ls.Model(H, N, rho, mu, prior=Pi)
    out = ls.loglik_grad(m, rec, prec, grad=True)
    plain = ls.loglik_grad(m, rec, prec, grad=False)
    # log P is the same bits with and without the gradient
    assert np.array_equal(out["loglik"].cpu().numpy(), plain["loglik"].cpu().numpy())
    ll = ref["loglik"].sum()
    assert abs(float(out["pac"].item()) - ll) <= (1e-12 if prec == "fp64" else F32_LOGLIK_RTOL) * abs(ll)
    tol = 1e-10 if prec == "fp64" else 1e-6
    if L > 1:
        g = out["grad_rho"].cpu().numpy()
        scale = max(np.abs(ref["grad_rho"]).sum(axis=0).max(), 1.0)
        assert np.abs(g - ref["grad_rho"].sum(axis=0)).max() <= tol * scale
    if np.ndim(mu) == 0:
        scale = max(np.abs(ref["grad_mu"]).sum(), 1.0)
        assert abs(float(out["grad_mu"].item()) - ref["grad_mu"].sum()) <= tol * scale
    else:
        gml = ref["grad_mu_l"]
        M = (gml + 1.0 / (1.0 - mu)) / (1.0 / mu + 1.0 / (1.0 - mu))
        parts = (M / mu + (1.0 - M) / (1.0 - mu)).sum(axis=0)
        err = np.abs(out["grad_mu"].cpu().numpy() - gml.sum(axis=0)) / parts
        assert err.max() <= (1e-12 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("N,L", [(2, 50), (40, 300), (130, 200), (40, 1), (40, 7), (40, 10)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_prior_gradient_vs_oracle(ls, N, L, prec):
    """d PAC / d rho and d PAC / d mu under a skewed prior, all recipients;
    L = 1, 7 and 10 give one-variant and short segments."""
    H, rho, mu, Pi = _case(N, L, seed=5 * N + L)
    _check_grad(ls, H, N, L, rho, mu, Pi, np.arange(N, dtype=np.int32), prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_prior_gradient_with_vector_mu(ls, prec):
    N, L = 90, 120
    H, rho, _, Pi = _case(N, L, seed=12)
    mu = 10.0 ** np.random.default_rng(12).uniform(-4, -1, L)
    _check_grad(ls, H, N, L, rho, mu, Pi, np.arange(N, dtype=np.int32), prec)


@pytest.mark.parametrize("prec,N,ns,nw", [("fp32", 10000, 16, 13), ("fp64", 4000, 8, 13)])
def test_prior_gradient_wide_groups(ls, prec, N, ns, nw):
    """Groups wider than the prefetching adjoint kernel allows (its wide
    variant, with the prior column), forced on a few recipients."""
    from _gpu import forced_shape
    L = 31
    H, rho, mu, Pi = _case(N, L, seed=N + 9)
    rec = np.array([0, 63, N // 2, N - 1], np.int32)
    with forced_shape(ns, nw):
        _check_grad(ls, H, N, L, rho, mu, Pi, rec, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_prior_large_n(ls, prec):
    """N = 16,384 (a 2 GiB prior): the widest groups the prior column leaves
    room for, on a few recipients against the oracle."""
    N, L = 16384, 8
    rng = np.random.default_rng(16384)
    h = (rng.random((L, N)) < 0.3).astype(np.uint8)
    rho = rho_from_spacings(rng.exponential(0.05, L - 1))
    Pi = rng.random((N, N))
    Pi **= 3
    np.fill_diagonal(Pi, 0.0)
    Pi /= Pi.sum(axis=0, keepdims=True)
    H = pack_haplotypes(h)
    rec = np.array([0, 4095, 8192, N - 1], np.int32)
    targets = np.array([0, 5], np.int32)
    ref = oracle.run_pass(H, N, L, rho, 0.01, rec, targets, want=("P", "logG"), prior=Pi)
    m = ls.Model(H, N, rho, 0.01, prior=Pi)
    r = ls.decode(m, targets, prec, recipients=rec, want=("P",))
    _check(prec, _np(r["P"]), ref["P"], "prob")
    _check(prec, _np(r["fwd"].log_scale), ref["llf"], "log")
    _check(prec, _np(r["bck"].log_scale), ref["logG"][0], "log")
