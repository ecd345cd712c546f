"""FP16-stored vectors (LS_FP32_F16STORE): every update is rounded to half,
so the error against the FP64 oracle is that of half storage, and tables
stored at any variant resume exactly. Through the C ABI (libls.so)."""

from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from lsinputs import make_inputs, pack_haplotypes, rho_from_spacings

from _gpu import F32_POST_ATOL, check_reduced, forced_shape, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    need_gpu()
    import paper_2212_11403_amd as m
    m.load()
    return m


def _np(t):
    return t.double().cpu().numpy()


def _case(N, L, seed, skew=3):
    """Mosaic haplotypes and a prior in which each recipient favours a few
    donors (weights u^skew), so that the donors it copies often carry a
    prior weight far below 1/(N-1)."""
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
    W = rng.random((N, N)) ** skew
    np.fill_diagonal(W, 0.0)
    Pi = W / W.sum(axis=0, keepdims=True)
    return pack_haplotypes(h), rho, 0.01, Pi


def test_half_storage_is_real(ls):
    """On the small workload the FP16-stored decode differs from the FP32
    one (every step rounds to half) and is within the FP16 bounds of the
    oracle, with an error well above FP32's."""
    x = make_inputs("c1")
    ref = oracle.run_pass(x["H"], x["N"], x["L"], x["rho"], x["mu"], np.arange(x["N"]),
                          x["targets"], want=("P",))
    m = ls.Model(x["H"], x["N"], x["rho"], x["mu"])
    p16 = _np(ls.decode(m, x["targets"], "f16", want=("P",))["P"])
    p32 = _np(ls.decode(m, x["targets"], "fp32", want=("P",))["P"])
    e16 = check_reduced("f16", p16, ref["P"], "prob")
    e32 = np.abs(p32 - ref["P"]).max()
    print(f"small workload: FP16-stored {e16:.3e}, FP32 {e32:.3e}")
    assert e16 > 10 * e32 and e32 <= F32_POST_ATOL


@pytest.mark.parametrize("prior", [False, True])
@pytest.mark.parametrize("vector_mu", [False, True])
def test_tables_in_steps_resume_exactly(ls, prior, vector_mu):
    """Tables advanced in several calls (each stores its vector in half and
    the next resumes from it) give the bits of one call, in both
    directions, with and without a skewed prior and a per-variant mu; the
    split into launches of LS_SWEEP_CHUNK variants does not change them."""
    N, L = 300, 700
    H, rho, mu, Pi = _case(N, L, seed=21)
    if vector_mu:
        mu = 10.0 ** np.random.default_rng(3).uniform(-4, -1, L)
    m = ls.Model(H, N, rho, mu, prior=Pi if prior else None)
    a = ls.Table(m, 0, "f16")
    ls.forward(a, m, L - 1)
    b = ls.Table(m, 0, "f16")
    for t in (0, 36, 37, 300, 301, 650, L - 1):
        ls.forward(b, m, t)
    assert np.array_equal(a.state.cpu().numpy(), b.state.cpu().numpy())
    # each call adds its own part of the log scale to the stored one
    assert np.allclose(_np(a.log_scale), _np(b.log_scale), rtol=1e-13, atol=0)
    c = ls.Table(m, 1, "f16")
    ls.backward(c, m, 0)
    d = ls.Table(m, 1, "f16")
    for t in (L - 1, 600, 599, 200, 1, 0):
        ls.backward(d, m, t)
    assert np.array_equal(c.state.cpu().numpy(), d.state.cpu().numpy())
    assert np.allclose(_np(c.log_scale), _np(d.log_scale), rtol=1e-13, atol=0)
    old = os.environ.get("LS_SWEEP_CHUNK")
    os.environ["LS_SWEEP_CHUNK"] = "53"
    try:
        e = ls.Table(m, 0, "f16")
        ls.forward(e, m, L - 1)
    finally:
        if old is None:
            os.environ.pop("LS_SWEEP_CHUNK")
        else:
            os.environ["LS_SWEEP_CHUNK"] = old
    assert np.array_equal(a.state.cpu().numpy(), e.state.cpu().numpy())
    assert np.allclose(_np(a.log_scale), _np(e.log_scale), rtol=1e-13, atol=0)


@pytest.mark.parametrize("skew", [3, 8])
def test_skewed_prior_stays_in_range(ls, skew):
    """A prior that gives the copied donors far less than average weight
    (weights u^skew: most prior entries tiny) once overflowed half in the
    backward table; the backward sweep normalised by the plain column sum
    keeps every entry below its scale, so the tables stay finite with a
    clean status at any skew. At skew 3 decoding at targets and the
    posterior from a forward and a backward half table at one variant both
    match the oracle within the FP16 bounds. At skew 8 the prior spans 48
    orders of magnitude and a posterior can be the product of an alpha and
    a beta entry each far below half's range relative to its vector's
    largest (about 2^-38): half storage itself loses it (a CPU emulation of
    the half-stored sweeps gives the same 0.8 error), so only the range is
    checked there."""
    import torch
    N, L = 500, 400
    H, rho, mu, Pi = _case(N, L, seed=40 + skew, skew=skew)
    targets = np.array([50, 200, 399], np.int32)
    rec = np.arange(N, dtype=np.int32)
    m = ls.Model(H, N, rho, mu, prior=Pi)
    r = ls.decode(m, targets, "f16", want=("P",))
    assert ls.status_check(r["fwd"]) == ls.LS_OK
    assert ls.status_check(r["bck"]) == ls.LS_OK
    assert torch.isfinite(r["bck"].state.float()).all()
    assert torch.isfinite(r["P"]).all()
    if skew > 3:
        return
    ref = oracle.run_pass(H, N, L, rho, mu, rec, targets, want=("P",), prior=Pi)
    check_reduced("f16", _np(r["P"]), ref["P"], "prob")
    check_reduced("f16", _np(r["fwd"].log_scale), ref["llf"], "log")
    fwd = ls.Table(m, 0, "f16")
    bck = ls.Table(m, 1, "f16")
    ls.forward(fwd, m, 200)
    ls.backward(bck, m, 200)
    P = torch.empty((N, N), dtype=torch.float32, device="cuda")
    ls.posterior_distance(fwd, bck, m, P, None)
    assert torch.isfinite(P).all()
    check_reduced("f16", _np(P), ref["P"][1], "prob")


@pytest.mark.parametrize("shape", [None, (196, 8)])
def test_widest_groups_at_full_size(ls, shape):
    """N = 100,000 with FP16 storage, in the 132-slot 12-wave groups the
    shape choice takes there (three waves per SIMD) and in the 196 x 8
    groups: posteriors and log-likelihoods within the FP16 bounds of the
    oracle on seeded recipients at both ends and in the middle."""
    N, L = 100_000, 9
    rng = np.random.default_rng(100)
    F = (rng.random((L, 6)) < 0.4).astype(np.uint8)
    h = F[np.arange(L)[:, None], rng.integers(0, 6, size=(L, N))]
    h = (h ^ (rng.random((L, N)) < 0.01)).astype(np.uint8)
    H = pack_haplotypes(h)
    rho = rho_from_spacings(rng.exponential(0.05, L - 1))
    mu = 0.01
    targets = np.array([2, 6], np.int32)
    rec = np.array([0, 1, 63, 64, N // 2, N - 2, N - 1], dtype=np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, targets, want=("P",))
    m = ls.Model(H, N, rho, mu)
    if shape is None:
        assert ls.kernel_shape(N, "f16") == (132, 12)
        r = ls.decode(m, targets, "f16", recipients=rec, want=("P",))
    else:
        with forced_shape(*shape):
            assert ls.kernel_shape(N, "f16") == shape
            r = ls.decode(m, targets, "f16", recipients=rec, want=("P",))
    check_reduced("f16", _np(r["P"]), ref["P"], "prob")
    check_reduced("f16", _np(r["fwd"].log_scale), ref["llf"], "log")
