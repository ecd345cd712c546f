"""The recombination map (eq. rho, the paper's CalcRho) and its chain rule on
the GPU against the FP64 oracle, and the PAC gradient with respect to the
map parameters (s, gamma) through the autograd functions."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from lsinputs import pack_haplotypes

from _gpu import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    need_gpu()
    import paper_2212_11403_amd as m
    m.load()
    return m


def _map(n, seed):
    rng = np.random.default_rng(seed)
    cM = rng.exponential(0.1, n)   # ~1e-3 Morgans per interval
    cM[::11] = 0.0                 # coincident positions
    cM[5] = 250.0                  # a long gap: rho close to 1
    return cM


@pytest.mark.parametrize("s,gamma", [(1.0, 1.0), (0.37, 1.6), (4.0, 0.5), (0.0, 1.0)])
def test_calc_rho_matches_oracle(ls, s, gamma):
    cM = _map(5000, 1)
    got = ls.calc_rho(cM, s, gamma).cpu().numpy()
    ref = oracle.calc_rho(cM, s, gamma)
    # device expm1/pow against the C library's: a few ulp
    assert np.all(np.abs(got - ref) <= 1e-14 * np.abs(ref) + 1e-300)
    assert np.all(got[cM == 0.0] == 0.0)


@pytest.mark.parametrize("s,gamma", [(1.0, 1.0), (0.37, 1.6), (4.0, 0.5)])
def test_rho_map_grad_matches_oracle(ls, s, gamma):
    cM = _map(20000, 2)
    g = np.random.default_rng(3).normal(size=cM.size)
    got = ls.rho_map_grad(cM, s, gamma, g).cpu().numpy()
    ref = np.array(oracle.rho_map_grad(cM, s, gamma, g))
    # sums of 20,000 terms in different orders: bound by the term magnitudes
    m = cM / 100.0
    mg = np.where(m > 0, m ** gamma, 0.0)
    e = np.exp(-s * mg)
    scale = np.array([np.sum(np.abs(g * mg * e)),
                      np.sum(np.abs(g * s * mg * np.log(np.where(m > 0, m, 1.0)) * e))])
    assert np.all(np.abs(got - ref) <= 1e-13 * scale + 1e-300)


def test_rho_map_argument_errors(ls):
    import torch
    c = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(ls.LsError):
        ls.calc_rho(c, 1.0, 0.0)        # gamma must be > 0
    with pytest.raises(ls.LsError):
        ls.calc_rho(c, -1.0, 1.0)       # s must be >= 0
    with pytest.raises(ls.LsError):
        ls.rho_map_grad(c, 1.0, float("nan"), c)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pac_gradient_wrt_map_parameters(ls, prec):
    """d PAC / d (s, gamma) through RhoMap and PACLoglik against the oracle's
    score chained with the oracle's map derivative, and (FP64) against
    central differences of the PAC."""
    import torch
    N, L = 60, 300
    rng = np.random.default_rng(8)
    K = 6
    F = (rng.random((L, K)) < 0.45).astype(np.uint8)
    h = F[:, rng.integers(0, K, size=N)].copy()
    h ^= (rng.random((L, N)) < 0.01).astype(np.uint8)
    H = pack_haplotypes(h)
    cM = _map(L - 1, 9)
    s0, g0, mu = 1.3, 0.9, 0.01
    s = torch.tensor(s0, dtype=torch.float64, device="cuda", requires_grad=True)
    ga = torch.tensor(g0, dtype=torch.float64, device="cuda", requires_grad=True)
    c = torch.tensor(cM, dtype=torch.float64, device="cuda")
    m_ = torch.tensor(mu, dtype=torch.float64, device="cuda")
    pac = ls.PACLoglik.apply(ls.RhoMap.apply(c, s, ga), m_, H, N, prec)
    pac.backward()
    rho = oracle.calc_rho(cM, s0, g0)
    ref = oracle.run_gradient(H, N, L, rho, mu, np.arange(N, dtype=np.int32))
    gr = ref["grad_rho"].sum(axis=0)
    gs_ref, gg_ref = oracle.rho_map_grad(cM, s0, g0, gr)
    # the chained sums have terms of both signs: bound by their magnitudes
    m = cM / 100.0
    pos = m > 0
    mg = np.where(pos, m ** g0, 0.0)
    e = np.exp(-s0 * mg)
    logm = np.log(np.where(pos, m, 1.0))
    scale_s = np.sum(np.abs(gr) * mg * e)
    scale_g = np.sum(np.abs(gr) * s0 * mg * np.abs(logm) * e)
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert abs(s.grad.item() - gs_ref) <= tol * scale_s
    assert abs(ga.grad.item() - gg_ref) <= tol * scale_g
    if prec == "fp64":
        def f(sv, gv):
            r = ls.calc_rho(cM, sv, gv)
            return float(ls.loglik_grad(ls.Model(H, N, r, mu), None, "fp64", grad=False)["pac"])
        h1, h2 = 1e-6 * s0, 1e-6 * g0
        fds = (f(s0 + h1, g0) - f(s0 - h1, g0)) / (2 * h1)
        fdg = (f(s0, g0 + h2) - f(s0, g0 - h2)) / (2 * h2)
        assert abs(fds - s.grad.item()) <= 1e-5 * abs(fds)
        assert abs(fdg - ga.grad.item()) <= 1e-5 * abs(fdg)
