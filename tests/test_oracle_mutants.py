"""The pins must catch plausible mistakes in the oracle.

Each case copies the oracle's C source, plants one mistake (a dropped term, a
wrong sign, a wrong index, a swapped operand), compiles the copy into a
temporary directory and checks that the exact-enumeration pins reject it.
Nothing here touches the real oracle build. CPU only.
"""

from __future__ import annotations

import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
from lsinputs import pack_haplotypes

from _pins import enumerate_exact, floor_checks, rho_map_checks

SRC = os.path.join(os.path.dirname(oracle.__file__), "ls_oracle.c")

MUTANTS = {
    "forward_drops_normalisation": ("(1.0 - r) * prev[j] / S", "(1.0 - r) * prev[j]"),
    "forward_rho_index": ("double r = m->rho[l - 1];\n    for (int j = 0; j < m->N; ++j) {\n        if (j == i) {\n            next[j] = 0.0;",
                          "double r = m->rho[l > 1 ? l - 2 : 0];\n    for (int j = 0; j < m->N; ++j) {\n        if (j == i) {\n            next[j] = 0.0;"),
    "emission_swapped": ("(double)(1 - Hm) * (1.0 - 2.0 * mu) + mu", "(double)(Hm) * (1.0 - 2.0 * mu) + mu"),
    "prior_keeps_self": ("    if (j == i)\n        return 0.0;\n    return m->Pi",
                         "    return m->Pi"),
    "backward_theta_index": ("cur[j] = (1.0 - r) * next[j] * theta(m, l + 1, j, i) / g + r;",
                             "cur[j] = (1.0 - r) * next[j] * theta(m, l, j, i) / g + r;"),
    "backward_rho_index": ("double r = m->rho[l];", "double r = m->rho[l + 1 < m->L - 1 ? l + 1 : l];"),
    "backward_drops_rho_term": ("/ g + r;", "/ g;"),
    "grad_rho_sign": ("grad_rho[l - 1] = (Sg - a) /", "grad_rho[l - 1] = (a - Sg) /"),
    "grad_rho_uses_wrong_alpha": ("const double *al = alpha + (int64_t)(l - 1) * N;",
                                  "const double *al = alpha + (int64_t)(l) * N;"),
    "grad_mu_sign": ("-p[j] / (1.0 - mu_at(m, l));", "p[j] / (1.0 - mu_at(m, l));"),
    "distance_not_halved": ("return -log(q) / 2.0;", "return -log(q);"),
    "posterior_not_normalised": ("p[j] = alpha[j] * beta[j] / Z;", "p[j] = alpha[j] * beta[j];"),
}


# mistakes in the recombination map (eq. rho) and its chain rule, caught by
# the map's own pins
RHO_MAP_MUTANTS = {
    "calc_rho_no_morgan_conversion": ("double m = cM[l] / 100.0;\n        rho[l]",
                                      "double m = cM[l];\n        rho[l]"),
    "rho_map_grad_drops_log": ("s * mg * log(m) * e", "s * mg * e"),
    "rho_map_grad_s_sign": ("gs += grad_rho[l] * mg * e;", "gs -= grad_rho[l] * mg * e;"),
}
# mistakes in the per-variant mu and prior-matrix paths, caught by the
# enumeration pins under a random rational prior and a per-variant mu
VARIANT_MUTANTS = {
    "prior_transposed": ("return m->Pi ? m->Pi[(int64_t)i * m->N + j]",
                         "return m->Pi ? m->Pi[(int64_t)j * m->N + i]"),
    "mu_of_previous_variant": ("    double mu = mu_at(m, l);", "    double mu = mu_at(m, l > 0 ? l - 1 : 0);"),
    "grad_mu_l_cumulative": ("            grad_mu_l[l] = gl;", "            grad_mu_l[l] = gmu;"),
    "backward_norm_uniform_prior": ("g += prior(m, j, i) * theta(m, l, j, i) * beta[j];",
                                    "g += (j == i ? 0.0 : theta(m, l, j, i) * beta[j] / (double)(m->N - 1));"),
}
# mistakes in the eps floor and the zero-total rule of the posterior (eq.
# postprob, eq. distmat), caught by the floor pins
FLOOR_MUTANTS = {
    "eps_single_precision": ("#define LSO_EPS 2.220446049250313080847e-16",
                             "#define LSO_EPS 1.1920928955078125e-07"),
    "zero_sum_branch_dropped": ("        else if (Z == 0.0)\n            p[j] = LSO_EPS;\n", ""),
    "zero_sum_gives_zero": ("            p[j] = LSO_EPS;\n        else", "            p[j] = 0.0;\n        else"),
    "floor_not_applied": ("double q = (p < LSO_EPS) ? LSO_EPS : p;", "double q = p;"),
}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")


def _rho_map_pins_pass(lib) -> bool:
    import json
    pairs = json.load(open(GOLDEN))["calc_rho"]["pairs"]
    return rho_map_checks(lambda c, s, g: oracle.calc_rho(c, s, g, lib=lib),
                          lambda c, s, g, gr: oracle.rho_map_grad(c, s, g, gr, lib=lib), pairs)


def _floor_pins_pass(lib) -> bool:
    def run(h01, rho, mu, rec, tg):
        L, N = h01.shape
        return oracle.run_pass(pack_haplotypes(h01), N, L, rho, mu, rec, tg, want=("P", "E"),
                               nthreads=1, lib=lib)
    return floor_checks(run)


def _build_mutant(tmp_path, name, find, repl):
    src = open(SRC).read()
    assert src.count(find) == 1, f"mutation {name!r} does not match the oracle source exactly once"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(find, repl))
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                    "-o", str(so), str(path), "-lm"], check=True)
    return oracle.bind(str(so))


def _pins_pass(lib) -> bool:
    """The exact-enumeration pins, as in test_oracle_pins, on two cases."""
    cases = [(5, 4, 1, Fraction(1, 16), [3, 17, 1, 29]), (4, 3, 3, Fraction(1, 4), [9, 2, 20])]
    for L, N, seed, mu, rnum in cases:
        h01 = (np.random.default_rng(seed).random((L, N)) < 0.5).astype(np.uint8)
        rho = [Fraction(k, 32) for k in rnum]
        rf = np.array([float(r) for r in rho])
        rec = np.arange(N, dtype=np.int32)
        tg = np.arange(L, dtype=np.int32)
        H = pack_haplotypes(h01)
        res = oracle.run_pass(H, N, L, rf, float(mu), rec, tg, want=("P", "E"), nthreads=1, lib=lib)
        gr = oracle.run_gradient(H, N, L, rf, float(mu), rec, nthreads=1, lib=lib)
        for i in range(N):
            ex = enumerate_exact(h01.tolist(), rho, mu, i)
            logP = np.log(float(ex["P"]))
            post = np.array([[float(x) for x in row] for row in ex["post"]])
            eps = 2.0 ** -52
            Eref = -np.log(np.maximum(post, eps)) / 2
            Eref[:, i] = 0.0
            ok = (abs(res["llf"][i] - logP) <= 1e-12 * abs(logP)
                  and abs(res["llb"][i] - logP) <= 1e-12 * abs(logP)
                  and np.allclose(res["P"][:, i, :], post, rtol=1e-11, atol=1e-15)
                  and np.allclose(res["E"][:, i, :], Eref, rtol=1e-11, atol=1e-15)
                  and np.allclose(gr["grad_rho"][i], [float(x) for x in ex["dlogP_drho"]],
                                  rtol=1e-9, atol=1e-12)
                  and abs(gr["grad_mu"][i] - float(ex["dlogP_dmu"]))
                  <= 1e-9 * abs(float(ex["dlogP_dmu"])) + 1e-9)
            if not ok:
                return False
    return True


def _variant_pins_pass(lib) -> bool:
    """Enumeration pins with a random rational prior matrix and a mutation
    probability per variant: posteriors, both likelihoods, d/d rho and
    d/d mu^l."""
    L, N = 5, 4
    h01 = (np.random.default_rng(21).random((L, N)) < 0.5).astype(np.uint8)
    W = np.random.default_rng(21).integers(1, 10, size=(N, N))
    Pi = [[Fraction(0)] * N for _ in range(N)]
    for i in range(N):
        tot = sum(int(W[j, i]) for j in range(N) if j != i)
        for j in range(N):
            if j != i:
                Pi[j][i] = Fraction(int(W[j, i]), tot)
    Pf = np.array([[float(x) for x in row] for row in Pi])
    rho = [Fraction(k, 32) for k in (3, 17, 1, 29)]
    mu = [Fraction(k, 32) for k in (1, 3, 2, 8, 1)]
    rf, mf = np.array([float(r) for r in rho]), np.array([float(m) for m in mu])
    H, rec, tg = pack_haplotypes(h01), np.arange(N, dtype=np.int32), np.arange(L, dtype=np.int32)
    res = oracle.run_pass(H, N, L, rf, mf, rec, tg, want=("P",), nthreads=1, lib=lib, prior=Pf)
    gr = oracle.run_gradient(H, N, L, rf, mf, rec, nthreads=1, lib=lib, prior=Pf)
    for i in range(N):
        ex = enumerate_exact(h01.tolist(), rho, mu, i, prior=Pi)
        logP = np.log(float(ex["P"]))
        post = np.array([[float(x) for x in row] for row in ex["post"]])
        ok = (abs(res["llf"][i] - logP) <= 1e-12 * abs(logP)
              and abs(res["llb"][i] - logP) <= 1e-12 * abs(logP)
              and np.allclose(res["P"][:, i, :], post, rtol=1e-11, atol=1e-15)
              and np.allclose(gr["grad_rho"][i], [float(x) for x in ex["dlogP_drho"]],
                              rtol=1e-9, atol=1e-12)
              and np.allclose(gr["grad_mu_l"][i], [float(x) for x in ex["dlogP_dmu_l"]],
                              rtol=1e-9, atol=1e-9))
        if not ok:
            return False
    return True


@pytest.mark.parametrize("name", sorted(VARIANT_MUTANTS))
def test_variant_pins_catch_mutant(tmp_path, name):
    find, repl = VARIANT_MUTANTS[name]
    lib = _build_mutant(tmp_path, name, find, repl)
    assert not _variant_pins_pass(lib), f"pins did not catch mutant {name}"


def test_unmutated_copy_passes(tmp_path):
    lib = _build_mutant(tmp_path, "identity", "LSO_EPS 2.220446049250313080847e-16",
                        "LSO_EPS 2.220446049250313080847e-16")
    assert _pins_pass(lib)
    assert _rho_map_pins_pass(lib)
    assert _variant_pins_pass(lib)
    assert _floor_pins_pass(lib)


@pytest.mark.parametrize("name", sorted(FLOOR_MUTANTS))
def test_floor_pins_catch_mutant(tmp_path, name):
    find, repl = FLOOR_MUTANTS[name]
    lib = _build_mutant(tmp_path, name, find, repl)
    assert not _floor_pins_pass(lib), f"pins did not catch mutant {name}"


@pytest.mark.parametrize("name", sorted(RHO_MAP_MUTANTS))
def test_rho_map_pins_catch_mutant(tmp_path, name):
    find, repl = RHO_MAP_MUTANTS[name]
    lib = _build_mutant(tmp_path, name, find, repl)
    assert not _rho_map_pins_pass(lib), f"pins did not catch mutant {name}"


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    find, repl = MUTANTS[name]
    lib = _build_mutant(tmp_path, name, find, repl)
    assert not _pins_pass(lib), f"pins did not catch mutant {name}"
