"""Pins for the clustering and standardisation oracle (oracle/ls_cluster.c):
average pairwise linkage (section 6) against a hand-worked example, the
definition (mean of the pairwise distances between the merged clusters),
scipy's average linkage, its own O(N^3) scan, and hand-worked ties; the
standardised distance column (section 2.2) against numpy and the
zero-deviation rule; planted mistakes are rejected. CPU only."""

from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(oracle.__file__), "ls_cluster.c")


def _rand_points(N, seed, dim=3):
    rng = np.random.default_rng(seed)
    X = rng.random((N, dim))
    return np.sqrt(((X[:, None] - X[None]) ** 2).sum(-1))


def _tie_matrix(N, seed, levels=4):
    """Symmetric matrix of small integers: many exact ties at every level."""
    rng = np.random.default_rng(seed)
    A = rng.integers(1, levels + 1, size=(N, N)).astype(np.float64)
    D = np.triu(A, 1)
    D = D + D.T
    return D


# --------------------------------------------------------------------------
# average linkage

def test_hand_worked_example():
    """Five taxa worked by hand: (a,b) at 2; (d,e) at 3; c with (d,e) at
    (4+5)/2; then (a,b) with (c,d,e) at the mean of the six cross distances,
    47/6."""
    d = {(0, 1): 2, (0, 2): 6, (0, 3): 10, (0, 4): 9, (1, 2): 5, (1, 3): 9, (1, 4): 8,
         (2, 3): 4, (2, 4): 5, (3, 4): 3}
    D = np.zeros((5, 5))
    for (i, j), v in d.items():
        D[i, j] = D[j, i] = v
    Z, order = oracle.average_linkage(D)
    expect = np.array([[0, 1, 2, 2], [3, 4, 3, 2], [2, 6, 4.5, 3], [5, 7, 47 / 6, 5]])
    np.testing.assert_allclose(Z, expect, rtol=1e-15, atol=0)
    assert order.tolist() == [0, 1, 2, 3, 4]


def test_ties_take_the_smallest_slots():
    """All distances equal: slot 0 absorbs slot 1, then slot 2, then slot 3
    (the reading for ties: the pair with the smallest slot, then the smallest
    partner)."""
    D = np.ones((4, 4))
    Z, order = oracle.average_linkage(D)
    assert Z.tolist() == [[0, 1, 1, 2], [2, 4, 1, 3], [3, 5, 1, 4]]
    # leaf order: root 6 = (3, 5), 5 = (2, 4), 4 = (0, 1): smaller id first
    assert order.tolist() == [3, 2, 0, 1]


def test_two_groups_with_ties():
    """Two groups of three at distance 1 inside and 5 across: the first
    group merges first (slots 0-2), then the second (slots 3-5), then the
    two at 5."""
    D = np.full((6, 6), 5.0)
    D[:3, :3] = 1.0
    D[3:, 3:] = 1.0
    np.fill_diagonal(D, 0.0)
    Z, _ = oracle.average_linkage(D)
    assert Z.tolist() == [[0, 1, 1, 2], [2, 6, 1, 3], [3, 4, 1, 2], [5, 8, 1, 3],
                          [7, 9, 5, 6]]


def _leaves(Z, N, c):
    if c < N:
        return [c]
    z = Z[c - N]
    return _leaves(Z, N, int(z[0])) + _leaves(Z, N, int(z[1]))


@pytest.mark.parametrize("N,seed", [(12, 1), (40, 2), (90, 3)])
def test_merge_heights_are_mean_pairwise_distances(N, seed):
    """The definition: each merge height is the mean of d(a, b) over the
    leaves of the two clusters, from the original matrix (brute force)."""
    D = _rand_points(N, seed)
    Z, order = oracle.average_linkage(D)
    for m in range(N - 1):
        A = _leaves(Z, N, int(Z[m, 0]))
        B = _leaves(Z, N, int(Z[m, 1]))
        assert Z[m, 3] == len(A) + len(B)
        mean = D[np.ix_(A, B)].mean()
        assert abs(Z[m, 2] - mean) <= 1e-13 * mean
    assert sorted(order.tolist()) == list(range(N))
    assert np.all(np.diff(Z[:, 2]) >= -1e-12)  # average linkage is monotone


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("N,seed", [(2, 0), (3, 1), (25, 2), (150, 3), (400, 4)])
def test_matches_scipy_average_linkage(dtype, N, seed):
    """scipy's average linkage (FP64) on distances without ties: the same
    merges and sizes, heights within the precision of D."""
    from scipy.cluster.hierarchy import linkage
    from scipy.spatial.distance import squareform
    D = _rand_points(N, seed).astype(dtype)
    Z, _ = oracle.average_linkage(D)
    Zs = linkage(squareform(D.astype(np.float64), checks=False), "average")
    assert np.array_equal(Z[:, [0, 1, 3]], Zs[:, [0, 1, 3]])
    tol = 1e-13 if dtype == np.float64 else 2e-6
    np.testing.assert_allclose(Z[:, 2], Zs[:, 2], rtol=tol, atol=0)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("maker,N,seed", [(_rand_points, 60, 5), (_tie_matrix, 60, 6),
                                          (_tie_matrix, 150, 7), (_rand_points, 200, 8)])
def test_nearest_slot_bookkeeping_equals_full_scan(dtype, maker, N, seed):
    """The O(N^2) evaluation gives the O(N^3) scan's merges bit for bit,
    including on matrices full of ties."""
    D = maker(N, seed).astype(dtype)
    Z1, o1 = oracle.average_linkage(D)
    Z2, o2 = oracle.average_linkage(D, naive=True)
    assert np.array_equal(Z1, Z2)
    assert np.array_equal(o1, o2)


def test_nan_distances_merge_last():
    """A NaN distance (a recipient column of a total underflow) comes after
    every number; NaN pairs among themselves by slot."""
    D = np.array([[0, 1, np.nan, 4], [1, 0, np.nan, 2], [np.nan, np.nan, 0, np.nan],
                  [4, 2, np.nan, 0]], dtype=np.float64)
    Z, order = oracle.average_linkage(D)
    assert Z[0].tolist() == [0, 1, 1, 2]
    assert Z[1].tolist() == [3, 4, 3, 3]
    assert Z[2, 0] == 2 and Z[2, 1] == 5 and np.isnan(Z[2, 2]) and Z[2, 3] == 4
    Zn, _ = oracle.average_linkage(D, naive=True)
    assert np.array_equal(Z, Zn, equal_nan=True)


def test_input_not_modified_and_sizes():
    D = _rand_points(30, 9).astype(np.float32)
    D0 = D.copy()
    Z, order = oracle.average_linkage(D)
    assert np.array_equal(D, D0)
    assert Z.shape == (29, 4) and order.shape == (30,)
    Z1, o1 = oracle.average_linkage(np.zeros((1, 1)))
    assert Z1.shape == (0, 4) and o1.tolist() == [0]


# --------------------------------------------------------------------------
# standardisation

def test_standardise_matches_numpy():
    rng = np.random.default_rng(3)
    e = rng.random(50) * 10
    i = 7
    z = oracle.standardise(e, i)
    donors = np.arange(50) != i
    ref = (e[donors] - e[donors].mean()) / e[donors].std(ddof=0)
    np.testing.assert_allclose(z[donors], ref, rtol=1e-13, atol=1e-14)
    assert z[i] == 0.0
    assert abs(z[donors].mean()) < 1e-13 and abs(z[donors].std(ddof=0) - 1) < 1e-13


def test_standardise_zero_deviation_gives_zeros():
    """Section 2.2: a column whose distances are all equal (the zero-total
    case, every p_ji = eps) standardises to 0."""
    e = np.full(9, 26 * np.log(2.0))
    e[4] = 0.0  # the recipient's own entry
    assert np.all(oracle.standardise(e, 4) == 0.0)
    e = np.full(1000, 0.1)  # a value whose rounded mean differs from it
    assert np.all(oracle.standardise(e, 0) == 0.0)
    e2 = np.array([1.0, np.nan, 2.0])
    assert np.isnan(oracle.standardise(e2, 0)[2])


def test_standardise_affine_invariance():
    rng = np.random.default_rng(4)
    e = rng.random(20)
    np.testing.assert_allclose(oracle.standardise(3.5 * e + 2.0, 3), oracle.standardise(e, 3),
                               rtol=1e-12, atol=1e-13)


# --------------------------------------------------------------------------
# planted mistakes

MUTANTS = {
    "unweighted_update": ("T s = t + u;", "T s = D[(int64_t)a * N + k] + D[(int64_t)b * N + k];"),
    "update_wrong_divisor": ("T d = s / n;", "T d = s / (na + nb + 1);"),
    "tie_takes_larger_slot": ("return p1 < p2 || (p1 == p2 && q1 < q2);",
                              "return p1 > p2 || (p1 == p2 && q1 > q2);"),
    "nan_first": ("            return n2;", "            return n1;"),
    "nn_not_rescanned": ("if (nn[k] == a || nn[k] == b) {", "if (nn[k] == b) {"),
    "leaf_order_swapped": ("stack[top++] = (int32_t)z[1]; /* right", "stack[top++] = (int32_t)z[0]; /* right"),
    "standardise_sample_sd": ("double sd = sqrt(v / (double)(N - 1));",
                              "double sd = sqrt(v / (double)(N - 2));"),
    "standardise_no_zero_rule": ("(j == i || all_equal) ? 0.0", "(j == i) ? 0.0"),
}


def _build_mutant(tmp_path, name, find, repl):
    src = open(SRC).read()
    assert src.count(find) >= 1, f"mutation {name!r} does not match the source"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(find, repl))
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(so), str(path), "-lm"], check=True)
    import ctypes
    lib = ctypes.CDLL(str(so))
    P, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.lso_average_linkage.argtypes = [P, i32, i32, i32, P, P]
    lib.lso_standardise.argtypes = [P, i32, i32, P]
    lib.lso_standardise.restype = None
    return lib


def _pins_pass(lib) -> bool:
    tests = [test_hand_worked_example, test_ties_take_the_smallest_slots,
             test_two_groups_with_ties, test_nan_distances_merge_last,
             test_standardise_matches_numpy,
             test_standardise_zero_deviation_gives_zeros]
    saved = oracle._lib
    try:
        oracle._lib = lib
        for t in tests:
            try:
                t()
            except (AssertionError, ValueError):
                return False
        try:
            test_merge_heights_are_mean_pairwise_distances(40, 2)
            for maker, N, seed in ((_tie_matrix, 60, 6), (_rand_points, 60, 5)):
                test_nearest_slot_bookkeeping_equals_full_scan(np.float32, maker, N, seed)
        except AssertionError:
            return False
    finally:
        oracle._lib = saved
    return True


def test_unmutated_copy_passes(tmp_path):
    lib = _build_mutant(tmp_path, "identity", "#include <math.h>", "#include <math.h>")
    assert _pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    find, repl = MUTANTS[name]
    lib = _build_mutant(tmp_path, name, find, repl)
    assert not _pins_pass(lib), f"pins did not catch mutant {name}"
