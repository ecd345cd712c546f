"""Average pairwise linkage (section 6) and standardised half-distance rows
(section 2.2) on the GPU against the oracle, through the C ABI (libls.so).

Merges, sizes and heights must equal the oracle's bit for bit: both take
every decision on the same FP32 (or FP64) values with the same update and
tie rule."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from lsinputs import make_inputs

from _gpu import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    need_gpu()
    import paper_2212_11403_amd as m
    m.load()
    return m


def _points(N, seed, dtype):
    rng = np.random.default_rng(seed)
    X = rng.random((N, 3))
    return np.sqrt(((X[:, None] - X[None]) ** 2).sum(-1)).astype(dtype)


def _ties(N, seed, dtype, levels=4):
    rng = np.random.default_rng(seed)
    A = np.triu(rng.integers(1, levels + 1, size=(N, N)).astype(np.float64), 1)
    return (A + A.T).astype(dtype)


def _gpu_linkage(ls, mats, dtype):
    import torch
    D = torch.from_numpy(np.ascontiguousarray(np.stack(mats))).cuda()
    Z, order = ls.average_linkage(D)
    torch.cuda.synchronize()
    return Z.cpu().numpy(), order.cpu().numpy()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_small_matrices_vs_oracle(ls, dtype):
    """Random and tie-heavy matrices of several sizes (one workgroup each)."""
    for N, mats in [(2, [_points(2, 0, dtype)]), (3, [_ties(3, 1, dtype)]),
                    (65, [_points(65, 2, dtype), _ties(65, 3, dtype), _ties(65, 4, dtype, 2)]),
                    (700, [_points(700, 5, dtype), _ties(700, 6, dtype, 8)])]:
        Z, order = _gpu_linkage(ls, mats, dtype)
        for t, D in enumerate(mats):
            Zr, orr = oracle.average_linkage(D)
            assert np.array_equal(Z[t], Zr), (N, t)
            assert np.array_equal(order[t], orr), (N, t)


def test_hand_worked_and_nan(ls):
    d = {(0, 1): 2, (0, 2): 6, (0, 3): 10, (0, 4): 9, (1, 2): 5, (1, 3): 9, (1, 4): 8,
         (2, 3): 4, (2, 4): 5, (3, 4): 3}
    D = np.zeros((5, 5))
    for (i, j), v in d.items():
        D[i, j] = D[j, i] = v
    Z, order = _gpu_linkage(ls, [D], np.float64)
    np.testing.assert_allclose(Z[0], [[0, 1, 2, 2], [3, 4, 3, 2], [2, 6, 4.5, 3],
                                      [5, 7, 47 / 6, 5]], rtol=1e-15, atol=0)
    assert order[0].tolist() == [0, 1, 2, 3, 4]
    Dn = np.array([[0, 1, np.nan, 4], [1, 0, np.nan, 2], [np.nan, np.nan, 0, np.nan],
                   [4, 2, np.nan, 0]], dtype=np.float32)
    Z, _ = _gpu_linkage(ls, [Dn], np.float32)
    Zr, _ = oracle.average_linkage(Dn)
    assert np.array_equal(Z[0], Zr, equal_nan=True)


@pytest.fixture(scope="module")
def c1_D(ls):
    """The small workload's ten FP32 distance matrices (decoded on the GPU
    and symmetrised), as the clustering input."""
    x = make_inputs("c1")
    m = ls.Model(x["H"], x["N"], x["rho"], x["mu"])
    out = ls.distance_matrices(m, x["targets"], "fp32")
    return out["D"].cpu().numpy()


def test_small_workload_distance_matrices(ls, c1_D):
    """All ten matrices of the small workload (N = 200): every merge and the
    leaf order equal the oracle's."""
    Z, order = _gpu_linkage(ls, list(c1_D), np.float32)
    for t in range(c1_D.shape[0]):
        Zr, orr = oracle.average_linkage(c1_D[t])
        assert np.array_equal(Z[t], Zr), t
        assert np.array_equal(order[t], orr), t


def test_benchmark_workload_distance_matrices(ls):
    """Three of the benchmark workload's matrices (N = 10,000, FP32, from the
    GPU decode of all recipients at three of its targets): every merge, its
    height and size, and the leaf order equal the oracle's."""
    import torch
    x = make_inputs("c2")
    m = ls.Model(x["H"], x["N"], x["rho"], x["mu"])
    tg = x["targets"][[0, 50, 99]]
    out = ls.distance_matrices(m, tg, "fp32")
    D = out["D"]
    Dh = D.cpu().numpy()
    Z, order = ls.average_linkage(D)
    torch.cuda.synchronize()
    Z, order = Z.cpu().numpy(), order.cpu().numpy()
    for t in range(len(tg)):
        Zr, orr = oracle.average_linkage(Dh[t])
        assert np.array_equal(Z[t], Zr), t
        assert np.array_equal(order[t], orr), t


def test_state_in_global_memory(ls):
    """A matrix whose per-slot state does not fit a workgroup's local memory
    (FP64, N = 13,000: 13 bytes per slot) runs the merge kernel with that
    state in the workspace; merges and order equal the oracle's."""
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(13)
    X = rng.random((13_000, 3))
    D = cdist(X, X)
    Z, order = _gpu_linkage(ls, [D], np.float64)
    Zr, orr = oracle.average_linkage(D)
    assert np.array_equal(Z[0], Zr)
    assert np.array_equal(order[0], orr)


def test_smaller_workgroups(ls, monkeypatch):
    """The merge kernel at 256 and 64 threads per matrix (LS_LINKAGE_THREADS)
    gives the same merges as the oracle."""
    mats = [_points(700, 21, np.float32), _ties(700, 22, np.float32, 8)]
    for th in ("256", "64"):
        monkeypatch.setenv("LS_LINKAGE_THREADS", th)
        Z, order = _gpu_linkage(ls, mats, np.float32)
        for t, D in enumerate(mats):
            Zr, orr = oracle.average_linkage(D)
            assert np.array_equal(Z[t], Zr), (th, t)
            assert np.array_equal(order[t], orr), (th, t)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_standardised_rows_vs_oracle(ls, prec):
    """Half-distance rows of the small workload standardised in place, in the
    strided layout of a window; plus a zero-total row (every entry equal)."""
    import torch
    x = make_inputs("c1")
    N, L = x["N"], x["L"]
    rec = np.arange(40, 90, dtype=np.int32)
    m = ls.Model(x["H"], N, x["rho"], x["mu"])
    r = ls.decode(m, x["targets"][:3], prec, recipients=rec, want=("E",))
    E = r["E"]
    E[1, 7] = 26.0 * float(np.log(2.0))
    E[1, 7, rec[7]] = 0.0
    Eh = E.double().cpu().numpy()
    ls.standardise_rows(E, rec)
    Z = E.double().cpu().numpy()
    tol = 1e-13 if prec == "fp64" else 2e-6
    for k in range(3):
        for q, i in enumerate(rec):
            ref = oracle.standardise(Eh[k, q], int(i))
            np.testing.assert_allclose(Z[k, q], ref, rtol=tol, atol=tol)
    assert np.all(Z[1, 7] == 0.0)
    # strided: rows of a [T][R + 2][N + 4] buffer
    buf = torch.full((3, len(rec) + 2, N + 4), 7.0, dtype=E.dtype, device="cuda")
    buf[:, :len(rec), :N] = torch.from_numpy(Eh).to(E.dtype).cuda()
    ls.standardise_rows(buf, rec, out_strides=((len(rec) + 2) * (N + 4), N + 4), N=N)
    assert torch.equal(buf[:, :len(rec), :N], E)
    assert bool((buf[:, :len(rec), N:] == 7.0).all()) and bool((buf[:, len(rec):] == 7.0).all())
