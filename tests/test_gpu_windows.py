"""Recipient windows writing into resident N x N distance matrices (section
3.9; the strided outputs of ls_forward), against the FP64 oracle and against
the contiguous path, through the C ABI (libls.so)."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from lsinputs import make_inputs, seeded_recipients

from _gpu import F32_POST_ATOL, F64_ATOL_LOG, F64_RTOL, need_gpu, rel_close
from test_gpu_parity import _random_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    need_gpu()
    import paper_2212_11403_amd as m
    m.load()
    return m


def _np(t):
    return t.double().cpu().numpy()


@pytest.mark.parametrize("N,L,window", [(700, 120, 128), (257, 60, 100), (130, 40, 130)])
def test_windowed_distances_fp64_vs_oracle(ls, N, L, window):
    H, rho, mu = _random_case(N, L, seed=N + L)
    targets = np.array([3, L // 2, L - 2], np.int32)
    m = ls.Model(H, N, rho, mu)
    out = ls.distance_matrices(m, targets, "fp64", window=window)
    Dref = oracle.distances(H, N, L, rho, mu, targets)
    rel_close(_np(out["D"]), Dref, F64_RTOL, F64_ATOL_LOG)
    ref = oracle.run_pass(H, N, L, rho, mu, np.arange(N, dtype=np.int32), targets, want=())
    rel_close(_np(out["loglik"]), ref["llf"], F64_RTOL, F64_ATOL_LOG)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_windowed_equals_one_window(ls, prec):
    """Windows of 96 recipients give the same bits as all recipients in one
    launch (the same kernels, shapes and summation order per recipient)."""
    N, L = 600, 150
    H, rho, mu = _random_case(N, L, seed=17)
    targets = np.array([10, 70, 140], np.int32)
    m = ls.Model(H, N, rho, mu)
    a = ls.distance_matrices(m, targets, prec, window=96)
    b = ls.distance_matrices(m, targets, prec, window=0)
    import torch
    assert torch.equal(a["D"], b["D"])
    assert torch.equal(a["loglik"], b["loglik"])
    r = ls.decode(m, targets, prec, want=("E",))
    E = r["E"]
    ls.distance_symmetrise(E, E, prec)
    assert torch.equal(a["D"], E)


@pytest.mark.parametrize("pad", [8, 5])
def test_strided_outputs_leave_padding_alone(ls, pad):
    """P and E rows at a row stride of N + pad and a target stride larger
    than the window: every row equals the contiguous output (bit for bit when
    the stride keeps 16-byte rows, so that the same posterior kernel runs;
    within FP32 rounding otherwise), and the padding keeps its sentinel."""
    import torch
    N, L, R = 200, 50, 37
    H, rho, mu = _random_case(N, L, seed=3)
    targets = np.array([7, 30], np.int32)
    rec = np.arange(50, 50 + R, dtype=np.int32)
    m = ls.Model(H, N, rho, mu)
    ref = ls.decode(m, targets, "fp32", recipients=rec, want=("P", "E"))
    rs, ts = N + pad, (R + 3) * (N + pad)
    T = len(targets)
    P = torch.full((T * ts,), float("nan"), dtype=torch.float32, device="cuda")
    E = torch.full((T * ts,), float("nan"), dtype=torch.float32, device="cuda")
    fwd = ls.Table(m, 0, "fp32", rec)
    ls.forward(fwd, m, L - 1, targets, ref["bsnap"], P, E, out_strides=(ts, rs))
    for k in range(T):
        blk_p = P[k * ts:(k + 1) * ts].view(R + 3, rs)
        blk_e = E[k * ts:(k + 1) * ts].view(R + 3, rs)
        if pad % 4 == 0:
            assert torch.equal(blk_p[:R, :N], ref["P"][k])
            assert torch.equal(blk_e[:R, :N], ref["E"][k])
        else:
            torch.testing.assert_close(blk_p[:R, :N], ref["P"][k], rtol=1e-5, atol=1e-12)
            torch.testing.assert_close(blk_e[:R, :N], ref["E"][k], rtol=1e-5, atol=1e-6)
        assert torch.isnan(blk_p[:R, N:]).all() and torch.isnan(blk_p[R:]).all()
        assert torch.isnan(blk_e[:R, N:]).all() and torch.isnan(blk_e[R:]).all()


def test_overlapping_strides_rejected(ls):
    import torch
    N, L = 100, 20
    H, rho, mu = _random_case(N, L, seed=4)
    m = ls.Model(H, N, rho, mu)
    fwd = ls.Table(m, 0, "fp32", np.arange(4, dtype=np.int32))
    bs = torch.zeros((2, 4, N), dtype=torch.float32, device="cuda")
    E = torch.zeros(10 * N * 4, dtype=torch.float32, device="cuda")
    for strides in ((0, N - 1), (3 * N, N), (-N, N)):
        with pytest.raises(ls.LsError) as ei:
            ls.forward(fwd, m, L - 1, [5, 9], bs, None, E, out_strides=strides)
        assert ei.value.code == 2  # LS_ERR_SHAPE
    assert fwd.l == -1


def test_large_workload_window_sampled(ls):
    """The large single-GPU workload's decode path (N = 100,000, L = 10,000,
    5 targets) on a window of 16 seeded recipients written into rows of
    full-width matrices at their own indices: FP32 posteriors against the
    FP64 oracle."""
    import torch
    x = make_inputs("c5")
    N, L, targets = x["N"], x["L"], x["targets"]
    rec = np.sort(seeded_recipients(N, 16, seed=555)).astype(np.int32)
    m = ls.Model(x["H"], N, x["rho"], x["mu"])
    r = ls.decode(m, targets, "fp32", recipients=rec, want=("P",))
    ref = oracle.run_pass(x["H"], N, L, x["rho"], x["mu"], rec, targets, want=("P",))
    err = np.abs(_np(r["P"]) - ref["P"]).max()
    print(f"c5 window: max abs posterior error {err:.3e}")
    assert err <= F32_POST_ATOL
