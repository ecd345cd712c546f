"""The allocation-free linkage entry point (ls_average_linkage_noalloc)
against ls_average_linkage, through the C ABI (libls.so): two calls in a row
on the library's fixed scratch, the second with fewer and smaller matrices
(so the scratch holds the first call's contents), and the size limit."""

from __future__ import annotations

import numpy as np
import pytest

from _gpu import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    need_gpu()
    import paper_2212_11403_amd as m
    m.load()
    return m


def _matrices(T, N, seed, dtype):
    rng = np.random.default_rng(seed)
    P = rng.random((T, N, 3))
    D = np.sqrt(((P[:, :, None, :] - P[:, None, :, :]) ** 2).sum(-1))
    D[:, np.arange(N), np.arange(N)] = 0.0
    # a few exact ties, so that the tie rule is exercised too
    D[:, 1, 2] = D[:, 2, 1] = D[:, 0, 1] = D[:, 1, 0]
    return D.astype(dtype)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_equals_workspace_call(ls, prec):
    import torch
    dtype = np.float64 if prec == "fp64" else np.float32
    for T, N, seed in ((6, 700, 1), (2, 129, 2)):
        print(f"noalloc {prec}: T={T} N={N} seed={seed}", flush=True)
        D = torch.from_numpy(_matrices(T, N, seed, dtype)).cuda()
        Zr, orr = ls.average_linkage(D.clone(), prec)
        Z = torch.empty((T, N - 1, 4), dtype=torch.float64, device="cuda")
        o = torch.empty((T, N), dtype=torch.int32, device="cuda")
        ls.average_linkage_noalloc(D.clone(), Z, o, prec)
        torch.cuda.synchronize()
        assert torch.equal(Z, Zr) and torch.equal(o, orr), (prec, T, N)


def test_noalloc_rejects_oversized_requests(ls):
    import ctypes
    import torch
    from paper_2212_11403_amd import _lib
    lib = _lib.load()
    N, T = 100_000, 20  # about 42 MB of workspace, over the 32 MiB scratch
    assert lib.ls_average_linkage_workspace_bytes(N, T, _lib.LS_FP32) > 32 << 20
    D = torch.empty(1, dtype=torch.float32, device="cuda")  # never read: rejected first
    Z = torch.empty(1, dtype=torch.float64, device="cuda")
    st = lib.ls_average_linkage_noalloc(ctypes.c_void_p(D.data_ptr()), N, T, _lib.LS_FP32,
                                        ctypes.c_void_p(Z.data_ptr()), None, None)
    assert st == _lib.LS_ERR_SCRATCH
    assert "scratch" in lib.ls_status_string(st).decode()
