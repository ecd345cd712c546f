"""The C ABI library loads and exports every symbol include/ls.h declares.
CPU only: no call here reaches the GPU (validation errors return before any
HIP call, and the shape query is host arithmetic)."""

from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ls.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2212_11403_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2212_11403_amd.build import build
        build()
    return _lib.load()


def test_header_and_binding_agree(lib):
    from paper_2212_11403_amd import _lib
    assert _declared() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    from paper_2212_11403_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in _declared():
        assert name in syms, name
        assert getattr(lib, name) is not None


def test_struct_layouts_match_header():
    from paper_2212_11403_amd._lib import LsModel, LsTable
    assert ctypes.sizeof(LsModel) == 88
    assert ctypes.sizeof(LsTable) == 56
    # the optional fields follow the ones ls_model_init sets, in header order
    assert LsModel.mu_vec.offset == 72 and LsModel.prior.offset == 80


def test_host_only_calls(lib):
    assert lib.ls_version().decode().startswith("libls")
    assert lib.ls_status_string(0).decode() == "ok"
    assert lib.ls_status_string(16).decode().startswith("a column sum")
    assert lib.ls_status_string(4).decode().startswith("N too large")
    assert lib.ls_model_workspace_bytes(1, 10) == 0
    # internal rows: two copies of floor(N/64) words plus the partial word,
    # padded to 64 B, the whole rounded up to 256 B; then five tables of L
    # FP32 coefficient pairs; then the emission tables of a per-variant mu
    # (L FP64 pairs, L FP32 pairs, L + 1 FP64 prefix sums)
    def emis(L):
        return L * 16 + L * 8 + (L + 1) * 8
    # and the [N][2] checks of a prior matrix
    assert lib.ls_model_workspace_bytes(200, 10) == 768 + 5 * 10 * 2 * 4 + emis(10) + 16 * 200
    assert lib.ls_model_workspace_bytes(10000, 3) == 7680 + 5 * 3 * 2 * 4 + emis(3) + 16 * 10000


def test_validation_errors_before_any_device_work(lib):
    from paper_2212_11403_amd._lib import LsModel, LsTable
    assert lib.ls_model_init(None, None, 0, None) == 1
    m = LsModel()
    m.N, m.L = 1, 5
    assert lib.ls_model_init(ctypes.byref(m), None, 0, None) == 1
    t = LsTable()
    assert lib.ls_forward(None, ctypes.byref(m), 0, None, 0, None, None, None, 0, 0, None) == 1
    assert lib.ls_forward(ctypes.byref(t), None, 0, None, 0, None, None, None, 0, 0, None) == 1
    assert lib.ls_table_init(ctypes.byref(t), 2, 1, None, None, None, None, 0, None) == 1
    assert lib.ls_distance_symmetrise(None, None, 3, 1, 1, None) == 1
    assert lib.ls_status_check(None, 1, None) == 1


def test_kernel_shapes_cover_every_size(lib):
    """Every N up to the per-precision limit gets a shape that places all
    donor words (host arithmetic only)."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    # FP64 without a prior reaches 53,248 (104 slots x 8 waves); with a prior
    # column every precision keeps half its plain limit (FP64: 22,500)
    limits = {0: 53248, 1: 100000, 2: 100000}
    for prec, nmax in limits.items():
        for prior in (0, 1):
            top = nmax if not prior else (22500 if prec == 0 else nmax // 2)
            for N in list(range(2, 3000, 1 + 6 * prior)) + list(range(3000, top + 1, 997)) + [top]:
                rc = lib.ls_kernel_shape(N, prec, prior, ctypes.byref(a), ctypes.byref(b))
                assert rc == 0, (prec, prior, N)
                ns, nw = a.value, b.value
                K = min(ns, 4)
                NW, NF = (N + 63) // 64, N // 64
                assert nw * (ns - K) <= NF and nw * ns >= NW, (prec, prior, N, ns, nw)
    assert lib.ls_kernel_shape(1, 1, 0, ctypes.byref(a), ctypes.byref(b)) == 1
    assert lib.ls_kernel_shape(100, 7, 0, ctypes.byref(a), ctypes.byref(b)) == 1


@pytest.mark.parametrize("N,L,R", [(2000, 50_000, 2000), (10_000, 100_000, 64), (300, 5000, 300)])
def test_gradient_workspace_size(lib, N, L, R):
    """ls_loglik_grad_workspace_bytes against the size the header states,
    e R N (1.5 sqrt(L) + 3) + 8 R L bytes, within 2% (alignment and the
    rounding of the segment length make up the rest). The query only reads
    N, L and the model's validity fields, so a host-side struct serves."""
    from paper_2212_11403_amd._lib import LsModel
    m = LsModel()
    m.N, m.L, m.hash, m.Hr = N, L, 1, 1
    for prec, e in ((0, 8), (1, 4)):
        got = lib.ls_loglik_grad_workspace_bytes(ctypes.byref(m), R, prec)
        est = e * R * N * (1.5 * L ** 0.5 + 3) + 8 * R * L
        assert abs(got - est) <= 0.02 * est, (prec, got, est)
    m.hash = 0
    assert lib.ls_loglik_grad_workspace_bytes(ctypes.byref(m), R, 1) == 0
