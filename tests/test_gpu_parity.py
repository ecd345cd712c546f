"""GPU path vs the FP64 oracle, through the C ABI (libls.so)."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from lsinputs import make_inputs, pack_haplotypes, rho_from_spacings

from _gpu import (F16_LOGLIK_RTOL, F16_POST_ATOL, F32_LOGLIK_RTOL, F32_POST_ATOL, F64_ATOL_LOG,
                  F64_ATOL_PROB, F64_RTOL, check_reduced, f64_rtol, forced_shape, need_gpu,
                  rel_close)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ls():
    need_gpu()
    import paper_2212_11403_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def c1():
    return make_inputs("c1")


@pytest.fixture(scope="module")
def c1_ref(c1):
    x = c1
    return oracle.run_pass(x["H"], x["N"], x["L"], x["rho"], x["mu"], np.arange(x["N"]),
                           x["targets"], want=("A", "B", "P", "E", "logF", "logG"))


def _np(t):
    return t.double().cpu().numpy()


def _random_case(N, L, seed, mu=0.01, d_mean=0.05):
    rng = np.random.default_rng(seed)
    # a few founders so that posteriors are not flat
    K = max(2, min(8, N // 3))
    F = (rng.random((L, K)) < 0.4).astype(np.uint8)
    which = rng.integers(0, K, size=(L, N))
    sw = rng.random((L, N)) < 0.05
    base = rng.integers(0, K, size=N)
    idx = np.where(np.cumsum(sw, axis=0) == 0, base[None, :], which)
    h = F[np.arange(L)[:, None], idx]
    flip = rng.random((L, N)) < 0.01
    h = (h ^ flip).astype(np.uint8)
    rho = rho_from_spacings(rng.exponential(d_mean, L - 1))
    return pack_haplotypes(h), rho, mu


# ---------------------------------------------------------------------------
# the small plain-FP64 workload in full

def test_c1_fp64_full_parity(ls, c1, c1_ref):
    x, ref = c1, c1_ref
    m = ls.Model(x["H"], x["N"], x["rho"], x["mu"])
    r = ls.decode(m, x["targets"], "fp64", want=("P", "E"))
    assert ls.status_check(r["fwd"]) == ls.LS_OK
    rel_close(_np(r["P"]), ref["P"], F64_RTOL, F64_ATOL_PROB)
    rel_close(_np(r["E"]), ref["E"], F64_RTOL, F64_ATOL_LOG)
    rel_close(_np(r["bsnap"]), ref["B"], F64_RTOL, F64_ATOL_PROB)
    rel_close(_np(r["fwd"].log_scale), ref["llf"], F64_RTOL, F64_ATOL_LOG)
    # the backward table ends at variant 0: beta^0 and log G^0
    ref0 = oracle.run_pass(x["H"], x["N"], x["L"], x["rho"], x["mu"], np.arange(x["N"]),
                           np.array([0], np.int32), want=("B", "logG"))
    rel_close(_np(r["bck"].state), ref0["B"][0], F64_RTOL, F64_ATOL_PROB)
    rel_close(_np(r["bck"].log_scale), ref0["logG"][0], F64_RTOL, F64_ATOL_LOG)


def test_c1_fp64_tables_at_every_target(ls, c1, c1_ref):
    """alpha^t, beta^t and the log scales of tables stopped at each target."""
    x, ref = c1, c1_ref
    m = ls.Model(x["H"], x["N"], x["rho"], x["mu"])
    fwd = ls.Table(m, 0, "fp64")
    bck = ls.Table(m, 1, "fp64")
    for k, t in enumerate(x["targets"]):
        ls.forward(fwd, m, int(t))
        rel_close(_np(fwd.state), ref["A"][k], F64_RTOL, F64_ATOL_PROB)
        rel_close(_np(fwd.log_scale), ref["logF"][k], F64_RTOL, F64_ATOL_LOG)
    for k in range(len(x["targets"]) - 1, -1, -1):
        ls.backward(bck, m, int(x["targets"][k]))
        rel_close(_np(bck.state), ref["B"][k], F64_RTOL, F64_ATOL_PROB)
        rel_close(_np(bck.log_scale), ref["logG"][k], F64_RTOL, F64_ATOL_LOG)


@pytest.mark.parametrize("prec", ["fp32", "f16"])
def test_c1_reduced_precision(ls, c1, c1_ref, prec):
    x, ref = c1, c1_ref
    m = ls.Model(x["H"], x["N"], x["rho"], x["mu"])
    r = ls.decode(m, x["targets"], prec, want=("P", "E"))
    check_reduced(prec, _np(r["P"]), ref["P"], "prob")
    check_reduced(prec, _np(r["fwd"].log_scale), ref["llf"], "log")


@pytest.mark.parametrize("prec", ["fp32", "f16"])
def test_c1_reduced_tables_hold_alpha_and_beta(ls, c1, c1_ref, prec):
    """Reduced-precision tables hold alpha^l and beta^l themselves (FP16:
    times the stated kappa), not the vectors of the divided emission pairs:
    each row within the precision's posterior bound of the oracle's, relative
    to the row's total. The log scales: FP32 within its log-likelihood bound
    (relative, at least 1 in the denominator: log F^l is near 0 at l = 0);
    FP16 storage adds a relative error of at most u = 2^-11 to each step's
    column sum, with no common sign, so after s steps the log scale is
    within 8 u sqrt(s) (a bound far outside the random walk's spread)."""
    x, ref = c1, c1_ref
    N = x["N"]
    kf, kb = (2.0 ** 14, 2.0 ** 14 / (N - 1)) if prec == "f16" else (1.0, 1.0)
    post = F16_POST_ATOL if prec == "f16" else F32_POST_ATOL
    logb = F16_LOGLIK_RTOL if prec == "f16" else F32_LOGLIK_RTOL
    m = ls.Model(x["H"], N, x["rho"], x["mu"])
    fwd = ls.Table(m, 0, prec)
    bck = ls.Table(m, 1, prec)

    def check(tab, kappa, vec, logs, steps):
        got = _np(tab.state) / kappa
        err = (np.abs(got - vec).max(axis=1) / vec.sum(axis=1)).max()
        dl = np.abs(_np(tab.log_scale) - logs)
        if prec == "f16":
            lerr = dl.max() / (8 * 2.0 ** -11 * np.sqrt(steps))
            assert err <= post and lerr <= 1.0, (err, lerr)
        else:
            lerr = (dl / np.maximum(np.abs(logs), 1.0)).max()
            assert err <= post and lerr <= logb, (err, lerr)
        return err, lerr

    worst = [0.0, 0.0]
    L = x["L"]
    for k, t in enumerate(x["targets"]):
        ls.forward(fwd, m, int(t))
        worst = np.maximum(worst, check(fwd, kf, ref["A"][k], ref["logF"][k], t + 1))
    for k in range(len(x["targets"]) - 1, -1, -1):
        t = int(x["targets"][k])
        ls.backward(bck, m, t)
        worst = np.maximum(worst, check(bck, kb, ref["B"][k], ref["logG"][k], L - t))
    print(f"{prec} tables: row error {worst[0]:.3e}, log scale error {worst[1]:.3e} "
          f"({'of the bound' if prec == 'f16' else 'relative'})")


# ---------------------------------------------------------------------------
# edge shapes: tiny N, word boundaries, partial words, several waves

EDGE = [(2, 30), (3, 25), (63, 20), (64, 20), (65, 20), (127, 15), (128, 15), (129, 15),
        (200, 12), (700, 8), (1031, 6)]


@pytest.mark.parametrize("N,L", EDGE)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_edge_sizes(ls, N, L, prec):
    H, rho, mu = _random_case(N, L, seed=N * 7 + L)
    targets = np.unique(np.array([0, L // 3, L - 1], np.int32))
    rec = np.arange(N, dtype=np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, targets, want=("P", "E", "A", "B"))
    m = ls.Model(H, N, rho, mu)
    r = ls.decode(m, targets, prec, want=("P", "E"))
    if prec == "fp64":
        rel_close(_np(r["P"]), ref["P"], F64_RTOL, F64_ATOL_PROB)
        rel_close(_np(r["E"]), ref["E"], F64_RTOL, F64_ATOL_LOG)
        rel_close(_np(r["fwd"].log_scale), ref["llf"], F64_RTOL, F64_ATOL_LOG)
    else:
        assert np.abs(_np(r["P"]) - ref["P"]).max() <= F32_POST_ATOL


SHAPES = [  # (N, slots, waves): every wave layout class
    (700, 4, 3), (700, 8, 2), (700, 3, 4), (700, 1, 11), (1031, 12, 2), (1031, 4, 5),
    (1031, 2, 9), (333, 1, 6), (333, 2, 3), (4160, 12, 6), (4160, 16, 5),
]


@pytest.mark.parametrize("N,ns,nw", SHAPES)
def test_forced_shapes_fp64(ls, N, ns, nw):
    L = 9
    H, rho, mu = _random_case(N, L, seed=N + 31 * ns + nw)
    targets = np.array([2, 5], np.int32)
    rec = np.array(sorted({0, 1, 63, 64, N // 2, N - 2, N - 1}), dtype=np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, targets, want=("P", "B", "A"))
    m = ls.Model(H, N, rho, mu)
    with forced_shape(ns, nw):
        assert ls.kernel_shape(N, "fp64") == (ns, nw)
        r = ls.decode(m, targets, "fp64", recipients=rec, want=("P",))
    rel_close(_np(r["P"]), ref["P"], F64_RTOL, F64_ATOL_PROB)
    rel_close(_np(r["bsnap"]), ref["B"], F64_RTOL, F64_ATOL_PROB)
    rel_close(_np(r["fwd"].log_scale), ref["llf"], F64_RTOL, F64_ATOL_LOG)


WIDE_SHAPES = [  # (precision, N, slots, waves): groups of 5..12 waves with wide slots, where
    # the cross-wave sum covers 8 or 12 lanes (the register budget of the slot
    # count caps the group at 8 or 12 waves); 128 and 132 slots in 12-wave groups
    # run three waves per SIMD, FP64 100 and 104 slots two
    ("fp64", 20000, 56, 6), ("fp64", 40000, 80, 8), ("fp64", 26000, 40, 11),
    ("fp32", 54000, 172, 5), ("fp32", 100000, 196, 8), ("fp32", 58000, 104, 9),
    ("fp32", 100000, 132, 12), ("fp32", 98000, 128, 12),
    ("fp64", 50000, 100, 8), ("fp64", 53248, 104, 8),
]


@pytest.mark.parametrize("prec,N,ns,nw", WIDE_SHAPES)
def test_forced_wide_shapes(ls, prec, N, ns, nw):
    L = 9
    H, rho, mu = _random_case(N, L, seed=N + ns + nw)
    targets = np.array([2, 5], np.int32)
    rec = np.array(sorted({0, 1, 63, 64, N // 2, N - 2, N - 1}), dtype=np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, targets, want=("P", "B"))
    m = ls.Model(H, N, rho, mu)
    with forced_shape(ns, nw):
        assert ls.kernel_shape(N, prec) == (ns, nw)
        r = ls.decode(m, targets, prec, recipients=rec, want=("P",))
    if prec == "fp64":
        tol = f64_rtol(N)
        rel_close(_np(r["P"]), ref["P"], tol, F64_ATOL_PROB)
        rel_close(_np(r["bsnap"]), ref["B"], tol, F64_ATOL_PROB)
        rel_close(_np(r["fwd"].log_scale), ref["llf"], tol, F64_ATOL_LOG)
    else:
        assert np.abs(_np(r["P"]) - ref["P"]).max() <= F32_POST_ATOL
        assert np.max(np.abs(_np(r["fwd"].log_scale) - ref["llf"]) / np.abs(ref["llf"])) <= F32_LOGLIK_RTOL


def test_stale_hip_error_is_not_reported(ls):
    """A failed HIP call made by someone else on this thread (here an invalid
    device ordinal, rejected on the host) must not surface as an error of the
    next library call."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    count = ctypes.c_int(0)
    assert hip.hipGetDeviceCount(ctypes.byref(count)) == 0
    assert hip.hipSetDevice(count.value + 5) != 0  # leaves a last-error behind
    N, L = 70, 12
    H, rho, mu = _random_case(N, L, seed=9)
    m = ls.Model(H, N, rho, mu)
    r = ls.decode(m, [3, 7], "fp64", want=("P",))
    assert np.all(np.isfinite(_np(r["P"])))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_many_recipients_equal_small_decode(ls, prec):
    """A decode of thousands of recipients (several rounds of workgroups per
    launch): every recipient's rows must equal those of a small decode bit
    for bit, and the oracle's."""
    N, L = 4500, 40
    H, rho, mu = _random_case(N, L, seed=45)
    targets = [7, 31]
    m = ls.Model(H, N, rho, mu)
    full = ls.decode(m, targets, prec, want=("P",))
    pick = np.array([0, 1, 2249, 2250, 2251, N - 1], np.int32)
    part = ls.decode(m, targets, prec, recipients=pick, want=("P",))
    assert np.array_equal(_np(full["P"])[:, pick, :], _np(part["P"]))
    assert np.array_equal(_np(full["fwd"].log_scale)[pick], _np(part["fwd"].log_scale))
    ref = oracle.run_pass(H, N, L, rho, mu, pick, targets, want=("P",))
    if prec == "fp64":
        rel_close(_np(part["P"]), ref["P"], F64_RTOL, F64_ATOL_PROB)
    else:
        assert np.abs(_np(part["P"]) - ref["P"]).max() <= F32_POST_ATOL


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sweep_chunk_length_does_not_change_results(ls, prec, monkeypatch):
    """Sweeps resume from the table at every chunk boundary: any chunk length
    gives the same vectors bit for bit (the log scales are summed per chunk,
    so they agree to rounding)."""
    N, L = 300, 500
    H, rho, mu = _random_case(N, L, seed=77)
    targets = [3, 160, 161, 499]
    m = ls.Model(H, N, rho, mu)
    res = {}
    for chunk in ("7", "64", "100000"):
        monkeypatch.setenv("LS_SWEEP_CHUNK", chunk)
        r = ls.decode(m, targets, prec, want=("P",))
        res[chunk] = (_np(r["P"]), _np(r["bsnap"]), _np(r["fwd"].log_scale),
                      _np(r["bck"].log_scale))
    for chunk in ("7", "64"):
        assert np.array_equal(res[chunk][0], res["100000"][0])
        assert np.array_equal(res[chunk][1], res["100000"][1])
        for q in (2, 3):
            assert np.allclose(res[chunk][q], res["100000"][q], rtol=1e-13, atol=1e-12)


def test_recipient_subset_equals_full(ls, c1):
    """Windows of recipients give the same columns (tables are independent
    HMMs, section 3.9)."""
    x = c1
    m = ls.Model(x["H"], x["N"], x["rho"], x["mu"])
    full = ls.decode(m, x["targets"], "fp64", want=("P",))
    sub = np.array([5, 199, 0, 77], np.int32)
    part = ls.decode(m, x["targets"], "fp64", recipients=sub, want=("P",))
    assert np.array_equal(_np(part["P"]), _np(full["P"])[:, sub, :])


def test_forward_in_steps_equals_direct(ls):
    N, L = 150, 40
    H, rho, mu = _random_case(N, L, seed=5)
    m = ls.Model(H, N, rho, mu)
    a = ls.Table(m, 0, "fp64")
    ls.forward(a, m, 30)
    b = ls.Table(m, 0, "fp64")
    for t in range(0, 31):
        ls.forward(b, m, t)
    assert np.array_equal(_np(a.state), _np(b.state))
    assert np.allclose(_np(a.log_scale), _np(b.log_scale), rtol=1e-13, atol=1e-12)
    c = ls.Table(m, 1, "fp64")
    ls.backward(c, m, 3)
    d = ls.Table(m, 1, "fp64")
    for t in range(L - 1, 2, -1):
        ls.backward(d, m, t)
    assert np.array_equal(_np(c.state), _np(d.state))
    assert np.allclose(_np(c.log_scale), _np(d.log_scale), rtol=1e-13, atol=1e-12)


def test_table_copy_then_propagate(ls):
    N, L = 90, 20
    H, rho, mu = _random_case(N, L, seed=6)
    m = ls.Model(H, N, rho, mu)
    a = ls.Table(m, 0, "fp32")
    ls.forward(a, m, 7)
    b = ls.Table(m, 0, "fp32")
    b.copy_from(a)
    ls.forward(b, m, 12)
    ls.forward(a, m, 12)
    assert np.array_equal(_np(a.state), _np(b.state))


def test_posterior_distance_from_tables(ls, c1, c1_ref):
    x, ref = c1, c1_ref
    m = ls.Model(x["H"], x["N"], x["rho"], x["mu"])
    import torch
    for prec in ("fp64", "fp32", "f16"):
        fwd = ls.Table(m, 0, prec)
        bck = ls.Table(m, 1, prec)
        t = int(x["targets"][3])
        ls.forward(fwd, m, t)
        ls.backward(bck, m, t)
        dt = ls.io_dtype(prec)
        P = torch.empty((x["N"], x["N"]), dtype=dt, device="cuda")
        E = torch.empty_like(P)
        ls.posterior_distance(fwd, bck, m, P, E)
        if prec == "fp64":
            rel_close(_np(P), ref["P"][3], F64_RTOL, F64_ATOL_PROB)
            rel_close(_np(E), ref["E"][3], F64_RTOL, F64_ATOL_LOG)
        else:
            # FP16: posteriors read straight from the two half tables
            check_reduced(prec, _np(P), ref["P"][3], "prob")


def test_distance_matrix(ls, c1, c1_ref):
    x, ref = c1, c1_ref
    m = ls.Model(x["H"], x["N"], x["rho"], x["mu"])
    r = ls.decode(m, x["targets"], "fp64", want=("E",))
    D = ls.distance_symmetrise(r["E"], prec="fp64")  # in place
    Dref = np.stack([oracle.symmetrise(ref["E"][k]) for k in range(len(x["targets"]))])
    rel_close(_np(D), Dref, F64_RTOL, F64_ATOL_LOG)
    Dn = _np(D)
    assert np.array_equal(Dn, np.transpose(Dn, (0, 2, 1)))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_symmetrise_ragged_tiles(ls, prec):
    """D = E + E^T with a zero diagonal, bit-exact: ragged tiles, N a
    multiple of the 16-byte vector or not, in place, and a base that is not
    16-byte aligned (which takes the scalar path)."""
    import torch
    td = torch.float32 if prec == "fp32" else torch.float64
    nd = np.float32 if prec == "fp32" else np.float64
    for N in (1, 5, 64, 65, 128, 130, 132, 196, 300):
        for inplace in (False, True):
            for offset in (0, 1):
                buf = torch.rand(3 * N * N + offset, dtype=td, device="cuda")
                E = buf[offset:].view(3, N, N)
                En = E.cpu().numpy().astype(np.float64)
                D = E if inplace else torch.empty_like(E)
                ls.distance_symmetrise(E, D, prec)
                ref = En + np.transpose(En, (0, 2, 1))
                for k in range(3):
                    np.fill_diagonal(ref[k], 0.0)
                got = D.cpu().numpy().astype(np.float64)
                assert np.array_equal(got, ref.astype(nd).astype(np.float64)), (N, inplace, offset)


def test_total_underflow_nan_columns(ls):
    """mu = 0 and a private allele of the recipient: its column becomes NaN
    (diagonal 0) and the status word says so (appendix A.3)."""
    L, N = 8, 6
    rng = np.random.default_rng(21)
    h = (rng.random((L, N)) < 0.5).astype(np.uint8)
    h[3, :] = 0
    h[3, 2] = 1
    H = pack_haplotypes(h)
    rho = np.full(L - 1, 0.1)
    rec = np.array([2, 4], np.int32)
    ref = oracle.run_pass(H, N, L, rho, 0.0, rec, np.array([5], np.int32), want=("P",))
    m = ls.Model(H, N, rho, 0.0)
    for prec in ("fp64", "fp32"):
        r = ls.decode(m, [5], prec, recipients=rec, want=("P",))
        P = _np(r["P"])[0]
        assert np.array_equal(np.isnan(P), np.isnan(ref["P"][0]))
        assert P[0, 2] == 0.0
        assert ls.status_check(r["fwd"]) == ls.LS_WARN_NONFINITE


@pytest.mark.parametrize("mu", [0.7, 1.0])
def test_mutation_probability_above_one_half(ls, mu):
    """For mu > 1/2 the mismatch emission is the larger one (the FP32 sweeps
    then carry both emissions divided by mu). At mu = 1 only donors that
    differ from the recipient at every variant keep mass between jumps; two
    donors here are complements of recipients 0 and 3."""
    N, L = 70, 40
    rng = np.random.default_rng(31)
    h = (rng.random((L, N)) < 0.5).astype(np.uint8)
    h[:, 5] = 1 - h[:, 0]
    h[:, 9] = 1 - h[:, 3]
    H = pack_haplotypes(h)
    rho = rho_from_spacings(rng.exponential(0.05, L - 1))
    rec = np.array([0, 3, 40], np.int32)
    targets = np.array([7, 30], np.int32)
    ref = oracle.run_pass(H, N, L, rho, mu, rec, targets, want=("P",))
    m = ls.Model(H, N, rho, mu)
    for prec in ("fp64", "fp32", "f16"):
        r = ls.decode(m, targets, prec, recipients=rec, want=("P",))
        P, ll = _np(r["P"]), _np(r["fwd"].log_scale)
        if prec == "fp64":
            rel_close(P, ref["P"], F64_RTOL, F64_ATOL_PROB)
            rel_close(ll, ref["llf"], F64_RTOL, F64_ATOL_LOG)
        else:
            check_reduced(prec, P, ref["P"], "prob")
            check_reduced(prec, ll, ref["llf"], "log")


def test_model_mismatch_is_rejected(ls):
    N, L = 70, 10
    H, rho, mu = _random_case(N, L, seed=8)
    m1 = ls.Model(H, N, rho, mu)
    m2 = ls.Model(H, N, rho * 0.5, mu)
    t = ls.Table(m1, 0, "fp32")
    ls.forward(t, m1, 3)
    with pytest.raises(ls.LsError) as e:
        ls.forward(t, m2, 5)
    assert e.value.code == 3  # LS_ERR_STATE


def test_argument_errors(ls):
    N, L = 70, 10
    H, rho, mu = _random_case(N, L, seed=9)
    m = ls.Model(H, N, rho, mu)
    t = ls.Table(m, 0, "fp32")
    with pytest.raises(ls.LsError):
        ls.forward(t, m, L)             # past the last variant
    with pytest.raises(ls.LsError):
        ls.forward(t, m, 5, targets=[4, 3], bsnap=t.state, E=t.state)  # not increasing
    b = ls.Table(m, 1, "fp32")
    with pytest.raises(ls.LsError):
        ls.forward(b, m, 3)             # backward table given to forward
    ls.forward(t, m, 6)
    with pytest.raises(ls.LsError):
        ls.forward(t, m, 4)             # cannot move backwards
