"""FP64 CPU oracle for the Li & Stephens all-vs-all copying model.

TEST INFRASTRUCTURE. Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU path: the arithmetic lives in ``ls_oracle.c`` (plain C, FP64,
built with ``-ffp-contract=off``), and this module only marshals arrays.

Every function here runs one recipient HMM at a time, exactly as the paper
writes the recursions (section 2.2, eq. fwd0/fwd1, bck0/bck1, postprob,
distmat). See ``ls_oracle.c`` for the definitions.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ls_oracle.c")
_SRC_CLUSTER = os.path.join(_HERE, "ls_cluster.c")
_LIB = os.path.join(_HERE, "libls_oracle.so")
_lib = None

EPS = 2.0 ** -52


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no GPU code)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_CLUSTER))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + f".{os.getpid()}.tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-pthread", "-o", tmp, _SRC, _SRC_CLUSTER, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def bind(path: str):
    """Load a compiled oracle library from ``path`` and declare its C API."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.lso_pass.argtypes = [P, i64, i32, i32, P, f64, P, i32, P, i32,
                             P, P, P, P, P, P, P, P, P, i32]
    lib.lso_pass.restype = ctypes.c_int
    lib.lso_pass_v.argtypes = [P, i64, i32, i32, P, P, P, i32, P, i32,
                               P, P, P, P, P, P, P, P, P, i32]
    lib.lso_pass_v.restype = ctypes.c_int
    lib.lso_gradient.argtypes = [P, i64, i32, i32, P, f64, P, i32, P, P, P, P, i32]
    lib.lso_gradient.restype = ctypes.c_int
    lib.lso_gradient_v.argtypes = [P, i64, i32, i32, P, P, P, i32, P, P, P, P, P, i32]
    lib.lso_gradient_v.restype = ctypes.c_int
    lib.lso_pass_x.argtypes = [P, i64, i32, i32, P, f64, P, P, P, i32, P, i32,
                               P, P, P, P, P, P, P, P, P, i32]
    lib.lso_pass_x.restype = ctypes.c_int
    lib.lso_gradient_x.argtypes = [P, i64, i32, i32, P, f64, P, P, P, i32, P, P, P, P, P, i32]
    lib.lso_gradient_x.restype = ctypes.c_int
    lib.lso_symmetrise.argtypes = [P, i32, P]
    lib.lso_symmetrise.restype = None
    lib.lso_calc_rho.argtypes = [P, i32, f64, f64, P]
    lib.lso_calc_rho.restype = None
    lib.lso_rho_map_grad.argtypes = [P, i32, f64, f64, P, P, P]
    lib.lso_rho_map_grad.restype = None
    lib.lso_version.restype = ctypes.c_char_p
    if hasattr(lib, "lso_average_linkage"):
        lib.lso_average_linkage.argtypes = [P, i32, i32, i32, P, P]
        lib.lso_average_linkage.restype = ctypes.c_int
        lib.lso_standardise.argtypes = [P, i32, i32, P]
        lib.lso_standardise.restype = None
    return lib


def _load():
    global _lib
    if _lib is None:
        _lib = bind(build())
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(n, int(os.environ.get("LSO_THREADS", n))))


def _prior_arg(prior, N):
    """The prior copying matrix Pi as an N x N array with Pi[j, i] the prior
    probability that recipient i copies donor j (column i belongs to
    recipient i), laid out for the library (row i of the buffer = column i)."""
    Pi = np.asarray(prior, dtype=np.float64)
    if Pi.shape != (N, N):
        raise ValueError("the prior matrix must be N x N")
    return np.ascontiguousarray(Pi.T)


def run_pass(H, N, L, rho, mu, recipients, targets=(), want=("P", "E"), nthreads=None, lib=None,
             prior=None):
    """Forward/backward pass for each recipient. ``mu`` is a scalar or a
    per-variant array of L values; ``prior`` the N x N prior copying matrix
    Pi (Pi[j, i]: recipient i copies donor j), or None for the uniform prior.

    Returns a dict with ``llf``/``llb`` (forward and backward log-likelihood,
    shape [R]) and, for each name in ``want`` among A (alpha), B (beta), P
    (posterior), E (half distance -log(p v eps)/2), arrays of shape [T][R][N];
    ``logF``/``logG`` are [T][R] (log F^t, log G^t); ``status`` [R] has bit 0
    for a forward and bit 1 for a backward zero or non-finite scale sum.
    """
    lib = lib or _load()
    H = np.ascontiguousarray(H, dtype=np.uint32)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    rec = np.ascontiguousarray(recipients, dtype=np.int32)
    tg = np.ascontiguousarray(targets, dtype=np.int32)
    R, T = rec.size, tg.size
    out = {}
    for k in ("A", "B", "P", "E"):
        out[k] = np.empty((T, R, N)) if k in want else None
    for k in ("logF", "logG"):
        out[k] = np.empty((T, R)) if k in want else None
    out["llf"] = np.empty(R)
    out["llb"] = np.empty(R)
    out["status"] = np.zeros(R, dtype=np.int32)
    if prior is not None:
        Pt = _prior_arg(prior, N)
        muv = None
        if np.ndim(mu) == 1:
            muv = np.ascontiguousarray(mu, dtype=np.float64)
            if muv.size != L:
                raise ValueError("a per-variant mu needs L values")
        rc = lib.lso_pass_x(_ptr(H), H.shape[1], N, L, _ptr(rho),
                            0.0 if muv is not None else float(mu), _ptr(muv), _ptr(Pt),
                            _ptr(rec), R, _ptr(tg), T, _ptr(out["A"]), _ptr(out["B"]),
                            _ptr(out["P"]), _ptr(out["E"]), _ptr(out["logF"]), _ptr(out["logG"]),
                            _ptr(out["llf"]), _ptr(out["llb"]), _ptr(out["status"]),
                            nthreads or default_threads())
    elif np.ndim(mu) == 1:
        muv = np.ascontiguousarray(mu, dtype=np.float64)
        if muv.size != L:
            raise ValueError("a per-variant mu needs L values")
        rc = lib.lso_pass_v(_ptr(H), H.shape[1], N, L, _ptr(rho), _ptr(muv), _ptr(rec), R,
                            _ptr(tg), T, _ptr(out["A"]), _ptr(out["B"]), _ptr(out["P"]),
                            _ptr(out["E"]), _ptr(out["logF"]), _ptr(out["logG"]),
                            _ptr(out["llf"]), _ptr(out["llb"]), _ptr(out["status"]),
                            nthreads or default_threads())
    else:
        rc = lib.lso_pass(_ptr(H), H.shape[1], N, L, _ptr(rho), float(mu), _ptr(rec), R,
                          _ptr(tg), T, _ptr(out["A"]), _ptr(out["B"]), _ptr(out["P"]),
                          _ptr(out["E"]), _ptr(out["logF"]), _ptr(out["logG"]), _ptr(out["llf"]),
                          _ptr(out["llb"]), _ptr(out["status"]), nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return {k: v for k, v in out.items() if v is not None}


def run_gradient(H, N, L, rho, mu, recipients, nthreads=None, lib=None, prior=None):
    """Per-recipient log-likelihood and its gradient w.r.t. rho (L-1) and mu.

    Returns dict(loglik [R], grad_rho [R][L-1], grad_mu [R], status [R]).
    With a per-variant ``mu`` (L values) also grad_mu_l [R][L], the
    derivative w.r.t. each mu^l (grad_mu is their sum). ``prior`` as in
    run_pass. Holds an L x N FP64 forward table per thread.
    """
    lib = lib or _load()
    H = np.ascontiguousarray(H, dtype=np.uint32)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    rec = np.ascontiguousarray(recipients, dtype=np.int32)
    R = rec.size
    g = np.zeros((R, max(L - 1, 0)))
    gm = np.empty(R)
    ll = np.empty(R)
    st = np.zeros(R, dtype=np.int32)
    if prior is not None:
        Pt = _prior_arg(prior, N)
        muv, gml = None, None
        if np.ndim(mu) == 1:
            muv = np.ascontiguousarray(mu, dtype=np.float64)
            if muv.size != L:
                raise ValueError("a per-variant mu needs L values")
            gml = np.zeros((R, L))
        rc = lib.lso_gradient_x(_ptr(H), H.shape[1], N, L, _ptr(rho),
                                0.0 if muv is not None else float(mu), _ptr(muv), _ptr(Pt),
                                _ptr(rec), R, _ptr(g) if L > 1 else None, _ptr(gml), _ptr(gm),
                                _ptr(ll), _ptr(st), nthreads or default_threads())
        if rc != 0:
            raise ValueError("oracle rejected its arguments")
        out = dict(loglik=ll, grad_rho=g, grad_mu=gm, status=st)
        if gml is not None:
            out["grad_mu_l"] = gml
        return out
    if np.ndim(mu) == 1:
        muv = np.ascontiguousarray(mu, dtype=np.float64)
        if muv.size != L:
            raise ValueError("a per-variant mu needs L values")
        gml = np.zeros((R, L))
        rc = lib.lso_gradient_v(_ptr(H), H.shape[1], N, L, _ptr(rho), _ptr(muv), _ptr(rec), R,
                                _ptr(g) if L > 1 else None, _ptr(gml), _ptr(gm), _ptr(ll),
                                _ptr(st), nthreads or default_threads())
        if rc != 0:
            raise ValueError("oracle rejected its arguments")
        return dict(loglik=ll, grad_rho=g, grad_mu=gm, grad_mu_l=gml, status=st)
    rc = lib.lso_gradient(_ptr(H), H.shape[1], N, L, _ptr(rho), float(mu), _ptr(rec), R,
                          _ptr(g) if L > 1 else None, _ptr(gm), _ptr(ll), _ptr(st),
                          nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return dict(loglik=ll, grad_rho=g, grad_mu=gm, status=st)


def symmetrise(E, lib=None):
    """D[a][b] = E[a][b] + E[b][a], D[a][a] = 0 for one N x N target."""
    lib = lib or _load()
    E = np.ascontiguousarray(E, dtype=np.float64)
    N = E.shape[0]
    D = np.empty_like(E)
    lib.lso_symmetrise(_ptr(E), N, _ptr(D))
    return D


def distances(H, N, L, rho, mu, targets, nthreads=None):
    """Full N x N distance matrices at the targets: [T][N][N]."""
    res = run_pass(H, N, L, rho, mu, np.arange(N, dtype=np.int32), targets, want=("E",),
                   nthreads=nthreads)
    return np.stack([symmetrise(res["E"][k]) for k in range(len(targets))])


def calc_rho(cM, s=1.0, gamma=1.0, lib=None):
    """rho_l = 1 - exp(-s (cM_l / 100)^gamma) (eq. rho; cM in centimorgans)."""
    lib = lib or _load()
    cM = np.ascontiguousarray(cM, dtype=np.float64)
    rho = np.empty_like(cM)
    lib.lso_calc_rho(_ptr(cM), cM.size, float(s), float(gamma), _ptr(rho))
    return rho


def rho_map_grad(cM, s, gamma, grad_rho, lib=None):
    """(d/ds, d/dgamma) of a function whose gradient w.r.t. rho = calc_rho(cM,
    s, gamma) is grad_rho."""
    lib = lib or _load()
    cM = np.ascontiguousarray(cM, dtype=np.float64)
    g = np.ascontiguousarray(grad_rho, dtype=np.float64)
    if g.size != cM.size:
        raise ValueError("grad_rho and cM differ in length")
    gs, gg = ctypes.c_double(), ctypes.c_double()
    lib.lso_rho_map_grad(_ptr(cM), cM.size, float(s), float(gamma), _ptr(g), ctypes.byref(gs),
                         ctypes.byref(gg))
    return gs.value, gg.value


def version() -> str:
    return _load().lso_version().decode()


def average_linkage(D, naive: bool = False, lib=None):
    """Average pairwise linkage of the symmetric distance matrix D (section
    6; float32 or float64, computed in that precision; D is not modified).
    Returns (Z [N-1][4] float64: smaller id, larger id, distance, size;
    order [N] int32: the dendrogram's leaf order). naive: the O(N^3) scan
    of every pair at every merge instead of the nearest-slot bookkeeping."""
    lib = lib or _load()
    D = np.array(D, copy=True, order="C")
    if D.dtype not in (np.float32, np.float64) or D.ndim != 2 or D.shape[0] != D.shape[1]:
        raise ValueError("D must be a square float32 or float64 matrix")
    N = D.shape[0]
    Z = np.zeros((max(N - 1, 0), 4))
    order = np.zeros(N, dtype=np.int32)
    rc = lib.lso_average_linkage(_ptr(D), N, int(D.dtype == np.float64), int(bool(naive)),
                                 _ptr(Z), _ptr(order))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return Z, order


def standardise(e, i, lib=None):
    """Standardised half-distance column of recipient i (section 2.2; zero
    deviation gives zeros): [N] float64."""
    lib = lib or _load()
    e = np.ascontiguousarray(e, dtype=np.float64)
    z = np.empty_like(e)
    lib.lso_standardise(_ptr(e), e.size, int(i), _ptr(z))
    return z
