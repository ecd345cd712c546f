"""Python binding of libls over torch device tensors.

Every function here only marshals arguments: it hands device pointers, sizes
and the current HIP stream to the C ABI (include/ls.h); all arithmetic runs in
the library's kernels. PyTorch provides device memory and streams.
"""

from __future__ import annotations

import ctypes
from typing import Iterable, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (LS_FP32, LS_FP32_F16STORE, LS_FP64, LS_MAX_TARGETS, LsModel, LsTable,
                   check)

PRECISIONS = {"fp64": LS_FP64, "fp32": LS_FP32, "f16": LS_FP32_F16STORE}
_STATE_DTYPE = {LS_FP64: torch.float64, LS_FP32: torch.float32, LS_FP32_F16STORE: torch.float16}
_IO_DTYPE = {LS_FP64: torch.float64, LS_FP32: torch.float32, LS_FP32_F16STORE: torch.float32}


def prec_code(prec) -> int:
    if isinstance(prec, str):
        return PRECISIONS[prec]
    return int(prec)


def io_dtype(prec) -> torch.dtype:
    return _IO_DTYPE[prec_code(prec)]


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _p(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _i32_host(x) -> Optional[ctypes.Array]:
    if x is None:
        return None
    arr = np.ascontiguousarray(np.asarray(x, dtype=np.int32))
    return (ctypes.c_int32 * arr.size)(*arr.tolist())


class Model:
    """Haplotypes and parameters on the device (cf. kalis Parameters).

    H: L x stride packed haplotypes (numpy uint32 or a device tensor).
    rho: L-1 recombination probabilities; mu: mutation probability, a scalar
    or one value per variant (L values; section 3.4 allows either).
    prior: optional N x N prior copying matrix Pi (section 2.1), Pi[j, i] the
    prior probability that recipient i copies donor j (columns sum to 1, the
    diagonal is not used); None for the uniform prior.
    """

    def __init__(self, H, N: int, rho, mu, device="cuda", stream=None, prior=None):
        lib = _lib.load()
        dev = torch.device(device)
        if isinstance(H, np.ndarray):
            H = torch.from_numpy(np.ascontiguousarray(H, dtype=np.uint32).view(np.int32))
        self.H = H.to(dev).contiguous()
        if self.H.dtype not in (torch.int32, torch.uint32):
            raise ValueError("H must hold 32-bit words")
        self.device = dev
        L = int(self.H.shape[0])
        self.c = LsModel()
        self.c.H = self.H.data_ptr()
        self.c.stride_words = int(self.H.shape[1])
        self.c.N = int(N)
        self.c.L = L
        self._set_params(rho, mu)
        self.prior = None
        if prior is not None:
            Pi = prior.to(torch.float64) if torch.is_tensor(prior) else \
                torch.as_tensor(np.asarray(prior, dtype=np.float64))
            if tuple(Pi.shape) != (int(N), int(N)):
                raise ValueError("the prior matrix must be N x N")
            # row i of the library's buffer is column i of Pi
            self.prior = Pi.to(dev).t().contiguous()
            self.c.prior = self.prior.data_ptr()
        nbytes = lib.ls_model_workspace_bytes(int(N), L)
        if nbytes == 0:
            raise ValueError("invalid N or L")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
        check(lib.ls_model_init(ctypes.byref(self.c), _p(self.workspace), nbytes,
                                _stream(stream)), "ls_model_init")

    def _set_params(self, rho, mu):
        L = self.c.L
        rho = torch.as_tensor(np.asarray(rho, dtype=np.float64) if not torch.is_tensor(rho)
                              else rho, dtype=torch.float64)
        self.rho = rho.to(self.device).contiguous()
        if self.rho.numel() != max(L - 1, 0):
            raise ValueError("rho must have L-1 entries")
        self.c.rho = self.rho.data_ptr() if self.rho.numel() else None
        self.mu_vec = None
        self.c.mu_vec = None
        if np.ndim(mu) == 0 and not (torch.is_tensor(mu) and mu.dim() > 0):
            self.c.mu = float(mu)
        else:
            muv = mu.to(torch.float64) if torch.is_tensor(mu) else \
                torch.as_tensor(np.asarray(mu, dtype=np.float64))
            self.mu_vec = muv.to(self.device).contiguous().reshape(-1)
            if self.mu_vec.numel() != L:
                raise ValueError("a per-variant mu must have L entries")
            self.c.mu = 0.0
            self.c.mu_vec = self.mu_vec.data_ptr()

    def update(self, rho, mu, stream=None):
        """New rho and mu for the same haplotypes (and prior): re-runs
        ls_model_init in the existing workspace. Tables made under the old
        parameters are refused afterwards (their model hash differs)."""
        self._set_params(rho, mu)
        lib = _lib.load()
        check(lib.ls_model_init(ctypes.byref(self.c), _p(self.workspace),
                                int(self.workspace.numel()), _stream(stream)), "ls_model_init")

    @property
    def N(self) -> int:
        return self.c.N

    @property
    def L(self) -> int:
        return self.c.L

    @property
    def mu(self):
        """The scalar mu, or the device tensor of per-variant values."""
        return self.c.mu if self.mu_vec is None else self.mu_vec


class Table:
    """Forward (direction 0) or backward (direction 1) table for a set of
    recipients (cf. MakeForwardTable / MakeBackwardTable)."""

    def __init__(self, model: Model, direction: int, prec="fp32", recipients=None, stream=None):
        lib = _lib.load()
        self.prec = prec_code(prec)
        dev = model.device
        if recipients is None:
            recipients = np.arange(model.N, dtype=np.int32)
        self.recipients = torch.as_tensor(np.asarray(recipients, dtype=np.int32)).to(dev) \
            if not torch.is_tensor(recipients) else recipients.to(dev, torch.int32).contiguous()
        R = int(self.recipients.numel())
        self.state = torch.zeros((R, model.N), dtype=_STATE_DTYPE[self.prec], device=dev)
        self.log_scale = torch.zeros(R, dtype=torch.float64, device=dev)
        self.status = torch.zeros(R, dtype=torch.int32, device=dev)
        self.c = LsTable()
        check(lib.ls_table_init(ctypes.byref(self.c), int(direction), self.prec, _p(self.state),
                                _p(self.log_scale), _p(self.status), _p(self.recipients), R,
                                _stream(stream)), "ls_table_init")
        self.N = model.N

    @property
    def l(self) -> int:
        return self.c.l

    @property
    def R(self) -> int:
        return self.c.R

    def reset(self, model: Model, recipients, stream=None):
        """Re-initialise this table's buffers for other recipients (at most
        as many as it was made for): "not yet propagated" (ResetTable)."""
        rec = recipients.to(model.device, torch.int32).contiguous() if torch.is_tensor(recipients) \
            else torch.as_tensor(np.asarray(recipients, dtype=np.int32)).to(model.device)
        R = int(rec.numel())
        if R < 1 or R > self.state.shape[0]:
            raise ValueError("reset: recipient count must be in [1, capacity]")
        self.recipients = rec
        check(_lib.load().ls_table_init(ctypes.byref(self.c), int(self.c.direction), self.prec,
                                        _p(self.state), _p(self.log_scale), _p(self.status),
                                        _p(rec), R, _stream(stream)), "ls_table_init")

    def copy_from(self, src: "Table", stream=None):
        """CopyTable(self, src)."""
        check(_lib.load().ls_table_copy(ctypes.byref(self.c), ctypes.byref(src.c), self.N,
                                        _stream(stream)), "ls_table_copy")
        self.recipients = src.recipients


def forward(table: Table, model: Model, t: int, targets=None, bsnap=None, P=None, E=None,
            stream=None, out_strides=(0, 0)):
    """Forward(table, model, t); at the targets, posteriors P and half
    distances E from the snapshots bsnap ([T][R][N]). out_strides = (target
    stride, row stride) of P and E in elements; (0, 0): contiguous
    [T][R][N]."""
    T = 0 if targets is None else len(targets)
    check(_lib.load().ls_forward(ctypes.byref(table.c), ctypes.byref(model.c), int(t),
                                 _i32_host(targets), T, _p(bsnap), _p(P), _p(E),
                                 int(out_strides[0]), int(out_strides[1]), _stream(stream)),
          "ls_forward")


def backward(table: Table, model: Model, t: int, targets=None, bsnap=None, stream=None):
    T = 0 if targets is None else len(targets)
    check(_lib.load().ls_backward(ctypes.byref(table.c), ctypes.byref(model.c), int(t),
                                  _i32_host(targets), T, _p(bsnap), _stream(stream)),
          "ls_backward")


def posterior_distance(fwd: Table, bck: Table, model: Model, P=None, E=None, stream=None):
    check(_lib.load().ls_posterior_distance(ctypes.byref(fwd.c), ctypes.byref(bck.c),
                                            ctypes.byref(model.c), _p(P), _p(E),
                                            _stream(stream)), "ls_posterior_distance")


def distance_symmetrise(E: torch.Tensor, D: Optional[torch.Tensor] = None, prec="fp32",
                        stream=None) -> torch.Tensor:
    """D[k] = E[k] + E[k]^T with a zero diagonal; E is [T][N][N] (or [N][N])."""
    if D is None:
        D = E
    T = 1 if E.dim() == 2 else int(E.shape[0])
    N = int(E.shape[-1])
    check(_lib.load().ls_distance_symmetrise(_p(E), _p(D), N, T, prec_code(prec),
                                             _stream(stream)), "ls_distance_symmetrise")
    return D


def status_check(table: Table, stream=None) -> int:
    """LS_OK, or LS_WARN_NONFINITE if a recipient's column under/overflowed."""
    code = _lib.load().ls_status_check(_p(table.status), table.R, _stream(stream))
    if code not in (_lib.LS_OK, _lib.LS_WARN_NONFINITE):
        check(code, "ls_status_check")
    return code


def kernel_shape(N: int, prec="fp32", prior: bool = False):
    """(slots per wave, waves per recipient) of the sweeps for N haplotypes;
    prior=True: for a model with a prior copying matrix."""
    a, b = ctypes.c_int32(0), ctypes.c_int32(0)
    check(_lib.load().ls_kernel_shape(int(N), prec_code(prec), int(bool(prior)), ctypes.byref(a),
                                      ctypes.byref(b)), "ls_kernel_shape")
    return a.value, b.value


def _f64_device(x) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float64)
    return (t if t.is_cuda else t.to("cuda")).contiguous()


def calc_rho(cM, s: float = 1.0, gamma: float = 1.0, stream=None) -> torch.Tensor:
    """rho = 1 - exp(-s (cM / 100)^gamma) (eq. rho; cM in centimorgans, one
    value per interval between consecutive variants) on the device."""
    c = _f64_device(cM)
    rho = torch.empty_like(c)
    check(_lib.load().ls_calc_rho(_p(c), int(c.numel()), float(s), float(gamma), _p(rho),
                                  _stream(stream)), "ls_calc_rho")
    return rho


def rho_map_grad(cM, s: float, gamma: float, grad_rho, stream=None) -> torch.Tensor:
    """(d/ds, d/dgamma) from a gradient w.r.t. rho = calc_rho(cM, s, gamma):
    a device float64 tensor of 2."""
    c = _f64_device(cM)
    g = _f64_device(grad_rho)
    if g.numel() != c.numel():
        raise ValueError("grad_rho and cM differ in length")
    out = torch.empty(2, dtype=torch.float64, device=c.device)
    check(_lib.load().ls_rho_map_grad(_p(c), int(c.numel()), float(s), float(gamma), _p(g),
                                      _p(out), _stream(stream)), "ls_rho_map_grad")
    return out


def loglik_grad(model: Model, recipients=None, prec="fp32", grad: bool = True, stream=None):
    """Per-recipient log-likelihood, their sum (PAC) and optionally the
    gradient of the sum w.r.t. rho (L-1) and mu (1 value, or L with a
    per-variant mu). Returns a dict of device tensors."""
    lib = _lib.load()
    pc = prec_code(prec)
    dev = model.device
    rec = None
    if recipients is not None:
        rec = torch.as_tensor(np.asarray(recipients, dtype=np.int32)).to(dev) \
            if not torch.is_tensor(recipients) else recipients.to(dev, torch.int32).contiguous()
    R = model.N if rec is None else int(rec.numel())
    ll = torch.empty(R, dtype=torch.float64, device=dev)
    pac = torch.empty(1, dtype=torch.float64, device=dev)
    g_rho = torch.empty(max(model.L - 1, 1), dtype=torch.float64, device=dev) if grad else None
    n_mu = 1 if model.mu_vec is None else model.L
    g_mu = torch.empty(n_mu, dtype=torch.float64, device=dev) if grad else None
    nbytes = lib.ls_loglik_grad_workspace_bytes(ctypes.byref(model.c), R, pc)
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
    check(lib.ls_loglik_grad(ctypes.byref(model.c), _p(rec), R, pc, _p(ll), _p(pac), _p(g_rho),
                             _p(g_mu), _p(ws), nbytes, _stream(stream)), "ls_loglik_grad")
    out = dict(loglik=ll, pac=pac)
    if grad:
        out["grad_rho"] = g_rho[: max(model.L - 1, 0)]
        out["grad_mu"] = g_mu
    return out


class Checkpoints:
    """Forward checkpoints of a log-likelihood evaluation kept for a later
    gradient (ls_loglik_checkpoint / ls_loglik_grad_adjoint). Holds the
    workspace; the model must not change in between."""

    def __init__(self, model: Model, recipients=None, prec="fp32", stream=None):
        lib = _lib.load()
        self.model = model
        self.prec = prec_code(prec)
        dev = model.device
        self.rec = None
        if recipients is not None:
            self.rec = torch.as_tensor(np.asarray(recipients, dtype=np.int32)).to(dev) \
                if not torch.is_tensor(recipients) else recipients.to(dev, torch.int32).contiguous()
        self.R = model.N if self.rec is None else int(self.rec.numel())
        self.nbytes = lib.ls_loglik_grad_workspace_bytes(ctypes.byref(model.c), self.R, self.prec)
        self.ws = torch.empty(int(self.nbytes), dtype=torch.uint8, device=dev)
        self.loglik = torch.empty(self.R, dtype=torch.float64, device=dev)
        self.pac = torch.empty(1, dtype=torch.float64, device=dev)
        self.hash = model.c.hash
        check(lib.ls_loglik_checkpoint(ctypes.byref(model.c), _p(self.rec), self.R, self.prec,
                                       _p(self.loglik), _p(self.pac), _p(self.ws), self.nbytes,
                                       _stream(stream)), "ls_loglik_checkpoint")

    def gradient(self, stream=None):
        """(grad_rho [L-1], grad_mu [1] or [L]) from the kept checkpoints."""
        model = self.model
        if model.c.hash != self.hash:
            raise RuntimeError("the model changed since the checkpoints were taken")
        dev = model.device
        g_rho = torch.empty(max(model.L - 1, 1), dtype=torch.float64, device=dev)
        g_mu = torch.empty(1 if model.mu_vec is None else model.L, dtype=torch.float64,
                           device=dev)
        check(_lib.load().ls_loglik_grad_adjoint(ctypes.byref(model.c), _p(self.rec), self.R,
                                                 self.prec, _p(g_rho), _p(g_mu), _p(self.ws),
                                                 self.nbytes, _stream(stream)),
              "ls_loglik_grad_adjoint")
        return g_rho[: max(model.L - 1, 0)], g_mu


def decode(model: Model, targets: Sequence[int], prec="fp32", recipients=None,
           want: Iterable[str] = ("E",), stream=None):
    """Posterior decoding at several targets: a backward sweep that keeps
    beta at the targets, then a forward sweep that combines alpha with it.

    Returns a dict with any of P (posteriors) and E (half distances), each
    [T][R][N], plus the two tables (whose log scales give the
    log-likelihood at variant 0 / L-1)."""
    targets = np.sort(np.asarray(targets, dtype=np.int32))
    want = set(want)
    pc = prec_code(prec)
    fwd = Table(model, 0, pc, recipients, stream)
    bck = Table(model, 1, pc, recipients, stream)
    T, R, N = len(targets), fwd.R, model.N
    dt = _IO_DTYPE[pc]
    dev = model.device
    P = torch.empty((T, R, N), dtype=dt, device=dev) if "P" in want else None
    E = torch.empty((T, R, N), dtype=dt, device=dev) if "E" in want else None
    bsnap = torch.empty((T, R, N), dtype=dt, device=dev)
    # backward in chunks of at most LS_MAX_TARGETS targets, from the end
    # (with T <= LS_MAX_TARGETS each direction is a single sweep launch)
    hi = T
    while hi > 0:
        lo = max(0, hi - LS_MAX_TARGETS)
        stop = 0 if lo == 0 else int(targets[lo])
        backward(bck, model, stop, targets[lo:hi], bsnap[lo:hi], stream)
        hi = lo
    if bck.l != 0:
        backward(bck, model, 0, None, None, stream)
    for lo in range(0, T, LS_MAX_TARGETS):
        hi = min(T, lo + LS_MAX_TARGETS)
        stop = model.L - 1 if hi == T else int(targets[hi - 1])
        forward(fwd, model, stop, targets[lo:hi], bsnap[lo:hi],
                P[lo:hi] if P is not None else None, E[lo:hi] if E is not None else None, stream)
    if fwd.l != model.L - 1:
        forward(fwd, model, model.L - 1, None, None, None, None, stream)
    return dict(P=P, E=E, fwd=fwd, bck=bck, bsnap=bsnap)


def distance_matrices(model: Model, targets: Sequence[int], prec="fp32", window: int = 0,
                      D: Optional[torch.Tensor] = None, stream=None):
    """Full N x N distance matrices at the targets (eq. distmat), resident on
    the device: recipients are decoded in windows of `window` (0: all at
    once; the recipient windows of section 3.9), each window writing its
    rows of the half distances straight into D ([T][N][N], allocated if
    None) through the strided output of ls_forward; then D = E + E^T in
    place. Returns dict(D=D, loglik=[N] per-recipient log-likelihoods)."""
    targets = np.sort(np.asarray(targets, dtype=np.int32))
    pc = prec_code(prec)
    N, T, dev = model.N, len(targets), model.device
    if T < 1 or T > LS_MAX_TARGETS:
        raise ValueError(f"between 1 and {LS_MAX_TARGETS} targets")
    dt = _IO_DTYPE[pc]
    if D is None:
        D = torch.empty((T, N, N), dtype=dt, device=dev)
    if tuple(D.shape) != (T, N, N) or D.dtype != dt or not D.is_contiguous():
        raise ValueError("D must be a contiguous [T][N][N] tensor of the precision's output type")
    w = N if window <= 0 else min(int(window), N)
    fwd = Table(model, 0, pc, np.arange(w, dtype=np.int32), stream)
    bck = Table(model, 1, pc, np.arange(w, dtype=np.int32), stream)
    bsnap = torch.empty((T, w, N), dtype=dt, device=dev)
    ll = torch.empty(N, dtype=torch.float64, device=dev)
    for r0 in range(0, N, w):
        r1 = min(N, r0 + w)
        rec = torch.arange(r0, r1, dtype=torch.int32, device=dev)
        fwd.reset(model, rec, stream)
        bck.reset(model, rec, stream)
        R = r1 - r0
        bs = bsnap.view(-1)[: T * R * N].view(T, R, N)
        backward(bck, model, 0, targets, bs, stream)
        rows = D.view(-1)[r0 * N:]  # row r0 of matrix 0 onwards
        check(_lib.load().ls_forward(ctypes.byref(fwd.c), ctypes.byref(model.c), model.L - 1,
                                     _i32_host(targets), T, _p(bs), None, _p(rows), N * N, N,
                                     _stream(stream)), "ls_forward")
        ll[r0:r1].copy_(fwd.log_scale[:R])
    distance_symmetrise(D, D, pc, stream)
    return dict(D=D, loglik=ll)


def average_linkage(D: torch.Tensor, prec=None, order: bool = True, stream=None):
    """Average pairwise linkage (section 6) of one [N][N] or T [T][N][N]
    symmetric distance matrices on the device (float32, or float64 for the
    FP64 path). D is overwritten. Returns (Z [T][N-1][4] float64: smaller
    id, larger id, merge distance, size; order [T][N] int32 leaf order, or
    None), with the leading T dropped for a single matrix."""
    single = D.dim() == 2
    Dm = D.unsqueeze(0) if single else D
    if not Dm.is_contiguous() or Dm.shape[-1] != Dm.shape[-2]:
        raise ValueError("D must be contiguous [T][N][N]")
    if prec is None:
        prec = "fp64" if D.dtype == torch.float64 else "fp32"
    pc = prec_code(prec)
    if (D.dtype == torch.float64) != (pc == LS_FP64):
        raise ValueError("D's dtype does not match the precision")
    T, N = int(Dm.shape[0]), int(Dm.shape[-1])
    lib = _lib.load()
    Z = torch.empty((T, max(N - 1, 0), 4), dtype=torch.float64, device=D.device)
    o = torch.empty((T, N), dtype=torch.int32, device=D.device) if order else None
    nbytes = lib.ls_average_linkage_workspace_bytes(N, T, pc)
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=D.device)
    check(lib.ls_average_linkage(_p(Dm), N, T, pc, _p(Z) if N > 1 else None, _p(o), _p(ws),
                                 nbytes, _stream(stream)), "ls_average_linkage")
    if single:
        return Z[0], (o[0] if o is not None else None)
    return Z, o


def average_linkage_noalloc(D: torch.Tensor, Z: torch.Tensor, order: torch.Tensor = None,
                            prec=None, stream=None):
    """average_linkage into caller-provided outputs through the entry point
    that allocates nothing (ls_average_linkage_noalloc: the workspace is the
    library's fixed per-device scratch). D [T][N][N] (overwritten), Z
    [T][N-1][4] float64, order [T][N] int32 or None; nothing is allocated
    here either. Calls on one GPU share the scratch and must not overlap."""
    if D.dim() != 3 or not D.is_contiguous() or D.shape[-1] != D.shape[-2]:
        raise ValueError("D must be contiguous [T][N][N]")
    T, N = int(D.shape[0]), int(D.shape[-1])
    if prec is None:
        prec = "fp64" if D.dtype == torch.float64 else "fp32"
    pc = prec_code(prec)
    if (D.dtype == torch.float64) != (pc == LS_FP64):
        raise ValueError("D's dtype does not match the precision")
    if N > 1 and (Z.dtype != torch.float64 or tuple(Z.shape) != (T, N - 1, 4)
                  or not Z.is_contiguous()):
        raise ValueError("Z must be contiguous float64 [T][N-1][4]")
    if order is not None and (order.dtype != torch.int32 or tuple(order.shape) != (T, N)
                              or not order.is_contiguous()):
        raise ValueError("order must be contiguous int32 [T][N]")
    check(_lib.load().ls_average_linkage_noalloc(_p(D), N, T, pc, _p(Z) if N > 1 else None,
                                                 _p(order), _stream(stream)),
          "ls_average_linkage_noalloc")


def standardise_rows(E: torch.Tensor, recipients, prec=None, stream=None,
                     out_strides=(0, 0), N=None) -> torch.Tensor:
    """Standardise half-distance rows in place (section 2.2): E [T][R][N]
    (or [R][N]) as ls_forward writes it, row r of recipient recipients[r];
    with out_strides, rows of N entries (default: E's last dimension) at
    those element strides from E's start."""
    if prec is None:
        prec = "fp64" if E.dtype == torch.float64 else "fp32"
    rec = recipients.to(E.device, torch.int32).contiguous() if torch.is_tensor(recipients) \
        else torch.as_tensor(np.asarray(recipients, dtype=np.int32)).to(E.device)
    R = int(rec.numel())
    N = int(E.shape[-1]) if N is None else int(N)
    T = 1 if E.dim() == 2 else int(E.shape[0])
    check(_lib.load().ls_standardise_rows(_p(E), _p(rec), R, T, N, int(out_strides[0]),
                                          int(out_strides[1]), prec_code(prec), _stream(stream)),
          "ls_standardise_rows")
    return E
