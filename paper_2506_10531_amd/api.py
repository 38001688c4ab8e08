"""Python binding of the gfx950 QAOA library: torch tensors in, torch tensors
out, all work queued on the current torch stream through the C ABI.

Conventions (arXiv 2506.10531, Sec. IV, Eq. (1)-(2)): bit i of z is qubit i;
layer 1 acts first on |+>; the mixer is e^{+i beta sum X} (H_X = -sum X);
C(z) = z^T Q z for any dense real Q.
"""
from __future__ import annotations

import ctypes
import threading

import torch

from . import _lib

PREC = {"c128": _lib.QAOA_C128, "c64": _lib.QAOA_C64}


def _prec(prec) -> int:
    if isinstance(prec, str):
        if prec not in PREC:
            raise ValueError(f"prec must be one of {list(PREC)}")
        return PREC[prec]
    return int(prec)


class Context:
    """A library context on one GPU (scratch memory, HBM budget)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        L = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(L.qaoa_create(ctypes.byref(h), int(device), int(hbm_budget)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            _lib.load().qaoa_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- measurement aids --
    def profile(self, enable: bool = True):
        _lib.check(_lib.load().qaoa_profile_enable(self.h, int(enable)))

    def profile_read(self, reset: bool = True):
        n = ctypes.c_longlong()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _lib.check(_lib.load().qaoa_profile_read(self.h, int(reset), ctypes.byref(n),
                                                 ctypes.byref(ms), ctypes.byref(by)))
        return n.value, ms.value, by.value

    def plan(self, prec, B, n, p, S=1, grad=False) -> dict:
        info = _lib.PlanInfo()
        _lib.check(_lib.load().qaoa_plan(self.h, _prec(prec), B, n, p, S, int(grad),
                                         ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in info._fields_}


_ctx_lock = threading.Lock()
_default = {}


def default_context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    with _ctx_lock:
        if device not in _default:
            _default[device] = Context(device)
        return _default[device]


def host_context() -> Context:
    """A context that validates and plans but runs nothing (no GPU needed)."""
    with _ctx_lock:
        if "host" not in _default:
            _default["host"] = Context(_lib.QAOA_DEVICE_NONE)
        return _default["host"]


def _dev(t: torch.Tensor, name: str, dtype=torch.float64) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    return t.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _shape_qp(Q, gammas, betas):
    """Q [B,n,n] or [n,n]; gammas/betas [B,S,p], [S,p] or [p]."""
    if Q.dim() == 2:
        Q = Q.unsqueeze(0)
    B, n, n2 = Q.shape
    if n != n2:
        raise ValueError("Q must be square")
    g, b = gammas, betas
    if g.shape != b.shape:
        raise ValueError("gammas and betas must have the same shape")
    if g.dim() == 1:
        g, b = g.view(1, 1, -1), b.view(1, 1, -1)
    elif g.dim() == 2:
        g, b = g.unsqueeze(0), b.unsqueeze(0)
    if g.shape[0] != B:
        raise ValueError("leading dimension of gammas must match Q's batch")
    return Q, g, b, B, n, g.shape[1], g.shape[2]


def expect(Q, gammas, betas, prec="c64", probs=False, norm=False, ctx=None):
    """<C> [B, S] of the Eq. (2) states (optionally norms and |psi|^2)."""
    Q = _dev(Q, "Q")
    gammas = _dev(gammas, "gammas")
    betas = _dev(betas, "betas")
    Q, g, b, B, n, S, p = _shape_qp(Q, gammas, betas)
    pc = _prec(prec)
    ctx = ctx or default_context(Q.device.index)
    dev = Q.device
    e = torch.empty((B, S), dtype=torch.float64, device=dev)
    nr = torch.empty((B, S), dtype=torch.float64, device=dev) if norm else None
    P = None
    if probs:
        dt = torch.float64 if pc == _lib.QAOA_C128 else torch.float32
        P = torch.empty((B, S, 1 << n), dtype=dt, device=dev)
    _lib.check(_lib.load().qaoa_expect(ctx.h, pc, B, n, p, S, _ptr(Q), _ptr(g), _ptr(b),
                                       _ptr(e), _ptr(nr), _ptr(P), _stream()))
    out = [e]
    if norm:
        out.append(nr)
    if probs:
        out.append(P)
    return out[0] if len(out) == 1 else tuple(out)


class Evaluator:
    """Repeated <C> evaluations of fixed problems, for optimiser loops.

    Q ([B,n,n] or [n,n]), the number of parameter sets S, the depth p, the
    precision and the output buffers are bound once; each call passes new
    gammas and betas (float64 [B,S,p], contiguous, on Q's GPU) to one
    qaoa_expect on the stream that was current when the evaluator was made,
    and returns the bound <C> tensor [B,S] (overwritten by the next call;
    `norm` and `probs` likewise when requested).  It saves the per-call
    argument handling and output allocation of expect()."""

    def __init__(self, Q, S: int, p: int, prec="c64", probs=False, norm=False, ctx=None):
        Q = _dev(Q, "Q")
        if Q.dim() == 2:
            Q = Q.unsqueeze(0)
        B, n, n2 = Q.shape
        if n != n2:
            raise ValueError("Q must be square")
        pc = _prec(prec)
        self.Q = Q
        self.shape = torch.Size((B, int(S), int(p)))
        self.device = Q.device
        self.ctx = ctx or default_context(Q.device.index)
        self.expect = torch.empty((B, S), dtype=torch.float64, device=Q.device)
        self.norm = torch.empty((B, S), dtype=torch.float64, device=Q.device) if norm else None
        self.probs = None
        if probs:
            dt = torch.float64 if pc == _lib.QAOA_C128 else torch.float32
            self.probs = torch.empty((B, S, 1 << n), dtype=dt, device=Q.device)
        self._fn = _lib.load().qaoa_expect
        self._head = (self.ctx.h, pc, B, n, int(p), int(S), Q.data_ptr())
        self._tail = (self.expect.data_ptr(),
                      self.norm.data_ptr() if norm else None,
                      self.probs.data_ptr() if probs else None,
                      torch.cuda.current_stream(Q.device).cuda_stream)

    def __call__(self, gammas: torch.Tensor, betas: torch.Tensor) -> torch.Tensor:
        for t in (gammas, betas):
            if (t.shape != self.shape or t.dtype != torch.float64 or t.device != self.device
                    or not t.is_contiguous()):
                raise ValueError(f"gammas and betas must be contiguous float64 {tuple(self.shape)} "
                                 f"on {self.device}")
        rc = self._fn(*self._head, gammas.data_ptr(), betas.data_ptr(), *self._tail)
        if rc:
            _lib.check(rc)
        return self.expect


def expect_noalloc(Q, gammas, betas, out, norm=None, probs=None, prec="c64", ctx=None):
    """qaoa_expect_noalloc: <C> into the caller's ``out`` [B, S] (and norms
    [B, S], |psi|^2 [B, S, 2^n] if given) with no device allocation by the
    library: its working memory is the library's fixed per-GPU scratch."""
    Q = _dev(Q, "Q")
    gammas = _dev(gammas, "gammas")
    betas = _dev(betas, "betas")
    Q, g, b, B, n, S, p = _shape_qp(Q, gammas, betas)
    pc = _prec(prec)
    for t, name in ((out, "out"), (norm, "norm")):
        if t is not None and (t.dtype != torch.float64 or not t.is_cuda or t.numel() != B * S
                              or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous GPU float64 tensor of {B * S}")
    if probs is not None:
        dt = torch.float64 if pc == _lib.QAOA_C128 else torch.float32
        if probs.dtype != dt or not probs.is_cuda or probs.numel() != B * S << n or \
                not probs.is_contiguous():
            raise ValueError(f"probs must be a contiguous GPU {dt} tensor of {B * S << n}")
    ctx = ctx or default_context(Q.device.index)
    _lib.check(_lib.load().qaoa_expect_noalloc(ctx.h, pc, B, n, p, S, _ptr(Q), _ptr(g), _ptr(b),
                                               _ptr(out), _ptr(norm), _ptr(probs), _stream()))
    return out


def state(Q, gammas, betas, prec="c64", ctx=None):
    """(psi [B, S, 2^n] complex128/complex64, <C> [B, S], norm [B, S])."""
    Q = _dev(Q, "Q")
    gammas = _dev(gammas, "gammas")
    betas = _dev(betas, "betas")
    Q, g, b, B, n, S, p = _shape_qp(Q, gammas, betas)
    pc = _prec(prec)
    ctx = ctx or default_context(Q.device.index)
    dev = Q.device
    dt = torch.complex128 if pc == _lib.QAOA_C128 else torch.complex64
    psi = torch.empty((B, S, 1 << n), dtype=dt, device=dev)
    e = torch.empty((B, S), dtype=torch.float64, device=dev)
    nr = torch.empty((B, S), dtype=torch.float64, device=dev)
    _lib.check(_lib.load().qaoa_state(ctx.h, pc, B, n, p, S, _ptr(Q), _ptr(g), _ptr(b),
                                      _ptr(psi), _ptr(e), _ptr(nr), _stream()))
    return psi, e, nr


def sample(Q, gammas, betas, shots: int, seed: int, prec="c64", ctx=None):
    """dict(z [B, shots] int64 view of uint64, cz, best_z [B], best_c [B],
    expect [B]).  Problem b uses SplitMix64 counters b*shots + s."""
    Q = _dev(Q, "Q")
    gammas = _dev(gammas, "gammas")
    betas = _dev(betas, "betas")
    if Q.dim() == 2:
        Q = Q.unsqueeze(0)
    B, n, _ = Q.shape
    g = gammas.view(B, -1)
    b = betas.view(B, -1)
    p = g.shape[1]
    ctx = ctx or default_context(Q.device.index)
    dev = Q.device
    z = torch.empty((B, shots), dtype=torch.int64, device=dev)
    cz = torch.empty((B, shots), dtype=torch.float64, device=dev)
    bz = torch.empty((B,), dtype=torch.int64, device=dev)
    bc = torch.empty((B,), dtype=torch.float64, device=dev)
    e = torch.empty((B,), dtype=torch.float64, device=dev)
    _lib.check(_lib.load().qaoa_sample(ctx.h, _prec(prec), B, n, p, _ptr(Q), _ptr(g), _ptr(b),
                                       int(shots), int(seed) & (2**64 - 1), _ptr(z), _ptr(cz),
                                       _ptr(bz), _ptr(bc), _ptr(e), _stream()))
    return dict(z=z, cz=cz, best_z=bz, best_c=bc, expect=e)


def grad(Q, gammas, betas, prec="c64", ctx=None):
    """(<C> [B,S], d<C>/dgamma [B,S,p], d<C>/dbeta [B,S,p]) by the adjoint
    method."""
    Q = _dev(Q, "Q")
    gammas = _dev(gammas, "gammas")
    betas = _dev(betas, "betas")
    Q, g, b, B, n, S, p = _shape_qp(Q, gammas, betas)
    ctx = ctx or default_context(Q.device.index)
    dev = Q.device
    e = torch.empty((B, S), dtype=torch.float64, device=dev)
    dg = torch.empty((B, S, p), dtype=torch.float64, device=dev)
    db = torch.empty((B, S, p), dtype=torch.float64, device=dev)
    _lib.check(_lib.load().qaoa_grad(ctx.h, _prec(prec), B, n, p, S, _ptr(Q), _ptr(g),
                                     _ptr(b), _ptr(e), _ptr(dg), _ptr(db), _stream()))
    return e, dg, db


class QAOAExpect(torch.autograd.Function):
    """<C>(gamma, beta) with the adjoint-kernel gradient.

    forward(Q [B,n,n], gammas [B,S,p], betas [B,S,p], prec) -> <C> [B,S];
    backward scales d<C>/dgamma and d<C>/dbeta by grad_output."""

    @staticmethod
    def forward(ctx, Q, gammas, betas, prec="c64"):
        e, dg, db = grad(Q.detach(), gammas.detach(), betas.detach(), prec=prec)
        ctx.save_for_backward(dg, db)
        ctx.gshape = gammas.shape
        return e.view(gammas.shape[:-1])

    @staticmethod
    def backward(ctx, go):
        dg, db = ctx.saved_tensors
        go = go.reshape(dg.shape[:-1]).unsqueeze(-1)
        return None, (dg * go).view(ctx.gshape), (db * go).view(ctx.gshape), None


# ---- DQAOA outer cycle (Sec. V) -------------------------------------------

def impact(Q, x, ctx=None):
    """Impact factors of the global solution x (uint8 [N]) on Q [N, N]:
    (impact [N], field (Q + Q^T) x [N], order [N] int32, energy [1])."""
    Q = _dev(Q, "Q")
    x = _dev(x, "x", torch.uint8)
    N = Q.shape[0]
    if Q.shape != (N, N) or x.shape != (N,):
        raise ValueError("Q must be [N, N] and x [N]")
    ctx = ctx or default_context(Q.device.index)
    dev = Q.device
    imp = torch.empty(N, dtype=torch.float64, device=dev)
    field = torch.empty(N, dtype=torch.float64, device=dev)
    order = torch.empty(N, dtype=torch.int32, device=dev)
    e = torch.empty(1, dtype=torch.float64, device=dev)
    _lib.check(_lib.load().qaoa_impact(ctx.h, N, _ptr(Q), _ptr(x), _ptr(imp), _ptr(field),
                                       _ptr(order), _ptr(e), _stream()))
    return imp, field, order, e


def ifd_choices(order, m: int, k: int, stride: int = 1, ctx=None):
    """IFD windows [m, k] int32 from a ranking (qaoa_ifd_choices)."""
    order = _dev(order, "order", torch.int32)
    N = order.shape[0]
    ctx = ctx or default_context(order.device.index)
    ch = torch.empty((m, k), dtype=torch.int32, device=order.device)
    _lib.check(_lib.load().qaoa_ifd_choices(ctx.h, N, _ptr(order), m, k, stride, _ptr(ch),
                                            _stream()))
    return ch


def traversal_choices(Q, impact, order, m: int, k: int, mode: str = "pfs", ctx=None):
    """BFS ("bfs") or PFS ("pfs") windows [m, k] int32 (qaoa_traversal_choices)
    from impact factors and their ranking (as api.impact returns them)."""
    Q = _dev(Q, "Q")
    impact = _dev(impact, "impact")
    order = _dev(order, "order", torch.int32)
    N = Q.shape[0]
    ctx = ctx or default_context(Q.device.index)
    md = {"bfs": _lib.QAOA_DECOMP_BFS, "pfs": _lib.QAOA_DECOMP_PFS}[mode]
    ch = torch.empty((m, k), dtype=torch.int32, device=Q.device)
    _lib.check(_lib.load().qaoa_traversal_choices(ctx.h, N, _ptr(Q), _ptr(impact), _ptr(order), md,
                                                  m, k, _ptr(ch), _stream()))
    return ch


def decompose(Q, choices, ctx=None):
    """Sub-QUBOs Q[S_t, S_t] [m, k, k] of the windows choices [m, k] int32."""
    Q = _dev(Q, "Q")
    choices = _dev(choices, "choices", torch.int32)
    N = Q.shape[0]
    m, k = choices.shape
    ctx = ctx or default_context(Q.device.index)
    sq = torch.empty((m, k, k), dtype=torch.float64, device=Q.device)
    _lib.check(_lib.load().qaoa_decompose(ctx.h, N, _ptr(Q), m, k, _ptr(choices), _ptr(sq),
                                          _stream()))
    return sq


def aggregate(Q, x, field, energy, choices, subsol, ctx=None):
    """Fold sub-solutions subsol [m] uint64 into x, field and energy in
    place (qaoa_aggregate); returns accepted [m] int32."""
    Q = _dev(Q, "Q")
    for t, nm, dt in ((x, "x", torch.uint8), (field, "field", torch.float64),
                      (energy, "energy", torch.float64)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise TypeError(f"{nm} must be a contiguous {dt} GPU tensor (updated in place)")
    choices = _dev(choices, "choices", torch.int32)
    subsol = _dev(subsol, "subsol",
                  subsol.dtype if subsol.dtype in (torch.int64, torch.uint64) else torch.uint64)
    N = Q.shape[0]
    m, k = choices.shape
    ctx = ctx or default_context(Q.device.index)
    acc = torch.empty(m, dtype=torch.int32, device=Q.device)
    _lib.check(_lib.load().qaoa_aggregate(ctx.h, N, _ptr(Q), _ptr(x), _ptr(field), _ptr(energy),
                                          m, k, _ptr(choices), _ptr(subsol), _ptr(acc),
                                          _stream()))
    return acc


def cvar(cz, alpha: float = 1.0, ctx=None):
    """CVaR_alpha [B] of shot energies cz [B, shots] (qaoa_cvar); alpha = 1
    is the shot mean."""
    cz = _dev(cz, "cz")
    if cz.dim() == 1:
        cz = cz.unsqueeze(0)
    B, K = cz.shape
    ctx = ctx or default_context(cz.device.index)
    out = torch.empty(B, dtype=torch.float64, device=cz.device)
    _lib.check(_lib.load().qaoa_cvar(ctx.h, B, K, _ptr(cz), float(alpha), _ptr(out), _stream()))
    return out


def sampled_objective(Q, gammas, betas, shots: int, seed: int, alpha: float = 1.0, prec="c64",
                      ctx=None):
    """The objective of a sampler-based QAOA: CVaR_alpha [B] of the energies
    of `shots` samples per problem (qaoa_sample, then qaoa_cvar)."""
    s = sample(Q, gammas, betas, shots, seed, prec=prec, ctx=ctx)
    return cvar(s["cz"], alpha, ctx=ctx)


def cobyla(Q, theta0, rhobeg: float = 0.5, rhoend: float = 1e-6, maxfun: int = 200,
           prec="c128", trace: bool = False, ctx=None):
    """COBYLA-type minimisation of <C> over (gamma, beta) for every problem
    Q [B, n, n] (GPU float64) from theta0 [B, 2p] (host array), batched:
    every round of requests is one qaoa_expect (qaoa_cobyla).  Returns
    dict(theta [B, 2p], expect [B], nfev [B], rounds), plus trace [B,
    maxfun, 2p + 1] (each evaluated point and its <C>) if ``trace``."""
    import numpy as np
    Q = _dev(Q, "Q")
    if Q.dim() == 2:
        Q = Q.unsqueeze(0)
    B, n, _ = Q.shape
    th0 = np.ascontiguousarray(theta0, dtype=np.float64).reshape(B, -1)
    if th0.shape[1] % 2:
        raise ValueError("theta0 must be [B, 2p]")
    p = th0.shape[1] // 2
    ctx = ctx or default_context(Q.device.index)
    th = np.empty_like(th0)
    e = np.empty(B)
    nf = np.empty(B, dtype=np.int32)
    tr = np.full((B, int(maxfun), 2 * p + 1), np.nan) if trace else None
    r = ctypes.c_int(0)
    cp = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None
    _lib.check(_lib.load().qaoa_cobyla(ctx.h, _prec(prec), B, n, p, _ptr(Q), cp(th0),
                                       float(rhobeg), float(rhoend), int(maxfun), cp(th), cp(e),
                                       cp(nf), ctypes.cast(ctypes.pointer(r), ctypes.c_void_p),
                                       cp(tr), _stream()))
    out = dict(theta=th, expect=e, nfev=nf, rounds=r.value)
    if trace:
        out["trace"] = tr
    return out
