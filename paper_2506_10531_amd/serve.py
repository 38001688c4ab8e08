"""Python handle on the library's solve queue (continuous batching of
sub-QUBO solves on one GPU).  The scheduler, admission control and all GPU
work live in the HIP library; this module marshals requests and results."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from .api import Context, PREC, default_context


class SolveQueue:
    def __init__(self, ctx: Context | None = None, *, max_slots=64, max_pending=1 << 16,
                 hbm_budget=0, prec="c64", p=3, evals=100, shots=1024, lr=0.05,
                 beta1=0.9, beta2=0.999, eps=1e-8, batched=True):
        self.ctx = ctx or default_context()
        o = _lib.QueueOpts(max_slots=max_slots, max_pending=max_pending,
                           hbm_budget=hbm_budget, prec=PREC[prec] if isinstance(prec, str) else prec,
                           p=p, evals=evals, shots=shots, lr=lr, beta1=beta1,
                           beta2=beta2, eps=eps, batched=int(batched))
        self.opts = o
        self.p = p
        self.shots = shots
        h = ctypes.c_void_p()
        _lib.check(_lib.load().qaoa_queue_create(self.ctx.h, ctypes.byref(o), ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            _lib.load().qaoa_queue_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, Q, gamma0, beta0, seed: int, raise_full=True):
        """Returns a ticket, or None when the queue is full and raise_full is
        False."""
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        g = np.ascontiguousarray(gamma0, dtype=np.float64).ravel()
        b = np.ascontiguousarray(beta0, dtype=np.float64).ravel()
        assert g.size == self.p and b.size == self.p
        dp = ctypes.POINTER(ctypes.c_double)
        req = _lib.SolveReq(n=Q.shape[0], Q=Q.ctypes.data_as(dp),
                            gamma0=g.ctypes.data_as(dp), beta0=b.ctypes.data_as(dp),
                            seed=int(seed) & (2**64 - 1))
        t = ctypes.c_uint64()
        rc = _lib.load().qaoa_submit(self.h, ctypes.byref(req), ctypes.byref(t))
        if rc == _lib.ERR_QUEUE_FULL and not raise_full:
            return None
        _lib.check(rc)
        return t.value

    def _result(self, r: _lib.SolveResult, samples):
        return dict(status=r.status, n=r.n, gamma=np.array(r.gamma[: self.p]),
                    beta=np.array(r.beta[: self.p]), expect=r.expect, best_z=r.best_z,
                    best_c=r.best_c, t_submit_ns=r.t_submit_ns, t_admit_ns=r.t_admit_ns,
                    t_done_ns=r.t_done_ns, samples=samples)

    def poll(self, ticket: int):
        """The result dict once done, else None."""
        r = _lib.SolveResult()
        s = np.empty(self.shots, dtype=np.uint64)
        rc = _lib.check(_lib.load().qaoa_poll(self.h, ticket, ctypes.byref(r),
                                              s.ctypes.data_as(ctypes.c_void_p)),
                        allow=(_lib.OK, _lib.PENDING))
        if rc == _lib.PENDING:
            return None
        return self._result(r, s)

    def wait(self, ticket: int, timeout_s: float | None = None):
        r = _lib.SolveResult()
        s = np.empty(self.shots, dtype=np.uint64)
        to = -1 if timeout_s is None else int(timeout_s * 1e9)
        _lib.check(_lib.load().qaoa_wait(self.h, ticket, to, ctypes.byref(r),
                                         s.ctypes.data_as(ctypes.c_void_p)))
        return self._result(r, s)

    def cancel(self, ticket: int):
        _lib.check(_lib.load().qaoa_cancel(self.h, ticket))

    def stats(self) -> dict:
        st = _lib.QueueStats()
        _lib.check(_lib.load().qaoa_queue_get_stats(self.h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def dqaoa_cycle(self, Q, x, gamma0, beta0, m: int, k: int, *, mode="ifd", stride=1,
                    choices=None, seed: int = 0):
        """One DQAOA cycle (qaoa_dqaoa_cycle) on this queue: decomposition of
        Q [N, N] (GPU float64) around the global solution x (GPU uint8 [N],
        updated in place), m sub-QUBO solves of k qubits, aggregation.
        mode "ifd", "bfs" or "pfs" (windows from impact factors) or "given"
        (choices [m, k] int32 on the GPU, e.g. random windows).  Returns (field, energy,
        stats dict)."""
        import torch
        from .api import _dev, _ptr, _stream
        Q = _dev(Q, "Q")
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.uint8
                and x.is_contiguous()):
            raise TypeError("x must be a contiguous uint8 GPU tensor (updated in place)")
        N = Q.shape[0]
        L = _lib.load()
        md = {"ifd": _lib.QAOA_DECOMP_IFD, "bfs": _lib.QAOA_DECOMP_BFS,
              "pfs": _lib.QAOA_DECOMP_PFS, "given": _lib.QAOA_DECOMP_GIVEN}[mode]
        ch = None
        if md == _lib.QAOA_DECOMP_GIVEN:
            ch = _dev(choices, "choices", torch.int32)
        g = np.ascontiguousarray(gamma0, dtype=np.float64).ravel()
        b = np.ascontiguousarray(beta0, dtype=np.float64).ravel()
        assert g.size == self.p and b.size == self.p
        field = torch.empty(N, dtype=torch.float64, device=Q.device)
        energy = torch.empty(1, dtype=torch.float64, device=Q.device)
        ws = L.qaoa_cycle_workspace(N, m, k)
        work = torch.empty(max(int(ws), 1), dtype=torch.uint8, device=Q.device)
        st = _lib.CycleStats()
        _lib.check(L.qaoa_dqaoa_cycle(
            self.ctx.h, self.h, N, _ptr(Q), _ptr(x), _ptr(field), _ptr(energy), md, m, k,
            stride, _ptr(ch), g.ctypes.data_as(ctypes.c_void_p),
            b.ctypes.data_as(ctypes.c_void_p), int(seed) & (2**64 - 1), _ptr(work),
            ctypes.byref(st), _stream()))
        return field, energy, {f: getattr(st, f) for f, _ in st._fields_}
