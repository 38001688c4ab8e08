"""CPU oracle for the QAOA state-vector path: TEST INFRASTRUCTURE ONLY.

A plain complex128 / FP64 implementation of Eq. (1)-(2) of arXiv 2506.10531
(Sec. IV), written in C++ (``oracle.cpp``) and reached through ctypes.  Only
the tests, the smoke check and the benchmark's CPU-baseline leg use it; the
HIP library never imports, links or calls anything here, and this module
imports nothing from the HIP package.

Every function takes NumPy arrays and returns NumPy arrays.  Parameter arrays
are laid out ``[S][p]`` (S parameter sets, p layers), row-major FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")

_dp = ctypes.POINTER(ctypes.c_double)
_up = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile ``oracle.cpp`` into ``liboracle.so`` with g++ and OpenMP."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
             "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_energy.restype = ctypes.c_double
        lib.oracle_energy.argtypes = [ctypes.c_int, _dp, ctypes.c_uint64]
        lib.oracle_uniform.restype = ctypes.c_double
        lib.oracle_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_cost_table.argtypes = [ctypes.c_int, _dp, _dp]
        lib.oracle_state.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp]
        lib.oracle_expect.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      _dp, _dp, _dp, _dp, _dp, _dp]
        lib.oracle_grad.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    _dp, _dp, _dp, _dp, _dp, _dp]
        lib.oracle_sample.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp,
                                      ctypes.c_int, ctypes.c_uint64, _up, _dp,
                                      _up, _dp, _dp]
        lib.oracle_adam_solve.argtypes = [
            ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int,
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_int, ctypes.c_uint64, _dp, _dp, _dp, _up, _dp, _up, _dp]
        lib.oracle_argmin.argtypes = [ctypes.c_int, _dp, _up, _dp]
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _pu(a):
    return a.ctypes.data_as(_up) if a is not None else None


def _params(gammas, betas):
    g = _f64(gammas)
    b = _f64(betas)
    if g.ndim == 1:
        g = g[None, :]
        b = b[None, :]
    assert g.shape == b.shape
    return g, b


def num_threads() -> int:
    """OpenMP threads the oracle uses (the host cores it runs on)."""
    return int(_load().oracle_num_threads())


def energy(Q, z: int) -> float:
    """C(z) = z^T Q z for one bit string (bit i of z is variable i)."""
    Q = _f64(Q)
    return float(_load().oracle_energy(Q.shape[0], _p(Q), int(z)))


def uniform(seed: int, s: int) -> float:
    """The sampler's uniform u_s in [0, 1) (SplitMix64 at counter s)."""
    return float(_load().oracle_uniform(int(seed), int(s)))


def cost_table(Q) -> np.ndarray:
    Q = _f64(Q)
    n = Q.shape[0]
    C = np.empty(1 << n)
    _load().oracle_cost_table(n, _p(Q), _p(C))
    return C


def state(Q, gammas, betas) -> np.ndarray:
    """|psi(theta)> of Eq. (2) as complex128 [2^n]."""
    Q = _f64(Q)
    g, b = _params(gammas, betas)
    n, p = Q.shape[0], g.shape[1]
    out = np.empty(2 << n)
    _load().oracle_state(n, p, _p(Q), _p(g[0]), _p(b[0]), _p(out))
    return out.view(np.complex128)


def expect(Q, gammas, betas, probs: bool = False):
    """(<C>[S], norm[S], probs[S][2^n] or None) for S parameter sets."""
    Q = _f64(Q)
    g, b = _params(gammas, betas)
    n, (S, p) = Q.shape[0], g.shape
    e = np.empty(S)
    nr = np.empty(S)
    P = np.empty((S, 1 << n)) if probs else None
    _load().oracle_expect(n, p, S, _p(Q), _p(g), _p(b), _p(e), _p(nr), _p(P))
    return e, nr, P


def grad(Q, gammas, betas):
    """(<C>[S], d<C>/dgamma[S][p], d<C>/dbeta[S][p]) by the adjoint method."""
    Q = _f64(Q)
    g, b = _params(gammas, betas)
    n, (S, p) = Q.shape[0], g.shape
    e = np.empty(S)
    dg = np.empty((S, p))
    db = np.empty((S, p))
    _load().oracle_grad(n, p, S, _p(Q), _p(g), _p(b), _p(e), _p(dg), _p(db))
    return e, dg, db


def sample(Q, gammas, betas, shots: int, seed: int):
    """dict(z, cz, best_z, best_c, gap) for one parameter set."""
    Q = _f64(Q)
    g, b = _params(gammas, betas)
    n, p = Q.shape[0], g.shape[1]
    z = np.empty(shots, dtype=np.uint64)
    cz = np.empty(shots)
    gap = np.empty(shots)
    bz = np.empty(1, dtype=np.uint64)
    bc = np.empty(1)
    _load().oracle_sample(n, p, _p(Q), _p(g[0]), _p(b[0]), shots, int(seed),
                          _pu(z), _p(cz), _pu(bz), _p(bc), _p(gap))
    return dict(z=z, cz=cz, best_z=int(bz[0]), best_c=float(bc[0]), gap=gap)


def adam_solve(Q, gamma0, beta0, evals=100, lr=0.05, b1=0.9, b2=0.999,
               eps=1e-8, shots=1024, seed=0):
    """One serving-loop solve: `evals` Adam steps on the exact gradient, then
    <C> and `shots` samples at the final parameters."""
    Q = _f64(Q)
    g0 = _f64(gamma0).ravel()
    b0 = _f64(beta0).ravel()
    n, p = Q.shape[0], g0.shape[0]
    go = np.empty(p)
    bo = np.empty(p)
    e = np.empty(1)
    z = np.empty(shots, dtype=np.uint64)
    cz = np.empty(shots)
    bz = np.empty(1, dtype=np.uint64)
    bc = np.empty(1)
    _load().oracle_adam_solve(n, p, _p(Q), _p(g0), _p(b0), int(evals), lr, b1,
                              b2, eps, int(shots), int(seed), _p(go), _p(bo),
                              _p(e), _pu(z), _p(cz), _pu(bz), _p(bc))
    return dict(gamma=go, beta=bo, expect=float(e[0]), z=z, cz=cz,
                best_z=int(bz[0]), best_c=float(bc[0]))


def argmin(Q):
    """Exhaustive (z*, C(z*)); ties to the smallest z."""
    Q = _f64(Q)
    z = np.empty(1, dtype=np.uint64)
    c = np.empty(1)
    _load().oracle_argmin(Q.shape[0], _p(Q), _pu(z), _p(c))
    return int(z[0]), float(c[0])
