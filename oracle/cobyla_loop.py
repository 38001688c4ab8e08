"""CPU oracle for the COBYLA variational loop: TEST INFRASTRUCTURE ONLY.

The paper's setting (Sec. IV): each sub-QUBO's (gamma, beta) start from
random values and are optimised by COBYLA on the exact objective <C> of
Eq. (1).  This is that loop, one sub-QUBO at a time, with SciPy's COBYLA as
the optimiser step and the complex128 oracle as the objective.  Only the
tests and the benchmark's CPU-baseline leg use it; it imports nothing from
the HIP package.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize

from . import expect


def cobyla_loop(Q, theta0, maxiter: int = 200, rhobeg: float = 0.5, tol: float = 1e-6):
    """Returns (theta, <C>, nfev) for theta0 = (gamma_1..p, beta_1..p)."""
    theta0 = np.asarray(theta0, dtype=np.float64)
    p = theta0.size // 2

    def f(x):
        e, _, _ = expect(Q, x[None, :p], x[None, p:])
        return float(e[0])

    r = minimize(f, theta0, method="COBYLA",
                 options=dict(maxiter=maxiter, rhobeg=rhobeg, tol=tol))
    return r.x, float(r.fun), int(r.nfev)
