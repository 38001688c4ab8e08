"""CPU oracle for the sampled objective: TEST INFRASTRUCTURE ONLY.

A sampler-based QAOA (the software the paper ran, Sec. IV) scores
parameters from the energies C(z_s) of K measured bit strings (the
measurement of Sec. IV) instead of the exact <C>.  The conditional value at
risk CVaR_alpha is the mean over the lowest alpha fraction of that
empirical distribution; alpha = 1 is the plain shot mean.  With the
energies sorted ascending, E_(1) <= ... <= E_(K):

    CVaR_alpha = ( sum_{k <= floor(alpha K)} E_(k)
                   + (alpha K - floor(alpha K)) E_(floor(alpha K) + 1) ) / (alpha K)

(the last term is absent when alpha K is an integer).  Only the tests use
this module; it imports nothing from the HIP package.
"""
from __future__ import annotations

import math

import numpy as np


def cvar(energies, alpha: float) -> float:
    e = np.sort(np.asarray(energies, dtype=np.float64))
    K = e.size
    a = alpha * K
    f = math.floor(a)
    s = float(e[:f].sum())
    if a > f:
        s += (a - f) * float(e[f])
    return s / a
