"""CPU oracle for the DQAOA outer cycle: TEST INFRASTRUCTURE ONLY.

Plain NumPy (FP64) versions of the classical steps around the QAOA solves
(arXiv 2506.10531, Sec. V): the energy of a global solution, the impact
factor of every variable, impact-factor directed (IFD) decomposition into
sub-QUBOs (Sec. V-A-2 and its algorithm), and the aggregation of
sub-solutions into the global solution (Sec. V, third step of the
workflow).  Each step is written from its definition, with no incremental
bookkeeping: energies are always evaluated in full.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg use this module; it imports
nothing from the HIP package.

Conventions (readings of the paper):
  * x is a 0/1 vector of the N global variables; E(x) = x^T Q x (Eq. (1)).
  * The impact factor of variable i is the energy change when x_i alone is
    flipped, E(x with x_i flipped) - E(x); variables are ranked by its
    magnitude, largest first, ties to the smaller index.
  * IFD window t (t = 0..m-1) takes the ranked variables at positions
    t*stride .. t*stride + k - 1 (cyclically), sorted ascending; stride 1 is
    the algorithm as printed.
  * A sub-QUBO is the full principal submatrix Q[S, S]; bit r of a sub-QUBO
    basis index is the r-th smallest variable of S.
  * Aggregation visits the sub-solutions in order; each overwrites the
    variables of its window and is kept only when the energy drops
    strictly.
"""
from __future__ import annotations

import numpy as np


def energy(Q, x) -> float:
    """E(x) = x^T Q x for a 0/1 vector x (Eq. (1))."""
    v = np.asarray(x, dtype=np.float64)
    return float(v @ np.asarray(Q, dtype=np.float64) @ v)


def impact(Q, x) -> np.ndarray:
    """Impact factor of every variable (Sec. V-A-2): flip it, evaluate the
    energy in full, subtract the current energy.  O(N^3), as the paper
    states for this step."""
    x = np.asarray(x, dtype=np.uint8)
    e0 = energy(Q, x)
    out = np.empty(x.size, dtype=np.float64)
    for i in range(x.size):
        y = x.copy()
        y[i] ^= 1
        out[i] = energy(Q, y) - e0
    return out


def rank(imp) -> np.ndarray:
    """Variables ordered by |impact factor|, largest first; ties go to the
    smaller index."""
    imp = np.asarray(imp, dtype=np.float64)
    idx = np.arange(imp.size)
    return np.lexsort((idx, -np.abs(imp))).astype(np.int32)


def ifd_choices(order, m: int, k: int, stride: int = 1) -> np.ndarray:
    """Variable windows of IFD decomposition: window t is the ranked list at
    positions t*stride + r (r < k, cyclic in N), sorted ascending."""
    order = np.asarray(order)
    N = order.size
    out = np.empty((m, k), dtype=np.int32)
    for t in range(m):
        out[t] = np.sort(order[(t * stride + np.arange(k)) % N])
    return out


def subqubos(Q, choices) -> np.ndarray:
    """The principal submatrices Q[S, S] of the windows, [m][k][k]."""
    Q = np.asarray(Q, dtype=np.float64)
    return np.stack([Q[np.ix_(c, c)] for c in np.asarray(choices)])


def aggregate(Q, x, choices, subsol):
    """Fold sub-solutions into the global solution in order: window t's
    variables take the bits of subsol[t] (bit r -> r-th smallest variable);
    the change is kept only if the full energy drops strictly.
    Returns (x, E(x), accepted[m])."""
    x = np.asarray(x, dtype=np.uint8).copy()
    e = energy(Q, x)
    acc = np.zeros(len(choices), dtype=bool)
    for t, (c, s) in enumerate(zip(np.asarray(choices), np.asarray(subsol, dtype=np.uint64))):
        bits = ((int(s) >> np.arange(len(c))) & 1).astype(np.uint8)
        y = x.copy()
        y[c] = bits
        e1 = energy(Q, y)
        if e1 < e:
            x, e = y, e1
            acc[t] = True
    return x, e, acc
