"""Seeded synthetic workloads: the only code shared by the HIP path's tests,
the benchmark and the oracle's tests.  It draws inputs; it holds none of the
method's arithmetic.

The paper's own instances (metamaterial-design QUBOs and Max-Cut graphs,
Sec. V-A) are not available, so dense QUBOs with i.i.d. uniform[-1, 1]
entries stand in for them, with sub-QUBO sizes 12..22 spanning the sizes the
paper uses (12 and 20, inside its 4..28 sweep, Sec. V-B).
"""
from __future__ import annotations

import numpy as np


def qubo(n: int, seed: int) -> np.ndarray:
    """Symmetric dense QUBO: the upper triangle (diagonal included) is i.i.d.
    uniform[-1, 1] from ``default_rng(seed)`` and is mirrored below."""
    rng = np.random.default_rng(seed)
    Q = np.zeros((n, n))
    iu = np.triu_indices(n)
    Q[iu] = rng.uniform(-1.0, 1.0, size=iu[0].shape[0])
    return Q + np.triu(Q, 1).T


def qubos(count: int, n: int, seed: int) -> np.ndarray:
    """``count`` independent symmetric QUBOs [count][n][n] from one stream."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count, n, n))
    iu = np.triu_indices(n)
    for b in range(count):
        out[b][iu] = rng.uniform(-1.0, 1.0, size=iu[0].shape[0])
        out[b] = out[b] + np.triu(out[b], 1).T
    return out


def params(sets: int, p: int, seed: int, lead=()):
    """(gammas, betas) of shape [*lead, sets, p]: gamma ~ U[0, pi],
    beta ~ U[0, pi/2]."""
    rng = np.random.default_rng(seed)
    shape = tuple(lead) + (sets, p)
    g = rng.uniform(0.0, np.pi, size=shape)
    b = rng.uniform(0.0, np.pi / 2, size=shape)
    return g, b


def subqubo_requests(count: int, N: int = 1000, n_lo: int = 12, n_hi: int = 22,
                     seed: int = 3):
    """Random decomposition of one dense N x N QUBO (Sec. V-A-1): each request
    takes n ~ U{n_lo..n_hi} distinct variables, sorted ascending, and the full
    principal submatrix Q[S, S] (qubit r = r-th smallest chosen variable).
    Returns (Qglobal, list of (indices, subQ))."""
    Qg = qubo(N, seed)
    rng = np.random.default_rng(seed + 1000003)
    reqs = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        idx = np.sort(rng.choice(N, size=n, replace=False))
        reqs.append((idx, np.ascontiguousarray(Qg[np.ix_(idx, idx)])))
    return Qg, reqs


def maxcut_qubo(N: int, seed: int, edges: int | None = None):
    """Unweighted Max-Cut instance of Sec. VI-B: floor(N(N-1)/8) distinct
    edges drawn uniformly from all node pairs (25% of a complete graph), as
    the QUBO minimising minus the cut: Q_ii = -deg(i), Q_ij = Q_ji = 1 per
    edge, so x^T Q x = -(number of cut edges).  Returns (Q, edges [E, 2])."""
    rng = np.random.default_rng(seed)
    E = N * (N - 1) // 8 if edges is None else edges
    pairs = rng.choice(N * (N - 1) // 2, size=E, replace=False)
    # pair index -> (i, j), i < j, in row-major order of the upper triangle
    i = (N - 2 - np.floor(np.sqrt(-8.0 * pairs + 4.0 * N * (N - 1) - 7) / 2.0 - 0.5)).astype(np.int64)
    j = (pairs + i + 1 - N * (N - 1) // 2 + (N - i) * ((N - i) - 1) // 2).astype(np.int64)
    Q = np.zeros((N, N))
    Q[i, j] = 1.0
    Q[j, i] = 1.0
    Q[np.arange(N), np.arange(N)] = -Q.sum(axis=1)
    return Q, np.stack([i, j], axis=1)


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


# The five workloads the library is measured and tested on.
WORKLOADS = {
    "plain_n10": dict(n=10, p=2, sets=64, prec="c128", q_seed=1, p_seed=11),
    "precision_n24": dict(n=24, p=4, sets=16, prec="c64", q_seed=2, p_seed=12),
    "serving": dict(requests=4096, N=1000, n_lo=12, n_hi=22, p=3, evals=100,
                    shots=1024, prec="c64", q_seed=3, arrival_seed=4),
    "diff_n16": dict(batch=512, n=16, p=6, prec="c64", q_seed=5, p_seed=15),
    "large_n32": dict(n=32, p=2, sets=4, prec="c64", q_seed=6, p_seed=16),
}
