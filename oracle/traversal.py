"""CPU oracle for BFS / PFS decomposition: TEST INFRASTRUCTURE ONLY.

Sec. V-A-3 and its figure: breadth-first search (BFS) starts at the variable
of largest impact factor and proceeds to strongly interacting variables;
priority-first search (PFS) instead takes, among the unselected variables
that interact with any selected one, the one of largest impact factor.
Readings:
  * variables i and j interact when W_ij = Q_ij + Q_ji != 0 (i != j); the
    strength of the interaction is |W_ij|;
  * window t (t = 0..m-1) starts at order[t mod N] (order: the variables
    ranked by |impact|, largest first), and grows to k variables;
  * BFS takes the neighbours of the variable it expands in order of
    strength, strongest first (ties to the smaller index), each when it is
    first discovered; PFS adds the interacting unselected variable of
    largest |impact| (ties to the smaller index);
  * when no unselected variable interacts with the window, both continue
    from the unselected variable of largest |impact| (ties: smaller index);
  * the window is returned sorted ascending, like the IFD windows.
Plain Python over the dense matrix; it imports nothing from the HIP package.
"""
from __future__ import annotations

import numpy as np


def _key(imp, i):
    return (-abs(imp[i]), i)


def _restart(N, imp, sel):
    cand = [i for i in range(N) if i not in sel]
    return min(cand, key=lambda i: _key(imp, i)) if cand else None


def bfs_window(Q, imp, seed: int, k: int):
    Q = np.asarray(Q, dtype=np.float64)
    N = Q.shape[0]
    W = Q + Q.T
    sel, queue = [seed], [seed]
    seen = {seed}
    while len(sel) < k:
        if not queue:
            s = _restart(N, imp, seen)
            sel.append(s)
            seen.add(s)
            queue.append(s)
            continue
        u = queue.pop(0)
        nb = [v for v in range(N) if v != u and v not in seen and W[u, v] != 0.0]
        nb.sort(key=lambda v: (-abs(W[u, v]), v))
        for v in nb:
            if len(sel) == k:
                break
            sel.append(v)
            seen.add(v)
            queue.append(v)
    return sorted(sel)


def pfs_window(Q, imp, seed: int, k: int):
    Q = np.asarray(Q, dtype=np.float64)
    N = Q.shape[0]
    W = Q + Q.T
    sel = [seed]
    chosen = {seed}
    while len(sel) < k:
        front = [v for v in range(N) if v not in chosen
                 and any(W[u, v] != 0.0 for u in sel if u != v)]
        nxt = min(front, key=lambda v: _key(imp, v)) if front else _restart(N, imp, chosen)
        sel.append(nxt)
        chosen.add(nxt)
    return sorted(sel)


def traversal_choices(Q, imp, order, m: int, k: int, mode: str) -> np.ndarray:
    """Windows [m][k] of BFS (mode "bfs") or PFS (mode "pfs")."""
    f = bfs_window if mode == "bfs" else pfs_window
    N = len(order)
    return np.array([f(Q, imp, int(order[t % N]), k) for t in range(m)], dtype=np.int32)
