"""Pins of the BFS / PFS decomposition oracle (oracle/traversal.py) and of
the Max-Cut QUBO generator: a hand-worked example shaped like the paper's
traversal figure (tests/golden/traversal_example.txt), connectivity of the
windows, and the Max-Cut energy as minus the number of cut edges (counted
edge by edge), with its brute-force optimum."""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle.traversal import bfs_window, pfs_window, traversal_choices
from paper_2506_10531_amd import workloads

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "traversal_example.txt")
GOLD_W = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "traversal_weighted.txt")


def _golden(path=GOLD):
    rec = {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            rec[k.strip()] = [float(x) for x in v.split()]
    return rec


def _example_q():
    Q = np.zeros((7, 7))
    for a, b in ((0, 1), (0, 3), (1, 6), (3, 4)):
        Q[a, b] = Q[b, a] = 0.5
    return Q


def test_hand_example():
    g = _golden()
    imp = np.array(g["impact"])
    Q = _example_q()
    assert bfs_window(Q, imp, 0, 3) == [int(v) for v in g["bfs_k3"]]
    assert pfs_window(Q, imp, 0, 3) == [int(v) for v in g["pfs_k3"]]
    assert bfs_window(Q, imp, 0, 5) == [int(v) for v in g["bfs_k5"]]
    assert pfs_window(Q, imp, 0, 4) == [int(v) for v in g["pfs_k4"]]
    assert bfs_window(Q, imp, 0, 6) == [int(v) for v in g["bfs_k6"]]
    assert pfs_window(Q, imp, 0, 6) == [int(v) for v in g["pfs_k6"]]


def weighted_example_q():
    """The eight-variable QUBO of tests/golden/traversal_weighted.txt: unequal,
    signed and asymmetric couplings (Q_ij, Q_ji)."""
    Q = np.zeros((8, 8))
    for (a, b), (qab, qba) in {(0, 1): (0.1, 0.1), (0, 3): (1.0, 0.0), (0, 5): (-1.2, 0.6),
                               (3, 4): (0.3, 0.0), (3, 6): (0.0, -0.9), (5, 2): (0.4, 0.4),
                               (1, 7): (0.25, 0.25)}.items():
        Q[a, b], Q[b, a] = qab, qba
    return Q


def test_bfs_strongest_first_by_coupling_sum():
    g = _golden(GOLD_W)
    imp = np.array(g["impact"])
    Q = weighted_example_q()
    for k in range(2, 9):
        assert bfs_window(Q, imp, 0, k) == [int(v) for v in g[f"bfs_k{k}"]], k


@pytest.mark.parametrize("mode", ["bfs", "pfs"])
def test_windows_are_connected_and_seeded(mode):
    Q, _ = workloads.maxcut_qubo(60, 3)
    W = Q + Q.T
    np.fill_diagonal(W, 0.0)
    imp = np.random.default_rng(1).normal(size=60)
    order = np.lexsort((np.arange(60), -np.abs(imp)))
    ch = traversal_choices(Q, imp, order, 20, 12, mode)
    for t, c in enumerate(ch):
        assert len(set(c.tolist())) == 12 and order[t] in c
        # the induced interaction graph of the window is connected (dense
        # enough graph: no restart was needed)
        seen, todo = {int(order[t])}, [int(order[t])]
        while todo:
            u = todo.pop()
            for v in c:
                if int(v) not in seen and W[u, v] != 0.0:
                    seen.add(int(v))
                    todo.append(int(v))
        assert seen == set(c.tolist())


def test_maxcut_energy_is_minus_cut():
    Q, edges = workloads.maxcut_qubo(11, 7)
    assert len(edges) == 11 * 10 // 8
    for z in (0, 5, 1023, 2047, 1234):
        x = (z >> np.arange(11)) & 1
        cut = sum(1 for a, b in edges if x[a] != x[b])
        assert oracle.energy(Q, z) == -cut
    best = max(sum(1 for a, b in edges if ((z >> a) & 1) != ((z >> b) & 1))
               for z in range(1 << 11))
    assert oracle.argmin(Q)[1] == -best
