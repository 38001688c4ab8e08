"""Pins of the outer-cycle oracle (oracle/cycle.py) against facts that do not
come from its own definitions: the one-flip closed form of the energy
change, decoupled (diagonal) QUBOs, hand-ranked and hand-windowed examples
(tests/golden/ifd_example.txt), sub-QUBO energies against the global energy,
and aggregation against brute-force optima."""
import itertools
import os

import numpy as np

import oracle
from oracle import cycle
from paper_2506_10531_amd import workloads

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_energy_matches_bitstring_energy():
    # x^T Q x equals the basis-state energy C(z) of the QAOA oracle
    Q = workloads.qubo(9, 31)
    for z in (0, 1, 5, 300, 511):
        x = ((z >> np.arange(9)) & 1).astype(np.uint8)
        assert abs(cycle.energy(Q, x) - oracle.energy(Q, z)) <= 1e-12


def test_impact_closed_form_nonsymmetric():
    # flipping x_i changes E by d_i (Q_ii + sum_{j != i} (Q_ij + Q_ji) x_j),
    # d_i = 1 - 2 x_i (expand (x + d e_i)^T Q (x + d e_i) with d^2 = 1)
    rng = np.random.default_rng(7)
    N = 40
    Q = rng.uniform(-1, 1, (N, N))
    x = rng.integers(0, 2, N).astype(np.uint8)
    imp = cycle.impact(Q, x)
    xf = x.astype(np.float64)
    for i in range(N):
        s = sum((Q[i, j] + Q[j, i]) * xf[j] for j in range(N) if j != i)
        assert abs(imp[i] - (1 - 2 * xf[i]) * (Q[i, i] + s)) <= 1e-12


def test_impact_diagonal_qubo_decouples():
    Q = np.diag(np.array([0.5, -2.0, 3.0, 0.0, -0.25]))
    x = np.array([1, 0, 1, 1, 0], dtype=np.uint8)
    assert np.array_equal(cycle.impact(Q, x), np.array([-0.5, -2.0, -3.0, 0.0, -0.25]))


def _golden():
    rec = {}
    for line in open(os.path.join(GOLD, "ifd_example.txt")):
        line = line.split("#")[0].strip()
        if line:
            key, val = line.split("=")
            rec[key.strip()] = [float(v) for v in val.split()]
    return rec


def test_rank_and_windows_hand_example():
    g = _golden()
    order = cycle.rank(np.array(g["impact"]))
    assert order.tolist() == [int(v) for v in g["order"]]
    ch = cycle.ifd_choices(order, m=3, k=2, stride=1)
    assert ch.tolist() == np.array(g["windows_k2_stride1"], dtype=int).reshape(3, 2).tolist()
    ch = cycle.ifd_choices(order, m=3, k=2, stride=2)
    assert ch.tolist() == np.array(g["windows_k2_stride2"], dtype=int).reshape(3, 2).tolist()


def test_subqubo_energy_is_global_energy_with_others_zero():
    rng = np.random.default_rng(3)
    N, k = 30, 6
    Q = workloads.qubo(N, 8)
    ch = np.stack([np.sort(rng.choice(N, size=k, replace=False)) for _ in range(4)])
    sq = cycle.subqubos(Q, ch)
    for t in range(4):
        for z in range(1 << k):
            x = np.zeros(N, dtype=np.uint8)
            x[ch[t]] = (z >> np.arange(k)) & 1
            assert abs(oracle.energy(sq[t], z) - cycle.energy(Q, x)) <= 1e-12


def test_aggregate_never_increases_and_reaches_brute_force_optimum():
    N = 10
    Q = workloads.qubo(N, 44)
    zmin, emin = oracle.argmin(Q)
    xopt = ((zmin >> np.arange(N)) & 1).astype(np.uint8)
    x0 = np.zeros(N, dtype=np.uint8)
    # a window holding every variable with the optimum as its sub-solution
    ch = np.arange(N, dtype=np.int32)[None, :]
    x1, e1, acc = cycle.aggregate(Q, x0, ch, np.array([zmin], dtype=np.uint64))
    assert abs(e1 - emin) <= 1e-12 and np.array_equal(x1, xopt)
    assert acc.tolist() == [emin < 0.0]
    # random proposals: energy never rises, the final energy is exact, and a
    # proposal equal to the current restriction is rejected
    rng = np.random.default_rng(9)
    ch = np.stack([np.sort(rng.choice(N, size=4, replace=False)) for _ in range(20)]).astype(np.int32)
    sub = rng.integers(0, 16, 20).astype(np.uint64)
    x, e = x0.copy(), cycle.energy(Q, x0)
    xf, ef, acc = cycle.aggregate(Q, x0, ch, sub)
    for t in range(20):
        y = x.copy()
        y[ch[t]] = (int(sub[t]) >> np.arange(4)) & 1
        if acc[t]:
            assert cycle.energy(Q, y) < e
            x, e = y, cycle.energy(Q, y)
        else:
            assert cycle.energy(Q, y) >= e
    assert np.array_equal(x, xf) and abs(ef - cycle.energy(Q, xf)) <= 1e-12
    same = np.array([sum(int(xf[c]) << r for r, c in enumerate(ch[0]))], dtype=np.uint64)
    _, _, acc = cycle.aggregate(Q, xf, ch[:1], same)
    assert not acc[0]


def test_aggregate_exhaustive_small():
    # every window of size 3 with its brute-force sub-optimum: the result is
    # at least as good as each single accepted move and never above E(x0)
    N = 7
    Q = workloads.qubo(N, 45)
    x0 = np.array([1, 0, 1, 0, 1, 0, 1], dtype=np.uint8)
    ch = np.array(list(itertools.combinations(range(N), 3)), dtype=np.int32)
    sub = []
    for c in ch:
        best = min(range(8), key=lambda z: (oracle.energy(Q[np.ix_(c, c)], z), z))
        sub.append(best)
    xf, ef, acc = cycle.aggregate(Q, x0, ch, np.array(sub, dtype=np.uint64))
    assert ef <= cycle.energy(Q, x0)
    assert abs(ef - cycle.energy(Q, xf)) <= 1e-12
    assert acc.any() == (ef < cycle.energy(Q, x0))
