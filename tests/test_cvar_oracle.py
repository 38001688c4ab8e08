"""Pins of the sampled-objective oracle (oracle/cvar.py): a hand-worked
example (tests/golden/cvar_example.txt), alpha = 1 is the mean, any alpha
K <= 1 is the minimum, CVaR never decreases with alpha, and a constant
sample is its own CVaR."""
import os

import numpy as np
import pytest

from oracle.cvar import cvar

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cvar_example.txt")


def _golden():
    rec = {}
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            rec[k.strip()] = [float(x) for x in v.split()]
    return rec


def test_hand_example():
    g = _golden()
    e = np.array(g["energies"])
    for a in ("0.25", "0.5", "1", "0.05"):
        assert abs(cvar(e, float(a)) - g["cvar_" + a][0]) <= 1e-12


@pytest.mark.parametrize("K", [1, 2, 17, 1024])
def test_limits_and_monotonicity(K):
    e = np.random.default_rng(K).normal(size=K)
    assert abs(cvar(e, 1.0) - e.mean()) <= 1e-12
    assert cvar(e, 0.5 / K) == e.min()
    assert cvar(e, 1.0 / K) == e.min()
    vals = [cvar(e, a) for a in np.linspace(0.01, 1.0, 40)]
    assert all(x <= y + 1e-12 for x, y in zip(vals, vals[1:]))
    assert abs(cvar(np.full(K, 3.25), 0.3) - 3.25) <= 1e-12
