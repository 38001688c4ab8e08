"""Pins of the oracle's COBYLA-type loop (oracle/cobyla_loop.py) by cases
whose optimum is known without it: two hand-worked trajectories
(tests/golden/cobyla_trajectory.txt) that fix every step rule (the initial
simplex, re-basing on a better vertex, trust steps and the vertex they drop,
geometry steps for a far and a flat vertex with both signs of g.v, rho
halving, the clamp to rhoend and the stop); a one-variable QUBO, whose
p = 1 objective is q times the probability of z = 1 (minimum min(0, q));
convex quadratics with a known minimiser, where SciPy's COBYLA (Powell's
reference code) reaches the same minimum; refinement of a dense objective
grid; and the evaluation budget."""
import os

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import expect
from oracle.cobyla_loop import cobyla_loop, cobyla_min, divergence


@pytest.mark.parametrize("q", [1.5, -0.7])
def test_one_variable_reaches_min_zero_q(q):
    Q = np.array([[q]])
    th, f, nfev = cobyla_loop(Q, np.array([0.4, 0.3]), rhoend=1e-8, maxfun=500)
    assert abs(f - min(0.0, q)) <= 1e-6 * abs(q)
    assert 3 <= nfev <= 500


@pytest.mark.parametrize("n,seed", [(2, 1), (4, 2), (6, 3)])
def test_convex_quadratic_minimiser_and_reference(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(n, n))
    H = M @ M.T + 0.5 * np.eye(n)
    c = rng.normal(size=n)

    def f(x):
        r = x - c
        return float(r @ H @ r) - 2.0

    x, fx, nfev = cobyla_min(f, np.zeros(n), rhobeg=0.5, rhoend=1e-7, maxfun=5000)
    assert np.max(np.abs(x - c)) <= 1e-3
    assert fx + 2.0 <= 1e-6
    ref = minimize(f, np.zeros(n), method="COBYLA",
                   options=dict(rhobeg=0.5, tol=1e-7, maxiter=5000))
    assert abs(fx - ref.fun) <= 1e-6


def test_refines_a_grid_minimum():
    Q = np.array([[0.3, -0.8], [-0.8, 0.6]])
    gs = np.linspace(0, 2 * np.pi, 181)
    bs = np.linspace(0, np.pi, 91)
    G, Bt = np.meshgrid(gs, bs, indexing="ij")
    e = expect(Q, G.reshape(-1, 1), Bt.reshape(-1, 1))[0]
    k = int(np.argmin(e))
    th, f, _ = cobyla_loop(Q, np.array([G.ravel()[k], Bt.ravel()[k]]), rhobeg=0.02,
                           rhoend=1e-8, maxfun=400)
    assert f <= e[k] + 1e-12
    assert e[k] - f <= 0.05 * np.abs(Q).sum()


def test_budget_and_descent():
    rng = np.random.default_rng(4)
    Q = rng.uniform(-1, 1, (5, 5))
    Q = np.triu(Q) + np.triu(Q, 1).T
    th0 = np.array([0.3, 0.9])
    e0 = expect(Q, th0[None, :1], th0[None, 1:])[0][0]
    _, f, nfev = cobyla_loop(Q, th0, maxfun=7)
    assert nfev == 7 and f <= e0
    _, f, nfev = cobyla_loop(Q, th0, maxfun=300)
    assert f <= e0 and nfev <= 300


GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cobyla_trajectory.txt")


def golden_cases():
    cases, cur = [], None
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if line.startswith("case "):
            cur = {"name": line.split()[1], "evals": []}
            cases.append(cur)
        elif line.startswith("eval "):
            _, _, kind, x, y, fx = line.split()
            cur["evals"].append((kind, float(x), float(y), float(fx)))
        elif line.startswith("final "):
            _, x, y, fx, nfev = line.split()
            cur["final"] = (float(x), float(y), float(fx), int(nfev))
        else:
            k, v = line.split("=")
            cur[k.strip()] = [float(t) for t in v.split()]
    return cases


@pytest.mark.parametrize("case", golden_cases(), ids=lambda c: c["name"])
def test_hand_worked_trajectory(case):
    a, b = case["minimiser"]
    h = case["weight"][0]

    def f(x):
        return (x[0] - a) ** 2 + h * (x[1] - b) ** 2

    trace = []
    x, fx, nfev = cobyla_min(f, np.array(case["x0"]), rhobeg=case["rhobeg"][0],
                             rhoend=case["rhoend"][0], maxfun=int(case["maxfun"][0]),
                             trace=trace)
    assert len(trace) == len(case["evals"]) == nfev
    for k, (rec, (kind, gx, gy, gf)) in enumerate(zip(trace, case["evals"])):
        assert rec["kind"] == kind, k
        assert abs(rec["x"][0] - gx) <= 1e-12 and abs(rec["x"][1] - gy) <= 1e-12, k
        assert abs(rec["f"] - gf) <= 1e-12 * max(1.0, abs(gf)), k
    fxg, fyg, ffg, nfg = case["final"]
    assert nfev == nfg
    assert abs(x[0] - fxg) <= 1e-12 and abs(x[1] - fyg) <= 1e-12 and abs(fx - ffg) <= 1e-12


def test_golden_covers_every_rule():
    kinds = [{e[0] for e in c["evals"]} for c in golden_cases()]
    assert set.union(*kinds) == {"start", "init", "trust", "geometry"}
    text = open(GOLD).read()
    for event in ("becomes x0", "drops vertex", "rho ->", "rho is rhoend: stop",
                  "(|d", "(face distance", "g.v = -"):
        assert event in text, event


def _perturbed(f, delta, k):
    """f plus a deterministic +-delta that depends on the point and on k."""
    import hashlib

    def g(x):
        h = hashlib.sha256(bytes([k]) + np.ascontiguousarray(x, dtype=np.float64).tobytes())
        return f(x) + (delta if h.digest()[0] & 1 else -delta)
    return g


def test_margins_flag_every_divergence():
    """The trace's decision margins are lower bounds of the objective change
    that flips a decision: wherever a run with its objective moved by
    +-delta leaves the unperturbed run, the decision taken there had a
    margin of at most 2 delta plus what the point drift accumulated before it
    moves the objective (2 gn drift), or a simplex test within a few times
    that drift of its threshold."""
    diverged = 0
    for seed in range(6):
        rng = np.random.default_rng(200 + seed)
        n, p = 5, 1 + seed % 2
        A = rng.uniform(-1, 1, size=(n, n))
        Q = np.triu(A) + np.triu(A, 1).T
        th0 = np.concatenate([rng.uniform(0, np.pi, p), rng.uniform(0, np.pi / 2, p)])

        def f(x, Q=Q, p=p):
            return float(expect(Q, x[None, :p], x[None, p:])[0][0])

        tr = []
        cobyla_min(f, th0, 0.5, 1e-6, 120, trace=tr)
        for delta in (1e-12, 1e-10):
            for k in range(3):
                other = []
                cobyla_min(_perturbed(f, delta, k), th0, 0.5, 1e-6, 120, trace=other)
                kd, drift = divergence(tr, [r["x"] for r in other])
                if kd == len(tr) == len(other):
                    continue
                diverged += 1
                r = tr[kd - 1]
                assert (r["margin"] <= 2 * delta + 2 * r["gn"] * drift
                        or r["gmargin"] <= 4 * drift), \
                    (seed, delta, k, kd, r["margin"], r["gn"], r["gmargin"], drift)
    assert diverged >= 3  # the check saw divergences to explain
