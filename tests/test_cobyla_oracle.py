"""Pins of the oracle's COBYLA loop (oracle/cobyla_loop.py) by cases whose
optimum is known without it: a one-variable QUBO, whose p = 1 objective is
q times the probability of z = 1 (minimum min(0, q)); a dense grid of the
two-variable objective, which COBYLA started at the best grid point may only
refine; and descent from a random start."""
import numpy as np
import pytest

from oracle.cobyla_loop import cobyla_loop


@pytest.mark.parametrize("q", [1.5, -0.7])
def test_one_variable_reaches_min_zero_q(q):
    Q = np.array([[q]])
    th, f, nfev = cobyla_loop(Q, np.array([0.4, 0.3]), maxiter=400, tol=1e-10)
    assert abs(f - min(0.0, q)) <= 1e-6 * abs(q)
    assert nfev > 2


def test_refines_a_grid_minimum():
    # a dense grid of the objective (the exact n = 2 expectation, p = 1),
    # then COBYLA from the best grid point: it may only improve on it, and
    # by no more than the grid spacing allows
    from oracle import expect
    Q = np.array([[0.3, -0.8], [-0.8, 0.6]])
    gs = np.linspace(0, 2 * np.pi, 181)
    bs = np.linspace(0, np.pi, 91)
    G, Bt = np.meshgrid(gs, bs, indexing="ij")
    e = expect(Q, G.reshape(-1, 1), Bt.reshape(-1, 1))[0]
    k = int(np.argmin(e))
    th, f, _ = cobyla_loop(Q, np.array([G.ravel()[k], Bt.ravel()[k]]), rhobeg=0.02,
                           maxiter=400, tol=1e-10)
    assert f <= e[k] + 1e-12
    assert e[k] - f <= 0.05 * (np.abs(Q).sum())


def test_never_worse_than_start():
    rng = np.random.default_rng(4)
    Q = rng.uniform(-1, 1, (5, 5))
    Q = np.triu(Q) + np.triu(Q, 1).T
    th0 = np.array([0.3, 0.9])
    from oracle import expect
    e0 = expect(Q, th0[None, :1], th0[None, 1:])[0][0]
    _, f, _ = cobyla_loop(Q, th0, maxiter=100)
    assert f <= e0
