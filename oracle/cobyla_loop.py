"""CPU oracle for the COBYLA variational loop: TEST INFRASTRUCTURE ONLY.

The paper optimises each sub-QUBO's (gamma, beta) from random values with
COBYLA at p = 1 (Sec. IV).  COBYLA (Powell, 1994) keeps a simplex of n + 1
points, fits the linear interpolant of the objective on it, steps to the
minimiser of that model inside a ball of radius rho (the trust region), and
keeps the simplex well shaped with geometry steps; rho shrinks from rhobeg
to rhoend.  Without constraints (the QAOA parameters are free) the method
reduces to the steps below, which the library implements the same way:

  * start: x_0 and x_0 + rho e_i (i = 1..n), each evaluated; the best point
    becomes the optimal vertex x_0, the others are held as displacements
    d_i from it, A = D^{-1} (D = [d_1 .. d_n]);
  * model gradient g = A^T (f_i - f_0);
  * acceptability: a vertex farther than beta rho (beta = 2.1) from x_0, or
    nearer than alpha rho (alpha = 0.25) to the face opposite it (distance
    1 / |row i of A|), is replaced by a geometry step: x_0 + gamma rho v
    (gamma = 1/2) with v the unit normal of that face, signed so that
    g . v <= 0; the farthest vertex first, else the flattest;
  * otherwise a trust step d = -rho g / |g| (predicted reduction rho |g|)
    replaces the vertex j maximising |(A d)_j| (the largest simplex volume;
    ties to the smaller j); a ratio of actual to predicted reduction below
    0.1 then halves rho (rho = rhoend once rho <= 1.5 rhoend), and when
    rho cannot shrink further the loop ends; g = 0 also shrinks rho;
  * a new point better than x_0 becomes the optimal vertex (the
    displacements are re-based on it);
  * the loop also ends after maxfun evaluations.

Only the tests and the benchmark's CPU-baseline leg use this module; it
imports nothing from the HIP package.
"""
from __future__ import annotations

import numpy as np

from . import expect

ALPHA, BETA, GAMMA, ETA = 0.25, 2.1, 0.5, 0.1


def _rebase(x0, f0, D, fv, j):
    """Vertex j (displacement D[:, j], value fv[j]) becomes the optimal
    vertex."""
    dj = D[:, j].copy()
    x0 = x0 + dj
    D = D - dj[:, None]
    D[:, j] = -dj
    fv = fv.copy()
    f0, fv[j] = fv[j], f0
    return x0, f0, D, fv


def cobyla_min(f, x0, rhobeg=0.5, rhoend=1e-6, maxfun=200, trace=None):
    """Minimise f from x0 by the steps above.  Returns (x, f(x), nfev).

    If ``trace`` is a list, one record per evaluation is appended: the kind
    of point ("start", "init", "geometry", "trust"), the point, its value,
    the vertex it replaced (-1 for start/init), whether it became the
    optimal vertex and whether rho shrank after it."""
    x0 = np.array(x0, dtype=np.float64)
    n = x0.size
    rho = float(rhobeg)
    rec = (lambda **kw: trace.append(kw)) if trace is not None else (lambda **kw: None)
    f0 = f(x0)
    nfev = 1
    rec(kind="start", x=x0.copy(), f=f0, j=-1, rebase=False, shrink=False)
    D = rho * np.eye(n)
    fv = np.empty(n)
    for i in range(n):
        if nfev >= maxfun:
            return x0, f0, nfev
        fv[i] = f(x0 + D[:, i])
        nfev += 1
        rec(kind="init", x=x0 + D[:, i], f=fv[i], j=-1, rebase=False, shrink=False)
    best = int(np.argmin(fv))
    if trace is not None:
        trace[-1]["rebase"] = bool(fv[best] < f0)
    if fv[best] < f0:
        x0, f0, D, fv = _rebase(x0, f0, D, fv, best)
    while nfev < maxfun:
        A = np.linalg.inv(D)
        g = A.T @ (fv - f0)
        dist = np.linalg.norm(D, axis=0)
        sigma = 1.0 / np.linalg.norm(A, axis=1)
        far = int(np.argmax(dist))
        flat = int(np.argmin(sigma))
        if dist[far] > BETA * rho or sigma[flat] < ALPHA * rho:
            j = far if dist[far] > BETA * rho else flat
            v = A[j] / np.linalg.norm(A[j])
            if g @ v > 0.0:
                v = -v
            d = GAMMA * rho * v
            fn = f(x0 + d)
            nfev += 1
            D[:, j] = d
            fv[j] = fn
            rec(kind="geometry", x=x0 + d, f=fn, j=j, rebase=bool(fn < f0), shrink=False)
            if fn < f0:
                x0, f0, D, fv = _rebase(x0, f0, D, fv, j)
            continue
        gn = float(np.linalg.norm(g))
        shrink = gn == 0.0
        if not shrink:
            d = -rho * g / gn
            fn = f(x0 + d)
            nfev += 1
            ratio = (f0 - fn) / (rho * gn)
            j = int(np.argmax(np.abs(A @ d)))
            rec(kind="trust", x=x0 + d, f=fn, j=j, rebase=bool(fn < f0),
                shrink=bool(ratio < ETA))
            D[:, j] = d
            fv[j] = fn
            if fn < f0:
                x0, f0, D, fv = _rebase(x0, f0, D, fv, j)
            shrink = ratio < ETA
        if shrink:
            if rho <= rhoend:
                break
            rho = 0.5 * rho
            if rho <= 1.5 * rhoend:
                rho = rhoend
    return x0, f0, nfev


def cobyla_loop(Q, theta0, rhobeg=0.5, rhoend=1e-6, maxfun=200, trace=None):
    """The paper's loop on one sub-QUBO: (theta, <C>, nfev) for theta0 =
    (gamma_1..p, beta_1..p), the objective being the complex128 oracle's
    exact <C>.  ``trace`` as in cobyla_min."""
    theta0 = np.asarray(theta0, dtype=np.float64)
    p = theta0.size // 2

    def fq(x):
        e, _, _ = expect(Q, x[None, :p], x[None, p:])
        return float(e[0])

    return cobyla_min(fq, theta0, rhobeg, rhoend, maxfun, trace)
