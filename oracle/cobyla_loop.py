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
    optimal vertex, whether rho shrank after it, and rho when the point was
    made.  Each record also carries how close the decisions taken after that
    evaluation (up to the next one) came to going the other way:
    ``margin``, the smallest change of the objective values that flips one
    of the comparisons that involve them (which vertex is best, the rebase
    test, the ratio test, the side of a geometry step, the vertex a trust
    step replaces), and ``gmargin``, the smallest distance of the simplex
    tests (farthest and flattest vertex against beta rho and alpha rho, and
    their runners-up) from their thresholds, in units of the parameters;
    ``gn`` is the model gradient's norm at those decisions, so that a run
    whose points have drifted by e sees objective values moved by about
    gn e.  The margins only read the loop's values; they change none of
    them."""
    x0 = np.array(x0, dtype=np.float64)
    n = x0.size
    rho = float(rhobeg)
    tr = trace is not None

    def rec(**kw):
        if tr:
            kw.update(rho=rho, margin=np.inf, gmargin=np.inf, gn=0.0)
            trace.append(kw)

    def near(m, key="margin"):  # a decision after the last evaluation
        if tr and trace:
            trace[-1][key] = min(trace[-1][key], float(m))

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
    if tr:
        trace[-1]["rebase"] = bool(fv[best] < f0)
        srt = np.sort(fv)
        near(abs(fv[best] - f0) / 2)
        if n > 1:
            near((srt[1] - srt[0]) / 2)
    if fv[best] < f0:
        x0, f0, D, fv = _rebase(x0, f0, D, fv, best)
    while nfev < maxfun:
        A = np.linalg.inv(D)
        g = A.T @ (fv - f0)
        dist = np.linalg.norm(D, axis=0)
        sigma = 1.0 / np.linalg.norm(A, axis=1)
        far = int(np.argmax(dist))
        flat = int(np.argmin(sigma))
        if tr:
            trace[-1]["gn"] = max(trace[-1]["gn"], float(np.linalg.norm(g)))
            near(abs(dist[far] - BETA * rho), "gmargin")
            near(abs(sigma[flat] - ALPHA * rho), "gmargin")
            if n > 1:
                sd, ss = np.sort(dist), np.sort(sigma)
                near(sd[-1] - sd[-2], "gmargin")
                near(ss[1] - ss[0], "gmargin")
        if dist[far] > BETA * rho or sigma[flat] < ALPHA * rho:
            j = far if dist[far] > BETA * rho else flat
            v = A[j] / np.linalg.norm(A[j])
            if tr:  # g . v = (fv - f0) . (A v): each value moved by delta moves it by 2 delta |A v|_1
                near(abs(g @ v) / (2.0 * np.sum(np.abs(A @ v))))
            if g @ v > 0.0:
                v = -v
            d = GAMMA * rho * v
            fn = f(x0 + d)
            nfev += 1
            D[:, j] = d
            fv[j] = fn
            rec(kind="geometry", x=x0 + d, f=fn, j=j, rebase=bool(fn < f0), shrink=False)
            near(abs(fn - f0) / 2)
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
            if tr:
                # values moved by delta move g by up to 2 delta sqrt(n) |A|_2
                an = float(np.linalg.norm(A, 2))
                sg = 2.0 * np.sqrt(n) * an
                near(abs(fn - f0) / 2)
                near(abs(ratio - ETA) / (2.0 / (rho * gn) + abs(ratio) * sg / gn))
                if n > 1:
                    ad = np.sort(np.abs(A @ d))
                    # the unit direction turns by up to 2 |dg| / |g|
                    near((ad[-1] - ad[-2]) / (2.0 * an * rho * 2.0 * sg / gn))
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


def divergence(trace, xs, frac=0.1):
    """Where another run leaves a traced one: xs are the other run's
    evaluated points in order.  Returns (k, drift): k is the first
    evaluation whose point differs from the traced one by more than frac
    times the trust radius it was made with (or the length of the shorter
    run when none does), so the decisions that sent the runs apart are those
    recorded with evaluation k - 1; drift is the largest point difference
    before k."""
    xs = np.asarray(xs, dtype=np.float64)
    m = min(len(trace), len(xs))
    xt = np.array([r["x"] for r in trace[:m]])
    rho = np.array([r["rho"] for r in trace[:m]])
    dx = np.max(np.abs(xt - xs[:m]), axis=1)
    off = np.nonzero(dx > frac * rho)[0]
    k = int(off[0]) if off.size else m
    return k, float(np.max(dx[:k])) if k > 0 else 0.0


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
