"""Writes tests/golden/cobyla_trajectory.txt: three hand-worked trajectories of
the unconstrained COBYLA steps (Powell's method as the paper's optimiser,
Sec. IV) on 2-parameter quadratics with known Hessians.

This is a pocket calculator for the worked example, not an implementation
to be trusted on its own: it follows the stated rules one step at a time
with 2 x 2 closed forms (the inverse by the adjugate, norms by hypot) and
prints every intermediate quantity next to the decision it drives, so each
line of the golden can be checked by hand.  It imports nothing from the
oracle or the library.  The rules, with alpha = 1/4, beta = 2.1,
gamma = 1/2, eta = 0.1:
  * evaluate x0 and x0 + rho e_1, x0 + rho e_2; the best becomes x0 and
    the other two are displacements d_1, d_2 from it; A = [d_1 d_2]^-1;
  * g = A^T (f_1 - f_0, f_2 - f_0);
  * a vertex with |d_j| > beta rho (the farther one if both), else one
    with 1 / |row j of A| < alpha rho (the flatter one), is replaced by
    x0 + gamma rho v, v = row j of A normalised and negated if g.v > 0;
  * otherwise the trust step d = -rho g / |g| replaces the vertex j of
    largest |(A d)_j| (ties: j = 1), and a ratio (f0 - f_new) / (rho |g|)
    below eta halves rho (rho = rhoend once rho <= 1.5 rhoend), or stops
    the run when rho is already rhoend;
  * a new point below f0 becomes x0.
Run from the repository root:  python tests/golden/cobyla_trajectory_calc.py
"""
import math
import os

ALPHA, BETA, GAMMA, ETA = 0.25, 2.1, 0.5, 0.1
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cobyla_trajectory.txt")

CASES = [
    # name, (a, b, h): f = (x - a)^2 + h (y - b)^2, x0, rhobeg, rhoend, maxfun
    ("A", (2.0, 1.0, 2.0), (0.0, 0.0), 1.0, 0.25, 40),
    ("B", (1.0, 2.0, 20.0), (0.0, 0.0), 1.0, 0.1, 60),
    ("C", (0.3, 0.7, 2.0), (0.7, -0.9), 1.0, 0.25, 40),
]


def g6(v):
    return f"{v:.6g}"


def vec(v):
    return "(" + ", ".join(g6(t) for t in v) + ")"


def run(name, abh, start, rho, rhoend, maxfun):
    a, b, h = abh
    lines = [f"case {name}", f"hessian_diag = 2 {g6(2 * h)}",
             f"minimiser = {a!r} {b!r}", f"weight = {h!r}",
             f"x0 = {start[0]!r} {start[1]!r}", f"rhobeg = {rho!r}", f"rhoend = {rhoend!r}",
             f"maxfun = {maxfun}"]

    def f(x, y):
        return (x - a) ** 2 + h * (y - b) ** 2

    evals = []

    def ev(p, kind):
        v = f(*p)
        evals.append(v)
        lines.append(f"eval {len(evals)} {kind} {p[0]!r} {p[1]!r} {v!r}")
        return v

    x0 = start
    f0 = ev(x0, "start")
    D = [[rho, 0.0], [0.0, rho]]
    fv = [ev((x0[0] + rho, x0[1]), "init"), ev((x0[0], x0[1] + rho), "init")]

    def rebase(j):
        nonlocal x0, f0, D, fv
        dj = D[j][:]
        x0 = (x0[0] + dj[0], x0[1] + dj[1])
        D = [[D[c][0] - dj[0], D[c][1] - dj[1]] for c in range(2)]
        D[j] = [-dj[0], -dj[1]]
        f0, fv[j] = fv[j], f0
        lines.append(f"#   vertex {j + 1} becomes x0 = {vec(x0)}, f0 = {g6(f0)}")

    j = 0 if fv[0] <= fv[1] else 1
    if fv[j] < f0:
        rebase(j)
    while len(evals) < maxfun:
        p, q, r, s = D[0][0], D[1][0], D[0][1], D[1][1]
        det = p * s - q * r
        A = [[s / det, -q / det], [-r / det, p / det]]
        df = [fv[0] - f0, fv[1] - f0]
        g = [A[0][0] * df[0] + A[1][0] * df[1], A[0][1] * df[0] + A[1][1] * df[1]]
        dist = [math.hypot(*D[0]), math.hypot(*D[1])]
        sig = [1.0 / math.hypot(*A[0]), 1.0 / math.hypot(*A[1])]
        lines.append(f"# rho = {g6(rho)}: d1 = {vec(D[0])}, d2 = {vec(D[1])}, "
                     f"g = {vec(g)}, |d| = {vec(dist)}, face distances = {vec(sig)}")
        far = 0 if dist[0] >= dist[1] else 1
        flat = 0 if sig[0] <= sig[1] else 1
        if dist[far] > BETA * rho or sig[flat] < ALPHA * rho:
            j = far if dist[far] > BETA * rho else flat
            why = (f"|d{j + 1}| > {g6(BETA * rho)}" if dist[far] > BETA * rho
                   else f"face distance {j + 1} < {g6(ALPHA * rho)}")
            nrm = math.hypot(*A[j])
            v = [A[j][0] / nrm, A[j][1] / nrm]
            gv = g[0] * v[0] + g[1] * v[1]
            if gv > 0.0:
                v = [-v[0], -v[1]]
            d = [GAMMA * rho * v[0], GAMMA * rho * v[1]]
            lines.append(f"#   geometry step on vertex {j + 1} ({why}); g.v = {g6(gv)}, "
                         f"d = {vec(d)}")
            fn = ev((x0[0] + d[0], x0[1] + d[1]), "geometry")
            D[j] = d
            fv[j] = fn
            if fn < f0:
                rebase(j)
            continue
        gn = math.hypot(*g)
        d = [-rho * g[0] / gn, -rho * g[1] / gn]
        lines.append(f"#   trust step d = {vec(d)}, predicted reduction {g6(rho * gn)}")
        fn = ev((x0[0] + d[0], x0[1] + d[1]), "trust")
        ratio = (f0 - fn) / (rho * gn)
        Ad = [A[0][0] * d[0] + A[0][1] * d[1], A[1][0] * d[0] + A[1][1] * d[1]]
        j = 0 if abs(Ad[0]) >= abs(Ad[1]) else 1
        lines.append(f"#   ratio {g6(ratio)}; |A d| = {vec([abs(Ad[0]), abs(Ad[1])])}: "
                     f"drops vertex {j + 1}")
        D[j] = d
        fv[j] = fn
        if fn < f0:
            rebase(j)
        if ratio < ETA:
            if rho <= rhoend:
                lines.append("#   rho is rhoend: stop")
                break
            rho *= 0.5
            if rho <= 1.5 * rhoend:
                rho = rhoend
            lines.append(f"#   rho -> {g6(rho)}")
    lines.append(f"final {x0[0]!r} {x0[1]!r} {f0!r} {len(evals)}")
    return lines


def main():
    out = ["# Hand-worked COBYLA trajectories (unconstrained steps of Powell's method,",
           "# the optimiser of Sec. IV) on f = (x - a)^2 + h (y - b)^2; written by",
           "# tests/golden/cobyla_trajectory_calc.py, whose docstring states the rules.",
           "# 'eval k kind x y f' lists every evaluated point in order; '#' lines give",
           "# the quantities behind each decision, rounded to 6 digits."]
    for c in CASES:
        out += run(*c)
    with open(OUT, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
