"""Batched COBYLA-type optimisation (qaoa_cobyla) against the oracle's
one-problem-at-a-time loop of the same steps (oracle/cobyla_loop.py, whose
step rules tests/golden/cobyla_trajectory.txt pins).  Every round is one
batched evaluation of the problems still running.

Per problem: the final <C> within 1e-10 relative, and the same evaluation
count and final parameters within rhoend / 10 -- unless the oracle's own loop
is that sensitive.  Near the end of a run the trust region is
~rhoend wide and the model gradient is a difference quotient of objective
values that differ by ~rhoend^2, so rounding-level differences of the
objective (measured here at every point the library evaluated: ~1e-15) can
legitimately steer two valid runs up to a last step apart.  That spread is
measured rather than assumed: the oracle's loop is rerun with its objective
perturbed by +-delta (delta = the measured library-oracle objective
difference) and a larger gap is accepted only within twice the largest
deviation those runs show; all of it is printed."""
import zlib

import numpy as np
import pytest

import oracle
from oracle.cobyla_loop import cobyla_loop, cobyla_min
from paper_2506_10531_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available()
    from paper_2506_10531_amd import api as a
    return a


RHOEND = 1e-6  # the default final trust-region radius of both loops


def subqubos(B, n, seed):
    _, rs = workloads.subqubo_requests(B, N=80, n_lo=n, n_hi=n, seed=seed)
    return np.stack([Q for _, Q in rs])


def oracle_objective(Q, p):
    def f(x):
        return float(oracle.expect(Q, x[None, :p], x[None, p:])[0][0])
    return f


def perturbed(f, delta, k):
    """f plus a deterministic +-delta that depends on the point and on k."""
    def g(x):
        h = zlib.crc32(np.ascontiguousarray(x, dtype=np.float64).tobytes() + bytes([k]))
        return f(x) + (delta if h & 1 else -delta)
    return g


@pytest.mark.parametrize("B,n,p,maxfun", [(6, 9, 1, 150), (1, 5, 1, 60), (4, 7, 2, 120),
                                          (3, 15, 1, 4), (2, 16, 1, 90)])
def test_batched_cobyla_matches_oracle_loop(api, B, n, p, maxfun):
    Qs = subqubos(B, n, 30 + n)
    g, b = workloads.params(B, p, 31 + n)
    th0 = np.concatenate([g, b], axis=1)
    print(f"cobyla B={B} n={n} p={p}", flush=True)
    r = api.cobyla(torch.as_tensor(Qs, device="cuda:0"), th0, maxfun=maxfun, prec="c128",
                   trace=True)
    assert r["rounds"] == int(r["nfev"].max())
    for t in range(B):
        th, f, nfev = cobyla_loop(Qs[t], th0[t], maxfun=maxfun)
        lib = r["trace"][t, :r["nfev"][t]]
        # the objective the library saw, against the oracle's at the same points
        f_or = oracle.expect(Qs[t], lib[:, :p], lib[:, p:2 * p])[0]
        delta = float(np.max(np.abs(lib[:, -1] - f_or)))
        assert delta <= 1e-12 * max(1.0, float(np.max(np.abs(f_or)))), delta
        assert np.all(np.isfinite(lib))  # one record per evaluation
        assert abs(r["expect"][t] - f) <= 1e-10 * max(1.0, abs(f))
        gap = float(np.max(np.abs(r["theta"][t] - th)))
        if gap <= RHOEND / 10 and r["nfev"][t] == nfev:
            continue
        fo = oracle_objective(Qs[t], p)
        dev = []
        for k in range(4):
            thk, _, nfk = cobyla_min(perturbed(fo, max(delta, 1e-15), k), th0[t], 0.5, RHOEND,
                                     maxfun)
            dev.append(float(np.max(np.abs(thk - th))))
        print(f"problem {t}: final gap {gap:.3e}, evaluations {r['nfev'][t]} vs {nfev}; "
              f"objective difference {delta:.2e}; the oracle's own runs under +-{delta:.1e} "
              f"perturbations move by {', '.join(f'{d:.2e}' for d in dev)}", flush=True)
        assert gap <= max(RHOEND / 10, 2.0 * max(dev)), (t, gap, dev)


def test_cobyla_complex64_descends(api):
    B, n, p = 5, 12, 1
    Qs = subqubos(B, n, 50)
    g, b = workloads.params(B, p, 51)
    th0 = np.concatenate([g, b], axis=1)
    r = api.cobyla(torch.as_tensor(Qs, device="cuda:0"), th0, maxfun=80, prec="c64")
    for t in range(B):
        cm = float(np.max(np.abs(oracle.cost_table(Qs[t]))))
        e0 = oracle.expect(Qs[t], th0[t:t + 1, :p], th0[t:t + 1, p:])[0][0]
        ef = oracle.expect(Qs[t], r["theta"][t:t + 1, :p], r["theta"][t:t + 1, p:])[0][0]
        assert abs(r["expect"][t] - ef) <= 1e-5 * cm
        assert ef <= e0 + 1e-5 * cm
