"""Batched COBYLA-type optimisation (qaoa_cobyla) against the oracle's
one-problem-at-a-time loop of the same steps (oracle/cobyla_loop.py, whose
step rules tests/golden/cobyla_trajectory.txt pins).  Every round is one
batched evaluation of the problems still running.

Per problem: the objective the library saw at every point it evaluated
against the oracle's (1e-12), the final <C> within 1e-10 relative, and the
same evaluation count and final parameters within rhoend / 10 -- unless the
two runs part at a near-tie.  COBYLA's decisions compare differences of
objective values that shrink to ~rhoend^2, so rounding-level differences of
the objective (~1e-15) can flip one and send two valid runs a last step or
two apart.  Where the runs part (the first point that differs by more than
a tenth of the trust radius), the oracle's trace gives how close its own
decision there came to going the other way; a larger gap is accepted only
when that margin is within what the measured objective difference and the
point drift before it can move (tests/test_cobyla_oracle.py checks those
margins against planted perturbations), and all of it is printed."""
import numpy as np
import pytest

import oracle
from oracle.cobyla_loop import cobyla_loop, divergence
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
        tr = []
        th, f, nfev = cobyla_loop(Qs[t], th0[t], maxfun=maxfun, trace=tr)
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
        k, drift = divergence(tr, lib[:, :2 * p])
        rk = tr[k - 1]
        bound = 2.0 * delta + 2.0 * rk["gn"] * drift
        print(f"problem {t}: final gap {gap:.3e}, evaluations {r['nfev'][t]} vs {nfev}; the "
              f"runs part after evaluation {k - 1} ({rk['kind']}, rho {rk['rho']:.1e}); "
              f"objective difference {delta:.1e}, point drift before it {drift:.1e}; the "
              f"oracle's decision there: margin {rk['margin']:.2e} against {bound:.2e}, "
              f"simplex margin {rk['gmargin']:.2e} against {4 * drift:.2e}", flush=True)
        assert rk["margin"] <= bound or rk["gmargin"] <= 4 * drift, (t, k, rk, delta, drift)


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
