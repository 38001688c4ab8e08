"""Batched COBYLA-type optimisation (qaoa_cobyla) against the oracle's
one-problem-at-a-time loop of the same steps (oracle/cobyla_loop.py).  In
complex128 the device objective equals the oracle's to ~1e-14, so every
problem takes the same steps: the same evaluation count and final <C> within
1e-10 relative.  The final parameters agree within 2 rhoend: the model
gradient divides objective differences by rho, so ~1e-14 objective
differences reach the last steps (of length ~rhoend) at ~1e-8, but where two
candidate vertices differ by ~1e-14 the choice between them (both valid
steps of the method) can differ, and the runs then end up to one final step
of the trust region apart.  Every round is one batched evaluation of the
problems still running."""
import numpy as np
import pytest

import oracle
from oracle.cobyla_loop import cobyla_loop
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
    r = api.cobyla(torch.as_tensor(Qs, device="cuda:0"), th0, maxfun=maxfun, prec="c128")
    assert r["rounds"] == int(r["nfev"].max())
    for t in range(B):
        th, f, nfev = cobyla_loop(Qs[t], th0[t], maxfun=maxfun)
        assert r["nfev"][t] == nfev, (t, r["nfev"][t], nfev)
        assert np.max(np.abs(r["theta"][t] - th)) <= 2 * RHOEND
        assert abs(r["expect"][t] - f) <= 1e-10 * max(1.0, abs(f))


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
