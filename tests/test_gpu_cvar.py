"""The sampled objective on the GPU (qaoa_cvar) against the CVaR oracle
(oracle/cvar.py): FP64 sums in another order, |d| <= 1e-12 * max(1, max|E|);
integer-valued energies with many ties give exactly the oracle's value; and
end to end from qaoa_sample's shot energies."""
import numpy as np
import pytest

from oracle.cvar import cvar
from paper_2506_10531_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available()
    from paper_2506_10531_amd import api as a
    return a


@pytest.mark.parametrize("B,K", [(1, 1), (3, 7), (5, 1024), (2, 3000)])
@pytest.mark.parametrize("alpha", [1e-4, 0.1, 0.25, 0.5, 1.0])
def test_cvar_random(api, B, K, alpha):
    e = np.random.default_rng(B * K).normal(scale=30.0, size=(B, K))
    out = api.cvar(torch.as_tensor(e, device="cuda:0"), alpha).cpu().numpy()
    for b in range(B):
        ref = cvar(e[b], alpha)
        assert abs(out[b] - ref) <= 1e-12 * max(1.0, np.abs(e[b]).max()), (b, out[b], ref)


def test_cvar_ties_exact(api):
    e = np.random.default_rng(3).integers(-5, 6, size=(4, 1000)).astype(np.float64)
    for alpha in (0.013, 0.2, 0.5, 1.0):
        out = api.cvar(torch.as_tensor(e, device="cuda:0"), alpha).cpu().numpy()
        assert np.allclose(out, [cvar(x, alpha) for x in e], rtol=0, atol=1e-12)


def test_sampled_objective_end_to_end(api):
    import oracle
    Q = workloads.qubo(10, 12)
    g, b = workloads.params(3, 2, 13)
    Qd = torch.as_tensor(np.stack([Q] * 3), device="cuda:0")
    s = api.sample(Qd, torch.as_tensor(g, device="cuda:0"), torch.as_tensor(b, device="cuda:0"),
                   512, 77, prec="c128")
    cz = s["cz"].cpu().numpy()
    z = s["z"].cpu().numpy().view(np.uint64)
    for t in range(3):
        # the shot energies are C(z_s) of the drawn bit strings
        assert all(abs(cz[t, i] - oracle.energy(Q, int(z[t, i]))) <= 1e-12 for i in range(0, 512, 37))
    for alpha in (0.1, 1.0):
        out = api.sampled_objective(Qd, torch.as_tensor(g, device="cuda:0"),
                                    torch.as_tensor(b, device="cuda:0"), 512, 77, alpha,
                                    prec="c128").cpu().numpy()
        assert np.allclose(out, [cvar(cz[t], alpha) for t in range(3)], rtol=0, atol=1e-11)
