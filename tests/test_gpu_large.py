"""Large single states on the GPU: the n = 24 precision workload against the
oracle (complex64 and complex128), n = 26 against the oracle, and n = 32
(a 32 GiB complex64 state, too large for the oracle's host memory budget)
through properties that hold at any size: beta = 0 leaves the distribution
uniform so <C> = (1'Q1 + tr Q)/4, unit norm, the p = 1 closed form, and the
diagonal-Q product formula; the largest states (n = 34 complex64, n = 33
complex128, 128 GiB each) against the p = 1 closed form."""
import numpy as np
import pytest

import oracle
from paper_2506_10531_amd import workloads
from tests import dense_ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available()
    from paper_2506_10531_amd import api as a
    return a


def cuda(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def test_precision_n24_all_sets(api):
    W = workloads.WORKLOADS["precision_n24"]
    n, p, S = W["n"], W["p"], W["sets"]
    Q = workloads.qubo(n, W["q_seed"])
    g, b = workloads.params(S, p, W["p_seed"])
    print("n=24 c64/c128 16 sets", flush=True)
    e64 = api.expect(cuda(Q), cuda(g), cuda(b), prec="c64").cpu().numpy()[0]
    e128 = api.expect(cuda(Q), cuda(g), cuda(b), prec="c128").cpu().numpy()[0]
    cm = float(np.max(np.abs(oracle.cost_table(Q))))
    sel = [0, S - 1]
    eo, _, _ = oracle.expect(Q, g[sel], b[sel])
    for i, s in enumerate(sel):
        assert abs(e128[s] - eo[i]) <= 1e-10 * max(1.0, abs(eo[i]))
        assert abs(e64[s] - eo[i]) <= 1e-5 * cm
    assert np.max(np.abs(e64 - e128)) <= 1e-5 * cm
    psi, _, nr = api.state(cuda(Q), cuda(g[:1]), cuda(b[:1]), prec="c64")
    ref = oracle.state(Q, g[0], b[0])
    l2 = np.linalg.norm(psi.cpu().numpy()[0, 0].astype(np.complex128) - ref)
    assert l2 <= 1e-4, l2
    assert abs(nr.item() - 1.0) <= 1e-5


def test_n26_against_oracle(api):
    n, p = 26, 2
    Q = workloads.qubo(n, 26)
    g, b = workloads.params(1, p, 27)
    print("n=26", flush=True)
    e64 = api.expect(cuda(Q), cuda(g), cuda(b), prec="c64").cpu().numpy()[0]
    e128 = api.expect(cuda(Q), cuda(g), cuda(b), prec="c128").cpu().numpy()[0]
    eo, _, _ = oracle.expect(Q, g, b)
    cm = float(np.max(np.abs(oracle.cost_table(Q))))
    assert abs(e128[0] - eo[0]) <= 1e-10 * max(1.0, abs(eo[0]))
    assert abs(e64[0] - eo[0]) <= 1e-5 * cm


N32 = 32


def _cmax_bound(Q):
    # max_z |C(z)| <= sum of |Q_ij| (used only to scale tolerances)
    return float(np.abs(Q).sum())


def test_n32_beta_zero_uniform_mean_and_norm(api):
    Q = workloads.qubo(N32, 6)
    g, b = workloads.params(2, 2, 16)
    b[:] = 0.0
    print("n=32 beta=0", flush=True)
    e, nr = api.expect(cuda(Q), cuda(g), cuda(b), prec="c64", norm=True)
    e, nr = e.cpu().numpy()[0], nr.cpu().numpy()[0]
    mean = dense_ref.mean_cost(Q)
    assert np.all(np.abs(nr - 1.0) <= 1e-5), nr
    assert np.all(np.abs(e - mean) <= 1e-5 * _cmax_bound(Q)), (e, mean)


def test_n32_p1_closed_form(api):
    Q = workloads.qubo(N32, 6)
    g, b = workloads.params(2, 1, 17)
    print("n=32 p=1 closed form", flush=True)
    e = api.expect(cuda(Q), cuda(g), cuda(b), prec="c64").cpu().numpy()[0]
    for s in range(2):
        cf = dense_ref.p1_closed_form(Q, g[s, 0], b[s, 0])
        assert abs(e[s] - cf) <= 1e-5 * _cmax_bound(Q), (s, e[s], cf)


def test_n32_diagonal_q_product_formula(api):
    rng = np.random.default_rng(32)
    d = rng.uniform(-1, 1, N32)
    Q = np.diag(d)
    g, b = workloads.params(1, 2, 18)
    print("n=32 diagonal", flush=True)
    e = api.expect(cuda(Q), cuda(g), cuda(b), prec="c64").cpu().numpy()[0]
    ref = dense_ref.diagonal_expect(d, g[0], b[0])
    assert abs(e[0] - ref) <= 1e-5 * np.abs(d).sum(), (e[0], ref)


@pytest.mark.parametrize("n", [27, 28, 30])
def test_three_sets_p1_closed_form(api, n):
    """Three-set complex64 plans whose kind-2 sets keep 6 to 8 contiguous low
    qubits (512-byte to 2 KiB runs): first, lead-only and last passes."""
    Q = workloads.qubo(n, 60 + n)
    g, b = workloads.params(2, 1, 70 + n)
    print(f"n={n} p=1 closed form", flush=True)
    e = api.expect(cuda(Q), cuda(g), cuda(b), prec="c64").cpu().numpy()[0]
    for s in range(2):
        cf = dense_ref.p1_closed_form(Q, g[s, 0], b[s, 0])
        assert abs(e[s] - cf) <= 1e-5 * _cmax_bound(Q), (s, e[s], cf)


@pytest.mark.parametrize("n", [28, 30])
def test_three_sets_diagonal_q_p3(api, n):
    """The same plans at p = 3 (middle passes on the kind-2 sets)."""
    rng = np.random.default_rng(n)
    d = rng.uniform(-1, 1, n)
    g, b = workloads.params(1, 3, 80 + n)
    print(f"n={n} diagonal p=3", flush=True)
    e = api.expect(cuda(np.diag(d)), cuda(g), cuda(b), prec="c64").cpu().numpy()[0]
    ref = dense_ref.diagonal_expect(d, g[0], b[0])
    assert abs(e[0] - ref) <= 1e-5 * np.abs(d).sum(), (e[0], ref)


@pytest.mark.parametrize("prec,n", [("c64", 34), ("c128", 33)])
def test_max_size_p1_closed_form(api, prec, n):
    """The largest states: n = QAOA_MAX_N = 34 in complex64 (a 128 GiB state;
    sets of 14, 10 and 10 qubits, the kind-2 tiles on 128-byte runs) and
    n = 33 in complex128 (128 GiB; 64-byte runs)."""
    Q = workloads.qubo(n, 90 + n)
    g, b = workloads.params(1, 1, 95 + n)
    print(f"n={n} {prec} p=1 closed form", flush=True)
    e, nr = api.expect(cuda(Q), cuda(g), cuda(b), prec=prec, norm=True)
    e, nr = float(e.cpu().numpy()[0][0]), float(nr.cpu().numpy()[0][0])
    cf = dense_ref.p1_closed_form(Q, g[0, 0], b[0, 0])
    bound = _cmax_bound(Q)
    tol = 1e-5 * bound if prec == "c64" else 1e-10 * max(1.0, bound)
    assert abs(e - cf) <= tol, (e, cf)
    assert abs(nr - 1.0) <= (1e-5 if prec == "c64" else 1e-12), nr


def test_large_n32_four_sets_runs_and_is_normalised(api):
    """The n = 32, p = 2, 4-set workload: every set keeps unit norm and the
    four <C> lie within [min C, max C] bounds."""
    W = workloads.WORKLOADS["large_n32"]
    Q = workloads.qubo(W["n"], W["q_seed"])
    g, b = workloads.params(W["sets"], W["p"], W["p_seed"])
    print("n=32 workload", flush=True)
    e, nr = api.expect(cuda(Q), cuda(g), cuda(b), prec="c64", norm=True)
    e, nr = e.cpu().numpy()[0], nr.cpu().numpy()[0]
    assert np.all(np.abs(nr - 1.0) <= 1e-5)
    assert np.all(np.abs(e) <= _cmax_bound(Q))
