"""GPU parity of the HIP path against the CPU oracle (called through the C ABI
by the Python binding).

Tolerances (FP64 accumulation everywhere; state arithmetic in the precision
named):
  complex128: |d<C>| <= 1e-10 * max(|<C>|, 1); state L2 error <= 1e-12.
  complex64:  |d<C>| <= 1e-5 * max_z |C(z)|; state L2 error <= 1e-4.
"""
import numpy as np
import pytest

import oracle
from paper_2506_10531_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_E = {"c128": lambda e, cmax: 1e-10 * max(abs(e), 1.0),
         "c64": lambda e, cmax: 1e-5 * cmax}
TOL_PSI = {"c128": 1e-12, "c64": 1e-4}


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2506_10531_amd import api as a
    return a


def cuda(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def cmax(Q):
    return float(np.max(np.abs(oracle.cost_table(Q))))


def run_case(api, n, p, S, prec, B=1, seed=0, state=True, probs=False):
    Qs = workloads.qubos(B, n, 1000 + 7 * n + seed)
    g, b = workloads.params(S, p, 2000 + n + seed, lead=(B,))
    print(f"case n={n} p={p} S={S} B={B} prec={prec}", flush=True)
    if state:
        psi, e, nr = api.state(cuda(Qs), cuda(g), cuda(b), prec=prec)
        psi = psi.cpu().numpy()
    else:
        e = api.expect(cuda(Qs), cuda(g), cuda(b), prec=prec)
    e = e.cpu().numpy()
    for bi in range(B):
        cm = cmax(Qs[bi])
        eo, no, Po = oracle.expect(Qs[bi], g[bi], b[bi], probs=probs)
        for s in range(S):
            err = abs(e[bi, s] - eo[s])
            assert err <= TOL_E[prec](eo[s], cm), (bi, s, e[bi, s], eo[s], err)
            if state:
                ref = oracle.state(Qs[bi], g[bi, s], b[bi, s])
                l2 = np.linalg.norm(psi[bi, s].astype(np.complex128) - ref)
                assert l2 <= TOL_PSI[prec], (bi, s, l2)
                assert abs(nr[bi, s].item() - 1.0) <= (1e-12 if prec == "c128" else 1e-5)
    return Qs, g, b


SMALL = [(n, p) for n in (1, 2, 3, 5, 8, 10, 12) for p in (1, 2, 3)]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n,p", SMALL)
def test_single_tile_state_and_expect(api, n, p, prec):
    run_case(api, n, p, S=3, prec=prec, B=2)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n,p", [(13, 2), (14, 3), (15, 1), (16, 2), (17, 4), (19, 3),
                                 (21, 2), (22, 2), (23, 1)])
def test_multipass_state_and_expect(api, n, p, prec):
    run_case(api, n, p, S=2, prec=prec, B=2 if n < 20 else 1)


@pytest.mark.parametrize("prec,n,p", [("c64", 13, 1), ("c64", 13, 64), ("c64", 14, 2),
                                      ("c64", 14, 64), ("c128", 13, 3), ("c128", 13, 64)])
def test_whole_state_32_and_64_amplitudes_per_thread(api, prec, n, p):
    """The whole-state launch at n = 13 and 14 (32 or 64 amplitudes per
    thread, C(z) formed at each use from the thread's fields and the shared
    register-bit table): state, <C>, norm and probabilities against the
    oracle, up to QAOA_MAX_P layers."""
    Qs, g, b = run_case(api, n, p, S=2, prec=prec, B=2, seed=5)
    e, P = api.expect(cuda(Qs), cuda(g), cuda(b), prec=prec, probs=True)
    psi = api.state(cuda(Qs), cuda(g), cuda(b), prec=prec)[0].cpu().numpy()
    P = P.cpu().numpy()
    u = 2.0 ** -52 if prec == "c128" else 2.0 ** -23
    for bi in range(2):
        for s in range(2):
            ref = oracle.state(Qs[bi], g[bi, s], b[bi, s])
            d = np.abs(psi[bi, s].astype(np.complex128) - ref)
            # |P_gpu - |ref|^2| <= |d| (2 |ref| + |d|) + rounding of |psi|^2
            bound = d * (2.0 * np.abs(ref) + d) + 4.0 * u * np.abs(ref) ** 2 + 1e-300
            err = np.abs(P[bi, s].astype(np.float64) - np.abs(ref) ** 2)
            assert np.all(err <= bound * 1.01 + 1e-18), float(np.max(err - bound))


@pytest.mark.parametrize("prec,n", [("c64", 15), ("c128", 14)])
def test_max_layers_state_and_expect(api, prec, n):
    """QAOA_MAX_P = 64 layers on register tiles (p + 1 = 65 passes on two
    qubit sets, all their tables from one launch)."""
    run_case(api, n, 64, S=2, prec=prec)


@pytest.mark.parametrize("n,p", [(23, 2), (25, 3)])
def test_multiset_c128_state(api, n, p):
    """complex128 register tiles: two sets up to n = 24, three beyond (with a
    lead-only pass for the middle set)."""
    run_case(api, n, p, S=1, prec="c128")


@pytest.mark.parametrize("B,S", [(4, 2), (3, 1)])
def test_xcd_grouped_tile_order(api, B, S):
    """complex128 passes on 64-byte runs deal 4 (first pass) or 16 (middle and
    last passes) consecutive tiles to one XCD when the grid, states x 2^(n-13)
    tiles, is a multiple of 8 x that group, and keep the launch order
    otherwise.  At n = 18 (32 tiles per state) 8 states take the grouped
    order in every pass; 3 states (96 tiles) take it in the first pass only."""
    run_case(api, 18, 3, S=S, prec="c128", B=B, seed=11)


def test_plain_n10_all_sets_with_probabilities(api):
    """64 parameter sets, p = 2, complex128, <C> and probabilities."""
    W = workloads.WORKLOADS["plain_n10"]
    Q = workloads.qubo(W["n"], W["q_seed"])
    g, b = workloads.params(W["sets"], W["p"], W["p_seed"])
    e, nr, P = api.expect(cuda(Q), cuda(g), cuda(b), prec="c128", probs=True, norm=True)
    eo, no, Po = oracle.expect(Q, g, b, probs=True)
    e = e.cpu().numpy()[0]
    P = P.cpu().numpy()[0]
    assert np.max(np.abs(e - eo) / np.maximum(np.abs(eo), 1.0)) <= 1e-10
    assert np.max(np.abs(P - Po)) <= 1e-14
    assert np.max(np.abs(nr.cpu().numpy() - 1.0)) <= 1e-12


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_mixer_mode_boundaries_and_large_gamma(api, prec):
    """beta at 0, pi/4 (tan = 1), pi/2 (cos = 0), negative, beyond pi/2; gamma
    large enough that gamma * C spans many turns (range reduction)."""
    n, p = 11, 6
    Q = workloads.qubo(n, 77)
    g = np.array([[0.3, 1.7, 40.0, -2.5, 0.0, 3.1]])
    b = np.array([[0.0, np.pi / 4, np.pi / 2, -0.7, 2.2, np.pi / 4 + 1e-9]])
    psi, e, _ = api.state(cuda(Q), cuda(g), cuda(b), prec=prec)
    ref = oracle.state(Q, g[0], b[0])
    l2 = np.linalg.norm(psi.cpu().numpy()[0, 0].astype(np.complex128) - ref)
    assert l2 <= TOL_PSI[prec], l2
    for nq in (17,):
        Q2 = workloads.qubo(nq, 78)
        psi2, _, _ = api.state(cuda(Q2), cuda(g), cuda(b), prec=prec)
        ref2 = oracle.state(Q2, g[0], b[0])
        l2 = np.linalg.norm(psi2.cpu().numpy()[0, 0].astype(np.complex128) - ref2)
        assert l2 <= TOL_PSI[prec], l2


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_nonsymmetric_q(api, prec):
    n, p = 15, 2
    rng = np.random.default_rng(5)
    Q = rng.uniform(-1, 1, (n, n))
    g, b = workloads.params(2, p, 6)
    e = api.expect(cuda(Q), cuda(g), cuda(b), prec=prec).cpu().numpy()[0]
    eo, _, _ = oracle.expect(Q, g, b)
    for s in range(2):
        assert abs(e[s] - eo[s]) <= TOL_E[prec](eo[s], cmax(Q))


def test_deterministic_repeat(api):
    n, p = 18, 3
    Q = workloads.qubo(n, 9)
    g, b = workloads.params(4, p, 10)
    a1 = api.expect(cuda(Q), cuda(g), cuda(b), prec="c64").cpu().numpy()
    a2 = api.expect(cuda(Q), cuda(g), cuda(b), prec="c64").cpu().numpy()
    assert np.array_equal(a1, a2)


@pytest.mark.parametrize("prec,n", [("c128", 10), ("c64", 13), ("c64", 16)])
def test_evaluator_matches_expect(api, prec, n):
    """api.Evaluator (problem and outputs bound once, one qaoa_expect per call)
    returns bitwise what api.expect returns for the same parameters, call
    after call, and refuses parameters of another shape."""
    B, S, p = 2, 5, 3
    Qs = workloads.qubos(B, n, 6100 + n)
    Qd = cuda(Qs)
    ev = api.Evaluator(Qd, S, p, prec=prec, probs=True, norm=True)
    for trial in range(3):
        g, b = workloads.params(S, p, 6200 + 10 * n + trial, lead=(B,))
        gd, bd = cuda(g), cuda(b)
        e = ev(gd, bd).clone()
        e2, nr2, P2 = api.expect(Qd, gd, bd, prec=prec, probs=True, norm=True)
        torch.cuda.synchronize()
        assert torch.equal(e, e2) and torch.equal(ev.norm, nr2) and torch.equal(ev.probs, P2)
    with pytest.raises(ValueError):
        ev(gd[:, :2].contiguous(), bd[:, :2].contiguous())


@pytest.mark.parametrize("prec,n,B,S,p", [("c128", 3, 3, 21845, 2), ("c64", 3, 3, 21845, 2),
                                          ("c64", 15, 1, 65535, 1)])
def test_max_states_per_call(api, prec, n, B, S, p):
    """B * S = 65535, the most states one call takes: the whole-state launch
    (one work-group per state, n = 3: every set against the oracle) and the
    register-tile passes (n = 15: 2 tiles per state, 131070 work-groups, 17 GB
    of state; 16 sets spread over the range against the oracle).  One state
    more is rejected before any work."""
    from paper_2506_10531_amd import _lib
    print(f"max states {prec} n={n} B={B} S={S} p={p}", flush=True)
    Qs = workloads.qubos(B, n, 7100 + n)
    g, b = workloads.params(S, p, 7200 + n, lead=(B,))
    ctx = api.Context(0)  # its 18 GB of scratch go with it
    e = api.expect(cuda(Qs), cuda(g), cuda(b), prec=prec, ctx=ctx).cpu().numpy()
    ctx.close()
    for bi in range(B):
        sets = np.arange(S) if n <= 8 else np.linspace(0, S - 1, 16).astype(int)
        eo = oracle.expect(Qs[bi], g[bi][sets], b[bi][sets])[0]
        tol = TOL_E[prec](0.0, cmax(Qs[bi]))
        if prec == "c128":
            tol = 1e-10 * np.maximum(np.abs(eo), 1.0)
        assert np.all(np.abs(e[bi][sets] - eo) <= tol), bi
    torch.cuda.synchronize()
    g1, b1 = workloads.params(65536, 1, 7300)
    with pytest.raises(_lib.QaoaError) as ei:
        api.expect(cuda(Qs[0]), cuda(g1), cuda(b1), prec=prec)
    assert ei.value.code == _lib.ERR_INVALID_ARG


@pytest.mark.parametrize("prec,n", [("c128", 5), ("c64", 13), ("c64", 18), ("c128", 16),
                                    ("c64", 25)])
def test_zero_q_is_exact(api, prec, n):
    """Q = 0: C(z) = 0 for every z, so <C> is exactly 0 and, |+> being an
    eigenstate of every mixer, the state stays uniform up to a global phase:
    every probability 2^-n, the norm 1."""
    B, S, p = 1, 2, 3
    Q = np.zeros((B, n, n))
    g, b = workloads.params(S, p, 7400 + n, lead=(B,))
    e, nr = api.expect(cuda(Q), cuda(g), cuda(b), prec=prec, norm=True)
    assert torch.all(e == 0.0), e
    tol = 1e-14 if prec == "c128" else 2e-6
    assert torch.all(torch.abs(nr - 1.0) <= tol), nr
    psi = api.state(cuda(Q), cuda(g), cuda(b), prec=prec)[0].cpu().numpy()
    P = np.abs(psi.astype(np.complex128)) ** 2
    assert np.max(np.abs(P * 2.0 ** n - 1.0)) <= (1e-12 if prec == "c128" else 1e-5)
