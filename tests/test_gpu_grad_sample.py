"""GPU parity of the adjoint gradient and of sampling against the oracle.

Gradient tolerances: complex128 within 1e-10 * max(1, max_z |C(z)|) of the
oracle's adjoint and within 1e-6 relative of central differences (h = 1e-6)
of the GPU's own complex128 <C>; complex64 within 1e-5 * max_z |C(z)| * p of
the oracle.  Sampling: every shot equals the oracle's draw unless the oracle's
u_s * total lies within twice the CDF error bound of an interval boundary.
That bound is rigorous and measured per problem: the running sums of |psi|^2
differ from the oracle's by at most
  sum_z | |a_z|^2 - |b_z|^2 | <= ||a - b||_2 ||a + b||_2 <= L2 (2 + L2)
(L2 = ||psi_gpu - psi_oracle||_2 of the state itself), plus the rounding of
|psi|^2 in the state's precision (2^-22 of the total for complex64) and of
the FP64 sums.
"""
import numpy as np
import pytest

import oracle
from paper_2506_10531_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = 0x9E3779B97F4A7C15


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available()
    from paper_2506_10531_amd import api as a
    return a


def cuda(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def cmax(Q):
    return float(np.max(np.abs(oracle.cost_table(Q))))


# the whole-state adjoint (n <= 12, complex64 n <= 13): one case per
# register-bit count (n = 1..8 none, 9..13 one to five) and partial waves
# (n < 6)
GRAD_CASES = [("c128", 1, 2), ("c128", 3, 1), ("c128", 7, 2), ("c128", 8, 3), ("c128", 9, 2),
              ("c128", 10, 3), ("c128", 11, 2), ("c128", 12, 2), ("c128", 13, 2),
              ("c128", 14, 1), ("c128", 16, 3), ("c128", 17, 4), ("c128", 18, 2),
              ("c128", 20, 6), ("c128", 22, 2), ("c64", 2, 3), ("c64", 5, 2), ("c64", 7, 1),
              ("c64", 9, 3), ("c64", 10, 2), ("c64", 11, 3), ("c64", 12, 4), ("c64", 13, 1), ("c64", 13, 4),
              ("c64", 14, 2), ("c64", 15, 1), ("c64", 16, 6), ("c64", 17, 5),
              ("c64", 18, 3), ("c64", 19, 3), ("c64", 20, 2), ("c64", 21, 1),
              ("c64", 22, 2)]


@pytest.mark.parametrize("prec,n,p", GRAD_CASES)
def test_grad_matches_oracle(api, prec, n, p):
    B, S = 2, 2
    Qs = workloads.qubos(B, n, 3000 + n)
    g, b = workloads.params(S, p, 3100 + n + p, lead=(B,))
    print(f"grad case prec={prec} n={n} p={p}", flush=True)
    e, dg, db = api.grad(cuda(Qs), cuda(g), cuda(b), prec=prec)
    e, dg, db = e.cpu().numpy(), dg.cpu().numpy(), db.cpu().numpy()
    for bi in range(B):
        eo, dgo, dbo = oracle.grad(Qs[bi], g[bi], b[bi])
        cm = cmax(Qs[bi])
        tol = 1e-10 * max(1.0, cm) if prec == "c128" else 1e-5 * cm * p
        assert np.max(np.abs(dg[bi] - dgo)) <= tol, (np.max(np.abs(dg[bi] - dgo)), tol)
        assert np.max(np.abs(db[bi] - dbo)) <= tol, (np.max(np.abs(db[bi] - dbo)), tol)
        etol = 1e-10 * max(1.0, cm) if prec == "c128" else 1e-5 * cm
        assert np.max(np.abs(e[bi] - eo)) <= etol


@pytest.mark.parametrize("n,p", [(23, 2), (24, 2), (25, 1), (26, 1)])
def test_grad_large_n_checkpointed(api, n, p):
    """n = 23..26 (served by qaoa_grad and by solve-queue requests): the
    LDS-tile adjoint with per-pass checkpoints over three qubit sets (two
    for complex64 at n <= 24), both precisions against one oracle gradient."""
    Q = workloads.qubo(n, 3700 + n)
    g, b = workloads.params(1, p, 3800 + n)
    eo, dgo, dbo = oracle.grad(Q, g, b)
    cm = cmax(Q)
    for prec in ("c128", "c64"):
        print(f"grad case prec={prec} n={n} p={p}", flush=True)
        e, dg, db = (x.cpu().numpy()[0] for x in api.grad(cuda(Q), cuda(g), cuda(b), prec=prec))
        tol = 1e-10 * max(1.0, cm) if prec == "c128" else 1e-5 * cm * p
        etol = 1e-10 * max(1.0, abs(eo[0])) if prec == "c128" else 1e-5 * cm
        assert np.max(np.abs(dg - dgo)) <= tol, (prec, np.max(np.abs(dg - dgo)), tol)
        assert np.max(np.abs(db - dbo)) <= tol, (prec, np.max(np.abs(db - dbo)), tol)
        assert abs(e[0] - eo[0]) <= etol, (prec, e[0], eo[0])


@pytest.mark.parametrize("prec,n", [("c64", 14), ("c128", 13), ("c64", 12), ("c128", 10),
                                    ("c64", 13)])
def test_grad_at_max_layers(api, prec, n):
    """QAOA_MAX_P = 64 layers: on register tiles p + 1 = 65 passes on two
    qubit sets, whose checkpoint and adjoint tables make 2p + 1 = 129 jobs of
    one tables launch; on the whole-state adjoint (n <= 12, complex64 13) 64
    layers undone in registers."""
    p = 64
    Q = workloads.qubos(1, n, 3300 + n)
    g, b = workloads.params(1, p, 3400 + n, lead=(1,))
    g, b = g * 0.1, b * 0.1
    print(f"grad case prec={prec} n={n} p={p}", flush=True)
    e, dg, db = api.grad(cuda(Q), cuda(g), cuda(b), prec=prec)
    eo, dgo, dbo = oracle.grad(Q[0], g[0], b[0])
    cm = cmax(Q[0])
    tol = 1e-10 * max(1.0, cm) if prec == "c128" else 1e-5 * cm * p
    assert np.max(np.abs(dg.cpu().numpy()[0] - dgo)) <= tol
    assert np.max(np.abs(db.cpu().numpy()[0] - dbo)) <= tol
    assert abs(e.cpu().numpy()[0] - eo).max() <= (1e-10 * max(1.0, cm) if prec == "c128" else 1e-5 * cm)


@pytest.mark.parametrize("n,p", [(9, 2), (16, 3)])
def test_grad_matches_central_differences(api, n, p):
    Q = workloads.qubo(n, 3200 + n)
    g, b = workloads.params(1, p, 3300 + n)
    _, dg, db = api.grad(cuda(Q), cuda(g), cuda(b), prec="c128")
    dg, db = dg.cpu().numpy()[0, 0], db.cpu().numpy()[0, 0]
    h = 1e-6
    # all shifted parameter sets in one batched expect call
    G = np.repeat(g, 4 * p, axis=0)
    Bt = np.repeat(b, 4 * p, axis=0)
    for j in range(p):
        G[4 * j + 0, j] += h
        G[4 * j + 1, j] -= h
        Bt[4 * j + 2, j] += h
        Bt[4 * j + 3, j] -= h
    e = api.expect(cuda(Q), cuda(G), cuda(Bt), prec="c128").cpu().numpy()[0]
    for j in range(p):
        fdg = (e[4 * j] - e[4 * j + 1]) / (2 * h)
        fdb = (e[4 * j + 2] - e[4 * j + 3]) / (2 * h)
        assert abs(dg[j] - fdg) <= 1e-6 * max(1.0, abs(fdg)), (j, dg[j], fdg)
        assert abs(db[j] - fdb) <= 1e-6 * max(1.0, abs(fdb)), (j, db[j], fdb)


def test_diff_n16_batch_512(api):
    """512 dense n = 16 QUBOs, p = 6, both precisions; the oracle checks a
    sample of 6 problems (first, last and spread)."""
    W = workloads.WORKLOADS["diff_n16"]
    B, n, p = W["batch"], W["n"], W["p"]
    Qs = workloads.qubos(B, n, W["q_seed"])
    g, b = workloads.params(1, p, W["p_seed"], lead=(B,))
    Qd, gd, bd = cuda(Qs), cuda(g), cuda(b)
    e64, dg64, db64 = (x.cpu().numpy() for x in api.grad(Qd, gd, bd, prec="c64"))
    e128, dg128, db128 = (x.cpu().numpy() for x in api.grad(Qd, gd, bd, prec="c128"))
    for bi in (0, 1, 101, 255, 400, 511):
        eo, dgo, dbo = oracle.grad(Qs[bi], g[bi], b[bi])
        cm = cmax(Qs[bi])
        assert np.max(np.abs(dg128[bi] - dgo)) <= 1e-10 * cm
        assert np.max(np.abs(db128[bi] - dbo)) <= 1e-10 * cm
        assert np.max(np.abs(dg64[bi] - dgo)) <= 1e-5 * cm * p
        assert np.max(np.abs(db64[bi] - dbo)) <= 1e-5 * cm * p
        assert abs(e128[bi, 0] - eo[0]) <= 1e-10 * max(1.0, abs(eo[0]))


def test_autograd_function(api):
    n, p, S = 12, 3, 2
    Q = cuda(workloads.qubo(n, 3400))
    g0, b0 = workloads.params(S, p, 3401)
    g = cuda(g0[None]).requires_grad_(True)
    b = cuda(b0[None]).requires_grad_(True)
    e = api.QAOAExpect.apply(Q[None], g, b, "c128")
    w = torch.tensor([[0.5, -2.0]], dtype=torch.float64, device="cuda:0")
    (e * w).sum().backward()
    _, dg, db = api.grad(Q, cuda(g0), cuda(b0), prec="c128")
    assert torch.allclose(g.grad, dg * w[..., None], atol=1e-12)
    assert torch.allclose(b.grad, db * w[..., None], atol=1e-12)


@pytest.mark.parametrize("prec,n,p", [("c128", 6, 2), ("c128", 13, 1), ("c128", 17, 2),
                                      ("c128", 19, 2), ("c128", 22, 3), ("c128", 24, 1),
                                      ("c64", 10, 3), ("c64", 14, 2), ("c64", 18, 2),
                                      ("c64", 19, 3), ("c64", 20, 2), ("c64", 21, 2),
                                      ("c64", 22, 3), ("c64", 24, 2), ("c64", 25, 2),
                                      ("c128", 25, 1)])
def test_sampling_matches_oracle_draws(api, prec, n, p):
    """Every register-tile probability store: complex64 n = 19..24 keep 7 down
    to 4 contiguous low qubits in the last pass's set (first mixed bit 4..7),
    complex128 n = 19..24 the 13-qubit plans, and n = 25 the three-set plans
    (their last pass on the last set after a lead-only pass)."""
    B, shots, seed = (3 if n <= 21 else 2 if n <= 24 else 1), 2048, 12345
    Qs = workloads.qubos(B, n, 3500 + n)
    g, b = workloads.params(1, p, 3600 + n, lead=(B,))
    r = api.sample(cuda(Qs), cuda(g[:, 0]), cuda(b[:, 0]), shots, seed, prec=prec)
    z = r["z"].cpu().numpy().astype(np.uint64)
    cz = r["cz"].cpu().numpy()
    bz = r["best_z"].cpu().numpy().astype(np.uint64)
    bc = r["best_c"].cpu().numpy()
    ex = r["expect"].cpu().numpy()
    psi = api.state(cuda(Qs), cuda(g), cuda(b), prec=prec)[0].cpu().numpy()[:, 0]
    eps_p = 2.0 ** -22 if prec == "c64" else 1e-14
    for bi in range(B):
        seed_b = (seed + bi * shots * GOLDEN) % 2**64
        o = oracle.sample(Qs[bi], g[bi, 0], b[bi, 0], shots, seed_b)
        l2 = float(np.linalg.norm(psi[bi].astype(np.complex128) - oracle.state(Qs[bi], g[bi], b[bi])))
        bound = 2.0 * (l2 * (2.0 + l2) + eps_p) + 1e-12
        diff = z[bi] != o["z"]
        print(f"sample {prec} n={n} problem {bi}: state L2 {l2:.2e}, {int(diff.sum())} draws "
              f"of {shots} differ, all within {bound:.2e} of a boundary", flush=True)
        # a mismatch is allowed only where the draw sits at a CDF boundary
        assert np.all(o["gap"][diff] <= bound), (o["gap"][diff], bound)
        assert l2 <= (1e-4 if prec == "c64" else 1e-10), l2
        C = oracle.cost_table(Qs[bi])
        assert np.allclose(cz[bi], C[z[bi].astype(np.int64)], atol=1e-12)
        order = np.lexsort((z[bi], cz[bi]))
        assert bz[bi] == z[bi][order[0]] and bc[bi] == cz[bi][order[0]]
        eo = oracle.expect(Qs[bi], g[bi], b[bi])[0][0]
        etol = 1e-10 * max(1.0, abs(eo)) if prec == "c128" else 1e-5 * np.max(np.abs(C))
        assert abs(ex[bi] - eo) <= etol


@pytest.mark.parametrize("prec,n", [("c64", 10), ("c128", 13), ("c64", 16)])
def test_sampling_nullable_outputs(api, prec, n):
    """qaoa_sample with cz and expect NULL (the whole-state launch at n <= 14 /
    13 then writes <C> to scratch) draws exactly what the call with every
    output does."""
    import ctypes

    from paper_2506_10531_amd import _lib
    B, shots, seed, p = 3, 512, 777, 2
    Qs = workloads.qubos(B, n, 3700 + n)
    g, b = workloads.params(1, p, 3800 + n, lead=(B,))
    Qd, gd, bd = cuda(Qs), cuda(g[:, 0]), cuda(b[:, 0])
    full = api.sample(Qd, gd, bd, shots, seed, prec=prec)
    z = torch.empty((B, shots), dtype=torch.int64, device="cuda:0")
    bz = torch.empty((B,), dtype=torch.int64, device="cuda:0")
    bc = torch.empty((B,), dtype=torch.float64, device="cuda:0")
    ctx = api.default_context(0)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = _lib.load().qaoa_sample(ctx.h, api.PREC[prec], B, n, p, vp(Qd), vp(gd), vp(bd), shots,
                                 seed, vp(z), None, vp(bz), vp(bc), None,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, _lib.load().qaoa_last_error()
    torch.cuda.synchronize()
    assert torch.equal(z, full["z"]) and torch.equal(bz, full["best_z"])
    assert torch.equal(bc, full["best_c"])
