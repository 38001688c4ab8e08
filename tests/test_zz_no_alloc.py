"""qaoa_expect_noalloc, the allocation-free variant of qaoa_expect, against
qaoa_expect itself (same kernels: bitwise equal results) and the oracle, on
two calls in a row, the second smaller than the first, then a size beyond its
fixed scratch (rejected).  Free device memory is the same before and after
its calls."""
import numpy as np
import pytest

import oracle
from paper_2506_10531_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def cuda(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def test_noalloc_matches_expect_on_two_calls():
    from paper_2506_10531_amd import _lib, api
    assert torch.cuda.is_available()
    # (prec, B, n, p, S): 2 x 4 complex64 n = 20 states (64 MiB of state),
    # then a smaller complex128 call with probabilities
    cases = [("c64", 2, 20, 3, 4), ("c128", 1, 11, 2, 3)]
    for prec, B, n, p, S in cases:
        print(f"noalloc case prec={prec} B={B} n={n} p={p} S={S}", flush=True)
        Qs = workloads.qubos(B, n, 4100 + n)
        g, b = workloads.params(S, p, 4200 + n, lead=(B,))
        Qd, gd, bd = cuda(Qs), cuda(g), cuda(b)
        want_probs = n <= 12
        ref = api.expect(Qd, gd, bd, prec=prec, norm=True, probs=want_probs)
        out = torch.full((B, S), float("nan"), dtype=torch.float64, device="cuda:0")
        nr = torch.full((B, S), float("nan"), dtype=torch.float64, device="cuda:0")
        pr = None
        if want_probs:
            dt = torch.float64 if prec == "c128" else torch.float32
            pr = torch.full((B, S, 1 << n), float("nan"), dtype=dt, device="cuda:0")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]  # after every tensor of the test exists
        api.expect_noalloc(Qd, gd, bd, out, norm=nr, probs=pr, prec=prec)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        assert torch.equal(out, ref[0]) and torch.equal(nr, ref[1])
        if want_probs:
            assert torch.equal(pr, ref[2])
        # the oracle's bar for the first problem
        eo = oracle.expect(Qs[0], g[0], b[0])[0]
        cm = float(np.max(np.abs(oracle.cost_table(Qs[0]))))
        tol = (1e-10 * np.maximum(np.abs(eo), 1.0)) if prec == "c128" else 1e-5 * cm
        assert np.all(np.abs(out.cpu().numpy()[0] - eo) <= tol)
    # beyond the fixed scratch: a clear error, nothing queued
    Q = cuda(workloads.qubo(26, 4300))
    g, b = workloads.params(1, 1, 4301)
    out = torch.empty((1, 1), dtype=torch.float64, device="cuda:0")
    with pytest.raises(_lib.QaoaError) as ei:
        api.expect_noalloc(Q, cuda(g), cuda(b), out, prec="c64")
    assert ei.value.code == _lib.ERR_OUT_OF_MEMORY
    assert "fixed scratch" in str(ei.value)
