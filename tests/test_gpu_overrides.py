"""The kernel-selection switches, read once per process: with
DQAOA_FWD_KERNEL=lds every forward evaluation runs the LDS-tile pass, and with
DQAOA_GRAD_KERNEL=lds every gradient runs the LDS-tile adjoint (otherwise
reached only above 22 qubits).  A child process with each switch set
evaluates seeded cases and prints them; its <C>, probabilities and gradients
must match the oracle within the tolerances of the default paths
(complex128: 1e-10 relative; complex64: 1e-5 of max |C|, gradients times p)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2506_10531_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_2506_10531_amd import api, workloads
cases = json.loads(sys.argv[2])
out = []
for prec, n, p, op in cases:
    Q = workloads.qubos(2, n, 5100 + n)
    g, b = workloads.params(2, p, 5200 + n, lead=(2,))
    d = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda:0")
    print(f"override case {prec} n={n} p={p} {op}", file=sys.stderr, flush=True)
    if op == "expect":
        e, P = api.expect(d(Q), d(g), d(b), prec=prec, probs=True)
        out.append({"e": e.cpu().numpy().tolist(), "P": P.cpu().double().numpy().tolist()})
    else:
        e, dg, db = api.grad(d(Q), d(g), d(b), prec=prec)
        out.append({"e": e.cpu().numpy().tolist(), "dg": dg.cpu().numpy().tolist(),
                    "db": db.cpu().numpy().tolist()})
print(json.dumps(out))
"""


def run_child(env_var, cases):
    env = dict(os.environ)
    env[env_var] = "lds"
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, json.dumps(cases)], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def cmax(Q):
    return float(np.max(np.abs(oracle.cost_table(Q))))


def test_lds_tile_forward_pass_matches_oracle():
    # single-tile (n <= 14 / 13) and multi-pass (above) LDS-tile plans
    cases = [("c64", 10, 2, "expect"), ("c64", 14, 3, "expect"), ("c64", 17, 2, "expect"),
             ("c128", 9, 3, "expect"), ("c128", 13, 2, "expect"), ("c128", 16, 2, "expect")]
    res = run_child("DQAOA_FWD_KERNEL", cases)
    for (prec, n, p, _), r in zip(cases, res):
        Q = workloads.qubos(2, n, 5100 + n)
        g, b = workloads.params(2, p, 5200 + n, lead=(2,))
        for bi in range(2):
            eo, _, Po = oracle.expect(Q[bi], g[bi], b[bi], probs=True)
            e = np.array(r["e"][bi])
            P = np.array(r["P"][bi])
            # a state within L2 of the oracle's moves each |psi(z)|^2 by at most
            # L2 (2 |psi(z)| + L2); L2 as for the default paths (1e-12 / 1e-4)
            l2 = 1e-12 if prec == "c128" else 1e-4
            assert np.max(np.abs(P - Po)) <= l2 * (2.0 * np.sqrt(np.max(Po)) + l2), n
            if prec == "c128":
                assert np.all(np.abs(e - eo) <= 1e-10 * np.maximum(np.abs(eo), 1.0)), (n, e, eo)
            else:
                assert np.all(np.abs(e - eo) <= 1e-5 * cmax(Q[bi])), (n, e, eo)


def test_lds_tile_adjoint_matches_oracle():
    cases = [("c64", 10, 2, "grad"), ("c64", 13, 3, "grad"), ("c64", 16, 2, "grad"),
             ("c128", 8, 3, "grad"), ("c128", 12, 2, "grad"), ("c128", 15, 2, "grad")]
    res = run_child("DQAOA_GRAD_KERNEL", cases)
    for (prec, n, p, _), r in zip(cases, res):
        Q = workloads.qubos(2, n, 5100 + n)
        g, b = workloads.params(2, p, 5200 + n, lead=(2,))
        for bi in range(2):
            eo, dgo, dbo = oracle.grad(Q[bi], g[bi], b[bi])
            cm = cmax(Q[bi])
            tol = 1e-10 * max(1.0, cm) if prec == "c128" else 1e-5 * cm * p
            assert np.max(np.abs(np.array(r["dg"][bi]) - dgo)) <= tol, (prec, n)
            assert np.max(np.abs(np.array(r["db"][bi]) - dbo)) <= tol, (prec, n)
            etol = 1e-10 * max(1.0, cm) if prec == "c128" else 1e-5 * cm
            assert np.max(np.abs(np.array(r["e"][bi]) - eo)) <= etol, (prec, n)
