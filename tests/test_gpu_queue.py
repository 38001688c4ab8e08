"""The solve queue on the GPU: results against the oracle's solve loop in
both precisions, the alone-versus-mix identity, FIFO admission, admission of
an arrival while a long step runs, backpressure, budget rejection and
cancellation."""
import time

import numpy as np
import pytest

import oracle
from paper_2506_10531_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = 0x9E3779B97F4A7C15


@pytest.fixture(scope="module")
def serve():
    assert torch.cuda.is_available()
    from paper_2506_10531_amd import serve as s
    return s


def reqs(count, p, seed, n_lo=4, n_hi=15):
    _, rs = workloads.subqubo_requests(count, N=60, n_lo=n_lo, n_hi=n_hi, seed=seed)
    g, b = workloads.params(count, p, seed + 1)
    return [(Q, g[i], b[i], 1000 + i) for i, (_, Q) in enumerate(rs)]


def test_queue_matches_oracle_solve_loop(serve):
    p, evals, shots = 2, 6, 256
    rs = reqs(6, p, 10, n_lo=5, n_hi=16)
    with serve.SolveQueue(prec="c128", p=p, evals=evals, shots=shots, max_slots=8) as q:
        tickets = [q.submit(Q, g, b, sd) for Q, g, b, sd in rs]
        res = [q.wait(t, timeout_s=60) for t in tickets]
    for (Q, g, b, sd), r in zip(rs, res):
        print(f"queue oracle n={Q.shape[0]}", flush=True)
        assert r["status"] == 0
        o = oracle.adam_solve(Q, g, b, evals=evals, shots=shots, seed=sd)
        assert np.allclose(r["gamma"], o["gamma"], atol=1e-9), (r["gamma"], o["gamma"])
        assert np.allclose(r["beta"], o["beta"], atol=1e-9)
        assert abs(r["expect"] - o["expect"]) <= 1e-9 * max(1.0, abs(o["expect"]))
        mism = (r["samples"] != o["z"]).sum()
        assert mism <= 2, mism
        assert r["best_c"] <= o["best_c"] + 1e-12 or mism > 0
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]


def test_queue_complex64_matches_oracle_solve_loop(serve):
    """Complex64 solves after 5 Adam evaluations against the complex128
    oracle loop: <C> within the complex64 tolerance 1e-5 max|C| (Adam
    normalises each step, so a gradient error dg moves theta by about
    lr dg / |g| and <C> by about lr dg, well inside it), parameters within
    1e-3, and samples equal except near CDF boundaries."""
    p, evals, shots = 3, 5, 512
    rs = reqs(8, p, 60, n_lo=8, n_hi=22)
    with serve.SolveQueue(prec="c64", p=p, evals=evals, shots=shots, max_slots=8) as q:
        tickets = [q.submit(Q, g, b, sd) for Q, g, b, sd in rs]
        res = [q.wait(t, timeout_s=120) for t in tickets]
    for (Q, g, b, sd), r in zip(rs, res):
        n = Q.shape[0]
        print(f"queue c64 oracle n={n}", flush=True)
        assert r["status"] == 0
        o = oracle.adam_solve(Q, g, b, evals=evals, shots=shots, seed=sd)
        cmax = float(np.max(np.abs(oracle.cost_table(Q))))
        dth = max(np.max(np.abs(r["gamma"] - o["gamma"])), np.max(np.abs(r["beta"] - o["beta"])))
        print(f"  |d<C>| = {abs(r['expect'] - o['expect']):.2e}  max|C| = {cmax:.2f}  "
              f"|dtheta| = {dth:.2e}", flush=True)
        assert abs(r["expect"] - o["expect"]) <= 1e-5 * cmax
        assert dth <= 1e-3
        mism = int((r["samples"] != o["z"]).sum())
        assert mism <= shots // 100, mism


def test_arrival_admitted_within_a_few_evaluations(serve):
    """A request that arrives while a long step runs and finds a free slot
    joins after at most a few evaluations (the scheduler ends a step early
    for it), not after the step's up to 16 evaluations."""
    p, evals = 3, 240
    long_q = [workloads.qubo(22, 70 + i) for i in range(8)]
    g, b = workloads.params(9, p, 71)
    small = workloads.qubo(12, 72)
    with serve.SolveQueue(prec="c64", p=p, evals=evals, shots=64, max_slots=11) as q:
        ts = [q.submit(Q, g[i], b[i], i) for i, Q in enumerate(long_q)]
        deadline = time.time() + 60
        while q.stats()["active"] != 8:
            assert time.time() < deadline
            time.sleep(0.001)
        tks = []
        for k in range(3):  # three arrivals while the long solves run
            time.sleep(0.023 + 0.011 * k)
            tks.append(q.submit(small, g[8], b[8], 100 + k))
        rs = [q.wait(t, timeout_s=120) for t in tks]
        rl = [q.wait(t, timeout_s=120) for t in ts]
    assert all(r["status"] == 0 for r in rs + rl)
    # the arrivals came while the long solves were still running
    assert all(r["t_submit_ns"] < rl[0]["t_done_ns"] for r in rs)
    waits = [r["t_admit_ns"] - r["t_submit_ns"] for r in rs]
    per_eval = (rl[0]["t_done_ns"] - rl[0]["t_admit_ns"]) / evals
    print(f"admission waits {[w / 1e6 for w in waits]} ms; one evaluation of the "
          f"eight n=22 solves {per_eval / 1e6:.3f} ms", flush=True)
    assert max(waits) <= 5 * per_eval + 2e6


def _run(serve, items, **kw):
    with serve.SolveQueue(**kw) as q:
        ts = [q.submit(Q, g, b, sd) for Q, g, b, sd in items]
        return [q.wait(t, timeout_s=120) for t in ts]


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_alone_equals_mix(serve, prec):
    p, evals, shots = 3, 5, 128
    mix = reqs(10, p, 20, n_lo=4, n_hi=16)
    kw = dict(prec=prec, p=p, evals=evals, shots=shots)
    in_mix = _run(serve, mix, max_slots=16, **kw)
    for i in (0, 3, 7):
        alone = _run(serve, [mix[i]], max_slots=1, **kw)[0]
        a, m = alone, in_mix[i]
        assert np.array_equal(a["gamma"], m["gamma"]) and np.array_equal(a["beta"], m["beta"])
        assert a["expect"] == m["expect"]
        assert np.array_equal(a["samples"], m["samples"])
        assert (a["best_z"], a["best_c"]) == (m["best_z"], m["best_c"])


def test_backpressure_budget_and_cancel(serve):
    from paper_2506_10531_amd import _lib
    p = 2
    Q = workloads.qubo(16, 1)
    g, b = workloads.params(1, p, 2)
    # one slot, two pending places, requests far longer than the test
    with serve.SolveQueue(prec="c64", p=p, evals=10**6, shots=16, max_slots=1,
                          max_pending=2) as q:
        t0 = q.submit(Q, g[0], b[0], 1)
        deadline = time.time() + 30
        while q.stats()["active"] != 1:
            assert time.time() < deadline
            time.sleep(0.001)
        t1 = q.submit(Q, g[0], b[0], 2)
        t2 = q.submit(Q, g[0], b[0], 3)
        assert q.submit(Q, g[0], b[0], 4, raise_full=False) is None  # full
        q.cancel(t1)  # pending: cancelled at once
        assert q.wait(t1, timeout_s=5)["status"] == _lib.ERR_CANCELLED
        q.cancel(t0)  # running: cancelled at the next step boundary
        assert q.wait(t0, timeout_s=30)["status"] == _lib.ERR_CANCELLED
        q.cancel(t2)
        assert q.wait(t2, timeout_s=30)["status"] == _lib.ERR_CANCELLED
        st = q.stats()
        assert st["rejected"] == 1 and st["cancelled"] == 3 and st["completed"] == 0
        with pytest.raises(_lib.QaoaError) as ei:
            q.cancel(t2)  # finished and released
        assert ei.value.code == _lib.ERR_NOT_FOUND
    # a request larger than the whole budget is refused at submit
    with serve.SolveQueue(prec="c64", p=p, evals=1, shots=16, max_slots=2,
                          hbm_budget=1 << 22) as q:
        Qb = workloads.qubo(20, 3)
        with pytest.raises(_lib.QaoaError) as ei:
            q.submit(Qb, g[0], b[0], 5)
        assert ei.value.code == _lib.ERR_OUT_OF_MEMORY


def test_admission_respects_budget(serve):
    """With a budget for two n = 18 requests, at most two are resident."""
    p = 2
    Q = workloads.qubo(18, 4)
    g, b = workloads.params(1, p, 5)
    from paper_2506_10531_amd import api
    ctx = api.default_context()
    one = ctx.plan("c64", 1, 18, p, 1, grad=True)["scratch_bytes"]
    with serve.SolveQueue(prec="c64", p=p, evals=3, shots=16, max_slots=8,
                          hbm_budget=int(2.6 * one) + (8 << 20)) as q:
        budget = int(2.6 * one) + (8 << 20)
        ts = [q.submit(Q, g[0], b[0], i) for i in range(5)]
        rs = [q.wait(t) for t in ts]
        # the scheduler's own high-water marks (sampling the current count
        # from here can miss short requests altogether)
        st = q.stats()
        assert st["completed"] == 5, st
        assert 1 <= st["peak_active"] <= 2, st
        assert st["peak_bytes"] <= budget, st
    # FIFO: admission times are ordered by submission
    adm = [r["t_admit_ns"] for r in rs]
    assert adm == sorted(adm)


def test_graph_replays_equal_eager_steps(serve, monkeypatch):
    """Evaluation steps replayed from captured graphs give bitwise the
    results of eager steps (every request runs many replays, with the index
    uploads and other groups' eager work in between)."""
    p, evals, shots = 2, 12, 64
    mix = reqs(12, p, 40, n_lo=4, n_hi=17)
    kw = dict(prec="c64", p=p, evals=evals, shots=shots, max_slots=6)
    monkeypatch.setenv("DQAOA_QUEUE_GRAPHS", "1")
    with_graphs = _run(serve, mix, **kw)
    monkeypatch.setenv("DQAOA_QUEUE_GRAPHS", "0")
    eager = _run(serve, mix, **kw)
    for a, b in zip(with_graphs, eager):
        assert a["status"] == 0 and b["status"] == 0
        assert np.array_equal(a["gamma"], b["gamma"]) and np.array_equal(a["beta"], b["beta"])
        assert a["expect"] == b["expect"]
        assert np.array_equal(a["samples"], b["samples"])
