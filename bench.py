#!/usr/bin/env python3
"""Benchmark of the QAOA state-vector hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): one dense
n = 24 QUBO (symmetric, upper triangle i.i.d. uniform[-1, 1], seed 2), p = 4
layers, 16 (gamma, beta) parameter sets (gamma ~ U[0, pi], beta ~ U[0, pi/2],
seed 12), complex64 state with FP64 phase range reduction and FP64 <C>
reductions.  One step = one qaoa_expect call over all 16 sets: 16 * 4 * 2^24
amplitude-layer updates, inputs resident in HBM.

Printed: one JSON line with the throughput (amplitude-layer updates/s), the
achieved HBM bandwidth of the dominant kernel (the forward tile pass) from HIP
events on its launch stream, a roofline record against MI355X's 8 TB/s, the
CPU oracle timed on a bounded sample on the host cores, and the numerical
error of the complex64 form against complex128 and the oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = ("amplitude-layer updates/s + HBM GB/s; sub-QUBO solves/s with p50/p99 "
          "latency")
# register-tile forward pass sources per precision, and the committed
# counter summary of each
KERNEL_SRC = {
    "c64": [os.path.join(ROOT, "paper_2506_10531_amd", "csrc", f)
            for f in ("fwd14.hip", "geom14.h", "regtile.h")],
    "c128": [os.path.join(ROOT, "paper_2506_10531_amd", "csrc", f)
             for f in ("fwd13d.hip", "geom13.h", "regtile.h")],
}
TRAFFIC_FILE = {
    "c64": os.path.join(ROOT, "profiles", "fwd_pass_precision_n24_traffic.json"),
    "c128": os.path.join(ROOT, "profiles", "fwd_pass_precision_n24_c128_traffic.json"),
}


def kernel_hash(prec: str = "c64") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRC[prec]:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def load_traffic(prec: str = "c64"):
    """HBM bytes per launch of the forward pass from the committed rocprofv3
    counter summary, if it was taken on the current kernel source (and the
    register-tile kernel is the one running)."""
    if os.environ.get("DQAOA_FWD_KERNEL") == "lds":
        return None
    try:
        rec = json.load(open(TRAFFIC_FILE[prec]))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha") != kernel_hash(prec):
        return None
    return rec.get("bytes_per_launch")


def timed_repeats(fn, min_s: float = 1.0, min_reps: int = 10) -> dict:
    """The timing protocol: calls of fn (each followed by a device
    synchronisation) until at least min_reps calls and min_s seconds have
    been timed; median and minimum per call."""
    import numpy as np
    import torch
    ts = []
    while len(ts) < min_reps or sum(ts) < min_s:
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return {"median_ms": 1e3 * float(np.median(ts)), "min_ms": 1e3 * float(np.min(ts)),
            "repeats": len(ts), "timed_s": float(sum(ts))}


def host_cpu() -> dict:
    """The host the CPU oracle runs on: model name and usable cores."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "usable_cores": len(os.sched_getaffinity(0))}


PAPER_CONTEXT = {
    "gpu_over_cpu": "up to 10x",
    "hardware": "Frontier: AMD Instinct MI250X GPUs against 64-core AMD EPYC CPUs",
    "workload": "DQAOA on dense QUBOs of N = 300/500/1000 split into sub-QUBOs of 20 "
                "variables, p = 1, COBYLA",
    "note": "context only: other hardware, simulators and workload; not a target",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="c64", choices=["c64", "c128"])
    ap.add_argument("--cpu-sets", type=int, default=16,
                    help="parameter sets the CPU oracle runs (bounded sample)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the complex128 comparison and error report")
    ap.add_argument("--serving-requests", type=int, default=4096,
                    help="requests replayed against the batched solve queue (0: skip)")
    ap.add_argument("--serving-single", type=int, default=-1,
                    help="requests of the same trace replayed against the one-at-a-time "
                         "queue (-1: all of them)")
    ap.add_argument("--serving-slots", type=int, default=256)
    ap.add_argument("--maxcut-cycles", type=int, default=3,
                    help="DQAOA cycles per decomposition on the sparse Max-Cut QUBO (0: skip)")
    ap.add_argument("--cobyla-subqubos", type=int, default=64,
                    help="sub-QUBOs of the COBYLA (p=1) versus device-Adam leg (0: skip)")
    ap.add_argument("--dqaoa-cycles", type=int, default=2,
                    help="DQAOA outer cycles on the N=1000 QUBO (0: skip)")
    ap.add_argument("--large-steps", type=int, default=3,
                    help="steps of the n=32 large-state workload (0: skip)")
    ap.add_argument("--grad-steps", type=int, default=5,
                    help="gradient calls per precision on the 512 x n=16, p=6 "
                         "differentiation workload (0: skip)")
    ap.add_argument("--legs", default="plain,p1,serving,large,dqaoa,cobyla,maxcut,grad",
                    help="comma-separated legs to run after the main workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a 2 GiB device copy (counter calibration)")
    return ap.parse_args()


def copy_probe():
    """A plain 2 GiB device-to-device copy: reads 2 GiB and writes 2 GiB, used
    to scale FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.copy_(a)
    t0.record()
    for _ in range(3):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / 3
    print(json.dumps({"copy_probe_bytes": a.numel() * 8, "launches": 4,
                      "copy_GBps": 2 * a.numel() * 8 / (ms * 1e-3) / 1e9}))


def serving_leg(requests: int, one_at_a_time: int, max_slots: int, calib: int,
                no_cpu: bool = False):
    """Sub-QUBO solves/s and p50/p99 latency of the solve queue.

    Requests come from one dense N = 1000 QUBO by random decomposition
    (n ~ U{12..22} sorted variables, principal submatrix), p = 3, 100 Adam
    evaluations + 1024 shots each, complex64.  A calibration run (all
    `calib` requests at once) gives the saturated rate mu; the Poisson trace
    arrives at 0.8 mu and is replayed against the batched queue and against
    the one-request-at-a-time queue (the first `one_at_a_time` requests, all
    of them by default).  Latency = done - submit (library clock)."""
    import threading

    import numpy as np

    from paper_2506_10531_amd import serve, workloads

    W = workloads.WORKLOADS["serving"]
    p, evals, shots = W["p"], W["evals"], W["shots"]
    _, reqs = workloads.subqubo_requests(requests, N=W["N"], n_lo=W["n_lo"],
                                         n_hi=W["n_hi"], seed=W["q_seed"])
    g0, b0 = workloads.params(requests, p, W["q_seed"] + 7)
    items = [(Q, g0[i], b0[i], 10_000 + i) for i, (_, Q) in enumerate(reqs)]

    def run(batch, items, arrivals):
        q = serve.SolveQueue(prec="c64", p=p, evals=evals, shots=shots,
                             max_slots=max_slots if batch else 1, batched=batch,
                             max_pending=len(items) + 1)
        tickets = [None] * len(items)

        def client():
            t0 = time.perf_counter()
            for i, (Q, g, b, sd) in enumerate(items):
                if arrivals is not None:
                    dt = arrivals[i] - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                tickets[i] = q.submit(Q, g, b, sd)

        th = threading.Thread(target=client)
        th.start()
        res = []
        for i in range(len(items)):
            while tickets[i] is None:
                time.sleep(0.0005)
            res.append(q.wait(tickets[i]))
        th.join()
        q.close()
        ok = [r for r in res if r["status"] == 0]
        lat = np.array([(r["t_done_ns"] - r["t_submit_ns"]) * 1e-6 for r in ok])
        span = (max(r["t_done_ns"] for r in ok) - min(r["t_submit_ns"] for r in ok)) * 1e-9
        return dict(solves=len(ok), failed=len(res) - len(ok),
                    solves_per_s=len(ok) / span, p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), span_s=span)

    ns = [Q.shape[0] for Q, _, _, _ in items]
    cal = run(True, items[:calib], None)
    rate = 0.8 * cal["solves_per_s"]
    arr = workloads.poisson_arrivals(requests, rate, W["arrival_seed"])
    batched = run(True, items, arr)
    if one_at_a_time < 0 or one_at_a_time > requests:
        one_at_a_time = requests
    single = (run(False, items[:one_at_a_time], arr[:one_at_a_time]) if one_at_a_time > 0
              else {"solves": 0})
    out = {
        "workload": (f"{requests} sub-QUBOs of one dense N={W['N']} QUBO, n~U{{"
                     f"{W['n_lo']}..{W['n_hi']}}}, p={p}, {evals} Adam evaluations + "
                     f"{shots} shots each, complex64, Poisson arrivals at 0.8 x the "
                     f"saturated rate"),
        "saturated_solves_per_s": cal["solves_per_s"],
        "arrival_rate_per_s": rate,
        "batched": batched,
        "one_at_a_time": dict(single, requests=one_at_a_time,
                              note=("the same trace" if one_at_a_time == requests
                                    else "first requests of the same trace")),
        "max_slots": max_slots,
    }
    if not no_cpu:
        out["cpu_oracle"] = serving_oracle(W["n_lo"], W["n_hi"], p, evals, shots, ns, 5000)
    return out


def plain_leg(no_cpu: bool):
    """The plain form: one dense n = 10 QUBO, p = 2, 64 parameter sets,
    complex128, <C> and the full probability vector of every set (one
    qaoa_expect per call, through api.Evaluator, and for comparison through
    api.expect).  Small enough that every state lives in one
    work-group's registers (one launch per call): the call is bound by FP64
    VALU latency and launch overhead, not HBM, so
    it reports updates/s and the FP64 rate of the counted arithmetic (6n
    flops of mixer butterflies and 6 of the phase multiply per
    amplitude-layer) against MI355X's 78.6 TFLOP/s FP64 vector peak."""
    import numpy as np
    import torch

    from paper_2506_10531_amd import api, workloads

    W = workloads.WORKLOADS["plain_n10"]
    n, p, S = W["n"], W["p"], W["sets"]
    Qh = workloads.qubo(n, W["q_seed"])
    g, b = workloads.params(S, p, W["p_seed"])
    dev = torch.device("cuda:0")
    Q, gd, bd = (torch.as_tensor(x, device=dev) for x in (Qh, g, b))
    ctx = api.Context(0)

    def call():
        api.expect(Q, gd, bd, prec="c128", probs=True, ctx=ctx)
    for _ in range(5):
        call()
    tx = timed_repeats(call)
    # the same evaluations with the problem and outputs bound once (one
    # qaoa_expect per call, as an optimiser loop makes them)
    ev = api.Evaluator(Q, S, p, prec="c128", probs=True, ctx=ctx)
    g3, b3 = gd.view(1, S, p).contiguous(), bd.view(1, S, p).contiguous()
    for _ in range(5):
        ev(g3, b3)
    tp = timed_repeats(lambda: ev(g3, b3))
    del ev
    ctx.close()
    updates = S * p * (1 << n)
    flops = updates * (6 * n + 6)
    out = {"workload": "plain_n10: one dense n=10 QUBO, p=2, 64 parameter sets, complex128, "
                       "<C> and probabilities",
           "value": updates / (tp["median_ms"] * 1e-3), "unit": "amplitude-layer updates/s",
           "timing": tp, "path": "api.Evaluator: one qaoa_expect per call",
           "api_expect": {"value": updates / (tx["median_ms"] * 1e-3), "timing": tx,
                          "path": "api.expect: arguments checked and outputs allocated per call"},
           "fp64_counted_flops_per_call": flops,
           "fp64_TFLOPs": flops / (tp["median_ms"] * 1e-3) / 1e12,
           "fp64_valu_frac": flops / (tp["median_ms"] * 1e-3) / 78.6e12}
    if not no_cpu:
        import oracle
        tc, calls = 0.0, 0
        while tc < 2.0 or calls < 3:
            t0 = time.perf_counter()
            oracle.expect(Qh, g, b, probs=True)
            tc += time.perf_counter() - t0
            calls += 1
        out["cpu_oracle"] = {"value": calls * updates / tc, "unit": "amplitude-layer updates/s",
                             "cores": oracle.num_threads(), "kind": "oracle",
                             "sample": f"{calls} whole calls (64 sets with probabilities)"}
    return out


def p1_leg():
    """The paper's depth: the n = 24 workload at p = 1 (16 sets, complex64),
    i.e. a first pass (generate |+>, phase, lead half-mixer, store) and a last
    pass (load, trail half-mixer, <C>) per evaluation, with their achieved
    bandwidth from the library's per-launch events."""
    import torch

    from paper_2506_10531_amd import api, workloads

    W = workloads.WORKLOADS["precision_n24"]
    n, S = W["n"], W["sets"]
    Q = torch.as_tensor(workloads.qubo(n, W["q_seed"]), device="cuda:0")
    g, b = workloads.params(S, 1, W["p_seed"])
    gd, bd = (torch.as_tensor(x, device="cuda:0") for x in (g, b))
    ctx = api.Context(0)

    def call():
        api.expect(Q, gd, bd, prec="c64", ctx=ctx)
    for _ in range(3):
        call()
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    tp = timed_repeats(call)
    ctx.profile(False)
    launches, pass_ms, pass_bytes = ctx.profile_read(reset=True)
    ctx.close()
    achieved = pass_bytes / (pass_ms * 1e-3) / 1e9
    return {"workload": "p1_n24: the n=24 QUBO of the main workload at p=1, 16 sets, complex64",
            "value": S * (1 << n) / (tp["median_ms"] * 1e-3), "unit": "amplitude-layer updates/s",
            "timing": tp, "pass_launches": launches, "achieved_GBps": achieved,
            "frac": achieved / PEAK_HBM_GBPS}


def serving_oracle(n_lo: int, n_hi: int, p: int, evals: int, shots: int, ns, seed: int) -> dict:
    """The oracle's one-request-at-a-time solve rate on the serving workload,
    extrapolated: one evaluation (exact <C> and adjoint gradient in
    complex128) is timed per qubit count, then a solve of n qubits costs
    `evals` evaluations plus a sampling pass, averaged over the trace's mix
    of n (a whole solve at n = 22 takes about a minute on the host)."""
    import numpy as np

    import oracle
    from paper_2506_10531_amd import workloads

    per_n = {}
    for n in range(n_lo, n_hi + 1):
        Q = workloads.qubo(n, seed + n)
        g, b = workloads.params(1, p, seed + 100 + n)
        t0 = time.perf_counter()
        oracle.grad(Q, g, b)
        t1 = time.perf_counter()
        oracle.sample(Q, g[0], b[0], shots, 1)
        t2 = time.perf_counter()
        per_n[n] = evals * (t1 - t0) + (t2 - t1)
    mean = float(np.mean([per_n[int(n)] for n in ns]))
    return {"solves_per_s": 1.0 / mean, "extrapolated": True, "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one timed complex128 evaluation (<C> + adjoint gradient) and one "
                      f"{shots}-shot sampling per n = {n_lo}..{n_hi}, scaled to {evals} "
                      f"evaluations per solve and averaged over the trace's n",
            "seconds_per_solve_by_n": {str(k): v for k, v in per_n.items()}}


def large_state_leg(steps: int, no_cpu: bool = False):
    """The n = 32, p = 2, 4-set complex64 workload (4 x 32 GiB states): one
    qaoa_expect per step, timed like the main workload, with the register-tile
    passes' achieved bandwidth from the library's per-launch events."""
    import torch

    from paper_2506_10531_amd import api, workloads

    W = workloads.WORKLOADS["large_n32"]
    n, p, S = W["n"], W["p"], W["sets"]
    dev = torch.device("cuda:0")
    Q = torch.as_tensor(workloads.qubo(n, W["q_seed"]), device=dev)
    g, b = workloads.params(S, p, W["p_seed"])
    gd, bd = torch.as_tensor(g, device=dev), torch.as_tensor(b, device=dev)
    ctx = api.Context(0)  # its own context: the 128 GiB scratch is freed at close
    plan = ctx.plan("c64", 1, n, p, S)
    api.expect(Q, gd, bd, prec="c64", ctx=ctx)  # warm-up (allocates the scratch)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        e = api.expect(Q, gd, bd, prec="c64", ctx=ctx)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile(False)
    launches, pass_ms, pass_bytes = ctx.profile_read(reset=True)
    en = e.cpu().numpy()[0]
    del e
    tp = timed_repeats(lambda: api.expect(Q, gd, bd, prec="c64", ctx=ctx), min_s=1.0,
                       min_reps=10)
    ctx.close()
    achieved = (pass_bytes / launches) / (pass_ms / launches * 1e-3) / 1e9
    floor = S * p * (1 << n) * 16
    cpu = None
    if not no_cpu:
        import oracle
        nc = 26  # the largest state the oracle takes on the host here (1 GiB complex128)
        Qc = workloads.qubo(nc, W["q_seed"])
        t0 = time.perf_counter()
        oracle.expect(Qc, g[:1], b[:1])
        tc = time.perf_counter() - t0
        cpu = {"value": p * (1 << nc) / tc, "unit": "amplitude-layer updates/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"one n={nc}, p={p} state (cost table + {p} layers), {tc:.1f} s; "
                         f"n=32 (64 GiB in complex128) is not run on the host"}
    return {
        "workload": "large_n32: one dense n=32 QUBO, p=2, 4 parameter sets, complex64 "
                    "(4 x 32 GiB states)",
        "value": S * p * (1 << n) * steps / wall,
        "unit": "amplitude-layer updates/s",
        "ms_per_step": 1e3 * wall / steps,
        "steps": steps,
        "hbm_GBps_floor": floor * steps / wall / 1e9,
        "passes": plan["passes"],
        "state_reads": plan["state_reads"],
        "state_writes": plan["state_writes"],
        "achieved_GBps": achieved,
        "frac": achieved / PEAK_HBM_GBPS,
        "expect": [float(x) for x in en],
        "timing": tp,
        "cpu_oracle": cpu,
    }


def grad_leg(steps: int, no_cpu: bool = False):
    """The differentiation workload (512 dense n = 16 QUBOs, p = 6): qaoa_grad
    in each precision, timed over `steps` calls, with the adjoint and
    checkpoint passes' bandwidth from the library's per-launch events."""
    import torch

    from paper_2506_10531_amd import api, workloads

    W = workloads.WORKLOADS["diff_n16"]
    B, n, p = W["batch"], W["n"], W["p"]
    dev = torch.device("cuda:0")
    Q = torch.as_tensor(workloads.qubos(B, n, W["q_seed"]), device=dev)
    g, b = workloads.params(B, p, W["p_seed"])
    gd = torch.as_tensor(g, device=dev).reshape(B, 1, p)
    bd = torch.as_tensor(b, device=dev).reshape(B, 1, p)
    ctx = api.Context(0)
    res = {"workload": f"diff_n16: {B} dense n={n} QUBOs, p={p}, one parameter set each",
           "steps": steps}
    for prec in ("c64", "c128"):
        plan = ctx.plan(prec, B, n, p, 1, grad=True)
        for _ in range(2):
            api.grad(Q, gd, bd, prec=prec, ctx=ctx)
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read(reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            api.grad(Q, gd, bd, prec=prec, ctx=ctx)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.profile(False)
        launches, pass_ms, pass_bytes = ctx.profile_read(reset=True)
        achieved = pass_bytes / (pass_ms * 1e-3) / 1e9
        res[prec] = {
            "ms_per_grad": 1e3 * wall / steps,
            "grads_per_s": B * steps / wall,
            "launches_per_grad": launches / steps,
            "pass_ms_per_grad": pass_ms / steps,
            "bytes_per_grad": pass_bytes / steps,
            "achieved_GBps": achieved,
            "frac": achieved / PEAK_HBM_GBPS,
            "tile_qubits": plan["tile_qubits"],
            "timing": timed_repeats(lambda: api.grad(Q, gd, bd, prec=prec, ctx=ctx)),
        }
    ctx.close()
    if not no_cpu:
        import oracle
        Qh = workloads.qubos(B, n, W["q_seed"])
        k = 16
        t0 = time.perf_counter()
        for i in range(k):
            oracle.grad(Qh[i], g[i:i + 1], b[i:i + 1])
        tc = time.perf_counter() - t0
        res["cpu_oracle"] = {"grads_per_s": k / tc, "extrapolated": True,
                             "cores": oracle.num_threads(), "kind": "oracle",
                             "sample": f"complex128 adjoint gradients of the first {k} of the "
                                       f"{B} problems, {tc:.1f} s"}
    return res


def dqaoa_leg(cycles: int, no_cpu: bool):
    """DQAOA outer cycles (Sec. V) on one dense N = 1000 QUBO with the
    paper's sub-QUBO count and size (160 windows of 20 variables, IFD
    windows with stride 1): impact factors, windows and the sub-QUBO gather,
    160 solves on the solve queue (p = 3, 100 Adam evaluations, 1024 shots,
    complex64), aggregation.  Beside it, the oracle's classical steps (full
    energy evaluations, as the paper's complexity counts them) on the host
    for the first cycle's inputs."""
    import numpy as np
    import torch

    from paper_2506_10531_amd import serve, workloads

    N, m, k, p = 1000, 160, 20, 3
    Qh = workloads.qubo(N, 3)
    x0 = np.random.default_rng(21).integers(0, 2, N).astype(np.uint8)
    g0, b0 = workloads.params(1, p, 22)
    Q = torch.as_tensor(Qh, device="cuda:0")
    x = torch.as_tensor(x0, device="cuda:0")
    rows = []
    with serve.SolveQueue(prec="c64", p=p, evals=100, shots=1024, max_slots=256) as q:
        for c in range(cycles):
            _, e, st = q.dqaoa_cycle(Q, x, g0[0], b0[0], m, k, mode="ifd", stride=1,
                                     seed=1000 * c)
            rows.append(st)
    out = {
        "workload": "dqaoa_n1000: one dense N=1000 QUBO, 160 IFD windows of 20 variables, "
                    "p=3, 100 Adam evaluations + 1024 shots per sub-QUBO, complex64",
        "cycles": rows,
        "ms_per_cycle": float(np.mean([r["decompose_ms"] + r["solve_ms"] + r["aggregate_ms"]
                                       for r in rows])),
        "solves_per_s": m / (np.mean([r["solve_ms"] for r in rows]) * 1e-3),
    }
    if not no_cpu:
        from oracle import cycle
        t0 = time.perf_counter()
        imp = cycle.impact(Qh, x0)
        ch = cycle.ifd_choices(cycle.rank(imp), m, k, 1)
        cycle.subqubos(Qh, ch)
        t1 = time.perf_counter()
        sub = np.random.default_rng(23).integers(0, 1 << k, m, dtype=np.uint64)
        cycle.aggregate(Qh, x0, ch, sub)
        t2 = time.perf_counter()
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()
                         if d.get("user_api") == "blas"] or [1])
        except Exception:  # noqa: BLE001 - the count is informational
            cores = None
        out["cpu_oracle_classical_steps"] = {
            "decompose_ms": 1e3 * (t1 - t0), "aggregate_ms": 1e3 * (t2 - t1),
            "cores": cores, "kind": "oracle",
            "sample": "impact factors by N full energy evaluations, IFD windows, sub-QUBOs; "
                      "aggregation of 160 random sub-solutions by full energy evaluations"}
    return out


def maxcut_leg(cycles: int):
    """DQAOA on a sparse Max-Cut QUBO (Sec. VI-B: N = 1000 nodes, N(N-1)/8
    random edges, sub-QUBOs of 12 variables, as many sub-QUBOs as half the
    nodes) with each decomposition: random windows, IFD, BFS and PFS; p = 1,
    30 Adam evaluations + 256 shots per sub-QUBO, complex64.  Reports the cut
    after each cycle (the paper's approximation ratio needs reference
    energies that are not available) and the cycle times."""
    import numpy as np
    import torch

    from paper_2506_10531_amd import serve, workloads

    N, k, p = 1000, 12, 1
    m = N // 2
    Qh, edges = workloads.maxcut_qubo(N, 41)
    x0 = np.random.default_rng(42).integers(0, 2, N).astype(np.uint8)
    g0, b0 = workloads.params(1, p, 43)
    Q = torch.as_tensor(Qh, device="cuda:0")
    out = {"workload": f"maxcut_n{N}: {len(edges)} edges, {m} sub-QUBOs of {k} variables, p=1, "
                       "30 Adam evaluations + 256 shots each, complex64",
           "initial_cut": int(-(x0.astype(np.float64) @ Qh @ x0))}
    rng = np.random.default_rng(44)
    with serve.SolveQueue(prec="c64", p=p, evals=30, shots=256, max_slots=512) as q:
        for mode in ("random", "ifd", "bfs", "pfs"):
            x = torch.as_tensor(x0, device="cuda:0")
            cuts, ms = [], []
            for c in range(cycles):
                ch = None
                if mode == "random":
                    ch = torch.as_tensor(np.stack([np.sort(rng.choice(N, size=k, replace=False))
                                                   for _ in range(m)]).astype(np.int32),
                                         device="cuda:0")
                _, e, st = q.dqaoa_cycle(Q, x, g0[0], b0[0], m, k,
                                         mode="given" if mode == "random" else mode,
                                         choices=ch, seed=7000 * c)
                cuts.append(int(round(-st["energy"])))
                ms.append(st["decompose_ms"] + st["solve_ms"] + st["aggregate_ms"])
            out[mode] = {"cut_per_cycle": cuts, "ms_per_cycle": float(np.mean(ms))}
    return out


def cobyla_leg(count: int):
    """The paper's variational loop (COBYLA-type steps from random
    parameters, p = 1; qaoa_cobyla batches every round of requests into one
    qaoa_expect) on `count` 20-variable sub-QUBOs of the N = 1000 QUBO,
    beside the solve queue's device Adam (100 evaluations) from the same
    initial parameters; both sampled with 1024 shots, complex64."""
    import numpy as np
    import torch

    from paper_2506_10531_amd import api, serve, workloads

    _, rs = workloads.subqubo_requests(count, N=1000, n_lo=20, n_hi=20, seed=3)
    Qs = np.stack([Q for _, Q in rs])
    g, b = workloads.params(count, 1, 24)
    th0 = np.concatenate([g, b], axis=1)
    Qd = torch.as_tensor(Qs, device="cuda:0")
    torch.cuda.synchronize()
    times = []
    for _ in range(5):  # one run takes tens of ms: the median of five
        t0 = time.perf_counter()
        r = api.cobyla(Qd, th0, rhobeg=0.5, rhoend=1e-4, maxfun=100, prec="c64")
        s = api.sample(Qd, torch.as_tensor(r["theta"][:, :1], device="cuda:0"),
                       torch.as_tensor(r["theta"][:, 1:], device="cuda:0"), 1024, 5, prec="c64")
        bc = s["best_c"].cpu().numpy()
        times.append(time.perf_counter() - t0)
    tc = float(np.median(times))
    tq = time.perf_counter()
    with serve.SolveQueue(prec="c64", p=1, evals=100, shots=1024, max_slots=count) as q:
        t0 = time.perf_counter()
        ts = [q.submit(Qs[i], g[i], b[i], 5 + i) for i in range(count)]
        res = [q.wait(t, timeout_s=300) for t in ts]
        ta = time.perf_counter() - t0
        tq = t0 - tq
    return {
        "workload": f"{count} sub-QUBOs of n=20 from the N=1000 QUBO, p=1, random initial "
                    "parameters, 1024 shots, complex64",
        "cobyla": {"solves_per_s": count / tc, "runs": len(times),
                   "min_solves_per_s": count / min(times),
                   "mean_expect": float(np.mean(r["expect"])),
                   "mean_best_c": float(np.mean(bc)),
                   "mean_evaluations": float(np.mean(r["nfev"])),
                   "batched_rounds": int(r["rounds"]), "rhoend": 1e-4, "maxfun": 100},
        "device_adam_100": {"solves_per_s": count / ta, "queue_create_s": tq,
                            "mean_expect": float(np.mean([x["expect"] for x in res])),
                            "mean_best_c": float(np.mean([x["best_c"] for x in res]))},
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only (--gpus 1); multi-GPU "
              "runs are not supported", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return

    import numpy as np
    import torch

    from paper_2506_10531_amd import api, workloads

    W = workloads.WORKLOADS["precision_n24"]
    n, p, S = W["n"], W["p"], W["sets"]
    prec = args.prec
    dev = torch.device("cuda:0")
    Q = workloads.qubo(n, W["q_seed"])
    g, b = workloads.params(S, p, W["p_seed"])
    Qd = torch.as_tensor(Q, device=dev)
    gd = torch.as_tensor(g, device=dev)
    bd = torch.as_tensor(b, device=dev)
    ctx = api.Context(0)
    plan = ctx.plan(prec, 1, n, p, S)
    el = 8 if prec == "c64" else 16
    updates_per_step = S * p * (1 << n)
    floor_bytes_per_step = updates_per_step * 2 * el  # one read + one write per layer

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        e = api.expect(Qd, gd, bd, prec=prec, ctx=ctx)
    torch.cuda.synchronize()

    ctx.profile(True)
    ctx.profile_read(reset=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        e = api.expect(Qd, gd, bd, prec=prec, ctx=ctx)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile(False)
    launches, pass_ms, pass_bytes = ctx.profile_read(reset=True)
    ev_ms = ev0.elapsed_time(ev1)

    # the timing protocol beside the contract's K steps: >= 10 calls and >= 1 s
    timing = timed_repeats(lambda: api.expect(Qd, gd, bd, prec=prec, ctx=ctx))
    ms_per_step = 1e3 * wall / args.steps
    value = updates_per_step * args.steps / wall
    avg_launch_ms = pass_ms / max(launches, 1)
    bytes_per_launch = pass_bytes / max(launches, 1)
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    # counter-derived HBM bytes per launch: taken for the complex64 register-tile pass
    traffic = load_traffic(prec)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "amplitude-layer updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "c64" else "f64",
        "precision": ("complex64 state, FP64 phase range reduction and FP64 "
                      "<C>/norm sums" if prec == "c64" else "complex128 state, FP64"),
        "data": "synthetic",
        "config": {"workload": "precision_n24: one dense n=24 QUBO, p=4, 16 "
                               "parameter sets", "n": n, "p": p, "sets": S,
                   "prec": prec, "q_seed": W["q_seed"], "p_seed": W["p_seed"]},
        "hbm_GBps": floor_bytes_per_step * args.steps / wall / 1e9,
        "event_ms_per_step": ev_ms / args.steps,
        "timing": timing,
        "host_cpu": host_cpu(),
        "paper_context": PAPER_CONTEXT,
        "plan": {"passes": plan["passes"], "sets": plan["sets"],
                 "tile_qubits": plan["tile_qubits"],
                 "state_reads": plan["state_reads"],
                 "state_writes": plan["state_writes"]},
        "roofline": {
            "kernel": ("fwd_pass_kernel<double>" if prec == "c128" and os.environ.get("DQAOA_FWD_KERNEL") == "lds" else
                       "fwd13d (complex128 register tile)" if prec == "c128" else
                       "fwd_pass_kernel<float>" if os.environ.get("DQAOA_FWD_KERNEL") == "lds"
                       else "fwd14_kernel (complex64 register tile)"),
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBPS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": avg_launch_ms,
            "launches": launches,
        },
    }

    if not args.no_extras:
        import oracle
        e_main = e.cpu().numpy()[0]
        other = "c128" if prec == "c64" else "c64"
        e_other = api.expect(Qd, gd, bd, prec=other, ctx=ctx).cpu().numpy()[0]
        # the other precision's throughput on the same workload
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read(reset=True)
        t0 = time.perf_counter()
        k2 = max(3, args.steps // 4)
        for _ in range(k2):
            api.expect(Qd, gd, bd, prec=other, ctx=ctx)
        torch.cuda.synchronize()
        w2 = time.perf_counter() - t0
        ctx.profile(False)
        l2, ms2, by2 = ctx.profile_read(reset=True)
        ach2 = (by2 / max(l2, 1)) / (ms2 / max(l2, 1) * 1e-3) / 1e9
        out[f"{other}_form"] = {"value": updates_per_step * k2 / w2,
                                "achieved_GBps": ach2, "frac": ach2 / PEAK_HBM_GBPS,
                                "ms_per_step": 1e3 * w2 / k2,
                                "traffic": load_traffic(other)}
        C = oracle.cost_table(Q)
        cmax = float(np.max(np.abs(C)))
        e64 = e_main if prec == "c64" else e_other
        e128 = e_other if prec == "c64" else e_main
        psi64, _, _ = api.state(Qd, gd[:1], bd[:1], prec="c64", ctx=ctx)
        ref = oracle.state(Q, g[0], b[0])
        l2err = float(np.linalg.norm(psi64.cpu().numpy()[0, 0].astype(np.complex128) - ref))
        del psi64
        out["errors"] = {
            "max_abs_C": cmax,
            "c64_vs_c128_expect_max_abs": float(np.max(np.abs(e64 - e128))),
            "c64_vs_c128_over_maxC": float(np.max(np.abs(e64 - e128)) / cmax),
            "c64_state_l2_vs_oracle_set0": l2err,
        }

    if not args.no_cpu_baseline:
        import oracle
        # whole oracle calls on the first k parameter sets, repeated until
        # about 10 s of host work have been timed
        k = max(1, min(S, args.cpu_sets))
        calls, tc = 0, 0.0
        while calls == 0 or (tc < 10.0 and calls < 8):
            t0 = time.perf_counter()
            eo, _, _ = oracle.expect(Q, g[:k], b[:k])
            tc += time.perf_counter() - t0
            calls += 1
        out["cpu_baseline"] = {
            "value": calls * k * p * (1 << n) / tc,
            "unit": "amplitude-layer updates/s",
            "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{calls} oracle call(s) on {k} of the {S} parameter sets of the same "
                      f"n=24, p=4 workload (cost table + {k} x {p} layers each), {tc:.1f} s",
        }
        if "errors" in out:
            ee = e_main if prec == "c64" else e_other
            out["errors"]["c64_vs_oracle_expect_max_abs"] = float(np.max(np.abs(ee[:k] - eo)))
            ec = e_other if prec == "c64" else e_main
            out["errors"]["c128_vs_oracle_expect_max_rel"] = float(
                np.max(np.abs(ec[:k] - eo) / np.maximum(np.abs(eo), 1.0)))
    legs = set(x for x in args.legs.split(",") if x)
    if "plain" in legs:
        out["plain"] = plain_leg(args.no_cpu_baseline)
    if "p1" in legs:
        out["p1_n24"] = p1_leg()
    if args.serving_requests > 0 and "serving" in legs:
        out["serving"] = serving_leg(args.serving_requests, args.serving_single,
                                     args.serving_slots,
                                     calib=min(256, args.serving_requests),
                                     no_cpu=args.no_cpu_baseline)
    if args.large_steps > 0 and "large" in legs:
        out["large_state"] = large_state_leg(args.large_steps, args.no_cpu_baseline)
    if args.dqaoa_cycles > 0 and "dqaoa" in legs:
        out["dqaoa"] = dqaoa_leg(args.dqaoa_cycles, args.no_cpu_baseline)
    if args.cobyla_subqubos > 0 and "cobyla" in legs:
        out["cobyla_p1"] = cobyla_leg(args.cobyla_subqubos)
    if args.maxcut_cycles > 0 and "maxcut" in legs:
        out["maxcut"] = maxcut_leg(args.maxcut_cycles)
    if args.grad_steps > 0 and "grad" in legs:
        out["grad"] = grad_leg(args.grad_steps, args.no_cpu_baseline)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
