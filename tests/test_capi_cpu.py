"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments before any device work, and plans the
state passes."""
import ctypes
import os
import re

import pytest

from paper_2506_10531_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dqaoa.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qaoa_[a-z_]+)\s*\(", text)))


def test_header_declares_what_binding_lists():
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.qaoa_version().startswith(b"dqaoa")


@pytest.fixture(scope="module")
def hctx():
    L = _lib.load()
    h = ctypes.c_void_p()
    assert L.qaoa_create(ctypes.byref(h), _lib.QAOA_DEVICE_NONE, 0) == _lib.OK
    yield h
    assert L.qaoa_destroy(h) == _lib.OK


def _expect(h, prec=1, B=1, n=10, p=2, S=1, Q=1, g=1, b=1, e=1):
    L = _lib.load()
    P = lambda x: ctypes.c_void_p(0x1000) if x else None  # never dereferenced
    return L.qaoa_expect(h, prec, B, n, p, S, P(Q), P(g), P(b), P(e), None, None, None)


def test_valid_call_on_host_context_reports_no_device(hctx):
    assert _expect(hctx) == _lib.ERR_NO_DEVICE
    assert b"host-only" in _lib.load().qaoa_last_error()


@pytest.mark.parametrize("kw", [
    dict(prec=2), dict(prec=-1), dict(B=0), dict(S=0), dict(n=0), dict(n=35),
    dict(p=0), dict(p=65), dict(Q=0), dict(g=0), dict(b=0), dict(e=0),
    dict(B=300, S=300),
])
def test_invalid_arguments_rejected_before_device_work(hctx, kw):
    assert _expect(hctx, **kw) == _lib.ERR_INVALID_ARG
    assert _lib.load().qaoa_last_error() != b""


def test_noalloc_validates_and_bounds_its_scratch(hctx):
    L = _lib.load()
    P = lambda x: ctypes.c_void_p(0x1000) if x else None  # never dereferenced

    def call(prec=1, B=1, n=10, p=2, S=1, e=1):
        return L.qaoa_expect_noalloc(hctx, prec, B, n, p, S, P(1), P(1), P(1), P(e), None,
                                     None, None)
    assert call() == _lib.ERR_NO_DEVICE
    assert call(n=24) == _lib.ERR_NO_DEVICE           # one 128 MiB state fits
    assert call(n=26) == _lib.ERR_OUT_OF_MEMORY       # 512 MiB does not
    assert b"fixed scratch" in L.qaoa_last_error()
    assert call(n=20, S=40) == _lib.ERR_OUT_OF_MEMORY  # 320 MiB of states
    for kw in (dict(prec=2), dict(B=0), dict(n=35), dict(p=0), dict(e=0)):
        assert call(**kw) == _lib.ERR_INVALID_ARG, kw


def test_null_context_rejected():
    assert _expect(None) == _lib.ERR_INVALID_ARG


def test_budget_overrun_is_out_of_memory():
    L = _lib.load()
    h = ctypes.c_void_p()
    assert L.qaoa_create(ctypes.byref(h), _lib.QAOA_DEVICE_NONE, 1 << 20) == _lib.OK
    try:
        # 2^24 complex64 amplitudes = 128 MiB of state: beyond a 1 MiB budget
        assert _expect(h, n=24) == _lib.ERR_OUT_OF_MEMORY
        # a single-tile state needs no state buffer: fits
        assert _expect(h, n=12) == _lib.ERR_NO_DEVICE
    finally:
        L.qaoa_destroy(h)


def test_sample_and_grad_validate(hctx):
    L = _lib.load()
    P = ctypes.c_void_p(0x1000)
    rc = L.qaoa_sample(hctx, 1, 1, 10, 2, P, P, P, 0, 0, P, None, P, P, None, None)
    assert rc == _lib.ERR_INVALID_ARG  # shots < 1
    rc = L.qaoa_sample(hctx, 1, 1, 10, 2, P, P, P, 16, 0, P, None, P, P, None, None)
    assert rc == _lib.ERR_NO_DEVICE
    rc = L.qaoa_grad(hctx, 1, 1, 10, 2, 1, P, P, P, None, None, P, None)
    assert rc == _lib.ERR_INVALID_ARG  # dgamma NULL
    rc = L.qaoa_grad(hctx, 1, 1, 10, 2, 1, P, P, P, None, P, P, None)
    assert rc == _lib.ERR_NO_DEVICE


def test_no_gpu_create_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = _lib.load()
    h = ctypes.c_void_p()
    assert L.qaoa_create(ctypes.byref(h), 0, 0) == _lib.ERR_NO_DEVICE


def _plan(h, prec, n, p, grad=0, B=1, S=1):
    info = _lib.PlanInfo()
    assert _lib.load().qaoa_plan(h, prec, B, n, p, S, grad, ctypes.byref(info)) == 0
    return info


def test_plan_two_sets_reach_the_algorithmic_floor(hctx):
    # n = 24 complex64 (14-qubit tiles, 4 contiguous low qubits): two qubit
    # sets, p + 1 passes, one read and one write of the state per layer.
    for p in (1, 2, 4, 6):
        info = _plan(hctx, 1, 24, p)
        assert (info.sets, info.passes) == (2, p + 1)
        assert (info.state_reads, info.state_writes) == (p, p)
        assert info.tile_qubits == 14 and info.chunk_qubits == 4


def test_plan_single_tile_and_three_sets(hctx):
    info = _plan(hctx, 1, 14, 3)
    assert (info.sets, info.passes, info.state_reads) == (1, 1, 0)
    info = _plan(hctx, 0, 13, 3)
    assert (info.sets, info.passes) == (1, 1)
    info = _plan(hctx, 1, 32, 2)
    assert info.sets == 3 and info.passes == 1 + 2 * 2
    # complex128 n = 24 fits two sets with 2 contiguous qubits (64-byte runs)
    info = _plan(hctx, 0, 24, 4)
    assert info.sets == 2 and info.chunk_qubits == 2


def test_plan_scratch_accounts_for_checkpoints(hctx):
    fwd = _plan(hctx, 1, 16, 6, grad=0, B=8)
    grd = _plan(hctx, 1, 16, 6, grad=1, B=8)
    state = 8 * (1 << 16) * 8
    assert fwd.scratch_bytes >= state
    # p + 1 passes: p checkpoints plus the adjoint state
    assert grd.scratch_bytes >= (6 + 1) * state


def test_package_imports_without_gpu():
    import paper_2506_10531_amd as pkg
    from paper_2506_10531_amd import api
    assert pkg.expect is api.expect and pkg.grad is api.grad
    assert pkg.workloads.qubo(3, 0).shape == (3, 3)
    h = api.host_context()
    info = h.plan("c64", 1, 24, 4)
    assert info["passes"] == 5


# ---- DQAOA outer cycle entry points ----------------------------------------

def _P(x):
    return ctypes.c_void_p(0x1000) if x else None  # never dereferenced


def test_cycle_workspace_sizes():
    L = _lib.load()
    assert L.qaoa_cycle_workspace(1000, 160, 20) >= 160 * 20 * 20 * 8 + 1000 * 12
    for args in ((0, 1, 1), (70000, 1, 1), (10, 0, 1), (10, 1, 0), (10, 1, 65)):
        assert L.qaoa_cycle_workspace(*args) == 0


@pytest.mark.parametrize("N,nulls,rc", [
    (100, (), _lib.ERR_NO_DEVICE), (0, (), _lib.ERR_INVALID_ARG),
    (70000, (), _lib.ERR_INVALID_ARG), (100, (0,), _lib.ERR_INVALID_ARG),
    (100, (1,), _lib.ERR_INVALID_ARG), (100, (2,), _lib.ERR_INVALID_ARG),
    (100, (3,), _lib.ERR_INVALID_ARG)])
def test_impact_arguments(hctx, N, nulls, rc):
    a = [_P(i not in nulls) for i in range(4)]
    assert _lib.load().qaoa_impact(hctx, N, a[0], a[1], a[2], a[3], None, None, None) == rc


@pytest.mark.parametrize("N,m,k,stride,rc", [
    (100, 10, 20, 1, _lib.ERR_NO_DEVICE), (100, 0, 20, 1, _lib.ERR_INVALID_ARG),
    (100, 10, 0, 1, _lib.ERR_INVALID_ARG), (100, 10, 65, 1, _lib.ERR_INVALID_ARG),
    (10, 10, 11, 1, _lib.ERR_INVALID_ARG), (100, 10, 20, 0, _lib.ERR_INVALID_ARG)])
def test_windows_decompose_aggregate_arguments(hctx, N, m, k, stride, rc):
    L = _lib.load()
    assert L.qaoa_ifd_choices(hctx, N, _P(1), m, k, stride, _P(1), None) == rc
    rc2 = _lib.ERR_NO_DEVICE if rc == _lib.ERR_NO_DEVICE or stride == 0 else rc
    assert L.qaoa_decompose(hctx, N, _P(1), m, k, _P(1), _P(1), None) == rc2
    assert L.qaoa_aggregate(hctx, N, _P(1), _P(1), _P(1), _P(1), m, k, _P(1), _P(1), None,
                            None) == rc2
    assert L.qaoa_decompose(hctx, N, None, m, k, _P(1), _P(1), None) == _lib.ERR_INVALID_ARG
    assert L.qaoa_aggregate(hctx, N, _P(1), _P(1), None, _P(1), m, k, _P(1), _P(1), None,
                            None) == _lib.ERR_INVALID_ARG


def test_dqaoa_cycle_arguments(hctx):
    L = _lib.load()
    st = _lib.CycleStats()

    def call(mode=_lib.QAOA_DECOMP_IFD, k=20, stride=1, ch=0, q=1, work=1):
        return L.qaoa_dqaoa_cycle(hctx, _P(q), 100, _P(1), _P(1), _P(1), _P(1), mode, 10, k,
                                  stride, _P(ch), _P(1), _P(1), 0, _P(work),
                                  ctypes.byref(st), None)
    assert call() == _lib.ERR_NO_DEVICE
    assert call(mode=5) == _lib.ERR_INVALID_ARG
    assert call(mode=_lib.QAOA_DECOMP_GIVEN) == _lib.ERR_INVALID_ARG   # no choices
    assert call(mode=_lib.QAOA_DECOMP_GIVEN, ch=1) == _lib.ERR_NO_DEVICE
    assert call(stride=0) == _lib.ERR_INVALID_ARG
    assert call(k=23) == _lib.ERR_INVALID_ARG                          # beyond the queue
    assert call(q=0) == _lib.ERR_INVALID_ARG
    assert call(work=0) == _lib.ERR_INVALID_ARG


@pytest.mark.parametrize("B,shots,alpha,ok", [
    (4, 1024, 0.25, True), (0, 10, 1.0, False), (70000, 10, 1.0, False), (1, 0, 1.0, False),
    (1, 70000, 1.0, False), (1, 10, 0.0, False), (1, 10, 1.5, False), (1, 10, float("nan"), False)])
def test_cvar_arguments(hctx, B, shots, alpha, ok):
    rc = _lib.load().qaoa_cvar(hctx, B, shots, _P(1), alpha, _P(1), None)
    assert rc == (_lib.ERR_NO_DEVICE if ok else _lib.ERR_INVALID_ARG)


def test_cobyla_arguments(hctx):
    L = _lib.load()

    def call(prec=0, B=4, n=10, p=1, rb=0.5, re=1e-6, mf=100, ptrs=(1, 1, 1, 1)):
        q, t0, t, e = (_P(v) for v in ptrs)
        return L.qaoa_cobyla(hctx, prec, B, n, p, q, t0, rb, re, mf, t, e, None, None, None,
                             None)
    assert call() == _lib.ERR_NO_DEVICE
    for kw in (dict(prec=3), dict(B=0), dict(n=0), dict(n=35), dict(p=0), dict(p=65),
               dict(rb=1e-7, re=1e-6), dict(re=0.0), dict(rb=float("inf")), dict(mf=0),
               dict(ptrs=(0, 1, 1, 1)), dict(ptrs=(1, 0, 1, 1)), dict(ptrs=(1, 1, 0, 1)),
               dict(ptrs=(1, 1, 1, 0))):
        assert call(**kw) == _lib.ERR_INVALID_ARG, kw


def test_traversal_arguments(hctx):
    L = _lib.load()

    def call(N=100, mode=_lib.QAOA_DECOMP_PFS, m=10, k=12, ptrs=(1, 1, 1, 1)):
        a = [_P(v) for v in ptrs]
        return L.qaoa_traversal_choices(hctx, N, a[0], a[1], a[2], mode, m, k, a[3], None)
    assert call() == _lib.ERR_NO_DEVICE
    assert call(mode=_lib.QAOA_DECOMP_BFS) == _lib.ERR_NO_DEVICE
    for kw in (dict(mode=_lib.QAOA_DECOMP_IFD), dict(mode=7), dict(N=20000), dict(k=0),
               dict(k=101), dict(m=0), dict(ptrs=(0, 1, 1, 1)), dict(ptrs=(1, 0, 1, 1)),
               dict(ptrs=(1, 1, 0, 1)), dict(ptrs=(1, 1, 1, 0))):
        assert call(**kw) == _lib.ERR_INVALID_ARG, kw


def test_ctypes_structs_match_the_header(tmp_path):
    """Every structure the binding passes through the C ABI has the size and
    field offsets of its typedef in include/dqaoa.h (compiled here with gcc)."""
    import shutil
    import subprocess
    from paper_2506_10531_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    pairs = [(_lib.PlanInfo, "qaoa_plan_info"), (_lib.QueueOpts, "qaoa_queue_opts"),
             (_lib.SolveReq, "qaoa_solve_req"), (_lib.SolveResult, "qaoa_solve_result"),
             (_lib.CycleStats, "qaoa_cycle_stats"), (_lib.QueueStats, "qaoa_queue_stats")]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dqaoa.h"', "int main(void) {"]
    want = []
    for cls, cname in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(cls))
        for f, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {f}));')
            want.append(getattr(cls, f).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == want
