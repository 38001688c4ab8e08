"""Exercises every host-side path of a libdqaoa build on a host-only context
(no GPU): the pass planner and scratch layouts over the whole (precision, n,
p, B, S, gradient) range, the pass-record export, and the argument checks of
every entry point, including the ones that reject sizes.  Run by
tests/test_sanitize_cpu.py under AddressSanitizer and UndefinedBehavior-
Sanitizer against a build whose host code carries them; any report aborts
the process.  Usage: python sanitize_driver.py <path to the .so>"""
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2506_10531_amd import _lib  # noqa: E402

L = _lib.load(sys.argv[1])
calls = 0
codes = set()


def call(fn, *args):
    global calls
    rc = getattr(L, fn)(*args)
    calls += 1
    codes.add(rc)
    L.qaoa_last_error()
    return rc


buf = (ctypes.c_double * 4096)()
ibuf = (ctypes.c_int * 4096)()
P = ctypes.cast(buf, ctypes.c_void_p)  # host memory; a host-only context reads none of it
IP = ctypes.cast(ibuf, ctypes.c_void_p)
h = ctypes.c_void_p()
assert call("qaoa_create", ctypes.byref(h), _lib.QAOA_DEVICE_NONE, 0) == _lib.OK
hb = ctypes.c_void_p()
assert call("qaoa_create", ctypes.byref(hb), _lib.QAOA_DEVICE_NONE, 1 << 20) == _lib.OK
assert call("qaoa_create", None, _lib.QAOA_DEVICE_NONE, 0) == _lib.ERR_INVALID_ARG

# planner and layouts
info = _lib.PlanInfo()
npass = ctypes.c_int()
for prec in (_lib.QAOA_C128, _lib.QAOA_C64):
    for n in range(0, 36):
        for p in (0, 1, 2, 3, 4, 6, 7, 33, 64, 65):
            for grad in (0, 1):
                for B, S in ((1, 1), (3, 5), (512, 1), (256, 256), (0, 1)):
                    call("qaoa_plan", h, prec, B, n, p, S, grad, ctypes.byref(info))
                for mp in (0, 1, 3, 256):
                    # exactly the records the call may write: an overrun hits a redzone
                    out = (ctypes.c_int * (10 * mp))() if mp else None
                    call("qaoa_plan_passes", h, prec, n, p, grad,
                         ctypes.cast(out, ctypes.c_void_p) if mp else None, mp,
                         ctypes.byref(npass))
for ctx in (h, hb):
    for prec in (0, 1, 2):
        for n in (1, 5, 13, 14, 15, 22, 24, 26, 30, 34, 35):
            for p in (1, 4, 64):
                call("qaoa_expect", ctx, prec, 2, n, p, 3, P, P, P, P, P, P, None)
                call("qaoa_expect_noalloc", ctx, prec, 2, n, p, 3, P, P, P, P, None, None, None)
                call("qaoa_state", ctx, prec, 1, n, p, 2, P, P, P, P, None, None, None)
                call("qaoa_sample", ctx, prec, 2, n, p, P, P, P, 1024, 7, P, P, P, P, P, None)
                call("qaoa_grad", ctx, prec, 2, n, p, 2, P, P, P, P, P, P, None)
# null pointers and bad sizes on every compute entry
call("qaoa_expect", h, 1, 1, 10, 2, 1, None, P, P, P, None, None, None)
call("qaoa_sample", h, 1, 1, 10, 2, P, P, P, 0, 7, P, P, P, P, P, None)
call("qaoa_grad", h, 1, 1, 10, 2, 1, P, P, P, P, None, P, None)
call("qaoa_cobyla", h, 0, 4, 10, 1, P, P, 0.5, 1e-6, 100, P, P, None, None, None, None)
call("qaoa_cobyla", h, 0, 4, 10, 1, P, P, 1e-7, 1e-6, 100, P, P, None, None, None, None)
call("qaoa_cvar", h, 4, 1024, P, 0.25, P, None)
call("qaoa_cvar", h, 70000, 10, P, 1.0, P, None)
for N, m, k in ((1000, 160, 20), (16384, 500, 12), (65537, 1, 1), (10, 5, 0), (100, 10, 65)):
    call("qaoa_impact", h, N, P, P, P, P, IP, P, None)
    call("qaoa_ifd_choices", h, N, IP, m, k, 1, IP, None)
    for mode in (_lib.QAOA_DECOMP_BFS, _lib.QAOA_DECOMP_PFS, 9):
        call("qaoa_traversal_choices", h, N, P, P, IP, mode, m, k, IP, None)
    call("qaoa_decompose", h, N, P, m, k, IP, P, None)
    call("qaoa_aggregate", h, N, P, P, P, P, m, k, IP, P, IP, None)
    L.qaoa_cycle_workspace(N, m, k)
# solve queue: options checked, then no device
opts = _lib.QueueOpts(max_slots=8, max_pending=16, hbm_budget=0, prec=_lib.QAOA_C64, p=3,
                      evals=10, shots=64, lr=0.05, beta1=0.9, beta2=0.999, eps=1e-8, batched=1)
q = ctypes.c_void_p()
call("qaoa_queue_create", h, ctypes.byref(opts), ctypes.byref(q))
for field, bad in (("max_slots", 0), ("p", 0), ("shots", 0), ("lr", 0.0), ("prec", 7)):
    o2 = _lib.QueueOpts.from_buffer_copy(opts)
    setattr(o2, field, bad)
    call("qaoa_queue_create", h, ctypes.byref(o2), ctypes.byref(q))
call("qaoa_submit", None, None, None)
call("qaoa_queue_destroy", None)
for ctx in (h, hb):
    assert call("qaoa_destroy", ctx) == _lib.OK
call("qaoa_destroy", None)
print(f"ok {calls} calls, return codes {sorted(codes)}")
