"""ctypes declarations of the C ABI in include/dqaoa.h (argument marshalling
only: every step of the state-vector path runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libdqaoa.so")

QAOA_C128 = 0
QAOA_C64 = 1
QAOA_MAX_N = 34
QAOA_MAX_P = 64
QAOA_DEVICE_NONE = -1

OK = 0
PENDING = 1
ERR_INVALID_ARG = -1
ERR_NO_DEVICE = -2
ERR_OUT_OF_MEMORY = -3
ERR_UNSUPPORTED = -4
ERR_HIP = -5
ERR_QUEUE_FULL = -6
ERR_CANCELLED = -7
ERR_TIMEOUT = -8
ERR_NOT_FOUND = -9

ERROR_NAMES = {
    ERR_INVALID_ARG: "QAOA_ERR_INVALID_ARG", ERR_NO_DEVICE: "QAOA_ERR_NO_DEVICE",
    ERR_OUT_OF_MEMORY: "QAOA_ERR_OUT_OF_MEMORY", ERR_UNSUPPORTED: "QAOA_ERR_UNSUPPORTED",
    ERR_HIP: "QAOA_ERR_HIP", ERR_QUEUE_FULL: "QAOA_ERR_QUEUE_FULL",
    ERR_CANCELLED: "QAOA_ERR_CANCELLED", ERR_TIMEOUT: "QAOA_ERR_TIMEOUT",
    ERR_NOT_FOUND: "QAOA_ERR_NOT_FOUND",
}

# Every symbol include/dqaoa.h declares.
EXPORTS = [
    "qaoa_last_error", "qaoa_version", "qaoa_create", "qaoa_destroy",
    "qaoa_expect", "qaoa_expect_noalloc", "qaoa_state", "qaoa_sample", "qaoa_grad", "qaoa_plan", "qaoa_plan_passes",
    "qaoa_profile_enable", "qaoa_profile_read", "qaoa_queue_create",
    "qaoa_queue_destroy", "qaoa_submit", "qaoa_poll", "qaoa_wait",
    "qaoa_cancel", "qaoa_queue_get_stats",
    "qaoa_impact", "qaoa_ifd_choices", "qaoa_decompose", "qaoa_aggregate",
    "qaoa_cycle_workspace", "qaoa_dqaoa_cycle", "qaoa_cvar", "qaoa_cobyla",
    "qaoa_traversal_choices",
]

QAOA_DECOMP_GIVEN = 0
QAOA_DECOMP_IFD = 1
QAOA_DECOMP_BFS = 2
QAOA_DECOMP_PFS = 3


class QaoaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class PlanInfo(ctypes.Structure):
    _fields_ = [("sets", ctypes.c_int), ("passes", ctypes.c_int),
                ("state_reads", ctypes.c_int), ("state_writes", ctypes.c_int),
                ("tile_qubits", ctypes.c_int), ("chunk_qubits", ctypes.c_int),
                ("scratch_bytes", ctypes.c_size_t)]


class QueueOpts(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int), ("max_pending", ctypes.c_int),
                ("hbm_budget", ctypes.c_size_t), ("prec", ctypes.c_int),
                ("p", ctypes.c_int), ("evals", ctypes.c_int),
                ("shots", ctypes.c_int), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("batched", ctypes.c_int)]


class SolveReq(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("Q", ctypes.POINTER(ctypes.c_double)),
                ("gamma0", ctypes.POINTER(ctypes.c_double)),
                ("beta0", ctypes.POINTER(ctypes.c_double)),
                ("seed", ctypes.c_uint64)]


class SolveResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n", ctypes.c_int),
                ("gamma", ctypes.c_double * QAOA_MAX_P),
                ("beta", ctypes.c_double * QAOA_MAX_P),
                ("expect", ctypes.c_double), ("best_z", ctypes.c_uint64),
                ("best_c", ctypes.c_double), ("t_submit_ns", ctypes.c_int64),
                ("t_admit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


class CycleStats(ctypes.Structure):
    _fields_ = [("decompose_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("aggregate_ms", ctypes.c_double), ("accepted", ctypes.c_int),
                ("energy", ctypes.c_double)]


class QueueStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("admitted", ctypes.c_longlong),
                ("completed", ctypes.c_longlong), ("cancelled", ctypes.c_longlong),
                ("rejected", ctypes.c_longlong), ("steps", ctypes.c_longlong),
                ("pending", ctypes.c_int), ("active", ctypes.c_int),
                ("bytes_in_use", ctypes.c_size_t), ("peak_active", ctypes.c_int),
                ("peak_bytes", ctypes.c_size_t)]


_lib = None


def load(path: str | None = None):
    """Loads the in-tree libdqaoa.so; raises if it has not been built (there
    is no fallback path).  ``path`` loads another build of the same sources
    instead (e.g. one with host-side sanitizers), uncached."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    so = path or SO
    if not os.path.exists(so):
        raise RuntimeError(
            f"{so} is missing: build the HIP library first "
            "(python -m paper_2506_10531_amd.build)")
    L = ctypes.CDLL(so)
    vp, i, u64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t
    dp = ctypes.c_void_p
    L.qaoa_last_error.restype = ctypes.c_char_p
    L.qaoa_version.restype = ctypes.c_char_p
    L.qaoa_create.argtypes = [ctypes.POINTER(vp), i, sz]
    L.qaoa_destroy.argtypes = [vp]
    L.qaoa_expect.argtypes = [vp, i, i, i, i, i, dp, dp, dp, dp, dp, dp, vp]
    L.qaoa_expect_noalloc.argtypes = [vp, i, i, i, i, i, dp, dp, dp, dp, dp, dp, vp]
    L.qaoa_state.argtypes = [vp, i, i, i, i, i, dp, dp, dp, dp, dp, dp, vp]
    L.qaoa_sample.argtypes = [vp, i, i, i, i, dp, dp, dp, i, u64, dp, dp, dp,
                              dp, dp, vp]
    L.qaoa_grad.argtypes = [vp, i, i, i, i, i, dp, dp, dp, dp, dp, dp, vp]
    L.qaoa_plan.argtypes = [vp, i, i, i, i, i, i, ctypes.POINTER(PlanInfo)]
    L.qaoa_plan_passes.argtypes = [vp, i, i, i, i, vp, i, ctypes.POINTER(i)]
    L.qaoa_profile_enable.argtypes = [vp, i]
    L.qaoa_profile_read.argtypes = [vp, i, ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
    L.qaoa_queue_create.argtypes = [vp, ctypes.POINTER(QueueOpts), ctypes.POINTER(vp)]
    L.qaoa_queue_destroy.argtypes = [vp]
    L.qaoa_submit.argtypes = [vp, ctypes.POINTER(SolveReq), ctypes.POINTER(u64)]
    L.qaoa_poll.argtypes = [vp, u64, ctypes.POINTER(SolveResult), vp]
    L.qaoa_wait.argtypes = [vp, u64, ctypes.c_int64, ctypes.POINTER(SolveResult), vp]
    L.qaoa_cancel.argtypes = [vp, u64]
    L.qaoa_queue_get_stats.argtypes = [vp, ctypes.POINTER(QueueStats)]
    L.qaoa_impact.argtypes = [vp, i, dp, dp, dp, dp, dp, dp, vp]
    L.qaoa_ifd_choices.argtypes = [vp, i, dp, i, i, i, dp, vp]
    L.qaoa_traversal_choices.argtypes = [vp, i, dp, dp, dp, i, i, i, dp, vp]
    L.qaoa_decompose.argtypes = [vp, i, dp, i, i, dp, dp, vp]
    L.qaoa_aggregate.argtypes = [vp, i, dp, dp, dp, dp, i, i, dp, dp, dp, vp]
    L.qaoa_cycle_workspace.argtypes = [i, i, i]
    L.qaoa_cvar.argtypes = [vp, i, i, dp, ctypes.c_double, dp, vp]
    L.qaoa_cobyla.argtypes = [vp, i, i, i, i, dp, dp, ctypes.c_double, ctypes.c_double, i,
                              dp, dp, dp, dp, dp, vp]
    L.qaoa_dqaoa_cycle.argtypes = [vp, vp, i, dp, dp, dp, dp, i, i, i, i, dp, dp, dp,
                                   u64, dp, ctypes.POINTER(CycleStats), vp]
    for name in EXPORTS:
        if name not in ("qaoa_last_error", "qaoa_version"):
            getattr(L, name).restype = ctypes.c_int
    L.qaoa_cycle_workspace.restype = sz
    if path is None:
        _lib = L
    return L


def check(rc: int, allow=(OK,)) -> int:
    if rc in allow:
        return rc
    msg = load().qaoa_last_error().decode(errors="replace")
    raise QaoaError(rc, msg)
