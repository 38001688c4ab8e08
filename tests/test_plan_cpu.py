"""CPU checks of the pass planner (no GPU): every pass's tile/block split of
the n index bits is a bijection onto [0, 2^n) that fits the LDS tile, and the
concatenated pass ops apply Eq. (2) exactly: phase 1, every qubit's mixer of
layer 1 once, phase 2, ..., every qubit's mixer of layer p once."""
import ctypes

import numpy as np
import pytest

from paper_2506_10531_amd import _lib

F_INIT, F_WRITE, F_REDUCE = 1, 2, 4


@pytest.fixture(scope="module")
def hctx():
    L = _lib.load()
    h = ctypes.c_void_p()
    assert L.qaoa_create(ctypes.byref(h), _lib.QAOA_DEVICE_NONE, 0) == 0
    yield h
    L.qaoa_destroy(h)


def passes(h, prec, n, p, grad):
    buf = (ctypes.c_int * (10 * 400))()
    np_ = ctypes.c_int()
    rc = _lib.load().qaoa_plan_passes(h, prec, n, p, grad, buf, 400, ctypes.byref(np_))
    assert rc == 0, _lib.load().qaoa_last_error()
    a = np.array(buf[: 10 * np_.value]).reshape(-1, 10)
    keys = ["set", "k", "c", "a", "mixlo", "lead", "ja", "jb", "flags", "kind"]
    return [dict(zip(keys, map(int, r))) for r in a]


def tile_bits(d, n):
    if d["c"] >= d["k"]:
        return list(range(d["k"]))
    return list(range(d["c"])) + list(range(d["a"], d["a"] + d["k"] - d["c"]))


def mixed_qubits(d, n):
    return tile_bits(d, n)[d["mixlo"]:]


CASES = [(prec, n, p, g) for prec in (0, 1) for g in (0, 1)
         for n in list(range(1, 35)) for p in (1, 2, 3, 5)]


@pytest.mark.parametrize("prec,n,p,grad", CASES)
def test_plan_geometry_and_semantics(hctx, prec, n, p, grad):
    kmax = (13 if prec == 0 else 14) - (1 if grad else 0)
    reg14 = prec == 1 and not grad and n >= 15
    reg13 = prec == 1 and grad and 14 <= n <= 22
    reg13d = prec == 0 and not grad and n >= 14
    reg12 = prec == 0 and grad and 13 <= n <= 22
    ps = passes(hctx, prec, n, p, grad)
    if reg13d:
        # 13-qubit complex128 tiles, 2 contiguous low bits in the other sets:
        # two sets (p + 1 passes) up to n = 24
        assert len(ps) == (p + 1 if n <= 24 else 2 * p + 1)
    for i, d in enumerate(ps):
        assert 1 <= d["k"] <= min(kmax, n)
        assert (d["kind"] != 0) == (reg14 or reg13 or reg13d or reg12)
        if reg14 or reg13 or reg13d or reg12:
            assert d["k"] == (14 if reg14 else 12 if reg12 else 13)
            assert d["kind"] == (1 if d["set"] == 0 else 2)
            # complex64 forward and gradient: each kind-2 set has min(MIXLO, 8)
            # contiguous low bits (its run of high bits holds exactly its qubits)
            assert d["c"] == (d["k"] if d["set"] == 0 else (2 if (reg13d or reg12) else
                                                            min(d["mixlo"], 8)))
        tb = tile_bits(d, n)
        assert len(tb) == d["k"] and len(set(tb)) == d["k"]
        assert all(0 <= b < n for b in tb)
        assert tb[: min(d["c"], d["k"])] == list(range(min(d["c"], d["k"])))
        assert 0 <= d["mixlo"] < d["k"]
        flags = d["flags"]
        assert bool(flags & F_INIT) == (i == 0)
        assert bool(flags & F_WRITE) == (i < len(ps) - 1)
        assert bool(flags & F_REDUCE) == (i == len(ps) - 1)
    # the ops in sequence
    events = []
    for d in ps:
        mq = mixed_qubits(d, n)
        if d["lead"] >= 0:
            events += [("M", d["lead"], q) for q in mq]
        for j in range(d["ja"], d["jb"] + 1):
            events.append(("P", j))
            events += [("M", j, q) for q in mq]
    ref_layers = []
    cur = None
    for ev in events:
        if ev[0] == "P":
            assert ev[1] == len(ref_layers), "phases out of order"
            cur = set()
            ref_layers.append(cur)
        else:
            assert cur is not None, "mixer before the first phase"
            assert ev[1] == len(ref_layers) - 1, "mixer of the wrong layer"
            assert ev[2] not in cur, "qubit mixed twice in one layer"
            cur.add(ev[2])
    assert len(ref_layers) == p
    for layer in ref_layers:
        assert layer == set(range(n))


def dep_local(l, d):
    if d["c"] >= d["k"]:
        return l
    return (l & ((1 << d["c"]) - 1)) | ((l >> d["c"]) << d["a"])


def dep_block(b, d):
    if d["c"] >= d["k"]:
        return b << d["k"]
    gap = d["a"] - d["c"]
    lo = b & ((1 << gap) - 1)
    hi = b >> gap
    return (lo << d["c"]) | (hi << (d["a"] + d["k"] - d["c"]))


@pytest.mark.parametrize("prec,n,grad", [(pr, n, g) for pr in (0, 1) for g in (0, 1)
                                         for n in (1, 5, 13, 14, 15, 16, 17, 19, 22)])
def test_tile_indexing_is_a_bijection(hctx, prec, n, grad):
    """The kernels address amplitude dep_block(tile) | dep_local(l): over all
    tiles and l it must hit every index of the 2^n state exactly once."""
    for d in passes(hctx, prec, n, 3, grad):
        k = d["k"]
        L = np.array([dep_local(l, d) for l in range(1 << k)], dtype=np.int64)
        Bz = np.array([dep_block(b, d) for b in range(1 << (n - k))], dtype=np.int64)
        assert not (L[:, None] & Bz[None, :]).any()
        idx = (L[:, None] | Bz[None, :]).ravel()
        assert idx.min() == 0 and idx.max() == (1 << n) - 1
        assert np.unique(idx).size == 1 << n


@pytest.mark.parametrize("n", [24, 28, 32, 34])
def test_large_state_bit_partition(hctx, n):
    for prec in (0, 1):
        for d in passes(hctx, prec, n, 2, 0):
            tb = set(tile_bits(d, n))
            blk = set(range(n)) - tb
            mask_b = sum(1 << b for b in blk)
            # block index deposits exactly onto the block bits, in order
            nb = n - d["k"]
            assert dep_block((1 << nb) - 1, d) == mask_b
            for i, b in enumerate(sorted(blk)):
                assert dep_block(1 << i, d) == 1 << b
            assert dep_local((1 << d["k"]) - 1, d) == sum(1 << b for b in tb)


@pytest.mark.parametrize("prec,grad", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_table_jobs_fit_at_max_layers(hctx, prec, grad):
    """One tables launch serves a register-tile call: one job per forward pass,
    a checkpoint and an adjoint job per gradient pass but the last.  At
    QAOA_MAX_P = 64 layers every plan's list fits the 193 jobs the library
    holds."""
    for n in range(1, 35):
        ps = passes(hctx, prec, n, 64, grad)
        if ps[0]["kind"] == 0:
            continue
        jobs = 2 * len(ps) - 1 if grad else len(ps)
        assert jobs <= 193, (n, jobs)
