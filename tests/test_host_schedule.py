"""CPU checks of the host logic behind the GPU kernels (no GPU needed).

* The persistent factorization kernel takes tasks in ticket order; the host
  replay checks that every ticket decodes to a distinct tile, that every flag
  a task waits on belongs to a task with a smaller ticket (no deadlock
  whatever the number of resident workgroups), and that every operand tile
  lies inside its array.
* The selected inversion is a sequence of launches; its dry run records every
  window each launch would read or write and checks it against array bounds.
"""
import ctypes

import numpy as np
import itertools

import pytest

from paper_2503_17528_amd import bta


@pytest.fixture(scope="module")
def L():
    lib = ctypes.CDLL(bta.LIB_PATH)
    lib.bta_internal_factor_schedule_check.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_void_p]
    lib.bta_internal_selinv_dry_check.argtypes = [ctypes.c_int64] * 3
    return lib


SHAPES = list(itertools.product([1, 2, 3, 7], [1, 5, 63, 64, 65, 130, 200], [0, 1, 4, 64, 65, 130]))


@pytest.mark.parametrize("n,b,a", SHAPES)
def test_factor_schedule_is_topological_and_in_bounds(L, n, b, a):
    counts = (ctypes.c_longlong * 7)()
    assert L.bta_internal_factor_schedule_check(n, b, a, counts) == 0
    T, TA = (b + 63) // 64, (a + 63) // 64
    assert sum(counts) == n * T * (T + 1) // 2 + (n - 1) * T * T + n * T * TA + n * TA * (TA + 1) // 2 + TA * (TA + 1) // 2


@pytest.mark.parametrize("n,b,a", [(128, 2048, 8), (256, 512, 4), (16, 64, 4), (96, 384, 6), (512, 1024, 256), (3, 128, 256)])
def test_factor_schedule_workload_sizes(L, n, b, a):
    assert L.bta_internal_factor_schedule_check(n, b, a, None) == 0


@pytest.mark.parametrize("n,b,a", SHAPES + [(128, 2048, 8), (256, 4096, 16), (256, 512, 4), (33, 384, 6), (512, 1024, 256), (3, 128, 257)])
def test_selinv_launch_windows_in_bounds(L, n, b, a):
    assert L.bta_internal_selinv_dry_check(n, b, a) == 0


def test_batched_factor_interleaving(L):
    """The batch's band-column ticket order: every ticket maps to its matrix in
    local order, every segment holds one band column, and a replay with every
    matrix's dependencies stays within the launch's bound on forward waits."""
    from paper_2503_17528_amd import synth

    L.bta_internal_factor_batch_check.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 3 + [ctypes.c_int, ctypes.c_void_p]
    arr = lambda xs: (ctypes.c_int64 * len(xs))(*xs)
    ahead = ctypes.c_longlong(-1)
    for seed in range(3):
        wls = synth.batched_workloads(seed)
        n = arr([w.n for w in wls]); b = arr([w.b for w in wls]); a = arr([w.a for w in wls])
        for cus in (256, 64, 8):
            assert L.bta_internal_factor_batch_check(len(wls), n, b, a, cus, ctypes.byref(ahead)) == 0, (seed, cus)
            assert 0 <= ahead.value < cus
    mixed = [(1, 5, 0), (3, 64, 2), (2, 130, 70), (5, 1, 1), (4, 200, 0), (6, 520, 3), (2, 600, 130)]
    for cus in (256, 32, 4, 2):
        assert L.bta_internal_factor_batch_check(len(mixed), arr([m[0] for m in mixed]), arr([m[1] for m in mixed]),
                                                 arr([m[2] for m in mixed]), cus, ctypes.byref(ahead)) == 0, cus
    # one matrix with lookahead: its DIAG tasks do wait ahead
    assert L.bta_internal_factor_batch_check(1, arr([8]), arr([1024]), arr([8]), 256, ctypes.byref(ahead)) == 0
    assert ahead.value > 0
    # no lookahead (many matrices per workgroup): nothing waits ahead
    assert L.bta_internal_factor_batch_check(1, arr([8]), arr([1024]), arr([8]), 1, ctypes.byref(ahead)) == 0
    assert ahead.value == 0


def test_batched_selinv_merge_is_independent(L):
    """Operations merged into one batched launch never write memory that
    another operation of the same launch reads or writes, and in the replayed
    graph no backward-sweep stage shares a written element with a
    preprocessing stage it is not ordered after (out of place and in place)."""
    from paper_2503_17528_amd import synth

    L.bta_internal_selinv_batch_check.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 3
    arr = lambda xs: (ctypes.c_int64 * len(xs))(*xs)
    for wls in (synth.batched_workloads(0)[:16], [synth.workload(*s) for s in [(1, 5, 0), (3, 64, 2), (2, 130, 70),
                                                                             (5, 40, 1), (4, 200, 0)]]):
        n, b, a = arr([w.n for w in wls]), arr([w.b for w in wls]), arr([w.a for w in wls])
        assert L.bta_internal_selinv_batch_check(len(wls), n, b, a) == 0
    # random batches of mixed lengths (each sweep spread over the longest one's steps)
    rng = np.random.default_rng(17)
    for _ in range(20):
        cnt = int(rng.integers(1, 13))
        n = [int(v) for v in rng.integers(1, 41, cnt)]
        b = [int(v) for v in rng.choice([5, 64, 130, 200], cnt)]
        a = [int(v) for v in rng.choice([0, 1, 4, 70], cnt)]
        assert L.bta_internal_selinv_batch_check(cnt, arr(n), arr(b), arr(a)) == 0, (n, b, a)


@pytest.mark.parametrize("look", [1, 4, 12, 16, 32])
def test_factor_schedule_other_lookaheads(L, look):
    """The schedule invariants hold for every DIAG lookahead the internal
    override can set (the ahead bound scales with it)."""
    L.bta_internal_factor_lookahead.argtypes = [ctypes.c_int]
    L.bta_internal_factor_lookahead.restype = ctypes.c_int
    prev = L.bta_internal_factor_lookahead(look)
    try:
        for n, b, a in [(3, 64 * 20 + 5, 3), (2, 64 * 40, 70), (4, 200, 0), (1, 64 * 33, 8)]:
            assert L.bta_internal_factor_schedule_check(n, b, a, None) == 0, (look, n, b, a)
    finally:
        L.bta_internal_factor_lookahead(prev)


def test_batched_factor_interleaving_random_batches(L):
    """Random batches (ragged tiles, T = 1, a = 0, arrow tips wider than the
    blocks) on several grids: the replayed forward waits never exceed the
    launch's bound, which stays below the number of workgroups."""
    import random

    L.bta_internal_factor_batch_check.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 3 + [ctypes.c_int, ctypes.c_void_p]
    arr = lambda xs: (ctypes.c_int64 * len(xs))(*xs)
    ahead = ctypes.c_longlong(-1)
    rng = random.Random(1)
    for _ in range(60):
        cnt = rng.randint(1, 40)
        ms = [(rng.randint(1, 12), rng.choice([1, 5, 64, 65, 128, 200, 300, 520, 700]), rng.choice([0, 1, 4, 64, 70, 130]))
              for _ in range(cnt)]
        cus = rng.choice([2, 4, 16, 64, 256])
        rc = L.bta_internal_factor_batch_check(cnt, arr([m[0] for m in ms]), arr([m[1] for m in ms]),
                                               arr([m[2] for m in ms]), cus, ctypes.byref(ahead))
        assert rc == 0, (rc, cus, ms)


@pytest.mark.parametrize("delay", [1, 2, 5, 64])
def test_factor_schedule_sub_delays(L, delay, monkeypatch):
    """The schedule invariants hold when the SUB tasks are dispatched `delay`
    columns after their own (BTA_FACTOR_SUB_DELAY; capped at the column count,
    the tail of a step then holds the SUB tasks of its last columns)."""
    monkeypatch.setenv("BTA_FACTOR_SUB_DELAY", str(delay))
    for n, b, a in [(3, 64 * 20 + 5, 3), (2, 64 * 40, 70), (4, 200, 0), (1, 64 * 33, 8), (5, 130, 65), (3, 64, 4)]:
        counts = (ctypes.c_longlong * 7)()
        assert L.bta_internal_factor_schedule_check(n, b, a, counts) == 0, (delay, n, b, a)
        T, TA = (b + 63) // 64, (a + 63) // 64
        assert sum(counts) == n * T * (T + 1) // 2 + (n - 1) * T * T + n * T * TA + n * TA * (TA + 1) // 2 + TA * (TA + 1) // 2
