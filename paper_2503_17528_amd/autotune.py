"""Autotuner of the factorization's and the selected inversion's tunables,
and access to the library's tuning table.

The library keeps its tuned decisions in a table keyed by
``<arch>|<op>|b=<b>|a=<a>|<knob>`` (``tune.hip``):

- the factorization's DIAG lookahead (``look``: how many band columns ahead of
  the diagonal-tile chain a diagonal task starts its accumulation);
- its SUB dispatch delay (``sub_delay``: how many band columns after their own
  the tasks of the coupling block's tiles are dispatched);
- its k-loop load path (``cached``: 1 reads published operand tiles through
  the L2);
- the largest split count of the selected inversion's sweep products at
  small b (op ``selinv``, knob ``split``);
- the batched selected inversion's tile shape per merged stage class
  (``tile128``, measured by the library itself on first use).

``BTA_TUNE_CACHE=<file.json>`` makes the library load the table from that file
on first use and write measured entries back; ``BTA_FACTOR_LOOKAHEAD``,
``BTA_FACTOR_CACHED``, ``BTA_FACTOR_SUB_DELAY`` and ``BTA_SELINV_SPLIT``
override the table for every shape.  The batched entry points take fixed
settings with measurement overrides: ``BTA_BATCH_ORDER`` (0 dispatches the
matrices' band columns in lockstep, 1 -- the default -- in proportion to each
chain's length), ``BTA_BATCH_LOOKAHEAD`` and ``BTA_BATCH_SUB_DELAY`` for the
batched factorization; ``BTA_BATCH_SPREAD=0`` (align every matrix's backward
sweep with the longest one's first steps instead of spreading it over them)
and ``BTA_BATCH_SKINNY=0`` (arrow rows through the 64 x 64 tile kernel) for
the batched selected inversion.

``tune_factor`` and ``tune_selinv_split`` time candidate settings on a seeded
synthetic matrix of the given block shape (the median of ``reps`` runs each,
HIP events on the current stream) and record the fastest in the table.
Command line::

    python -m paper_2503_17528_amd.autotune --n 32 --b 2048 --a 8 --out tune.json
"""
from __future__ import annotations

import argparse
import ctypes
import json
import statistics
import sys
from typing import Dict, Iterable, Optional

from . import bta, synth


def _lib():
    L = bta.lib()
    L.bta_internal_tune_set.argtypes = [ctypes.c_char_p, ctypes.c_longlong]
    L.bta_internal_tune_set.restype = ctypes.c_int
    L.bta_internal_tune_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_longlong)]
    L.bta_internal_tune_get.restype = ctypes.c_int
    L.bta_internal_tune_key.argtypes = [ctypes.c_char_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_char_p,
                                        ctypes.c_char_p, ctypes.c_int]
    L.bta_internal_tune_key.restype = ctypes.c_int
    L.bta_internal_tune_save.argtypes = [ctypes.c_char_p]
    L.bta_internal_tune_save.restype = ctypes.c_int
    L.bta_internal_tune_load.argtypes = [ctypes.c_char_p]
    L.bta_internal_tune_load.restype = ctypes.c_int
    L.bta_internal_tune_clear.argtypes = []
    L.bta_internal_tune_clear.restype = ctypes.c_int
    L.bta_internal_autotune_dump.argtypes = [ctypes.c_char_p, ctypes.c_int]
    L.bta_internal_autotune_dump.restype = ctypes.c_int
    L.bta_internal_factor_lookahead.argtypes = [ctypes.c_int]
    L.bta_internal_factor_lookahead.restype = ctypes.c_int
    L.bta_internal_factor_cached_loads.argtypes = [ctypes.c_int]
    L.bta_internal_factor_cached_loads.restype = ctypes.c_int
    return L


def key(op: str, b: int, a: int, knob: str) -> str:
    buf = ctypes.create_string_buffer(256)
    if _lib().bta_internal_tune_key(op.encode(), b, a, knob.encode(), buf, 256) != 0:
        raise ValueError("tuning key too long")
    return buf.value.decode()


def set_entry(k: str, value: int) -> None:
    if _lib().bta_internal_tune_set(k.encode(), int(value)) != 0:
        raise ValueError(f"invalid tuning key {k!r}")


def get_entry(k: str) -> Optional[int]:
    v = ctypes.c_longlong(0)
    return int(v.value) if _lib().bta_internal_tune_get(k.encode(), ctypes.byref(v)) == 0 else None


def table() -> Dict[str, int]:
    buf = ctypes.create_string_buffer(1 << 20)
    _lib().bta_internal_autotune_dump(buf, len(buf))
    out = {}
    for line in buf.value.decode().splitlines():
        k, _, v = line.rpartition("=")
        out[k] = int(v)
    return out


def save(path: str) -> None:
    if _lib().bta_internal_tune_save(path.encode()) != 0:
        raise OSError(f"could not write {path}")


def load(path: str) -> None:
    if _lib().bta_internal_tune_load(path.encode()) != 0:
        raise OSError(f"could not read a tuning table from {path}")


def clear() -> None:
    _lib().bta_internal_tune_clear()


def tune_factor(n: int, b: int, a: int, looks: Iterable[int] = (2, 4, 6, 8, 12, 16), cached: Iterable[int] = (0, 1),
                reps: int = 3, seed: int = 0, log=None, sub_delays: Iterable[int] = (0, 2, 4, 8, 16)) -> Dict[str, float]:
    """Time bta_factor on a seeded n x (b, a) matrix for every (lookahead,
    load path) candidate, the median of ``reps`` runs each, and record the
    fastest as the table's ``look`` and ``cached`` entries for (b, a); then,
    with those, every SUB dispatch delay (``sub_delay``: columns by which the
    tasks of the coupling block's tiles follow their own column), recording
    the fastest.  ``BTA_FACTOR_SUB_DELAY``, when set, overrides the table.
    Returns {"look=<L>,cached=<c>": median ms, "sub_delay=<d>": median ms}."""
    import torch

    if reps < 3:
        raise ValueError("reps >= 3 (the median of at least three runs)")
    L = _lib()
    reading = "scaled" if b >= 2048 else "literal"
    wl = synth.workload(n, b, a, reading)
    dev = torch.device("cuda", torch.cuda.current_device())
    Q = synth.make_torch(wl, seed, dev)
    out = tuple(torch.empty_like(Q[k]) for k in "DBRT")
    work, _ = bta.workspace(bta.BTA_OP_FACTOR, n, b, a, dev)
    T = (b + 63) // 64

    def median_ms() -> float:
        ms = []
        for _ in range(reps + 1):  # the first run warms up
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            info = bta.factor(Q["D"], Q["B"], Q["R"], Q["T"], out=out, work=work, check=False)[4]
            e1.record()
            torch.cuda.synchronize()
            if int(info.item()) != 0:
                raise bta.BTAError(bta.BTA_EHIP, f"factorization failed during tuning (info {int(info.item())})")
            ms.append(e0.elapsed_time(e1))
        return statistics.median(ms[1:])

    times: Dict[str, float] = {}
    prev_look = L.bta_internal_factor_lookahead(-1)
    prev_cached = L.bta_internal_factor_cached_loads(-2)
    try:
        for look in sorted(set(min(max(1, int(x)), max(1, T - 1)) for x in looks)):
            for c in cached:
                L.bta_internal_factor_lookahead(look)
                L.bta_internal_factor_cached_loads(int(c))
                med = median_ms()
                times[f"look={look},cached={int(c)}"] = med
                if log:
                    log(f"factor n={n} b={b} a={a} look={look} cached={int(c)}: {med:.3f} ms")
    finally:
        L.bta_internal_factor_lookahead(prev_look)
        L.bta_internal_factor_cached_loads(prev_cached)
    best = min(times, key=times.get)
    look_s, cached_s = best.split(",")
    set_entry(key("factor", b, a, "look"), int(look_s.split("=")[1]))
    set_entry(key("factor", b, a, "cached"), int(cached_s.split("=")[1]))
    # the SUB dispatch delay, with the lookahead and load path just recorded
    kd = key("factor", b, a, "sub_delay")
    delays: Dict[str, float] = {}
    for d in sorted(set(min(max(0, int(x)), T) for x in sub_delays)):
        set_entry(kd, d)
        delays[f"sub_delay={d}"] = median_ms()
        if log:
            log(f"factor n={n} b={b} a={a} sub_delay={d}: {delays[f'sub_delay={d}']:.3f} ms")
    set_entry(kd, int(min(delays, key=delays.get).split("=")[1]))
    times.update(delays)
    return times


def tune_selinv_split(n: int, b: int, a: int, splits: Iterable[int] = (1, 2, 3, 4), reps: int = 3, seed: int = 0,
                      log=None) -> Dict[str, float]:
    """Time bta_selinv on the factor of a seeded n x (b, a) matrix for every
    largest split count of the sweep products (``split``: 1 = no split; the
    library splits only where a product's 64 x 64 tiles fill under half the
    CUs), the median of ``reps`` runs each, and record the fastest as the
    table's ``split`` entry for (b, a).  ``BTA_SELINV_SPLIT``, when set,
    overrides the table and makes the candidates equal.
    Returns {"split=<s>": median ms}."""
    import torch

    if reps < 3:
        raise ValueError("reps >= 3 (the median of at least three runs)")
    reading = "scaled" if b >= 2048 else "literal"
    wl = synth.workload(n, b, a, reading)
    dev = torch.device("cuda", torch.cuda.current_device())
    Q = synth.make_torch(wl, seed, dev)
    L = bta.factor(Q["D"], Q["B"], Q["R"], Q["T"])[:4]
    out = tuple(torch.empty_like(t) for t in L)
    work, _ = bta.workspace(bta.BTA_OP_SELINV, n, b, a, dev)
    k = key("selinv", b, a, "split")
    prev = get_entry(k)
    times: Dict[str, float] = {}
    try:
        for sp in sorted(set(int(x) for x in splits)):
            set_entry(k, sp)
            ms = []
            for _ in range(reps + 1):  # the first run warms up
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                bta.selinv(*L, out=out, work=work)
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            med = statistics.median(ms[1:])
            times[f"split={sp}"] = med
            if log:
                log(f"selinv n={n} b={b} a={a} split={sp}: {med:.3f} ms")
    finally:
        if prev is not None:
            set_entry(k, prev)
    best = min(times, key=times.get)
    set_entry(k, int(best.split("=")[1]))
    return times


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="tune the BTA factorization and selected inversion for one block shape")
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--b", type=int, required=True)
    ap.add_argument("--a", type=int, default=0)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", required=True, help="JSON tuning table to update (read first if it exists)")
    args = ap.parse_args(argv)
    import os

    if os.path.exists(args.out):
        load(args.out)
    say = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    times = tune_factor(args.n, args.b, args.a, reps=args.reps, log=say)
    times.update(tune_selinv_split(args.n, args.b, args.a, reps=args.reps, log=say))
    save(args.out)
    print(json.dumps({"times_ms": times, "table": table()}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
