"""Reentrancy per stream: bta_selinv (which leases helper streams and events
for its preprocessing and copy-outs) called from two host threads at once,
each on its own stream with its own workspace and outputs, several times in a
row; both results compared block by block with the oracle."""
import threading

import numpy as np
import pytest

import oracle
from paper_2503_17528_amd import synth
from tests.gpu_util import TOL, errs, say, to_np

pytestmark = pytest.mark.gpu


def test_selinv_two_threads_two_streams():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_17528_amd import bta

    bta.lib()
    shapes = [(12, 192, 5), (9, 256, 3)]
    say(f"case concurrency: selinv on two threads and two streams, shapes {shapes}")
    ref, Ls, outs, works = [], [], [], []
    for k, s in enumerate(shapes):
        wl = synth.workload(*s)
        Q = synth.make_np(wl, 40 + k)
        F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
        Xo = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
        ref.append({"D": Xo["XD"], "B": Xo["XB"], "R": Xo["XR"], "T": Xo["XT"]})
        D, B, R, T = (torch.from_numpy(Q[x]).to("cuda") for x in "DBRT")
        L = bta.factor(D, B, R, T)[:4]
        Ls.append(L)
        outs.append(tuple(torch.empty_like(t) for t in L))
        works.append(bta.workspace(bta.BTA_OP_SELINV, *s, "cuda")[0])
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    start = threading.Barrier(2)
    failures = []

    def run(k):
        try:
            start.wait()
            for _ in range(4):
                with torch.cuda.stream(streams[k]):
                    bta.selinv(*Ls[k], out=outs[k], work=works[k], stream=streams[k])
        except Exception as e:  # reported below, on the main thread
            failures.append((k, repr(e)))

    threads = [threading.Thread(target=run, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not failures, failures
    for k in range(2):
        e = errs(dict(zip("DBRT", to_np(outs[k]))), ref[k], lower=())
        say(f"   thread {k} {shapes[k]}: {e}")
        assert max(e.values()) < TOL, e
