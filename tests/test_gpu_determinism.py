"""Bitwise run-to-run reproducibility of every entry point.

The library fixes the order of every sum: a tile's k loop runs its sources in
a fixed order whichever workgroup takes the task, the tip updates are summed
in step order, split-k partials are added in split order, and the solve's and
log-determinant's reductions have fixed trees.  Repeated calls on the same
input -- on different streams, in place or out of place, eager or replayed
from the batched graph -- must therefore give identical bits.  Each case also
checks one run against the oracle, so the bits compared are right ones.
"""
import numpy as np
import pytest

import oracle
from paper_2503_17528_amd import synth
from tests.gpu_util import TOL, errs, say, to_dev, to_np

pytestmark = pytest.mark.gpu

# ragged tiles, a tip wider than the blocks, and b = 512 (split-k sweep products)
SHAPES = [(16, 64, 4), (5, 192, 6), (3, 257, 2), (4, 128, 256), (8, 512, 4)]


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_17528_amd import bta

    bta.lib()
    return torch


def _bits(torch, t):
    """The tensor's bytes as int64 words (so -0.0 != 0.0 and NaNs compare)."""
    return t.contiguous().reshape(-1).view(torch.int64)


def _same(torch, xs, ys, what):
    for k, (x, y) in enumerate(zip(xs, ys)):
        if x is None:
            assert y is None
            continue
        bx, by = _bits(torch, x), _bits(torch, y)
        nd = int((bx != by).sum().item())
        assert nd == 0, f"{what}: array {k} differs in {nd} of {bx.numel()} words"


def _pipeline(torch, bta, Qd, y, stream, inplace=False):
    """factor, selinv, solve, logdet, logdet_quad and the gradient on `stream`."""
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        if inplace:
            A = tuple(t.clone() for t in Qd)
            L = bta.factor(*A, out=A, stream=stream, check=False)
        else:
            L = bta.factor(*Qd, stream=stream, check=False)
        Ls = tuple(t.clone() for t in L[:4])  # selinv in place overwrites L
        x = bta.solve(*Ls, y, stream=stream)
        ld = bta.logdet(Ls[0], Ls[3], stream=stream)
        f = bta.logdet_quad(Ls[0], Ls[3], y, x, stream=stream)
        X = bta.selinv(*L[:4], out=L[:4] if inplace else None, stream=stream)
        G = bta.grad_logdet_quad(X, x, stream=stream)
    stream.synchronize()
    assert int(L[4].item()) == 0
    return {"L": Ls, "X": X, "x": (x,), "ld": (ld, f), "G": G}


@pytest.mark.parametrize("n,b,a", SHAPES)
def test_repeat_bitwise(torch_cuda, n, b, a):
    torch = torch_cuda
    from paper_2503_17528_amd import bta

    say(f"case determinism n={n} b={b} a={a}")
    wl = synth.workload(n, b, a)
    Q = synth.make_np(wl, 21)
    Qd = to_dev(Q)
    N = n * b + a
    y = torch.from_numpy(np.random.default_rng(5).standard_normal((N, 2))).to("cuda")
    s0 = torch.cuda.current_stream()
    s1 = torch.cuda.Stream()
    runs = [_pipeline(torch, bta, Qd, y, s0), _pipeline(torch, bta, Qd, y, s1), _pipeline(torch, bta, Qd, y, s0),
            _pipeline(torch, bta, Qd, y, s1, inplace=True)]
    for r, run in enumerate(runs[1:], 1):
        for key in ("L", "X", "x", "ld", "G"):
            _same(torch, runs[0][key], run[key], f"run {r} {key}")
    say(f"   {len(runs)} runs bitwise identical (2 streams, in place and out of place)")

    # the bits are the right ones
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    Xo = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    eL = errs(dict(zip("DBRT", to_np(runs[0]["L"]))), {"D": F["LD"], "B": F["LB"], "R": F["LR"], "T": F["LT"]})
    eX = errs(dict(zip("DBRT", to_np(runs[0]["X"]))), {"D": Xo["XD"], "B": Xo["XB"], "R": Xo["XR"], "T": Xo["XT"]},
              lower=())
    assert max(eL.values()) < TOL, eL
    assert max(eX.values()) < TOL, eX


def test_batched_bitwise(torch_cuda):
    """The eager first call of the batched entry points (which also tunes the
    merged GEMM stages) and two graph replays give identical bits."""
    torch = torch_cuda
    from paper_2503_17528_amd import bta

    shapes = [(1, 5, 0), (3, 64, 2), (2, 130, 70), (5, 40, 1), (4, 200, 0), (6, 64, 4), (3, 384, 6)]
    say("case determinism batched")
    Qs = [synth.make_np(synth.workload(*s), 40 + k) for k, s in enumerate(shapes)]
    mats = [{k: torch.from_numpy(q[k]).to("cuda") for k in "DBRT"} for q in Qs]
    batch = bta.Batch(mats)
    outs = []
    for call in range(3):
        for L in batch.L:
            for t in L:
                t.fill_(float("nan"))
        for X in batch.X:
            for t in X:
                t.fill_(float("nan"))
        batch.factor()
        batch.selinv()
        torch.cuda.synchronize()
        outs.append([tuple(t.clone() for t in L) + tuple(t.clone() for t in X) for L, X in zip(batch.L, batch.X)])
    for call in (1, 2):
        for m in range(len(shapes)):
            _same(torch, outs[0][m], outs[call][m], f"call {call} matrix {m} {shapes[m]}")
    say(f"   3 calls bitwise identical over {len(shapes)} matrices")
    m = len(shapes) - 1
    Q = Qs[m]
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    Xo = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    eX = errs(dict(zip("DBRT", to_np(outs[0][m][4:]))), {"D": Xo["XD"], "B": Xo["XB"], "R": Xo["XR"], "T": Xo["XT"]},
              lower=())
    assert max(eX.values()) < TOL, eX
