"""GPU parity of the batched entry points (many BTA matrices of uneven n, b,
a in one persistent factor launch, then the batched selected inversion),
every matrix against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2503_17528_amd import synth
from tests.gpu_util import TOL, errs, say, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_17528_amd import bta

    bta.lib()
    return torch


def _check_matrix(Q, Lg, Xg, m):
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    Xo = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    eL = errs(dict(zip("DBRT", to_np(Lg))), {"D": F["LD"], "B": F["LB"], "R": F["LR"], "T": F["LT"]})
    eX = errs(dict(zip("DBRT", to_np(Xg))), {"D": Xo["XD"], "B": Xo["XB"], "R": Xo["XR"], "T": Xo["XT"]}, lower=())
    worst = max(max(eL.values()), max(eX.values()))
    return worst, eL, eX


@pytest.mark.parametrize("inplace", [False, True])
def test_small_mixed_batch(torch_cuda, inplace):
    torch = torch_cuda
    from paper_2503_17528_amd import bta

    shapes = [(1, 5, 0), (3, 64, 2), (2, 130, 70), (5, 40, 1), (4, 200, 0), (6, 64, 4)]
    say(f"case batched small inplace={inplace}")
    Qs = [synth.make_np(synth.workload(*s), 10 + k) for k, s in enumerate(shapes)]
    mats = [{k: torch.from_numpy(q[k]).to("cuda") for k in "DBRT"} for q in Qs]
    batch = bta.Batch(mats, inplace=inplace)
    batch.factor()
    if not inplace:
        Ls = [tuple(t.clone() for t in L) for L in batch.L]
    batch.selinv()
    torch.cuda.synchronize()
    for m, (s, Q) in enumerate(zip(shapes, Qs)):
        if inplace:
            F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
            Xo = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
            e = errs(dict(zip("DBRT", to_np(batch.X[m]))), {"D": Xo["XD"], "B": Xo["XB"], "R": Xo["XR"], "T": Xo["XT"]},
                     lower=())
            worst = max(e.values())
        else:
            worst, _, _ = _check_matrix(Q, Ls[m], batch.X[m], m)
        say(f"   matrix {m} {s}: max rel err {worst:.3e}")
        assert worst < TOL


def test_hyperparameter_sweep_batch(torch_cuda):
    """64 matrices, n ~ U{16..96}, b in {128, 256, 384}, a in {2, 4, 6}: every
    block of every matrix's L against the factor its input was drawn from, and
    every block of every matrix's Sigma against the oracle's Algorithm 2 run on
    that factor, on the first call (eager, autotuned) and on the second (graph
    replay)."""
    torch = torch_cuda
    from threadpoolctl import threadpool_limits

    from paper_2503_17528_amd import bta

    wls = synth.batched_workloads(0)
    say(f"case batched sweep: {len(wls)} matrices, {sum(w.block_bytes() for w in wls) / 1e9:.2f} GB")
    full = [synth.make_torch(w, 100 + k, "cuda", with_factor=True) for k, w in enumerate(wls)]
    mats = [{k: f[k] for k in "DBRT"} for f in full]
    batch = bta.Batch(mats)
    ref = []
    # small blocks: one BLAS thread per call is several times faster than many
    with threadpool_limits(1):
        for m in range(len(wls)):
            Lh = {k: full[m][k].cpu().numpy() for k in ("LD", "LB", "LR", "LT")}
            Xo = oracle.pobtasi(Lh["LD"], Lh["LB"], Lh["LR"], Lh["LT"])
            ref.append(({"D": Lh["LD"], "B": Lh["LB"], "R": Lh["LR"], "T": Lh["LT"]},
                        {"D": Xo["XD"], "B": Xo["XB"], "R": Xo["XR"], "T": Xo["XT"]}))
            if m % 16 == 15:
                say(f"   oracle done for {m + 1} matrices")
    for call in range(2):
        for L in batch.X:
            for t in L:
                t.zero_()
        batch.factor()
        Ls = [tuple(t.clone() for t in L) for L in batch.L]
        batch.selinv()
        torch.cuda.synchronize()
        worst_all = 0.0
        for m in range(len(wls)):
            eL = errs(dict(zip("DBRT", to_np(Ls[m]))), ref[m][0])
            eX = errs(dict(zip("DBRT", to_np(batch.X[m]))), ref[m][1], lower=())
            worst = max(max(eL.values()), max(eX.values()))
            worst_all = max(worst_all, worst)
            assert worst < TOL, (call, m, wls[m].name, eL, eX)
        say(f"   call {call}: all {len(wls)} matrices, max rel err {worst_all:.3e}")


def test_failure_is_reported_per_matrix(torch_cuda):
    torch = torch_cuda
    from paper_2503_17528_amd import bta

    shapes = [(3, 64, 2), (4, 80, 3), (2, 64, 0)]
    Qs = [synth.make_np(synth.workload(*s), 20 + k) for k, s in enumerate(shapes)]
    Qs[1]["D"][2][7, 7] = -1e6
    expect = oracle.pobtaf(Qs[1]["D"], Qs[1]["B"], Qs[1]["R"], Qs[1]["T"])["info"]
    mats = [{k: torch.from_numpy(q[k]).to("cuda") for k in "DBRT"} for q in Qs]
    batch = bta.Batch(mats)
    batch.factor(check=False)
    torch.cuda.synchronize()
    infos = [int(i.item()) for i in batch.info]
    say(f"case batched failure: infos {infos}, expected matrix 1 -> {expect}")
    assert infos == [0, expect, 0]
