"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Every block of L and of the selected inverse must match the oracle within
1e-10 relative Frobenius error; strict upper triangles of the diagonal
factor blocks must be exact zeros; symmetric outputs exactly symmetric.
"""
import numpy as np
import pytest

import oracle
from paper_2503_17528_amd import synth
from tests.gpu_util import TOL, errs, say, to_dev, to_np

pytestmark = pytest.mark.gpu

# (n, b, a): ragged tiles, a = 0, n = 1, a wider than one tile, several tiles
SHAPES = [
    (1, 3, 0), (1, 64, 4), (2, 5, 1), (3, 64, 0), (4, 100, 3), (2, 130, 70),
    (16, 64, 4), (5, 192, 6), (3, 257, 2), (6, 128, 0), (2, 64, 64), (1, 200, 17),
    # arrow tip wider than the diagonal blocks (the paper's b = 1024, a = 256 ratio and beyond)
    (4, 128, 256), (3, 96, 257),
]


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_17528_amd import bta

    bta.lib()  # raises if the library is missing: never a silent fallback
    return torch


def _run(torch, Q, inplace=False):
    from paper_2503_17528_amd import bta

    D, B, R, T = to_dev(Q)
    if inplace:
        L = bta.factor(D, B, R, T, out=(D, B, R, T))
        X = bta.selinv(*L[:4], out=L[:4])
    else:
        L = bta.factor(D, B, R, T)
        X = bta.selinv(*L[:4])
    torch.cuda.synchronize()
    return to_np(L[:4]), int(L[4].item()), to_np(X)


def _check(Lg, Xg, F, Xo, n, b, a):
    eL = errs(dict(zip("DBRT", Lg)), {"D": F["LD"], "B": F["LB"], "R": F["LR"], "T": F["LT"]})
    eX = errs(dict(zip("DBRT", Xg)), {"D": Xo["XD"], "B": Xo["XB"], "R": Xo["XR"], "T": Xo["XT"]}, lower=())
    say(f"   L err {eL}\n   X err {eX}")
    assert max(eL.values()) < TOL, eL
    assert max(eX.values()) < TOL, eX
    for i in range(n):
        assert np.all(np.triu(Lg[0][i], 1) == 0.0)
        assert np.array_equal(Xg[0][i], Xg[0][i].T)
    if a:
        assert np.all(np.triu(Lg[3], 1) == 0.0)
        assert np.array_equal(Xg[3], Xg[3].T)


@pytest.mark.parametrize("n,b,a", SHAPES)
def test_factor_selinv_parity(torch_cuda, n, b, a):
    say(f"case factor+selinv n={n} b={b} a={a}")
    wl = synth.workload(n, b, a)
    Q = synth.make_np(wl, 3)
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    Xo = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    Lg, info, Xg = _run(torch_cuda, Q)
    assert info == 0
    _check(Lg, Xg, F, Xo, n, b, a)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("n,b,a", [(3, 384, 6), (2, 520, 8), (4, 136, 2), (2, 64, 130), (5, 192, 0)])
def test_selinv_gemm_kernels(torch_cuda, n, b, a, mode):
    """Both GEMM kernel families of the selected inversion (register-staged,
    direct-to-LDS with 128 and 64 tiles) against the oracle."""
    from paper_2503_17528_amd import bta

    say(f"case selinv gemm mode={mode} n={n} b={b} a={a}")
    wl = synth.workload(n, b, a)
    Q = synth.make_np(wl, 4)
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    Xo = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    prev = bta.gemm_mode(mode)
    try:
        Lg, info, Xg = _run(torch_cuda, Q)
    finally:
        bta.gemm_mode(prev)
    assert info == 0
    _check(Lg, Xg, F, Xo, n, b, a)


@pytest.mark.parametrize("n,b,a", [(4, 100, 3), (3, 64, 0), (2, 130, 70), (3, 128, 256)])
def test_inplace_matches(torch_cuda, n, b, a):
    say(f"case in-place n={n} b={b} a={a}")
    Q = synth.make_np(synth.workload(n, b, a), 8)
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    Xo = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    Lg, info, Xg = _run(torch_cuda, Q, inplace=True)
    assert info == 0
    # in place: the L outputs were overwritten by X; check X only
    eX = errs(dict(zip("DBRT", Xg)), {"D": Xo["XD"], "B": Xo["XB"], "R": Xo["XR"], "T": Xo["XT"]}, lower=())
    say(f"   X err {eX}")
    assert max(eX.values()) < TOL


def test_garbage_upper_triangle_is_ignored(torch_cuda):
    n, b, a = 3, 96, 5
    say(f"case garbage-upper n={n} b={b} a={a}")
    Q = synth.make_np(synth.workload(n, b, a), 4)
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    Xo = oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
    G = {k: v.copy() for k, v in Q.items()}
    for i in range(n):
        G["D"][i] += np.triu(np.full((b, b), np.nan), 1)
    G["T"] += np.triu(np.full((a, a), 1e300), 1)
    Lg, info, Xg = _run(torch_cuda, G)
    assert info == 0
    _check(Lg, Xg, F, Xo, n, b, a)


@pytest.mark.parametrize("where", ["first", "middle", "tip", "nan"])
def test_not_positive_definite_reports_row(torch_cuda, where):
    from paper_2503_17528_amd import bta

    n, b, a = 4, 80, 3
    say(f"case not-PD {where}")
    Q = synth.make_np(synth.workload(n, b, a), 6)
    if where == "first":
        Q["D"][0][5, 5] = -1.0
    elif where == "middle":
        Q["D"][2][70, 70] = -1e6
    elif where == "tip":
        Q["T"][1, 1] = -1e6
    else:
        Q["D"][1][10, 10] = np.nan
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    assert F["info"] > 0
    D, B, R, T = to_dev(Q)
    L = bta.factor(D, B, R, T, check=False)
    torch_cuda.cuda.synchronize()
    assert int(L[4].item()) == F["info"]
    with pytest.raises(bta.NotPositiveDefinite) as ei:
        bta.factor(D, B, R, T)
    assert ei.value.row == F["info"]


@pytest.mark.parametrize("n,b,a,nrhs", [(1, 3, 0, 1), (4, 100, 3, 1), (3, 64, 0, 2), (2, 130, 70, 3), (16, 64, 4, 1),
                                            (4, 128, 256, 2)])
def test_solve_and_logdet(torch_cuda, n, b, a, nrhs):
    from paper_2503_17528_amd import bta

    say(f"case solve/logdet n={n} b={b} a={a} nrhs={nrhs}")
    wl = synth.workload(n, b, a)
    Q = synth.make_np(wl, 9)
    y = synth.rhs_np(wl, 9, nrhs)
    F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
    xo = oracle.pobtas(F["LD"], F["LB"], F["LR"], F["LT"], y)
    ldo = oracle.logdet(F["LD"], F["LT"])
    D, B, R, T = to_dev(Q)
    L = bta.factor(D, B, R, T)
    yd = torch_cuda.from_numpy(y).to("cuda")
    x = bta.solve(*L[:4], yd)
    ld = bta.logdet(L[0], L[3])
    torch_cuda.cuda.synchronize()
    xg = x.cpu().numpy()
    e = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    say(f"   solve rel err {e:.3e}  logdet {float(ld.item())} vs {ldo}")
    assert e < TOL
    assert abs(float(ld.item()) - ldo) <= TOL * abs(ldo)


def test_abi_rejects_bad_workspace_on_device(torch_cuda):
    from paper_2503_17528_amd import bta

    n, b, a = 2, 64, 4
    Q = synth.make_np(synth.workload(n, b, a), 1)
    D, B, R, T = to_dev(Q)
    work = torch_cuda.empty(16, dtype=torch_cuda.uint8, device="cuda")
    with pytest.raises(bta.BTAError) as ei:
        bta.factor(D, B, R, T, work=work)
    assert ei.value.status == bta.BTA_EINVAL


@pytest.mark.parametrize("delay", [0, 1, 3, 10])
def test_factor_sub_delays(torch_cuda, delay):
    """Every SUB dispatch delay gives the oracle's factor (the delay only
    reorders the tickets of the coupling block's tiles): a 10 x 10 tile band
    with ragged tiles and a two-tile tip, the delay set through the tuning
    table (10 = every SUB task after its step's last column)."""
    from paper_2503_17528_amd import autotune, bta

    n, b, a = 4, 610, 70
    say(f"case sub_delay={delay} n={n} b={b} a={a}")
    k = autotune.key("factor", b, a, "sub_delay")
    autotune.set_entry(k, delay)
    try:
        wl = synth.workload(n, b, a)
        Q = synth.make_np(wl, 12)
        F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
        D, B, R, T = to_dev(Q)
        L = bta.factor(D, B, R, T)
        torch_cuda.cuda.synchronize()
        e = errs(dict(zip("DBRT", to_np(L[:4]))), {"D": F["LD"], "B": F["LB"], "R": F["LR"], "T": F["LT"]})
        say(f"   L err {e}")
        assert max(e.values()) < TOL, e
    finally:
        autotune.clear()
