"""GPU parity at the full workload sizes, in the launch configuration that
bench.py times (out-of-place bta_factor + bta_selinv on one stream).

Every block of L is compared with the factor the inputs were drawn from
(Q = L_gen L_gen^T exactly, and the Cholesky factor is unique).  Every block
of Sigma is compared with the oracle's Algorithm 2 run on that factor, where
the oracle finishes in a minute or two on the host (n=128/b=2048,
n=256/b=512, n=512/b=1024/a=256).  At n=256, b=4096, a=16 (68.7 GB of
blocks, about 20 minutes of oracle time) the oracle runs on the trailing
blocks only: the backward sweep of Algorithm 2 produces blocks K..n-1 and the
tip from L blocks K..n-1 and the tip factor alone, so its run on that tail is
exactly the tail of the full selected inverse.  Property checks that hold at
any size complete the picture:

* the block identities (Sigma Q)_jj = I, (Sigma Q)_{n,j} = 0, (Sigma Q)_nn = I,
  which use selected blocks only (evaluated with torch on the device: a
  property check, not a second implementation of the method);
* sampled exact columns of Sigma from the oracle's block substitution with
  L_gen (``oracle.pobtas``), compared with the selected entries of the GPU's X.
"""
import numpy as np
import pytest

import oracle
from paper_2503_17528_amd import synth
from tests.gpu_util import TOL, errs, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_17528_amd import bta

    bta.lib()
    return torch


def _block_rel(torch, got, ref, lower):
    if lower:
        got, ref = torch.tril(got), torch.tril(ref)
    d = torch.linalg.matrix_norm(got - ref)
    r = torch.linalg.matrix_norm(ref)
    return (d / r).max().item()


def _diag_identity(torch, X, Din, Bprev, Bnext, Rin, j, n, a):
    """max |(Sigma Q)_jj - I| from the selected blocks around j."""
    XD, XB, XR, XT = X
    acc = XD[j] @ Din
    if a:
        acc += XR[j].T.contiguous() @ Rin
    if j > 0:
        acc += XB[j - 1] @ Bprev.T.contiguous()
    if j < n - 1:
        acc += XB[j].T.contiguous() @ Bnext
    acc -= torch.eye(acc.shape[0], dtype=torch.float64, device=acc.device)
    return acc.abs().max().item()


def _arrow_identity(torch, X, Din, Bprev, Bnext, Rin, j, n):
    """max |(Sigma Q)_{n,j}| (must vanish)."""
    XD, XB, XR, XT = X
    acc = XR[j] @ Din + XT @ Rin
    if j > 0:
        acc += XR[j - 1] @ Bprev.T.contiguous()
    if j < n - 1:
        acc += XR[j + 1] @ Bnext
    return acc.abs().max().item()


def _tip_identity(torch, X, Rall, Tin, n):
    """max |(Sigma Q)_nn - I| = |X_nn Q_nn + sum_j X_{n,j} Q_{n,j}^T - I|."""
    XD, XB, XR, XT = X
    acc = XT @ Tin
    for j in range(n):
        acc += XR[j] @ Rall[j].T.contiguous()
    acc -= torch.eye(acc.shape[0], dtype=torch.float64, device=acc.device)
    return acc.abs().max().item()


def _exact_columns(torch, Lh, X, n, b, a, cols):
    """Sigma e_c from the oracle's substitution with the drawn factor (CPU),
    compared with the selected entries of column c of the GPU's X."""
    N = n * b + a
    E = np.zeros((N, len(cols)))
    for q, c in enumerate(cols):
        E[c, q] = 1.0
    S = oracle.pobtas(Lh["LD"], Lh["LB"], Lh["LR"], Lh["LT"], E)
    XD, XB, XR, XT = (t.cpu() for t in X)
    worst = 0.0
    for q, c in enumerate(cols):
        col = S[:, q]
        got = []
        ref = []
        if c < n * b:
            j, cc = divmod(c, b)
            got.append(XD[j][:, cc].numpy()); ref.append(col[j * b:(j + 1) * b])
            if j < n - 1:
                got.append(XB[j][:, cc].numpy()); ref.append(col[(j + 1) * b:(j + 2) * b])
            if a:
                got.append(XR[j][:, cc].numpy()); ref.append(col[n * b:])
        else:
            cc = c - n * b
            got.append(XT[:, cc].numpy()); ref.append(col[n * b:])
            for j in range(n):
                got.append(XR[j][cc, :].numpy()); ref.append(col[j * b:(j + 1) * b])
        g, r = np.concatenate(got), np.concatenate(ref)
        worst = max(worst, float(np.linalg.norm(g - r) / np.linalg.norm(r)))
    return worst


@pytest.mark.parametrize("wl", [synth.BENCH, synth.AUTOGRAD, synth.ARROW], ids=lambda w: w.name)
def test_fullsize_factor_selinv(torch_cuda, wl):
    from paper_2503_17528_amd import bta

    torch = torch_cuda
    n, b, a = wl.n, wl.b, wl.a
    say(f"case fullsize {wl.name}: drawing")
    Q = synth.make_torch(wl, 0, "cuda", with_factor=True)
    say("   factor + selinv")
    L = bta.factor(Q["D"], Q["B"], Q["R"], Q["T"])
    X = bta.selinv(*L[:4])
    torch.cuda.synchronize()
    eL = {
        "D": _block_rel(torch, L[0], Q["LD"], True),
        "B": _block_rel(torch, L[1], Q["LB"], False) if n > 1 else 0.0,
        "R": _block_rel(torch, L[2], Q["LR"], False) if a else 0.0,
        "T": _block_rel(torch, L[3][None], Q["LT"][None], True) if a else 0.0,
    }
    say(f"   every L block vs drawn factor: {eL}")
    assert max(eL.values()) < TOL

    # every block of Sigma against the oracle's Algorithm 2 on the drawn factor
    Lh = {k: Q[k].cpu().numpy() for k in ("LD", "LB", "LR", "LT")}
    say("   oracle selected inversion on the host")
    Xo = oracle.pobtasi(Lh["LD"], Lh["LB"], Lh["LR"], Lh["LT"])
    Xg = dict(zip("DBRT", (t.cpu().numpy() for t in X)))
    eX = errs(Xg, {"D": Xo["XD"], "B": Xo["XB"], "R": Xo["XR"], "T": Xo["XT"]}, lower=())
    say(f"   every Sigma block vs oracle: {eX}")
    assert max(eX.values()) < TOL, eX
    del Xg, Xo

    rng = np.random.default_rng(0)
    js = sorted(set([0, n - 1] + list(rng.integers(0, n, 4))))
    worst = 0.0
    for j in js:
        Bp = Q["B"][j - 1] if j > 0 else None
        Bn = Q["B"][j] if j < n - 1 else None
        worst = max(worst, _diag_identity(torch, X, Q["D"][j], Bp, Bn, Q["R"][j], j, n, a))
        if a:
            worst = max(worst, _arrow_identity(torch, X, Q["D"][j], Bp, Bn, Q["R"][j], j, n))
    if a:
        worst = max(worst, _tip_identity(torch, X, Q["R"], Q["T"], n))
    say(f"   Sigma Q identities, blocks {js} and the tip: max abs deviation {worst:.3e}")
    assert worst < 1e-10
    N = n * b + a
    cols = sorted(set([0, b - 1, N - 1] + list(rng.integers(0, N, 5))))
    ec = _exact_columns(torch, Lh, X, n, b, a, cols)
    say(f"   exact columns {cols}: max rel err {ec:.3e}")
    assert ec < TOL


def test_largest_workload_in_place(torch_cuda):
    """n=256, b=4096, a=16 (68.7 GB of blocks), in place: every L block
    against the drawn factor; the trailing Sigma blocks and the tip against
    the oracle's Algorithm 2 on the trailing factor blocks; the Sigma Q
    identities at the first, middle and last blocks and at the tip."""
    from paper_2503_17528_amd import bta

    torch = torch_cuda
    wl = synth.LARGE
    n, b, a = wl.n, wl.b, wl.a
    K = 4  # trailing blocks checked against the oracle
    free, total = torch.cuda.mem_get_info()
    need = wl.block_bytes() * 1.15 + 6e9
    if free < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB free, have {free / 1e9:.0f} GB")
    say(f"case largest {wl.name}: drawing")
    Q = synth.make_torch(wl, 0, "cuda")
    js = [0, 1, n // 2, n - 2, n - 1]
    # the input blocks needed by the identity checks (the arrays are overwritten in place)
    Din = {j: Q["D"][j].clone() for j in js}
    Bin = {j: Q["B"][j].clone() for j in sorted(set(k for j in js for k in (j - 1, j) if 0 <= k < n - 1))}
    Rin = Q["R"].clone()
    Tin = Q["T"].clone()
    say("   factor (in place)")
    L = bta.factor(Q["D"], Q["B"], Q["R"], Q["T"], out=(Q["D"], Q["B"], Q["R"], Q["T"]))
    torch.cuda.synchronize()
    worst = {"D": 0.0, "B": 0.0, "R": 0.0, "T": 0.0}
    for j in range(n):
        Lg = synth.factor_block_torch(wl, 0, synth.KIND_DIAG, j, "cuda")
        worst["D"] = max(worst["D"], _block_rel(torch, L[0][j][None], Lg[None], True))
        if j < n - 1:
            Lg = synth.factor_block_torch(wl, 0, synth.KIND_SUB, j, "cuda")
            worst["B"] = max(worst["B"], _block_rel(torch, L[1][j][None], Lg[None], False))
        Lg = synth.factor_block_torch(wl, 0, synth.KIND_ARROW, j, "cuda")
        worst["R"] = max(worst["R"], _block_rel(torch, L[2][j][None], Lg[None], False))
    Lg = synth.factor_block_torch(wl, 0, synth.KIND_TIP, 0, "cuda")
    worst["T"] = _block_rel(torch, L[3][None], Lg[None], True)
    say(f"   every L block vs drawn factor: {worst}")
    assert max(worst.values()) < TOL

    # the oracle's inputs: the trailing K blocks of the drawn factor and its tip
    tail = {
        "LD": np.stack([synth.factor_block_torch(wl, 0, synth.KIND_DIAG, j, "cuda").cpu().numpy() for j in range(n - K, n)]),
        "LB": np.stack([synth.factor_block_torch(wl, 0, synth.KIND_SUB, j, "cuda").cpu().numpy() for j in range(n - K, n - 1)]),
        "LR": np.stack([synth.factor_block_torch(wl, 0, synth.KIND_ARROW, j, "cuda").cpu().numpy() for j in range(n - K, n)]),
        "LT": Lg.cpu().numpy(),
    }
    say("   selinv (in place)")
    X = bta.selinv(*L[:4], out=L[:4])
    torch.cuda.synchronize()
    XD, XB, XR, XT = X

    say(f"   oracle selected inversion of the trailing {K} blocks on the host")
    Xo = oracle.pobtasi(tail["LD"], tail["LB"], tail["LR"], tail["LT"])
    Xg = {"D": XD[n - K:].cpu().numpy(), "B": XB[n - K:n - 1].cpu().numpy(), "R": XR[n - K:].cpu().numpy(),
          "T": XT.cpu().numpy()}
    eX = errs(Xg, {"D": Xo["XD"], "B": Xo["XB"], "R": Xo["XR"], "T": Xo["XT"]}, lower=())
    say(f"   Sigma blocks {n - K}..{n - 1} and the tip vs oracle: {eX}")
    assert max(eX.values()) < TOL, eX

    dev = 0.0
    for j in js:
        Bp = Bin.get(j - 1)
        Bn = Bin.get(j)
        dev = max(dev, _diag_identity(torch, X, Din[j], Bp, Bn, Rin[j], j, n, a))
        dev = max(dev, _arrow_identity(torch, X, Din[j], Bp, Bn, Rin[j], j, n))
    dev = max(dev, _tip_identity(torch, X, Rin, Tin, n))
    say(f"   Sigma Q identities at blocks {js} and the tip: max abs deviation {dev:.3e}")
    assert dev < 1e-10
