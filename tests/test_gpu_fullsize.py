"""GPU parity at the full workload sizes, in the launch configuration that
bench.py times (out-of-place bta_factor + bta_selinv on one stream).

At these sizes the oracle cannot run whole, so parity is checked on outputs
that can be computed one by one, and on properties that hold at any size:

* L against the factor the inputs were drawn from (Q = L_gen L_gen^T exactly,
  and the Cholesky factor is unique): per block relative Frobenius <= 1e-10.
* Sampled exact columns of Sigma: the oracle's block substitution with L_gen
  (``oracle.pobtas``, on the CPU) gives Sigma e_c; its selected entries are
  compared with the GPU's X blocks.
* The block identities (Sigma Q)_jj = I, (Sigma Q)_{n,j} = 0, (Sigma Q)_nn = I,
  which use selected blocks only, for sampled j (evaluated with torch on the
  device: a property check, not a second implementation of the method).
"""
import numpy as np
import pytest

import oracle
from paper_2503_17528_amd import synth
from tests.gpu_util import TOL, say

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


def _sigma_q_identities(torch, Q, X, n, b, a, js):
    D, B, R, T = Q["D"], Q["B"], Q["R"], Q["T"]
    XD, XB, XR, XT = X
    worst = 0.0
    I_b = torch.eye(b, dtype=torch.float64, device=D.device)
    for j in js:
        acc = XD[j] @ D[j]
        if a:
            acc += XR[j].T.contiguous() @ R[j]
        if j > 0:
            acc += XB[j - 1] @ B[j - 1].T.contiguous()
        if j < n - 1:
            acc += XB[j].T.contiguous() @ B[j]
        worst = max(worst, (acc - I_b).abs().max().item())
        if a:
            acc = XR[j] @ D[j] + XT @ R[j]
            if j > 0:
                acc += XR[j - 1] @ B[j - 1].T.contiguous()
            if j < n - 1:
                acc += XR[j + 1] @ B[j]
            worst = max(worst, acc.abs().max().item())
    if a:
        acc = XT @ T
        for j in range(n):
            acc += XR[j] @ R[j].T.contiguous()
        worst = max(worst, (acc - torch.eye(a, dtype=torch.float64, device=D.device)).abs().max().item())
    return worst


def _exact_columns(torch, Lgen, X, n, b, a, cols):
    """Sigma e_c from the oracle's substitution with the drawn factor (CPU),
    compared with the selected entries of column c of the GPU's X."""
    LD, LB, LR, LT = (t.cpu().numpy() for t in (Lgen["LD"], Lgen["LB"], Lgen["LR"], Lgen["LT"]))
    N = n * b + a
    E = np.zeros((N, len(cols)))
    for q, c in enumerate(cols):
        E[c, q] = 1.0
    S = oracle.pobtas(LD, LB, LR, LT, E)
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
    say(f"   L vs drawn factor: {eL}")
    assert max(eL.values()) < TOL
    rng = np.random.default_rng(0)
    js = sorted(set([0, n - 1] + list(rng.integers(0, n, 4))))
    ident = _sigma_q_identities(torch, Q, X, n, b, a, js)
    say(f"   Sigma Q identities, blocks {js}: max abs deviation {ident:.3e}")
    assert ident < 1e-10
    N = n * b + a
    cols = sorted(set([0, b - 1, N - 1] + list(rng.integers(0, N, 5))))
    ec = _exact_columns(torch, Q, X, n, b, a, cols)
    say(f"   exact columns {cols}: max rel err {ec:.3e}")
    assert ec < TOL


def test_largest_workload_in_place(torch_cuda):
    """n=256, b=4096, a=16 (68.7 GB of blocks): in place, checked block by
    block against the drawn factor and through the Sigma Q identities."""
    from paper_2503_17528_amd import bta

    torch = torch_cuda
    wl = synth.LARGE
    n, b, a = wl.n, wl.b, wl.a
    free, total = torch.cuda.mem_get_info()
    need = wl.block_bytes() * 1.15 + 6e9
    if free < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB free, have {free / 1e9:.0f} GB")
    say(f"case largest {wl.name}: drawing")
    Q = synth.make_torch(wl, 0, "cuda")
    js = [0, 1, n // 2, n - 2, n - 1]
    # keep the input blocks needed by the identity check
    keep = {j: (Q["D"][j].clone(), Q["B"][j].clone() if j < n - 1 else None, Q["R"][j].clone()) for j in js}
    keep_prev = {j: Q["B"][j - 1].clone() for j in js if j > 0}
    Tin = Q["T"].clone()
    say("   factor (in place)")
    L = bta.factor(Q["D"], Q["B"], Q["R"], Q["T"], out=(Q["D"], Q["B"], Q["R"], Q["T"]))
    torch.cuda.synchronize()
    worst = 0.0
    for j in js:
        Lg = synth.factor_block_torch(wl, 0, synth.KIND_DIAG, j, "cuda")
        worst = max(worst, _block_rel(torch, L[0][j][None], Lg[None], True))
        if j < n - 1:
            Lg = synth.factor_block_torch(wl, 0, synth.KIND_SUB, j, "cuda")
            worst = max(worst, _block_rel(torch, L[1][j][None], Lg[None], False))
        Lg = synth.factor_block_torch(wl, 0, synth.KIND_ARROW, j, "cuda")
        worst = max(worst, _block_rel(torch, L[2][j][None], Lg[None], False))
    Lg = synth.factor_block_torch(wl, 0, synth.KIND_TIP, 0, "cuda")
    worst = max(worst, _block_rel(torch, L[3][None], Lg[None], True))
    say(f"   sampled L blocks vs drawn factor: max rel err {worst:.3e}")
    assert worst < TOL
    say("   selinv (in place)")
    X = bta.selinv(*L[:4], out=L[:4])
    torch.cuda.synchronize()
    XD, XB, XR, XT = X
    dev = 0.0
    for j in js[1:-1]:
        Dj, Bj, Rj = keep[j]
        acc = XD[j] @ Dj + XR[j].T.contiguous() @ Rj + XB[j - 1] @ keep_prev[j].T.contiguous() + XB[j].T.contiguous() @ Bj
        dev = max(dev, (acc - torch.eye(b, dtype=torch.float64, device="cuda")).abs().max().item())
    acc = XT @ Tin
    say(f"   Sigma Q diagonal identities at blocks {js[1:-1]}: max abs deviation {dev:.3e}")
    assert dev < 1e-10
