"""bta_factor_noalloc (the factorization with the library's fixed device
scratch, for callers that cannot allocate): through the C ABI, two calls in a
row, the second on a smaller problem, each compared block by block with
bta_factor (the workspace entry point) on the same input, to the 1e-10
relative Frobenius bar per block (the same kernels run, so the results are
expected to agree exactly), and with the oracle."""
import numpy as np
import pytest

import oracle
from paper_2503_17528_amd import synth
from tests.gpu_util import TOL, errs, say, to_np

pytestmark = pytest.mark.gpu


def test_factor_noalloc_matches_factor():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_17528_amd import bta

    bta.lib()
    # the second problem is smaller: the scratch keeps the first call's contents
    for k, shape in enumerate([(10, 200, 7), (3, 96, 2)]):
        wl = synth.workload(*shape)
        need = bta.bta_workspace_bytes(bta.BTA_OP_FACTOR, *shape)
        say(f"case no-alloc factor call {k}: shape {shape}, scratch {need} bytes")
        Q = synth.make_np(wl, 60 + k)
        D, B, R, T = (torch.from_numpy(Q[x]).to("cuda") for x in "DBRT")
        Ln = bta.factor_noalloc(D, B, R, T)
        Lw = bta.factor(D, B, R, T, check=False)
        torch.cuda.synchronize()
        assert int(Ln[4].item()) == 0 and int(Lw[4].item()) == 0
        got = dict(zip("DBRT", to_np(Ln[:4])))
        ref = dict(zip("DBRT", to_np(Lw[:4])))
        e = errs(got, ref)
        same = all(np.array_equal(got[x], ref[x]) for x in "DBRT")
        F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
        eo = errs(got, {"D": F["LD"], "B": F["LB"], "R": F["LR"], "T": F["LT"]})
        say(f"   vs bta_factor: {e} (bitwise equal: {same}); vs oracle: {eo}")
        assert max(e.values()) < TOL, e
        assert max(eo.values()) < TOL, eo


def test_factor_noalloc_rejects_oversize():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_17528_amd import bta

    bta.lib()
    shape = (64, 2048, 8)  # 32 MiB of diagonal-tile inverses per 8 blocks: far above the limit
    assert bta.bta_workspace_bytes(bta.BTA_OP_FACTOR, *shape) > (64 << 20)
    n, b, a = shape
    D = torch.zeros((n, b, b), dtype=torch.float64, device="cuda")
    B = torch.zeros((n - 1, b, b), dtype=torch.float64, device="cuda")
    R = torch.zeros((n, a, b), dtype=torch.float64, device="cuda")
    T = torch.zeros((a, a), dtype=torch.float64, device="cuda")
    with pytest.raises(bta.BTAError) as ei:
        bta.factor_noalloc(D, B, R, T, out=(D, B, R, T))
    assert ei.value.status == bta.BTA_EINVAL
    assert "scratch" in str(ei.value)
