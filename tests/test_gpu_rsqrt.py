"""Error bound of the pivot reciprocal square root used by the diagonal-tile
Cholesky (the hardware estimate refined by one third-order step): within
1.5 units in the last place of 1/sqrt(d) over positive normal pivots, and NaN
for every pivot that is not a positive finite number (the factorization's
failure check reads NaN as a failed pivot).  The reference is 1/sqrt(d) in
the host's extended precision (64-bit significand), rounded only for the ulp
measure."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _gpu_rsqrt(torch, L, x):
    d_in = torch.from_numpy(x).to("cuda")
    d_out = torch.empty_like(d_in)
    L.bta_internal_rsqrt.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    L.bta_internal_rsqrt.restype = ctypes.c_int
    rc = L.bta_internal_rsqrt(d_in.data_ptr(), d_out.data_ptr(), x.size, torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    return d_out.cpu().numpy()


def _ulp_err(x, y):
    ref = np.longdouble(1.0) / np.sqrt(x.astype(np.longdouble))
    ulp = np.spacing(ref.astype(np.float64)).astype(np.longdouble)
    return np.abs(y.astype(np.longdouble) - ref) / ulp


def test_rsqrt_refined_error_bound():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_17528_amd import bta

    L = bta.lib()
    assert np.finfo(np.longdouble).nmant >= 63, "needs an extended-precision host long double"
    rng = np.random.default_rng(7)
    # every binade of the normal range (log-uniform), a dense sweep of [1, 4)
    # (both parities of the exponent), and the range pivots take in practice
    x = np.concatenate([
        np.exp(rng.uniform(np.log(np.finfo(np.float64).tiny), np.log(np.finfo(np.float64).max), 2_000_000)),
        rng.uniform(1.0, 4.0, 2_000_000),
        np.exp(rng.uniform(np.log(1e-6), np.log(1e6), 1_000_000)),
    ])
    x = x[np.isfinite(x) & (x >= np.finfo(np.float64).tiny)]
    y = _gpu_rsqrt(torch, L, x)
    e = _ulp_err(x, y)
    say(f"rsqrt_refined over {x.size} pivots: max {float(e.max()):.3f} ulp, mean {float(e.mean()):.3f} ulp")
    assert float(e.max()) <= 1.5

    bad = np.array([0.0, -0.0, -1.0, -1e-300, np.inf, -np.inf, np.nan])
    yb = _gpu_rsqrt(torch, L, bad)
    say(f"non-positive or non-finite pivots -> {yb}")
    # 0 gives inf * 0 inside the step, +inf gives 0 * inf: NaN either way
    assert np.all(np.isnan(yb)), yb
