"""GPU checks of the grouped FP64 MFMA GEMM used by the selected inversion
(internal entry point), against float64 torch products on the CPU: operand
layouts, triangular k ranges, lower / lower-plus-mirror stores, ragged edges,
and every kernel family (register-staged, direct-to-LDS 64 and 128 tiles)."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

TRI_NONE, TRI_K_GE_COL, TRI_K_GE_ROW, TRI_K_LE_ROW, TRI_K_LE_COL = 0, 1, 2, 3, 4
ST_FULL, ST_LOWER, ST_LOWER_MIRROR = 0, 1, 3


@pytest.fixture(scope="module")
def lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_17528_amd import bta

    L = bta.lib()
    L.bta_internal_gemm.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                                         ctypes.c_void_p]
    L.bta_internal_gemm.restype = ctypes.c_int
    return L


def _operands(rng, M, N, K, at, bt, tri):
    """Random operands in their stored layout; a triangular k range means the
    operand is zero outside that triangle (the kernel may skip the zeros)."""
    Am = rng.standard_normal((M, K))   # A(m, k)
    Bm = rng.standard_normal((N, K))   # B(c, k)
    k = np.arange(K)
    if tri == TRI_K_GE_COL:
        Bm = Bm * (k[None, :] >= np.arange(N)[:, None])
    elif tri == TRI_K_LE_COL:
        Bm = Bm * (k[None, :] <= np.arange(N)[:, None])
    elif tri == TRI_K_GE_ROW:
        Am = Am * (k[None, :] >= np.arange(M)[:, None])
    elif tri == TRI_K_LE_ROW:
        Am = Am * (k[None, :] <= np.arange(M)[:, None])
    A = np.ascontiguousarray(Am.T) if at else Am
    B = np.ascontiguousarray(Bm.T) if bt else Bm
    return A, B, Am @ Bm.T


CASES = [
    # M, N, K, at, bt, tri, store, lower_tiles
    (130, 70, 96, 0, 0, TRI_NONE, ST_FULL, 0),
    (200, 200, 150, 0, 1, TRI_NONE, ST_FULL, 0),
    (256, 256, 256, 1, 1, TRI_K_GE_ROW, ST_LOWER_MIRROR, 1),
    (192, 192, 192, 0, 1, TRI_K_GE_COL, ST_FULL, 0),
    (264, 256, 264, 0, 1, TRI_NONE, ST_FULL, 0),
    (256, 256, 264, 1, 0, TRI_NONE, ST_LOWER, 1),
    (8, 256, 256, 0, 1, TRI_NONE, ST_FULL, 0),
    (160, 160, 160, 0, 1, TRI_K_LE_ROW, ST_FULL, 0),
]


@pytest.mark.parametrize("mode", [1, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(str(v) for v in c))
def test_gemm_kernels_match_reference(lib, case, mode):
    import torch

    from paper_2503_17528_amd import bta

    M, N, K, at, bt, tri, store, lower_tiles = case
    say(f"case gemm mode={mode} {case}")
    rng = np.random.default_rng(hash(case) % (2 ** 31))
    A, B, prod = _operands(rng, M, N, K, at, bt, tri)
    Cin = rng.standard_normal((M, N)) if store == ST_FULL else rng.standard_normal((max(M, N), max(M, N)))[:M, :N].copy()
    alpha, beta = -1.0, (1.0 if store != ST_LOWER_MIRROR else 0.0)
    dA, dB = torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")
    dC = torch.tensor(Cin, device="cuda")
    prev = bta.gemm_mode(mode)
    try:
        rc = lib.bta_internal_gemm(M, N, K, dA.data_ptr(), A.shape[1], at, dB.data_ptr(), B.shape[1], bt, tri,
                                   dC.data_ptr() if beta != 0.0 else None, dC.data_ptr(), N, alpha, beta, store,
                                   lower_tiles, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        bta.gemm_mode(prev)
    assert rc == 0
    got = dC.cpu().numpy()
    ref = alpha * prod + (beta * Cin if beta != 0.0 else 0.0)
    if store == ST_FULL:
        err = np.abs(got - ref).max() / np.abs(ref).max()
    else:
        il = np.tril_indices(min(M, N))
        err = np.abs(got[il] - ref[il]).max() / np.abs(ref[il]).max()
        if store == ST_LOWER_MIRROR:
            assert np.array_equal(got[:N, :N], got[:N, :N].T)
        else:  # strict upper part untouched
            iu = np.triu_indices(min(M, N), 1)
            assert np.array_equal(got[iu], Cin[iu])
    say(f"   max rel err {err:.2e}")
    assert err < 1e-12


SPLIT_CASES = [
    # M, N, K, at, bt, store, lower_tiles, beta: the sweep's b x b product and its lower X_ii product
    (512, 512, 512, 0, 1, ST_FULL, 0, 0.0),
    (512, 512, 512, 1, 1, ST_LOWER_MIRROR, 1, 1.0),
    (520, 520, 520, 0, 1, ST_FULL, 0, 0.0),
    (256, 256, 264, 1, 1, ST_LOWER_MIRROR, 1, 1.0),
]


@pytest.mark.parametrize("case", SPLIT_CASES, ids=lambda c: "x".join(str(v) for v in c))
def test_gemm_split_k_matches_reference(lib, case):
    """The split-k path (partials over k ranges in one launch, then an
    in-order sum with alpha, beta and the store mode) against the product in
    float64 on the CPU."""
    import torch

    M, N, K, at, bt, store, lower_tiles, beta = case
    say(f"case gemm split-k {case}")
    L = lib
    L.bta_internal_gemm_split.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                                               ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                               ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                               ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                                               ctypes.POINTER(ctypes.c_int), ctypes.c_void_p]
    L.bta_internal_gemm_split.restype = ctypes.c_int
    rng = np.random.default_rng(hash(case) % (2 ** 31))
    A, B, prod = _operands(rng, M, N, K, at, bt, TRI_NONE)
    Cin = rng.standard_normal((M, N))
    if store != ST_FULL:
        Cin = Cin + Cin.T
    alpha = -1.0
    dA, dB = torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")
    dC = torch.tensor(Cin, device="cuda")
    ws = torch.empty(4 * M * N, dtype=torch.float64, device="cuda")
    splits = ctypes.c_int(0)
    rc = L.bta_internal_gemm_split(M, N, K, dA.data_ptr(), A.shape[1], at, dB.data_ptr(), B.shape[1], bt,
                                   dC.data_ptr() if beta != 0.0 else None, dC.data_ptr(), N, alpha, beta, store,
                                   lower_tiles, ws.data_ptr(), ws.numel(), ctypes.byref(splits),
                                   torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert rc == 0
    got = dC.cpu().numpy()
    ref = alpha * prod + (beta * Cin if beta != 0.0 else 0.0)
    if store == ST_FULL:
        err = np.abs(got - ref).max() / np.abs(ref).max()
    else:
        il = np.tril_indices(M)
        err = np.abs(got[il] - ref[il]).max() / np.abs(ref[il]).max()
        assert np.array_equal(got, got.T)
    say(f"   splits {splits.value}, max rel err {err:.2e}")
    assert splits.value >= 2
    assert err < 1e-12


SKINNY_CASES = [
    # M, N, K, K1, alpha, beta: the arrow-row product (a rows, K = b + a in two segments) and ragged edges
    (6, 384, 390, 384, -1.0, 0.0),
    (16, 200, 700, 300, 0.5, 1.5),
    (1, 64, 5, 0, 1.0, 0.0),
    (3, 1000, 33, 33, -1.0, 0.0),
    (11, 130, 257, 256, -1.0, 2.0),
]


@pytest.mark.parametrize("case", SKINNY_CASES, ids=lambda c: "x".join(str(v) for v in c))
def test_gemm_skinny_matches_reference(lib, case):
    """The skinny list kernel (at most 16 rows; one workgroup per 64 columns,
    k residues summed in a fixed order) against the product in float64 on the
    CPU, over two k segments, with alpha, beta and ragged column edges; run
    twice for identical bits."""
    import torch

    M, N, K, K1, alpha, beta = case
    say(f"case gemm skinny {case}")
    L = lib
    L.bta_internal_gemm_skinny.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                                                ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                                ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                                                ctypes.c_void_p, ctypes.c_void_p]
    L.bta_internal_gemm_skinny.restype = ctypes.c_int
    rng = np.random.default_rng(hash(case) % (2 ** 31))
    A = rng.standard_normal((M, K))     # A(m, k), by rows
    B = rng.standard_normal((K, N))     # B(c, k) stored as B[k, c]
    Cin = rng.standard_normal((M, N))
    dA, dB = torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")
    dlist = torch.empty(512, dtype=torch.uint8, device="cuda")
    outs = []
    for _ in range(2):
        dC = torch.tensor(Cin, device="cuda")
        rc = L.bta_internal_gemm_skinny(M, N, K, K1, dA.data_ptr(), K, dB.data_ptr(), N,
                                        dC.data_ptr() if beta != 0.0 else None, dC.data_ptr(), N, alpha, beta,
                                        dlist.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert rc == 0
        outs.append(dC.cpu().numpy())
    ref = alpha * (A @ B) + (beta * Cin if beta != 0.0 else 0.0)
    err = np.abs(outs[0] - ref).max() / np.abs(ref).max()
    say(f"   max rel err {err:.2e}")
    assert err < 1e-12
    assert np.array_equal(outs[0].view(np.int64), outs[1].view(np.int64))
    # more than 16 rows does not qualify
    assert L.bta_internal_gemm_skinny(17, N, K, K1, dA.data_ptr(), K, dB.data_ptr(), N, None, dC.data_ptr(), N,
                                      alpha, 0.0, dlist.data_ptr(), torch.cuda.current_stream().cuda_stream) == -1


LIST_CASES = [
    # M, N, K, at, bt, tri, store, lower_tiles, nprob: k loops of 1, 2, 3 and many stages (the deep
    # pipeline's tail waits), an odd K (the register-staged body), transposes, triangular k ranges,
    # lower stores and several problems per launch
    (64, 64, 16, 0, 1, TRI_NONE, ST_FULL, 0, 3),
    (70, 130, 32, 0, 1, TRI_NONE, ST_FULL, 0, 2),
    (128, 96, 48, 1, 0, TRI_NONE, ST_FULL, 0, 2),
    (384, 384, 390, 0, 1, TRI_NONE, ST_FULL, 0, 4),
    (256, 256, 256, 1, 1, TRI_K_GE_ROW, ST_LOWER_MIRROR, 1, 2),
    (192, 192, 192, 0, 1, TRI_K_GE_COL, ST_FULL, 0, 3),
    (200, 200, 5, 0, 1, TRI_NONE, ST_FULL, 0, 2),
]


@pytest.mark.parametrize("big", [0, 1])
@pytest.mark.parametrize("case", LIST_CASES, ids=lambda c: "x".join(str(v) for v in c))
def test_gemm_list_kernels_match_reference(lib, case, big):
    """The batched list kernels (64 x 64 tiles with four LDS stages, 128 x 128
    tiles) over several problems in one launch, against float64 products on
    the CPU."""
    import torch

    M, N, K, at, bt, tri, store, lower_tiles, nprob = case
    say(f"case gemm list big={big} {case}")
    L = lib
    L.bta_internal_gemm_list.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                                              ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                                              ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                              ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                                              ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                              ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                                              ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.bta_internal_gemm_list.restype = ctypes.c_int
    rng = np.random.default_rng(hash(case) % (2 ** 31))
    ops = [_operands(rng, M, N, K, at, bt, tri) for _ in range(nprob)]
    A = np.stack([o[0] for o in ops])
    B = np.stack([o[1] for o in ops])
    S = max(M, N)
    Cin = rng.standard_normal((nprob, M, N)) if store == ST_FULL else rng.standard_normal((nprob, S, S))[:, :M, :N].copy()
    alpha, beta = -1.0, (1.0 if store != ST_LOWER_MIRROR else 0.0)
    dA, dB = torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")
    dC = torch.tensor(Cin, device="cuda")
    dlist = torch.empty(512 * (nprob + 1), dtype=torch.uint8, device="cuda")
    rc = L.bta_internal_gemm_list(M, N, K, dA.data_ptr(), A.shape[2], at, dB.data_ptr(), B.shape[2], bt, tri,
                                  dC.data_ptr() if beta != 0.0 else None, dC.data_ptr(), N, alpha, beta, store,
                                  lower_tiles, nprob, A[0].size, B[0].size, M * N, big, dlist.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    got = dC.cpu().numpy()
    worst = 0.0
    for q in range(nprob):
        ref = alpha * ops[q][2] + (beta * Cin[q] if beta != 0.0 else 0.0)
        if store == ST_FULL:
            err = np.abs(got[q] - ref).max() / np.abs(ref).max()
        else:
            il = np.tril_indices(min(M, N))
            err = np.abs(got[q][il] - ref[il]).max() / np.abs(ref[il]).max()
            if store == ST_LOWER_MIRROR:
                assert np.array_equal(got[q][:N, :N], got[q][:N, :N].T)
        worst = max(worst, err)
    say(f"   max rel err {worst:.2e}")
    assert worst < 1e-12
