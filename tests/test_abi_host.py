"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol that include/bta.h declares, sizes its workspace, and rejects
invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bta.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"BTA_API\s+[\w\s\*]*?\b(bta_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def bta():
    from paper_2503_17528_amd import bta as m

    if not os.path.exists(m.LIB_PATH):
        pytest.fail("libbta.so is not built (run __graft_entry__.build())")
    m.lib()
    return m


def test_header_declares_the_four_operations():
    names = _declared()
    for n in ("bta_factor", "bta_selinv", "bta_solve", "bta_logdet", "bta_workspace_bytes", "bta_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol(bta):
    L = ctypes.CDLL(bta.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(bta.EXPORTED)


def test_workspace_bytes(bta):
    for op in range(4):
        assert bta.bta_workspace_bytes(op, 4, 64, 4, 1) > 0
    assert bta.bta_workspace_bytes(0, 0, 64, 4, 0) == 0      # n < 1
    assert bta.bta_workspace_bytes(0, 4, 0, 4, 0) == 0       # b < 1
    assert bta.bta_workspace_bytes(0, 4, 64, -1, 0) == 0     # a < 0
    assert bta.bta_workspace_bytes(9, 4, 64, 4, 0) == 0      # unknown op
    assert bta.bta_workspace_bytes(2, 4, 64, 4, 0) == 0      # solve needs nrhs >= 1
    # grows with the problem
    assert bta.bta_workspace_bytes(0, 8, 256, 4, 0) > bta.bta_workspace_bytes(0, 4, 256, 4, 0)


def test_status_strings(bta):
    for st in (bta.BTA_OK, bta.BTA_EINVAL, bta.BTA_EHIP, bta.BTA_ENOTSUP):
        assert bta.bta_status_string(st).startswith("BTA_")
    # 2 is not a status: a failed pivot is reported on the device (d_info)
    for st in (2, 99):
        assert "unknown" in bta.bta_status_string(st)


FAKE = 1 << 40  # never dereferenced: every call below fails validation first


def _factor(bta, n=2, b=8, a=2, ptrs=None, work=FAKE, wbytes=1 << 30, info=FAKE + 4096 * 64):
    base = [FAKE + k * (1 << 32) for k in range(8)] if ptrs is None else ptrs
    return bta.bta_factor(n, b, a, *base, work, wbytes, info, None)


def test_factor_rejects_bad_sizes(bta):
    assert _factor(bta, n=0) == bta.BTA_EINVAL
    assert _factor(bta, b=0) == bta.BTA_EINVAL
    assert _factor(bta, a=-1) == bta.BTA_EINVAL
    assert "invalid sizes" in bta.bta_last_error()


def test_factor_rejects_null_and_misaligned(bta):
    ptrs = [FAKE + k * (1 << 32) for k in range(8)]
    ptrs[0] = None
    assert _factor(bta, ptrs=ptrs) == bta.BTA_EINVAL
    assert "D is NULL" in bta.bta_last_error()
    ptrs = [FAKE + k * (1 << 32) for k in range(8)]
    ptrs[5] = FAKE + 5 * (1 << 32) + 4
    assert _factor(bta, ptrs=ptrs) == bta.BTA_EINVAL
    assert "aligned" in bta.bta_last_error()
    assert _factor(bta, info=None) == bta.BTA_EINVAL


def test_factor_rejects_partial_overlap_but_not_exact_aliasing(bta):
    ptrs = [FAKE + k * (1 << 32) for k in range(8)]
    ptrs[4] = ptrs[0] + 8  # LD overlaps D partially
    assert _factor(bta, ptrs=ptrs) == bta.BTA_EINVAL
    assert "overlaps" in bta.bta_last_error()
    ptrs = [FAKE + k * (1 << 32) for k in range(8)]
    ptrs[5] = ptrs[0]  # LB on top of D: not a pair
    assert _factor(bta, ptrs=ptrs) == bta.BTA_EINVAL
    # exact in-place aliasing passes argument checks; it then fails on the
    # workspace check below (too small), still before any device call
    ptrs = [FAKE + k * (1 << 32) for k in range(4)] * 2
    assert _factor(bta, ptrs=ptrs, wbytes=16) == bta.BTA_EINVAL
    assert "workspace too small" in bta.bta_last_error()


def test_factor_rejects_bad_workspace(bta):
    assert _factor(bta, work=None) == bta.BTA_EINVAL
    assert _factor(bta, work=FAKE + 8) == bta.BTA_EINVAL
    assert "256-byte" in bta.bta_last_error()


def test_a0_and_n1_accept_null_arrays(bta):
    # a = 0: R, T, LR, LT may be NULL; n = 1: B, LB may be NULL.  These pass
    # the array checks and stop at the (too small) workspace.
    p = [FAKE + k * (1 << 32) for k in range(8)]
    for k in (2, 3, 6, 7):
        p[k] = None
    assert bta.bta_factor(3, 8, 0, *p, FAKE, 16, FAKE + (9 << 32), None) == bta.BTA_EINVAL
    assert "workspace" in bta.bta_last_error()
    p = [FAKE + k * (1 << 32) for k in range(8)]
    for k in (1, 5):
        p[k] = None
    assert bta.bta_factor(1, 8, 2, *p, FAKE, 16, FAKE + (9 << 32), None) == bta.BTA_EINVAL
    assert "workspace" in bta.bta_last_error()


def test_selinv_solve_logdet_validate(bta):
    p = [FAKE + k * (1 << 32) for k in range(8)]
    assert bta.bta_selinv(0, 8, 2, *p, FAKE, 1 << 30, None) == bta.BTA_EINVAL
    q = list(p)
    q[4] = q[0] + 64
    assert bta.bta_selinv(2, 8, 2, *q, FAKE, 1 << 30, None) == bta.BTA_EINVAL
    assert bta.bta_solve(2, 8, 2, *p[:4], p[4], 0, FAKE, 1 << 30, None) == bta.BTA_EINVAL
    assert bta.bta_solve(2, 8, 2, *p[:4], p[0], 1, FAKE, 1 << 30, None) == bta.BTA_EINVAL  # rhs overlaps LD
    assert bta.bta_logdet(2, 8, 2, p[0], p[3], None, FAKE, 1 << 30, None) == bta.BTA_EINVAL
    assert bta.bta_logdet(2, 8, 2, p[0], p[3], p[1], FAKE, 1, None) == bta.BTA_EINVAL


def test_build_rejects_scratch_kernels():
    """The build's parser of the compiler's per-kernel resource report flags
    every kernel with scratch and only those."""
    from paper_2503_17528_amd import build

    lines = [
        "gemm.hip:1:1: remark: Function Name: _Zk1 [-Rpass-analysis=kernel-resource-usage]",
        "gemm.hip:1:1: remark:     VGPRs: 104 [-Rpass-analysis=kernel-resource-usage]",
        "gemm.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "gemm.hip:9:1: remark: Function Name: _Zk2 [-Rpass-analysis=kernel-resource-usage]",
        "gemm.hip:9:1: remark:     ScratchSize [bytes/lane]: 352 [-Rpass-analysis=kernel-resource-usage]",
    ]
    assert build.scratch_kernels(lines) == [("_Zk2", 352)]
    assert build.scratch_kernels(lines[:3]) == []


def test_factor_noalloc_rejects_problems_above_its_scratch(bta):
    """The fixed-scratch factorization refuses problems whose scratch exceeds
    its limit before any HIP work (host-only: fake, aligned, disjoint device
    addresses)."""
    import ctypes as ct

    n, b, a = 64, 2048, 8
    assert bta.bta_workspace_bytes(bta.BTA_OP_FACTOR, n, b, a, 0) > (64 << 20)
    base = 1 << 44
    span = 1 << 36
    p = [base + k * span for k in range(9)]
    st = bta.bta_factor_noalloc(n, b, a, *p[:8], p[8], None)
    assert st == bta.BTA_EINVAL
    assert "scratch" in bta.bta_last_error()
    # a small problem passes the size check (and then needs a device)
    assert bta.bta_workspace_bytes(bta.BTA_OP_FACTOR, 4, 64, 2, 0) <= (64 << 20)
