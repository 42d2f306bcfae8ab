"""ctypes binding of the C ABI in ``include/bta.h`` (argument marshalling only).

The raw entry points keep the C names (``bta_factor``, ``bta_selinv``,
``bta_solve``, ``bta_logdet``, ``bta_workspace_bytes``, ``bta_status_string``)
and take integers / raw device addresses.  ``factor``, ``selinv``, ``solve``
and ``logdet`` wrap them for contiguous float64 torch tensors on the current
HIP device and stream: they allocate outputs and workspace with torch and
pass pointers; every step of the computation runs in the HIP library.

The library must be built (``paper_2503_17528_amd.build``); there is no
fallback: if ``libbta.so`` is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbta.so")

BTA_OK, BTA_EINVAL, BTA_EHIP, BTA_ENOTSUP = 0, 1, 3, 4
# Binding-level code of NotPositiveDefinite: the C ABI reports a failed pivot
# on the device (d_info), never as a status.
NOT_POSITIVE_DEFINITE = 2
BTA_OP_FACTOR, BTA_OP_SELINV, BTA_OP_SOLVE, BTA_OP_LOGDET = 0, 1, 2, 3

EXPORTED = ("bta_workspace_bytes", "bta_factor", "bta_factor_noalloc", "bta_selinv", "bta_solve", "bta_logdet",
            "bta_logdet_quad", "bta_grad_logdet_quad", "bta_batched_workspace_bytes", "bta_factor_batched",
            "bta_selinv_batched", "bta_status_string", "bta_last_error")


class bta_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("b", ctypes.c_int64), ("a", ctypes.c_int64)] + \
               [(k, ctypes.c_void_p) for k in ("D", "B", "R", "T", "LD", "LB", "LR", "LT", "XD", "XB", "XR", "XT",
                                               "d_info")]

_lib = None


class BTAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class NotPositiveDefinite(BTAError):
    def __init__(self, row: int):
        super().__init__(NOT_POSITIVE_DEFINITE, f"matrix is not positive definite: first failing pivot at global row {row} (1-based)")
        self.row = row


def lib() -> ctypes.CDLL:
    """Load ``libbta.so`` (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run paper_2503_17528_amd.build.build())")
    L = ctypes.CDLL(LIB_PATH)
    i64, vp, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    L.bta_workspace_bytes.argtypes = [ctypes.c_int, i64, i64, i64, i64]
    L.bta_workspace_bytes.restype = sz
    L.bta_factor.argtypes = [i64, i64, i64] + [vp] * 8 + [vp, sz, vp, vp]
    L.bta_factor.restype = ctypes.c_int
    L.bta_factor_noalloc.argtypes = [i64, i64, i64] + [vp] * 8 + [vp, vp]
    L.bta_factor_noalloc.restype = ctypes.c_int
    L.bta_selinv.argtypes = [i64, i64, i64] + [vp] * 8 + [vp, sz, vp]
    L.bta_selinv.restype = ctypes.c_int
    L.bta_solve.argtypes = [i64, i64, i64] + [vp] * 4 + [vp, i64, vp, sz, vp]
    L.bta_solve.restype = ctypes.c_int
    L.bta_logdet.argtypes = [i64, i64, i64, vp, vp, vp, vp, sz, vp]
    L.bta_logdet.restype = ctypes.c_int
    L.bta_logdet_quad.argtypes = [i64, i64, i64, vp, vp, vp, vp, i64, vp, vp, sz, vp]
    L.bta_logdet_quad.restype = ctypes.c_int
    L.bta_grad_logdet_quad.argtypes = [i64, i64, i64] + [vp] * 5 + [i64, vp] + [vp] * 5 + [vp]
    L.bta_grad_logdet_quad.restype = ctypes.c_int
    L.bta_batched_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, vp]
    L.bta_batched_workspace_bytes.restype = sz
    L.bta_factor_batched.argtypes = [ctypes.c_int, vp, vp, sz, vp]
    L.bta_factor_batched.restype = ctypes.c_int
    L.bta_selinv_batched.argtypes = [ctypes.c_int, vp, vp, sz, vp]
    L.bta_selinv_batched.restype = ctypes.c_int
    L.bta_status_string.argtypes = [ctypes.c_int]
    L.bta_status_string.restype = ctypes.c_char_p
    L.bta_internal_gemm_mode.argtypes = [ctypes.c_int]
    L.bta_internal_gemm_mode.restype = ctypes.c_int
    L.bta_last_error.argtypes = []
    L.bta_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


# ---------------------------------------------------------------- raw entry points (C names)



def gemm_mode(mode: int = -1) -> int:
    """Select the GEMM kernels of the selected inversion (0 automatic,
    1 register-staged, 2 direct-to-LDS where the operands allow, 3 .. 7 one
    direct-to-LDS kernel: 64 / 128 tiles, lean 64 x 64 / 128 x 64 / 128 x 128);
    -1 only queries.  Returns the previous mode."""
    return int(lib().bta_internal_gemm_mode(int(mode)))

def bta_workspace_bytes(op: int, n: int, b: int, a: int, nrhs: int = 0) -> int:
    return int(lib().bta_workspace_bytes(op, n, b, a, nrhs))


def bta_factor(n, b, a, D, B, R, T, LD, LB, LR, LT, work, work_bytes, d_info, stream) -> int:
    return int(lib().bta_factor(n, b, a, D, B, R, T, LD, LB, LR, LT, work, work_bytes, d_info, stream))


def bta_factor_noalloc(n, b, a, D, B, R, T, LD, LB, LR, LT, d_info, stream) -> int:
    return int(lib().bta_factor_noalloc(n, b, a, D, B, R, T, LD, LB, LR, LT, d_info, stream))


def bta_selinv(n, b, a, LD, LB, LR, LT, XD, XB, XR, XT, work, work_bytes, stream) -> int:
    return int(lib().bta_selinv(n, b, a, LD, LB, LR, LT, XD, XB, XR, XT, work, work_bytes, stream))


def bta_solve(n, b, a, LD, LB, LR, LT, rhs, nrhs, work, work_bytes, stream) -> int:
    return int(lib().bta_solve(n, b, a, LD, LB, LR, LT, rhs, nrhs, work, work_bytes, stream))


def bta_logdet(n, b, a, LD, LT, d_out, work, work_bytes, stream) -> int:
    return int(lib().bta_logdet(n, b, a, LD, LT, d_out, work, work_bytes, stream))


def bta_logdet_quad(n, b, a, LD, LT, y, x, nrhs, d_out, work, work_bytes, stream) -> int:
    return int(lib().bta_logdet_quad(n, b, a, LD, LT, y, x, nrhs, d_out, work, work_bytes, stream))


def bta_grad_logdet_quad(n, b, a, XD, XB, XR, XT, x, nrhs, d_scale, GD, GB, GR, GT, gy, stream) -> int:
    return int(lib().bta_grad_logdet_quad(n, b, a, XD, XB, XR, XT, x, nrhs, d_scale, GD, GB, GR, GT, gy, stream))


def bta_batched_workspace_bytes(op, count, descs) -> int:
    return int(lib().bta_batched_workspace_bytes(op, count, descs))


def bta_factor_batched(count, descs, work, work_bytes, stream) -> int:
    return int(lib().bta_factor_batched(count, descs, work, work_bytes, stream))


def bta_selinv_batched(count, descs, work, work_bytes, stream) -> int:
    return int(lib().bta_selinv_batched(count, descs, work, work_bytes, stream))


def bta_status_string(status: int) -> str:
    return lib().bta_status_string(status).decode()


def bta_last_error() -> str:
    return lib().bta_last_error().decode()


# ---------------------------------------------------------------- torch wrappers


def _check(status: int, what: str):
    if status != BTA_OK:
        raise BTAError(status, f"{what}: {bta_status_string(status)}: {bta_last_error()}")


def _ptr(t) -> Optional[int]:
    if t is None or t.numel() == 0:
        return None
    return t.data_ptr()


def _stream(stream=None) -> Optional[int]:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream or None


def _dims(D, R, T) -> Tuple[int, int, int]:
    n, b = int(D.shape[0]), int(D.shape[1])
    a = int(T.shape[0]) if T is not None else 0
    return n, b, a


def _validate(t, shape, name):
    import torch

    if t is None:
        return
    if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != tuple(shape) or not t.is_cuda:
        raise ValueError(f"{name}: expected a contiguous float64 HIP tensor of shape {tuple(shape)}, "
                         f"got {tuple(t.shape)} {t.dtype} contiguous={t.is_contiguous()} device={t.device}")


def workspace(op: int, n: int, b: int, a: int, device, nrhs: int = 0):
    import torch

    nbytes = bta_workspace_bytes(op, n, b, a, nrhs)
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device), nbytes


def factor(D, B, R, T, out=None, work=None, stream=None, check: bool = True):
    """L = POBTAF(A).  Returns (LD, LB, LR, LT, info) with info a 0-dim int64
    device tensor; with ``check`` the call synchronizes and raises
    NotPositiveDefinite on a failed pivot.  ``out`` may be (D, B, R, T)
    itself for an in-place factorization."""
    import torch

    n, b, a = _dims(D, R, T)
    _validate(D, (n, b, b), "D"); _validate(B, (max(n - 1, 0), b, b), "B")
    _validate(R, (n, a, b), "R"); _validate(T, (a, a), "T")
    dev = D.device
    if out is None:
        out = (torch.empty_like(D), torch.empty_like(B), torch.empty_like(R), torch.empty_like(T))
    LD, LB, LR, LT = out
    info = torch.zeros((), dtype=torch.int64, device=dev)
    if work is None:
        work, nbytes = workspace(BTA_OP_FACTOR, n, b, a, dev)
    else:
        nbytes = work.numel()
    st = bta_factor(n, b, a, _ptr(D), _ptr(B), _ptr(R), _ptr(T), _ptr(LD), _ptr(LB), _ptr(LR), _ptr(LT),
                    work.data_ptr(), nbytes, info.data_ptr(), _stream(stream))
    _check(st, "bta_factor")
    if check:
        check_info(info)
    return LD, LB, LR, LT, info


def check_info(info) -> None:
    """Raise for a failed factorization: NotPositiveDefinite for a positive
    info (the 1-based row of the first bad pivot), BTAError for the watchdog's
    -1.  Synchronizes with the device (reads the 0-dim info tensor)."""
    v = int(info.item())
    if v > 0:
        raise NotPositiveDefinite(v)
    if v < 0:
        raise BTAError(BTA_EHIP, "bta_factor: progress watchdog fired")


def factor_noalloc(D, B, R, T, out=None, stream=None):
    """bta_factor_noalloc: L = POBTAF(A) with the library's fixed device
    scratch instead of a workspace (no allocation inside the call; problems
    above the scratch limit raise BTAError with BTA_EINVAL).  Returns
    (LD, LB, LR, LT, info) without synchronizing."""
    import torch

    n, b, a = _dims(D, R, T)
    _validate(D, (n, b, b), "D"); _validate(B, (max(n - 1, 0), b, b), "B")
    _validate(R, (n, a, b), "R"); _validate(T, (a, a), "T")
    if out is None:
        out = (torch.empty_like(D), torch.empty_like(B), torch.empty_like(R), torch.empty_like(T))
    LD, LB, LR, LT = out
    info = torch.zeros((), dtype=torch.int64, device=D.device)
    st = bta_factor_noalloc(n, b, a, _ptr(D), _ptr(B), _ptr(R), _ptr(T), _ptr(LD), _ptr(LB), _ptr(LR), _ptr(LT),
                            info.data_ptr(), _stream(stream))
    _check(st, "bta_factor_noalloc")
    return LD, LB, LR, LT, info


def selinv(LD, LB, LR, LT, out=None, work=None, stream=None):
    """X = POBTASI(L): blocks of A^{-1} at the BTA pattern.  ``out`` may be
    (LD, LB, LR, LT) itself for an in-place selected inversion."""
    import torch

    n, b, a = _dims(LD, LR, LT)
    _validate(LD, (n, b, b), "LD"); _validate(LB, (max(n - 1, 0), b, b), "LB")
    _validate(LR, (n, a, b), "LR"); _validate(LT, (a, a), "LT")
    if out is None:
        out = (torch.empty_like(LD), torch.empty_like(LB), torch.empty_like(LR), torch.empty_like(LT))
    XD, XB, XR, XT = out
    if work is None:
        work, nbytes = workspace(BTA_OP_SELINV, n, b, a, LD.device)
    else:
        nbytes = work.numel()
    st = bta_selinv(n, b, a, _ptr(LD), _ptr(LB), _ptr(LR), _ptr(LT), _ptr(XD), _ptr(XB), _ptr(XR), _ptr(XT),
                    work.data_ptr(), nbytes, _stream(stream))
    _check(st, "bta_selinv")
    return XD, XB, XR, XT


def solve(LD, LB, LR, LT, rhs, inplace: bool = False, work=None, stream=None):
    """x = A^{-1} rhs from the factor; rhs of shape (N,) or (N, nrhs)."""
    n, b, a = _dims(LD, LR, LT)
    N = n * b + a
    x = rhs if inplace else rhs.clone()
    vec = x.dim() == 1
    x2 = x.view(N, 1) if vec else x
    nrhs = int(x2.shape[1])
    _validate(x2, (N, nrhs), "rhs")
    if work is None:
        work, nbytes = workspace(BTA_OP_SOLVE, n, b, a, LD.device, nrhs)
    else:
        nbytes = work.numel()
    st = bta_solve(n, b, a, _ptr(LD), _ptr(LB), _ptr(LR), _ptr(LT), x2.data_ptr(), nrhs, work.data_ptr(), nbytes,
                   _stream(stream))
    _check(st, "bta_solve")
    return x


def logdet(LD, LT, work=None, stream=None):
    """log det A from the factor, as a 0-dim float64 device tensor."""
    import torch

    n, b = int(LD.shape[0]), int(LD.shape[1])
    a = int(LT.shape[0]) if LT is not None else 0
    out = torch.empty((), dtype=torch.float64, device=LD.device)
    if work is None:
        work, nbytes = workspace(BTA_OP_LOGDET, n, b, a, LD.device)
    else:
        nbytes = work.numel()
    st = bta_logdet(n, b, a, _ptr(LD), _ptr(LT), out.data_ptr(), work.data_ptr(), nbytes, _stream(stream))
    _check(st, "bta_logdet")
    return out


def logdet_quad(LD, LT, y, x, work=None, stream=None):
    """log det A + sum(y * x) (x = A^{-1} y) as a 0-dim float64 device tensor."""
    import torch

    n, b = int(LD.shape[0]), int(LD.shape[1])
    a = int(LT.shape[0]) if LT is not None else 0
    N = n * b + a
    y2 = y.reshape(N, -1)
    x2 = x.reshape(N, -1)
    nrhs = int(y2.shape[1])
    _validate(y2, (N, nrhs), "y")
    _validate(x2, (N, nrhs), "x")
    out = torch.empty((), dtype=torch.float64, device=LD.device)
    if work is None:
        work, nbytes = workspace(BTA_OP_LOGDET, n, b, a, LD.device)
    else:
        nbytes = work.numel()
    st = bta_logdet_quad(n, b, a, _ptr(LD), _ptr(LT), y2.data_ptr(), x2.data_ptr(), nrhs, out.data_ptr(),
                         work.data_ptr(), nbytes, _stream(stream))
    _check(st, "bta_logdet_quad")
    return out


def grad_logdet_quad(X, x, scale=None, out=None, want_gy=True, stream=None):
    """Gradient blocks (GD, GB, GR, GT, gy) of log det Q + y^T Q^{-1} y from the
    selected inverse X = (XD, XB, XR, XT) and x = Q^{-1} y.  ``scale`` is an
    optional 0-dim device tensor multiplying every gradient; ``out`` may be X
    itself (in place)."""
    import torch

    XD, XB, XR, XT = X
    n, b, a = _dims(XD, XR, XT)
    N = n * b + a
    x2 = x.reshape(N, -1)
    nrhs = int(x2.shape[1])
    _validate(x2, (N, nrhs), "x")
    if out is None:
        out = tuple(torch.empty_like(t) for t in X)
    GD, GB, GR, GT = out
    gy = torch.empty_like(x2) if want_gy else None
    if scale is not None:
        _validate(scale, (), "scale")
    st = bta_grad_logdet_quad(n, b, a, _ptr(XD), _ptr(XB), _ptr(XR), _ptr(XT), x2.data_ptr(), nrhs,
                              _ptr(scale) if scale is not None else None, _ptr(GD), _ptr(GB), _ptr(GR), _ptr(GT),
                              _ptr(gy), _stream(stream))
    _check(st, "bta_grad_logdet_quad")
    return GD, GB, GR, GT, (gy.reshape(x.shape) if gy is not None else None)


class Batch:
    """A batch of independent BTA matrices held as torch tensors: ``mats`` is
    a list of dicts with keys D, B, R, T (inputs).  Allocates L and X outputs
    and per-matrix info tensors, builds the descriptor array once, and runs
    the batched entry points."""

    def __init__(self, mats, inplace: bool = False):
        import torch

        self.mats = mats
        self.count = len(mats)
        arr = (bta_desc * self.count)()
        self.L, self.X, self.info = [], [], []
        for m, q in enumerate(mats):
            D, B, R, T = q["D"], q["B"], q["R"], q["T"]
            n, b, a = _dims(D, R, T)
            L = (D, B, R, T) if inplace else tuple(torch.empty_like(t) for t in (D, B, R, T))
            X = L if inplace else tuple(torch.empty_like(t) for t in (D, B, R, T))
            info = torch.zeros((), dtype=torch.int64, device=D.device)
            self.L.append(L); self.X.append(X); self.info.append(info)
            arr[m] = bta_desc(n, b, a, _ptr(D), _ptr(B), _ptr(R), _ptr(T), _ptr(L[0]), _ptr(L[1]), _ptr(L[2]),
                              _ptr(L[3]), _ptr(X[0]), _ptr(X[1]), _ptr(X[2]), _ptr(X[3]), info.data_ptr())
        self.descs = arr
        dev = mats[0]["D"].device
        nf = bta_batched_workspace_bytes(BTA_OP_FACTOR, self.count, ctypes.byref(arr))
        ns = bta_batched_workspace_bytes(BTA_OP_SELINV, self.count, ctypes.byref(arr))
        self.wf = torch.empty(max(nf, 1), dtype=torch.uint8, device=dev)
        self.ws = torch.empty(max(ns, 1), dtype=torch.uint8, device=dev)
        self.nf, self.ns = nf, ns

    def factor(self, stream=None, check: bool = True):
        st = bta_factor_batched(self.count, ctypes.byref(self.descs), self.wf.data_ptr(), self.nf, _stream(stream))
        _check(st, "bta_factor_batched")
        if check:
            for m, info in enumerate(self.info):
                v = int(info.item())
                if v != 0:
                    raise BTAError(NOT_POSITIVE_DEFINITE, f"matrix {m}: info={v}")
        return self.L

    def selinv(self, stream=None):
        st = bta_selinv_batched(self.count, ctypes.byref(self.descs), self.ws.data_ptr(), self.ns, _stream(stream))
        _check(st, "bta_selinv_batched")
        return self.X
