"""CPU FP64 oracle for the BTA block Cholesky and selected inversion.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here.  The
product path (the HIP library and its binding) never touches this module, and
this module imports nothing from the product path: the two share no code.

Plain, slow, obviously correct numpy/scipy code in float64.  Each block step is
a LAPACK/BLAS call (POTRF, TRSM, GEMM), exactly as the paper describes its own
block operations, in the order of the paper's listings:

* ``pobtaf``  -- Algorithm 1 (POBTAF), block-sequential Cholesky factorization.
* ``pobtasi`` -- Algorithm 2 (POBTASI), block-sequential selected inversion.
* ``pobtas``  -- block forward/back substitution with the factor (not in the
  paper; the textbook triangular solves with the BTA factor).
* ``logdet``  -- ``2 * sum(log diag L)`` over all diagonal blocks and the tip.
* ``grad_logdet_quad`` -- blocks of ``G = Sigma - x x^T`` restricted to the BTA
  pattern, the gradient of ``f(Q) = logdet Q + y^T Q^{-1} y``.
* ``dense``/``pattern`` helpers assemble the full matrix for brute-force checks.

Readings of the paper taken here (its text is silent or ambiguous on them):

* "TRSM" in Algorithm 1 is the right-side solve ``X = A_{j,i} L_ii^{-T}``: it
  follows from ``A_{j,i} = L_{j,i} L_ii^T``.
* "TRSM" in Algorithm 2 is the right-side solve ``X = U L_ii^{-1}``: it follows
  from ``Sigma L = L^{-T}`` read block column by block column.
* The dagger is the plain transpose (real FP64 matrices).
* Only the lower triangles of the diagonal blocks and the tip are read; ``L``
  has exact zeros above its diagonal; ``X_ii`` and ``X_nn`` are returned as
  full symmetric blocks (lower triangle mirrored).
* Cholesky needs strict positive definiteness.  A non-positive or non-finite
  pivot is reported LAPACK-style as the 1-based global row of the first
  failing pivot (tip rows are ``n*b+1 .. n*b+a``).
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack


# ----------------------------------------------------------------------------
# dense block primitives (one LAPACK/BLAS call each)


def _potrf(A: np.ndarray) -> Tuple[np.ndarray, int]:
    """Lower Cholesky factor of the lower triangle of ``A`` (LAPACK dpotrf).
    Returns (L, info) with info = 1-based order of the first non-positive
    leading minor, 0 on success."""
    m = A.shape[0]
    if m == 0:
        return np.zeros((0, 0)), 0
    c, info = lapack.dpotrf(np.array(A, dtype=np.float64, order="F"), lower=1, clean=1)
    c = np.tril(np.asarray(c))
    info = int(info)
    # A non-finite pivot is a failed pivot too (some LAPACK builds only test
    # d <= 0, which a NaN passes): report the first non-finite diagonal entry.
    upto = m if info == 0 else info - 1
    bad = np.nonzero(~np.isfinite(np.diagonal(c)[:upto]))[0]
    if bad.size:
        info = int(bad[0]) + 1
    return c, info


def _trsm_right_lower_trans(L: np.ndarray, Bm: np.ndarray) -> np.ndarray:
    """X with X L^T = Bm, i.e. X = Bm L^{-T} (right side, lower, transposed)."""
    if Bm.size == 0:
        return np.zeros_like(Bm)
    # X L^T = Bm  <=>  L X^T = Bm^T
    return sla.solve_triangular(L, Bm.T, lower=True, trans="N").T


def _trsm_right_lower(L: np.ndarray, U: np.ndarray) -> np.ndarray:
    """X with X L = U, i.e. X = U L^{-1} (right side, lower, no transpose)."""
    if U.size == 0:
        return np.zeros_like(U)
    # X L = U  <=>  L^T X^T = U^T
    return sla.solve_triangular(L, U.T, lower=True, trans="T").T


def _inv_lower(L: np.ndarray) -> np.ndarray:
    m = L.shape[0]
    if m == 0:
        return np.zeros((0, 0))
    return sla.solve_triangular(L, np.eye(m), lower=True)


def _sym_from_lower(X: np.ndarray) -> np.ndarray:
    lo = np.tril(X)
    return lo + np.tril(X, -1).T


# ----------------------------------------------------------------------------
# Algorithm 1: POBTAF


def pobtaf(D, B, R, T) -> Dict[str, np.ndarray]:
    """Block Cholesky factorization of a BTA matrix (Algorithm 1, POBTAF).

    Inputs are the blocks of ``A`` (D[n,b,b], B[n-1,b,b], R[n,a,b], T[a,a]);
    they are not modified.  Returns ``{"LD","LB","LR","LT","info"}``.  On a
    failed pivot, ``info`` is the 1-based global row and the returned blocks
    hold whatever had been computed so far."""
    A_D = np.array(D, dtype=np.float64, copy=True)
    A_B = np.array(B, dtype=np.float64, copy=True)
    A_R = np.array(R, dtype=np.float64, copy=True)
    A_T = np.array(T, dtype=np.float64, copy=True)
    n, b = A_D.shape[0], A_D.shape[1]
    a = A_T.shape[0]
    LD = np.zeros_like(A_D)
    LB = np.zeros_like(A_B)
    LR = np.zeros_like(A_R)
    out = {"LD": LD, "LB": LB, "LR": LR, "LT": np.zeros_like(A_T), "info": 0}

    # forward pass over the first n-1 block columns
    for i in range(n - 1):
        LD[i], info = _potrf(A_D[i])                               # L_ii = POTRF(A_ii)
        if info:
            out["info"] = i * b + info
            return out
        LB[i] = _trsm_right_lower_trans(LD[i], A_B[i])              # L_{i+1,i} = A_{i+1,i} L_ii^{-T}
        LR[i] = _trsm_right_lower_trans(LD[i], A_R[i])              # L_{n,i}   = A_{n,i}   L_ii^{-T}
        A_D[i + 1] -= LB[i] @ LB[i].T                               # A_{i+1,i+1} -= L_{i+1,i} L_{i+1,i}^T
        A_R[i + 1] -= LR[i] @ LB[i].T                               # A_{n,i+1}   -= L_{n,i} L_{i+1,i}^T
        A_T -= LR[i] @ LR[i].T                                      # A_{n,n}     -= L_{n,i} L_{n,i}^T

    # last block column, then the tip
    LD[n - 1], info = _potrf(A_D[n - 1])
    if info:
        out["info"] = (n - 1) * b + info
        return out
    LR[n - 1] = _trsm_right_lower_trans(LD[n - 1], A_R[n - 1])
    A_T -= LR[n - 1] @ LR[n - 1].T
    out["LT"], info = _potrf(A_T)
    if info:
        out["info"] = n * b + info
    return out


# ----------------------------------------------------------------------------
# Algorithm 2: POBTASI


def pobtasi(LD, LB, LR, LT) -> Dict[str, np.ndarray]:
    """Selected inversion of a BTA matrix from its block Cholesky factor
    (Algorithm 2, POBTASI): the blocks of ``Sigma = A^{-1}`` at the nonzero
    block positions of ``A``.  Returns ``{"XD","XB","XR","XT"}``."""
    LD = np.asarray(LD, dtype=np.float64)
    LB = np.asarray(LB, dtype=np.float64)
    LR = np.asarray(LR, dtype=np.float64)
    LT = np.asarray(LT, dtype=np.float64)
    n, b = LD.shape[0], LD.shape[1]
    a = LT.shape[0]
    XD = np.zeros_like(LD)
    XB = np.zeros_like(LB)
    XR = np.zeros_like(LR)

    # X_nn = L_nn^{-T} L_nn^{-1}
    Wt = _inv_lower(LT)
    XT = Wt.T @ Wt
    XT = _sym_from_lower(XT)

    # last block column (i = n-1)
    j = n - 1
    U = -XT @ LR[j]                                                 # U_{n,n-1} = -X_nn L_{n,n-1}
    XR[j] = _trsm_right_lower(LD[j], U)                             # X_{n,n-1} = U L_{n-1,n-1}^{-1}
    U = _inv_lower(LD[j]).T - XR[j].T @ LR[j]                       # U_{n-1,n-1}
    XD[j] = _sym_from_lower(_trsm_right_lower(LD[j], U))            # X_{n-1,n-1}

    # backward pass
    for i in range(n - 2, -1, -1):
        U = -XD[i + 1] @ LB[i] - XR[i + 1].T @ LR[i]                # U_{i+1,i}
        XB[i] = _trsm_right_lower(LD[i], U)                         # X_{i+1,i}
        U = -XR[i + 1] @ LB[i] - XT @ LR[i]                         # U_{n,i}
        XR[i] = _trsm_right_lower(LD[i], U)                         # X_{n,i}
        U = _inv_lower(LD[i]).T - XB[i].T @ LB[i] - XR[i].T @ LR[i] # U_{i,i}
        XD[i] = _sym_from_lower(_trsm_right_lower(LD[i], U))        # X_{i,i}
    return {"XD": XD, "XB": XB, "XR": XR, "XT": XT}


# ----------------------------------------------------------------------------
# Triangular solves with the factor and the log-determinant (not in the paper)


def pobtas(LD, LB, LR, LT, rhs) -> np.ndarray:
    """Solve ``A x = rhs`` with the BTA factor: ``z = L^{-1} rhs`` by block
    forward substitution, then ``x = L^{-T} z`` by block back substitution.
    ``rhs`` has shape (N,) or (N, nrhs) with N = n*b + a."""
    LD = np.asarray(LD, dtype=np.float64)
    LB = np.asarray(LB, dtype=np.float64)
    LR = np.asarray(LR, dtype=np.float64)
    LT = np.asarray(LT, dtype=np.float64)
    n, b = LD.shape[0], LD.shape[1]
    a = LT.shape[0]
    y = np.array(rhs, dtype=np.float64, copy=True)
    vec = y.ndim == 1
    if vec:
        y = y[:, None]
    z = np.zeros_like(y)
    blk = lambda i: slice(i * b, (i + 1) * b)
    tip = slice(n * b, n * b + a)

    def lsolve(L, v, trans):
        if v.size == 0:
            return v.copy()
        return sla.solve_triangular(L, v, lower=True, trans=trans)

    # forward: z_i = L_ii^{-1} (y_i - L_{i,i-1} z_{i-1});  z_n = L_nn^{-1} (y_n - sum_i L_{n,i} z_i)
    acc_tip = y[tip].copy()
    for i in range(n):
        v = y[blk(i)].copy()
        if i > 0:
            v -= LB[i - 1] @ z[blk(i - 1)]
        z[blk(i)] = lsolve(LD[i], v, "N")
        acc_tip -= LR[i] @ z[blk(i)]
    z[tip] = lsolve(LT, acc_tip, "N")

    # backward: x_n = L_nn^{-T} z_n;  x_i = L_ii^{-T} (z_i - L_{i+1,i}^T x_{i+1} - L_{n,i}^T x_n)
    x = np.zeros_like(z)
    x[tip] = lsolve(LT, z[tip], "T")
    for i in range(n - 1, -1, -1):
        v = z[blk(i)] - LR[i].T @ x[tip]
        if i < n - 1:
            v -= LB[i].T @ x[blk(i + 1)]
        x[blk(i)] = lsolve(LD[i], v, "T")
    return x[:, 0] if vec else x


def logdet(LD, LT) -> float:
    """``log det A = 2 * sum_k log L_kk`` over every diagonal block and the tip
    (pairwise summation of the logs)."""
    d = [np.log(np.diagonal(np.asarray(LD, dtype=np.float64), axis1=1, axis2=2)).ravel(),
         np.log(np.diagonal(np.asarray(LT, dtype=np.float64)))]
    return float(2.0 * np.sum(np.concatenate(d)))


def grad_logdet_quad(X: Dict[str, np.ndarray], x: np.ndarray, n: int, b: int, a: int) -> Dict[str, np.ndarray]:
    """Gradient blocks of ``f = logdet Q + y^T Q^{-1} y`` with respect to the
    block arrays, where ``Q_ii = (D_i + D_i^T)/2``, ``Q_nn = (T + T^T)/2`` and
    the lower blocks B_i, R_i also stand at their mirrored upper positions:
    with ``G = Sigma - x x^T`` (``x = Q^{-1} y``) restricted to the pattern,
    grad_D = G_D, grad_T = G_T, grad_B = 2 G_B, grad_R = 2 G_R."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    xb = lambda i: x[i * b:(i + 1) * b]
    xn = x[n * b:n * b + a]
    gD = np.stack([X["XD"][i] - np.outer(xb(i), xb(i)) for i in range(n)])
    gB = np.stack([2.0 * (X["XB"][i] - np.outer(xb(i + 1), xb(i))) for i in range(n - 1)]) if n > 1 else np.zeros((0, b, b))
    gR = np.stack([2.0 * (X["XR"][i] - np.outer(xn, xb(i))) for i in range(n)])
    gT = X["XT"] - np.outer(xn, xn)
    return {"D": gD, "B": gB, "R": gR, "T": gT}


# ----------------------------------------------------------------------------
# dense assembly / pattern extraction (for brute-force checks at tiny sizes)


def dense(D, B, R, T) -> np.ndarray:
    """The full symmetric N x N matrix of a BTA block set (lower triangles of
    D and T mirrored; B and R mirrored into the upper blocks)."""
    D = np.asarray(D, dtype=np.float64)
    n, b = D.shape[0], D.shape[1]
    T = np.asarray(T, dtype=np.float64)
    a = T.shape[0]
    N = n * b + a
    Q = np.zeros((N, N))
    for i in range(n):
        s = slice(i * b, (i + 1) * b)
        Q[s, s] = _sym_from_lower(D[i])
        if i < n - 1:
            s1 = slice((i + 1) * b, (i + 2) * b)
            Q[s1, s] = B[i]
            Q[s, s1] = np.asarray(B[i]).T
        Q[n * b:, s] = R[i]
        Q[s, n * b:] = np.asarray(R[i]).T
    Q[n * b:, n * b:] = _sym_from_lower(T)
    return Q


def dense_lower_factor(LD, LB, LR, LT) -> np.ndarray:
    """The full N x N lower-triangular matrix of a BTA factor."""
    LD = np.asarray(LD, dtype=np.float64)
    n, b = LD.shape[0], LD.shape[1]
    a = np.asarray(LT).shape[0]
    N = n * b + a
    L = np.zeros((N, N))
    for i in range(n):
        s = slice(i * b, (i + 1) * b)
        L[s, s] = np.tril(LD[i])
        if i < n - 1:
            L[(i + 1) * b:(i + 2) * b, s] = LB[i]
        L[n * b:, s] = LR[i]
    L[n * b:, n * b:] = np.tril(LT)
    return L


def pattern(M: np.ndarray, n: int, b: int, a: int) -> Dict[str, np.ndarray]:
    """Blocks of a full N x N matrix at the BTA pattern positions."""
    D = np.stack([M[i * b:(i + 1) * b, i * b:(i + 1) * b] for i in range(n)])
    B = np.stack([M[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] for i in range(n - 1)]) if n > 1 else np.zeros((0, b, b))
    R = np.stack([M[n * b:, i * b:(i + 1) * b] for i in range(n)])
    T = M[n * b:, n * b:].copy()
    return {"D": D, "B": B, "R": R, "T": T}


def rel_block_errors(got: Dict[str, np.ndarray], ref: Dict[str, np.ndarray], keys=("D", "B", "R", "T"),
                     lower_keys=("D", "T")) -> Dict[str, float]:
    """Max over blocks of ``||got - ref||_F / ||ref||_F`` per block type
    (lower triangles for the symmetric/triangular slots).  A block whose
    reference norm is below 1e-300 is compared absolutely against the mean
    block norm of its type."""
    res = {}
    for k in keys:
        g = np.asarray(got[k], dtype=np.float64)
        r = np.asarray(ref[k], dtype=np.float64)
        if r.size == 0:
            res[k] = 0.0
            continue
        if r.ndim == 2:
            g, r = g[None], r[None]
        if k in lower_keys:
            g = np.tril(g)
            r = np.tril(r)
        diff = np.sqrt(np.sum((g - r) ** 2, axis=(1, 2)))
        nrm = np.sqrt(np.sum(r ** 2, axis=(1, 2)))
        mean = max(float(np.mean(nrm)), 1e-300)
        e = np.where(nrm > 1e-300, diff / np.maximum(nrm, 1e-300), diff / mean)
        res[k] = float(np.max(e))
    return res
