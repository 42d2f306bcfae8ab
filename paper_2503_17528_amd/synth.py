"""Seeded synthetic BTA inputs shared by the tests, the bench and the smoke run.

This module only draws random numbers and assembles ``Q = L L^T`` from a
randomly drawn block lower-triangular factor ``L`` with the BTA pattern.  It
holds none of the factorization or selected-inversion arithmetic, so both the
CPU oracle and the HIP path can take their inputs from here.

Block storage (row-major, contiguous, float64), for a BTA matrix with ``n``
diagonal blocks of size ``b`` and an arrow tip of size ``a`` (the paper's
notation, Section 2.1, Table 2; total size ``N = n*b + a``):

* ``D[n, b, b]``   diagonal blocks ``A_{i,i}`` (only the lower triangle is read)
* ``B[n-1, b, b]`` lower blocks ``A_{i+1,i}``
* ``R[n, a, b]``   arrowhead blocks ``A_{n,i}`` (last block row)
* ``T[a, a]``      arrow tip ``A_{n,n}`` (only the lower triangle is read)

The factor drawn here follows the recipe of the synthetic workloads: ``L_ii``
lower triangular with diagonal ``U[lo, hi]`` and strictly-lower entries
``N(0, s_diag^2)``; ``L_{i+1,i}`` and ``L_{n,i}`` dense ``N(0, (0.1/sqrt(b))^2)``;
the tip factor lower triangular with diagonal ``U[lo, hi]``.  Two readings of
the off-diagonal spread inside ``L_ii`` exist: ``literal`` uses standard
deviation 0.1, ``scaled`` uses 0.1/sqrt(b) (needed at b >= 2048, where the
literal reading makes the inverse grow by orders of magnitude per block and
no FP64 method can reach 1e-10 relative accuracy).

Every block is drawn from its own seed ``(seed, kind, i)``, so any block can be
regenerated on its own (streaming for very large workloads).  On the CPU the
stream is numpy's PCG64 (``default_rng(SeedSequence([seed, kind, i]))``); on a
GPU device it is torch's Philox generator seeded with a mix of the same triple.
The two streams differ: a given (workload, seed, device) names one matrix, and
whoever checks a result receives a host copy of the exact input.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

KIND_DIAG, KIND_SUB, KIND_ARROW, KIND_TIP, KIND_RHS, KIND_BATCH = 0, 1, 2, 3, 4, 5


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and value recipe of one synthetic BTA matrix."""

    name: str
    n: int
    b: int
    a: int
    diag_lo: float = 1.0
    diag_hi: float = 2.0
    reading: str = "literal"  # "literal" | "scaled"

    @property
    def N(self) -> int:
        return self.n * self.b + self.a

    @property
    def diag_offdiag_std(self) -> float:
        return 0.1 if self.reading == "literal" else 0.1 / math.sqrt(self.b)

    @property
    def tip_offdiag_std(self) -> float:
        if self.reading == "literal" or self.a == 0:
            return 0.1
        return 0.1 / math.sqrt(self.a)

    @property
    def coupling_std(self) -> float:
        return 0.1 / math.sqrt(self.b)

    def block_bytes(self) -> int:
        n, b, a = self.n, self.b, self.a
        return 8 * (n * b * b + (n - 1) * b * b + n * a * b + a * a)

    def flops(self) -> Dict[str, float]:
        """Minimum-work algorithmic flop count of the factorization and the
        selected inversion (triangular/symmetric products counted at half
        price), the count the throughput metric divides by."""
        n, b, a = float(self.n), float(self.b), float(self.a)
        f_fact = n * (b ** 3 / 3 + a * b * b + a * a * b) + (n - 1) * (2 * b ** 3 + 2 * a * b * b) + a ** 3 / 3
        f_si = n * (2 * b ** 3 / 3 + 2 * a * b * b + 2 * a * a * b) + (n - 1) * (4 * b ** 3 + 4 * a * b * b) + 2 * a ** 3 / 3
        return {"factor": f_fact, "selinv": f_si, "total": f_fact + f_si}


def workload(n: int, b: int, a: int, reading: str = "literal", diag=(1.0, 2.0), name: Optional[str] = None) -> Workload:
    if name is None:
        name = f"bta_n{n}_b{b}_a{a}_{reading}"
    return Workload(name=name, n=n, b=b, a=a, diag_lo=float(diag[0]), diag_hi=float(diag[1]), reading=reading)


# The synthetic workloads (shapes of spatio-temporal GMRF precision matrices:
# b spatial nodes per time step, n time steps, a fixed effects).
SMALL = workload(16, 64, 4, "literal", name="bta_n16_b64_a4")
BENCH = workload(128, 2048, 8, "scaled", name="bta_n128_b2048_a8")
AUTOGRAD = workload(256, 512, 4, "literal", name="bta_n256_b512_a4")
LARGE = workload(256, 4096, 16, "scaled", diag=(1.0, 3.0), name="bta_n256_b4096_a16")
# wide arrowhead, the shape of the paper's synthetic scaling set (b = 1024, a = 256, largest n)
ARROW = workload(512, 1024, 256, "scaled", name="bta_n512_b1024_a256")


def batched_workloads(seed: int, count: int = 64) -> list:
    """Draw ``count`` independent workloads: n ~ U{16..96}, b in {128,256,384},
    a in {2,4,6} (the hyper-parameter-sweep batch)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, KIND_BATCH, 99]))
    out = []
    for j in range(count):
        n = int(rng.integers(16, 97))
        b = int(rng.choice([128, 256, 384]))
        a = int(rng.choice([2, 4, 6]))
        out.append(workload(n, b, a, "literal", name=f"batch{j}_n{n}_b{b}_a{a}"))
    return out


# ----------------------------------------------------------------------------
# CPU (numpy) draw


def _rng(seed: int, kind: int, i: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(kind), int(i)]))


def _lower_block_np(rng, m: int, lo: float, hi: float, std: float) -> np.ndarray:
    x = np.tril(rng.standard_normal((m, m)) * std, -1)
    x[np.diag_indices(m)] = rng.uniform(lo, hi, size=m)
    return x


def factor_block_np(wl: Workload, seed: int, kind: int, i: int) -> np.ndarray:
    """Regenerate one block of the drawn factor on the CPU."""
    b, a = wl.b, wl.a
    rng = _rng(seed, kind, i)
    if kind == KIND_DIAG:
        return _lower_block_np(rng, b, wl.diag_lo, wl.diag_hi, wl.diag_offdiag_std)
    if kind == KIND_SUB:
        return rng.standard_normal((b, b)) * wl.coupling_std
    if kind == KIND_ARROW:
        return rng.standard_normal((a, b)) * wl.coupling_std
    if kind == KIND_TIP:
        return _lower_block_np(rng, a, wl.diag_lo, wl.diag_hi, wl.tip_offdiag_std)
    raise ValueError(kind)


def factor_np(wl: Workload, seed: int) -> Dict[str, np.ndarray]:
    """The drawn factor ``L`` as block arrays LD, LB, LR, LT (numpy)."""
    n, b, a = wl.n, wl.b, wl.a
    LD = np.empty((n, b, b))
    LB = np.empty((max(n - 1, 0), b, b))
    LR = np.empty((n, a, b))
    for i in range(n):
        LD[i] = factor_block_np(wl, seed, KIND_DIAG, i)
        LR[i] = factor_block_np(wl, seed, KIND_ARROW, i)
        if i < n - 1:
            LB[i] = factor_block_np(wl, seed, KIND_SUB, i)
    LT = factor_block_np(wl, seed, KIND_TIP, 0)
    return {"LD": LD, "LB": LB, "LR": LR, "LT": LT}


def assemble_np(L: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    """Q = L L^T blockwise (exactly the BTA pattern, since the pattern is
    closed under this product)."""
    LD, LB, LR, LT = L["LD"], L["LB"], L["LR"], L["LT"]
    n, b = LD.shape[0], LD.shape[1]
    a = LT.shape[0]
    D = np.empty_like(LD)
    B = np.empty_like(LB)
    R = np.empty_like(LR)
    T = LT @ LT.T
    for i in range(n):
        D[i] = LD[i] @ LD[i].T
        R[i] = LR[i] @ LD[i].T
        if i > 0:
            D[i] += LB[i - 1] @ LB[i - 1].T
            R[i] += LR[i - 1] @ LB[i - 1].T
        if i < n - 1:
            B[i] = LB[i] @ LD[i].T
        T += LR[i] @ LR[i].T
    # exact symmetry of the symmetric blocks
    D = 0.5 * (D + np.transpose(D, (0, 2, 1)))
    T = 0.5 * (T + T.T)
    return {"D": D, "B": B, "R": R, "T": T}


def make_np(wl: Workload, seed: int, with_factor: bool = False) -> Dict[str, np.ndarray]:
    L = factor_np(wl, seed)
    Q = assemble_np(L)
    if with_factor:
        Q.update(L)
    return Q


def rhs_np(wl: Workload, seed: int, nrhs: int = 1) -> np.ndarray:
    """y ~ N(0, 1), shape (N, nrhs)."""
    return _rng(seed, KIND_RHS, 0).standard_normal((wl.N, nrhs))


# ----------------------------------------------------------------------------
# Device (torch) draw, for workloads too large to draw on the host


def _torch_seed(seed: int, kind: int, i: int) -> int:
    # splitmix64 finaliser over the packed triple: a distinct 63-bit seed per block
    z = (int(seed) * 0x9E3779B97F4A7C15 + int(kind) * 0xBF58476D1CE4E5B9 + int(i) * 0x94D049BB133111EB) & (2**64 - 1)
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & (2**64 - 1)
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & (2**64 - 1)
    z ^= z >> 31
    return z & (2**63 - 1)


def factor_block_torch(wl: Workload, seed: int, kind: int, i: int, device):
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(_torch_seed(seed, kind, i))
    f64 = torch.float64
    b, a = wl.b, wl.a

    def lower(m, std):
        x = torch.randn((m, m), generator=g, device=device, dtype=f64).mul_(std).tril_(-1)
        d = torch.rand((m,), generator=g, device=device, dtype=f64).mul_(wl.diag_hi - wl.diag_lo).add_(wl.diag_lo)
        x.diagonal().copy_(d)
        return x

    if kind == KIND_DIAG:
        return lower(b, wl.diag_offdiag_std)
    if kind == KIND_SUB:
        return torch.randn((b, b), generator=g, device=device, dtype=f64).mul_(wl.coupling_std)
    if kind == KIND_ARROW:
        return torch.randn((a, b), generator=g, device=device, dtype=f64).mul_(wl.coupling_std)
    if kind == KIND_TIP:
        return lower(a, wl.tip_offdiag_std)
    raise ValueError(kind)


def make_torch(wl: Workload, seed: int, device, with_factor: bool = False, out: Optional[dict] = None,
               progress=None):
    """Draw the factor on ``device`` block by block and assemble ``Q = L L^T``
    there.  Only two factor block-columns are alive at a time unless
    ``with_factor`` is set.  ``out`` may pass preallocated D, B, R, T;
    ``progress(done, n)`` (optional) is called every 32 blocks."""
    import torch

    n, b, a = wl.n, wl.b, wl.a
    f64 = torch.float64
    if out is None:
        out = {
            "D": torch.empty((n, b, b), device=device, dtype=f64),
            "B": torch.empty((max(n - 1, 0), b, b), device=device, dtype=f64),
            "R": torch.empty((n, a, b), device=device, dtype=f64),
            "T": torch.empty((a, a), device=device, dtype=f64),
        }
    D, B, R, T = out["D"], out["B"], out["R"], out["T"]
    if with_factor:
        out["LD"] = torch.empty((n, b, b), device=device, dtype=f64)
        out["LB"] = torch.empty((max(n - 1, 0), b, b), device=device, dtype=f64)
        out["LR"] = torch.empty((n, a, b), device=device, dtype=f64)
    LT = factor_block_torch(wl, seed, KIND_TIP, 0, device)
    T.copy_(LT @ LT.T)
    prev_sub = prev_arrow = None
    for i in range(n):
        Ld = factor_block_torch(wl, seed, KIND_DIAG, i, device)
        Lr = factor_block_torch(wl, seed, KIND_ARROW, i, device)
        Di = Ld @ Ld.T
        Ri = Lr @ Ld.T
        if prev_sub is not None:
            Di += prev_sub @ prev_sub.T
            Ri += prev_arrow @ prev_sub.T
        D[i].copy_(0.5 * (Di + Di.T))
        R[i].copy_(Ri)
        T.add_(Lr @ Lr.T)
        if i < n - 1:
            Ls = factor_block_torch(wl, seed, KIND_SUB, i, device)
            B[i].copy_(Ls @ Ld.T)
        else:
            Ls = None
        if with_factor:
            out["LD"][i].copy_(Ld)
            out["LR"][i].copy_(Lr)
            if Ls is not None:
                out["LB"][i].copy_(Ls)
        prev_sub, prev_arrow = Ls, Lr
        if progress is not None and (i % 32 == 31 or i == n - 1):
            progress(i + 1, n)
    T.copy_(0.5 * (T + T.T))
    if with_factor:
        out["LT"] = LT
    return out


def rhs_torch(wl: Workload, seed: int, device, nrhs: int = 1):
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(_torch_seed(seed, KIND_RHS, 0))
    return torch.randn((wl.N, nrhs), generator=g, device=device, dtype=torch.float64)
