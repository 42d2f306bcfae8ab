"""Helpers shared by the GPU parity tests (device tensors <-> oracle blocks)."""
import sys
import time

import numpy as np

TOL = 1e-10  # relative Frobenius error per block


_T0 = time.perf_counter()


def say(*args):
    """Progress line with the seconds since the GPU tests started."""
    print(f"[{time.perf_counter() - _T0:7.1f}s]", *args, flush=True)
    sys.stdout.flush()


def to_dev(blocks, keys=("D", "B", "R", "T")):
    import torch

    return [torch.from_numpy(np.ascontiguousarray(blocks[k])).to("cuda") for k in keys]


def to_np(ts):
    return [t.detach().cpu().numpy() for t in ts]


def errs(got, ref, lower=("D", "T")):
    """Max per-block relative Frobenius error by block type (lower triangles
    for the symmetric/triangular slots)."""
    out = {}
    for k in ("D", "B", "R", "T"):
        g = np.asarray(got[k], dtype=np.float64)
        r = np.asarray(ref[k], dtype=np.float64)
        if r.size == 0:
            out[k] = 0.0
            continue
        if r.ndim == 2:
            g, r = g[None], r[None]
        if k in lower:
            g, r = np.tril(g), np.tril(r)
        d = np.sqrt(np.sum((g - r) ** 2, axis=(1, 2)))
        nr = np.sqrt(np.sum(r ** 2, axis=(1, 2)))
        mean = max(float(np.mean(nr)), 1e-300)
        e = np.where(nr > 1e-300, d / np.maximum(nr, 1e-300), d / mean)
        out[k] = float(np.max(e))
    return out
