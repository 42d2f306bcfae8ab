"""Throughput of the BTA block Cholesky factorization + selected inversion
(POBTAF + POBTASI) in FP64 on one MI355X.

A step is one full pass of the hot path over one synthetic BTA matrix:
bta_factor (A -> L) followed by bta_selinv (L -> Sigma at the BTA pattern),
out of place, inputs resident in HBM.  The default workload is the largest
single-GPU one: n=256 diagonal blocks of b=4096 with an a=16 arrow tip
(68.7 GB of blocks per copy), drawn by the seeded L L^T generator (scaled
off-diagonal reading, diagonal of L_ii in [1,3]), the shape of a
spatio-temporal GMRF precision matrix.  ``--workload bench`` runs n=128,
b=2048, a=8.

Prints one JSON line: TFLOP/s over the algorithmic flop count (whole timed
region), the median step time with a distribution-free 95% confidence
interval, the roofline record of the dominant kernel (HIP events on the
launch stream over the timed region), the CPU oracle timed on a bounded
sample of the same workload, and the parity gate: after timing, every block
of the timed L is compared with the factor the input was drawn from, and
every diagonal, arrow and tip block identity of Sigma Q = I is evaluated with
the timed X; the line is printed only if all of them hold to 1e-10.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X FP64 matrix (MFMA) peak
PEAK_HBM_GBS = 8000.0
TOL = 1e-10
METRIC = "POBTAF+POBTASI FP64 TFLOP/s and % FP64 MFMA peak on 1 MI355X at err<=1e-10"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--b", type=int, default=2048)
    ap.add_argument("--a", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", choices=["large", "bench", "custom", "arrow", "batched", "autograd"], default="large",
                    help="large (default): the n=256, b=4096, a=16 workload (diagonal of L_ii in [1,3]); "
                         "bench: n=128, b=2048, a=8; "
                         "arrow: the wide-arrowhead workload n=512, b=1024, a=256; "
                         "batched: 64 matrices, n in [16,96], b in {128,256,384}, a in {2,4,6}, one batched "
                         "factorization + selected inversion per step (graph-replayed); "
                         "autograd: f = logdet Q + y^T Q^-1 y at n=256, b=512, a=4, forward + backward per step; "
                         "custom: --n/--b/--a with the default generator")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-target-s", type=float, default=15.0, help="CPU oracle sample budget (seconds)")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the parity gate (profiling runs only: the line then carries parity null)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before the warmup, one device-to-device copy of this many MiB (a dispatch of known "
                         "traffic that calibrates hardware byte counters in a profile of this command)")
    return ap.parse_args()


def profiled_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    this workload, if the kernel's sources are still the profiled ones (their
    hash is recorded in the summary); None otherwise."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}_bytes_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for f in fields["sources"].split():
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != fields["source_sha256_16"]:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def cpu_baseline(b, a, seed, target_s):
    """The oracle (numpy/scipy, host BLAS threads) on n_s blocks of the same
    b and a, scaled to TFLOP/s with the same flop count."""
    import numpy as np  # noqa: F401

    import oracle
    from paper_2503_17528_amd import synth

    try:
        from threadpoolctl import threadpool_info

        cores = max([int(i.get("num_threads", 0)) for i in threadpool_info() if i.get("user_api") == "blas"] or [0])
    except Exception:
        cores = 0
    if cores <= 0:
        cores = os.cpu_count() or 1

    def run(ns):
        wl = synth.workload(ns, b, a, "scaled" if b >= 2048 else "literal")
        Q = synth.make_np(wl, seed)
        t0 = time.perf_counter()
        F = oracle.pobtaf(Q["D"], Q["B"], Q["R"], Q["T"])
        oracle.pobtasi(F["LD"], F["LB"], F["LR"], F["LT"])
        dt = time.perf_counter() - t0
        return wl, dt

    wl, dt = run(2)
    rate = wl.flops()["total"] / dt
    ns = int(max(2, min(64, round(target_s * rate / (wl.flops()["total"] / 2)))))
    if ns > 2:
        wl, dt = run(ns)
    tf = wl.flops()["total"] / dt / 1e12
    return {"value": round(tf, 4), "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"POBTAF+POBTASI oracle on n={ns} blocks of b={b}, a={a} (same block shape), {dt:.1f} s"}


def step_stats(ms):
    """Median of the per-step times with a distribution-free 95% confidence
    interval (order statistics of the binomial(K, 1/2) law; min..max for K < 6)."""
    import math

    x = sorted(ms)
    k = len(x)
    med = x[k // 2] if k % 2 else 0.5 * (x[k // 2 - 1] + x[k // 2])
    if k < 6:
        lo, hi = x[0], x[-1]
    else:
        j = int(math.floor((k - 1.96 * math.sqrt(k)) / 2.0))
        u = int(math.ceil(1 + (k + 1.96 * math.sqrt(k)) / 2.0))
        lo, hi = x[max(j, 1) - 1], x[min(u, k) - 1]
    return {"median": round(med, 3), "ci95": [round(lo, 3), round(hi, 3)], "min": round(x[0], 3),
            "max": round(x[-1], 3), "n": k}


def timed_steps(torch, step, steps, warmup):
    """Warm up, then time `steps` calls of step() between synchronizations
    (events on the current stream); returns (ms per step over the whole timed
    region, per-step ms list, wall seconds)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        step()
        ev[k + 1].record()
    torch.cuda.synchronize()
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    return ev[0].elapsed_time(ev[-1]) / steps, per, time.perf_counter() - t0


def kernel_line(L, steps):
    """Per-kernel HIP-event totals of the timed region (factor kernels only are
    timed outside graphs)."""
    kms = (ctypes.c_double * 4)()
    kcnt = (ctypes.c_longlong * 4)()
    L.bta_internal_timing_read(kms, kcnt)
    L.bta_internal_timing(0, 0)
    return kms, kcnt


def mfma_probe(torch, L, dev):
    """Sustained FP64 MFMA rate of this device: a register-only MFMA loop
    (bta_internal_mfma_probe) at 1, 2, 4 and 8 workgroups of 4 waves per CU
    with 4, 8 and 16 independent chains per wave (the same number of MFMAs per
    launch in every configuration), timed with events on the current stream;
    the best configuration's rate."""
    L.bta_internal_mfma_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    L.bta_internal_mfma_probe.restype = ctypes.c_int
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    out = torch.empty(8 * cus * 256, dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    best = 0.0
    for per_cu in (1, 2, 4, 8):
        for chains in (4, 8, 16):
            grid = per_cu * cus
            iters = 4000 * 128 // (per_cu * chains)
            for _ in range(2):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                rc = L.bta_internal_mfma_probe(out.data_ptr(), grid, iters, chains, s)
                e1.record()
                torch.cuda.synchronize()
                if rc != 0:
                    return None
                best = max(best, grid * 4.0 * iters * chains * 2048 / (e0.elapsed_time(e1) * 1e-3) / 1e12)
    return round(best, 2)


def parity_gate(torch, synth, wl, seed, Q, L, X):
    """Check the timed outputs: every L block against the factor the input was
    drawn from (regenerated block by block on the device), and every block
    identity of Sigma Q = I that uses selected blocks only:
    (Sigma Q)_jj = I, (Sigma Q)_{n,j} = 0 for every j, and (Sigma Q)_nn = I."""
    n, b, a = wl.n, wl.b, wl.a
    LD, LB, LR, LT = L
    XD, XB, XR, XT = X
    D, B, R, T = Q["D"], Q["B"], Q["R"], Q["T"]

    def rel(g, r, lower):
        if lower:
            g, r = torch.tril(g), torch.tril(r)
        return (torch.linalg.matrix_norm(g - r) / torch.linalg.matrix_norm(r)).item()

    eL = {"D": 0.0, "B": 0.0, "R": 0.0, "T": 0.0}
    ident = {"diag": 0.0, "arrow": 0.0, "tip": 0.0}
    I_b = torch.eye(b, dtype=torch.float64, device=D.device)
    for j in range(n):
        eL["D"] = max(eL["D"], rel(LD[j], synth.factor_block_torch(wl, seed, synth.KIND_DIAG, j, D.device), True))
        if j < n - 1:
            eL["B"] = max(eL["B"], rel(LB[j], synth.factor_block_torch(wl, seed, synth.KIND_SUB, j, D.device), False))
        if a:
            eL["R"] = max(eL["R"], rel(LR[j], synth.factor_block_torch(wl, seed, synth.KIND_ARROW, j, D.device), False))
        acc = XD[j] @ D[j]
        if a:
            acc += XR[j].T.contiguous() @ R[j]
        if j > 0:
            acc += XB[j - 1] @ B[j - 1].T.contiguous()
        if j < n - 1:
            acc += XB[j].T.contiguous() @ B[j]
        acc -= I_b
        ident["diag"] = max(ident["diag"], acc.abs().max().item())
        if a:
            acc = XR[j] @ D[j] + XT @ R[j]
            if j > 0:
                acc += XR[j - 1] @ B[j - 1].T.contiguous()
            if j < n - 1:
                acc += XR[j + 1] @ B[j]
            ident["arrow"] = max(ident["arrow"], acc.abs().max().item())
        if j % 64 == 63:
            print(f"[bench] parity gate: {j + 1}/{n} blocks", file=sys.stderr, flush=True)
    if a:
        eL["T"] = rel(LT, synth.factor_block_torch(wl, seed, synth.KIND_TIP, 0, D.device), True)
        acc = XT @ T
        for j in range(n):
            acc += XR[j] @ R[j].T.contiguous()
        acc -= torch.eye(a, dtype=torch.float64, device=D.device)
        ident["tip"] = acc.abs().max().item()
    worst = max(max(eL.values()), max(ident.values()))
    return {"ok": bool(worst < TOL), "tol": TOL, "blocks_checked": "all",
            "L_vs_drawn_factor_max_rel_fro": {k: float(f"{v:.3e}") for k, v in eL.items()},
            "sigma_q_identity_max_abs": {k: float(f"{v:.3e}") for k, v in ident.items()}}


def run_batched(args, torch, bta, synth, L):
    """The batched workload: one bta_factor_batched + bta_selinv_batched per step."""
    wls = synth.batched_workloads(args.seed)
    print(f"[bench] drawing {len(wls)} matrices ({sum(w.block_bytes() for w in wls) / 1e9:.2f} GB of blocks)",
          file=sys.stderr, flush=True)
    mats = [synth.make_torch(w, 100 + k, "cuda") for k, w in enumerate(wls)]
    batch = bta.Batch(mats)

    def step():
        batch.factor(check=False)
        batch.selinv()

    step()  # first call: autotuning and graph capture
    torch.cuda.synchronize()
    L.bta_internal_timing(1, 4096 * max(1, args.steps))
    ms, per, wall = timed_steps(torch, step, args.steps, args.warmup)
    kms, kcnt = kernel_line(L, args.steps)
    bad = [m for m, i in enumerate(batch.info) if int(i.item()) != 0]
    if bad:
        raise RuntimeError(f"factorization failed for matrices {bad}")
    fl = sum(w.flops()["total"] for w in wls)
    ffac = sum(w.flops()["factor"] for w in wls)
    tfl = fl / (ms * 1e-3) / 1e12
    roof = None
    if kcnt[0]:
        avg = kms[0] / kcnt[0]
        ach = ffac / (kcnt[0] / args.steps) / (avg * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": "factor_batched_kernel", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4), "traffic": None,
                "flops_per_launch": ffac / (kcnt[0] / args.steps), "avg_launch_ms": round(avg, 4)}
    return {"metric": METRIC,
            "value": round(tfl, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "bta_batched64", "matrices": len(wls), "seed": args.seed, "flops_per_step": fl},
            "step_ms": step_stats(per),
            "pct_fp64_peak": round(100.0 * tfl / PEAK_FP64_TFLOPS, 2), "roofline": roof, "cpu_baseline": None,
            "wall_s_timed": round(wall, 3)}


def run_autograd(args, torch, bta, synth, L):
    """f = logdet Q + y^T Q^{-1} y: forward and backward per step."""
    from paper_2503_17528_amd import autograd

    wl = synth.AUTOGRAD
    Q = synth.make_torch(wl, args.seed, "cuda")
    n, b, a = wl.n, wl.b, wl.a
    g = torch.Generator(device="cuda").manual_seed(args.seed)
    y = torch.randn(n * b + a, dtype=torch.float64, device="cuda", generator=g)
    leaves = [Q[k].clone().requires_grad_(True) for k in "DBRT"]

    def step():
        for t in leaves:
            t.grad = None
        f = autograd.logdet_quad(*leaves, y)
        f.backward()

    L.bta_internal_timing(1, 4096 * max(1, args.steps))
    ms, per, wall = timed_steps(torch, step, args.steps, args.warmup)
    kms, kcnt = kernel_line(L, args.steps)
    fl = wl.flops()
    # factor + selected inversion (the O(n b^2) solves and gradient assembly are not counted)
    tfl = fl["total"] / (ms * 1e-3) / 1e12
    roof = None
    if kcnt[0]:
        avg = kms[0] / kcnt[0]
        ach = fl["factor"] / (kcnt[0] / args.steps) / (avg * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": "factor_kernel", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4), "traffic": None,
                "flops_per_launch": fl["factor"] / (kcnt[0] / args.steps), "avg_launch_ms": round(avg, 4)}
    return {"metric": METRIC,
            "value": round(tfl, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": wl.name + "_logdet_quad_fwd_bwd", "n": n, "b": b, "a": a, "seed": args.seed,
                       "flops_per_step": fl["total"]},
            "step_ms": step_stats(per),
            "pct_fp64_peak": round(100.0 * tfl / PEAK_FP64_TFLOPS, 2), "roofline": roof, "cpu_baseline": None,
            "wall_s_timed": round(wall, 3)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}): this build has no multi-GPU path; "
              "the single-GPU throughput is the reported value.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2503_17528_amd import bta, synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L = bta.lib()
    L.bta_internal_timing.argtypes = [ctypes.c_int, ctypes.c_int]
    L.bta_internal_timing_read.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    if args.workload in ("batched", "autograd"):
        run = run_batched if args.workload == "batched" else run_autograd
        print(json.dumps(run(args, torch, bta, synth, L)), flush=True)
        return

    if args.workload == "large":
        wl = synth.LARGE
    elif args.workload == "bench":
        wl = synth.BENCH
    elif args.workload == "arrow":
        wl = synth.ARROW
    else:
        reading = "scaled" if args.b >= 2048 else "literal"
        wl = synth.workload(args.n, args.b, args.a, reading, name=f"bta_n{args.n}_b{args.b}_a{args.a}")
    n, b, a, reading = wl.n, wl.b, wl.a, wl.reading
    print(f"[bench] drawing {wl.name} ({wl.block_bytes() / 1e9:.2f} GB of blocks) on {dev}", file=sys.stderr, flush=True)
    Q = synth.make_torch(wl, args.seed, dev,
                         progress=lambda i, m: print(f"[bench] drawn {i}/{m} blocks", file=sys.stderr, flush=True))
    D, B, R, T = Q["D"], Q["B"], Q["R"], Q["T"]
    outL = tuple(torch.empty_like(x) for x in (D, B, R, T))
    outX = tuple(torch.empty_like(x) for x in (D, B, R, T))
    wf, nf = bta.workspace(bta.BTA_OP_FACTOR, n, b, a, dev)
    ws, nsel = bta.workspace(bta.BTA_OP_SELINV, n, b, a, dev)
    torch.cuda.synchronize()
    probe = mfma_probe(torch, L, dev)
    print(f"[bench] FP64 MFMA probe: {probe} TFLOP/s", file=sys.stderr, flush=True)

    if args.copy_probe_mb > 0:
        src = torch.ones(args.copy_probe_mb * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        LD, LB, LR, LT, info = bta.factor(D, B, R, T, out=outL, work=wf, check=False)
        bta.selinv(LD, LB, LR, LT, out=outX, work=ws)
        return info

    print(f"[bench] {args.warmup} warmup steps", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        info = step()
    torch.cuda.synchronize()
    if args.warmup and int(info.item()) != 0:
        raise RuntimeError(f"factorization failed: info={int(info.item())}")

    # timed region: K steps between synchronizations; HIP events on the launch stream around every
    # factorization launch (kind 0 only: events around every launch would add two records per GEMM)
    print(f"[bench] {args.steps} timed steps", file=sys.stderr, flush=True)
    L.bta_internal_timing(1, 4096 * max(1, args.steps))
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps + 1)]
    t_wall0 = time.perf_counter()
    evs[0].record()
    for k in range(args.steps):
        LD, LB, LR, LT, info = bta.factor(D, B, R, T, out=outL, work=wf, check=False)
        evs[2 * k + 1].record()
        bta.selinv(LD, LB, LR, LT, out=outX, work=ws)
        evs[2 * k + 2].record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0
    ms_total = evs[0].elapsed_time(evs[-1])
    per_step = [evs[2 * k].elapsed_time(evs[2 * k + 2]) for k in range(args.steps)]
    ms_factor = sum(evs[2 * k].elapsed_time(evs[2 * k + 1]) for k in range(args.steps)) / args.steps
    ms_selinv = sum(evs[2 * k + 1].elapsed_time(evs[2 * k + 2]) for k in range(args.steps)) / args.steps
    kms = (ctypes.c_double * 4)()
    kcnt = (ctypes.c_longlong * 4)()
    rd = L.bta_internal_timing_read(kms, kcnt)
    L.bta_internal_timing(0, 0)
    if int(info.item()) != 0:
        raise RuntimeError(f"factorization failed: info={int(info.item())}")

    parity = None
    if not args.no_check:
        print("[bench] parity gate on the timed outputs (every block)", file=sys.stderr, flush=True)
        parity = parity_gate(torch, synth, wl, args.seed, Q, outL, outX)
        print(f"[bench] parity: {parity}", file=sys.stderr, flush=True)
        if not parity["ok"]:
            print(json.dumps({"metric": METRIC, "error": "parity gate failed", "parity": parity}), file=sys.stderr)
            sys.exit(1)

    # one more step, untimed, with events around every launch of every kind: the per-kernel breakdown
    L.bta_internal_timing(15, 4096)
    bta.factor(D, B, R, T, out=outL, work=wf, check=False)
    bta.selinv(outL[0], outL[1], outL[2], outL[3], out=outX, work=ws)
    torch.cuda.synchronize()
    kms1 = (ctypes.c_double * 4)()
    kcnt1 = (ctypes.c_longlong * 4)()
    L.bta_internal_timing_read(kms1, kcnt1)
    L.bta_internal_timing(0, 0)

    fl = wl.flops()
    ms_step = ms_total / args.steps
    tflops = fl["total"] / (ms_step * 1e-3) / 1e12
    st = step_stats(per_step)

    # timing categories: single kernels, except "gemm_all_variants", which sums every GEMM kernel variant
    # (128x128, 128x64, 64x64 and lower-triangle bodies, on both streams); algorithmic flops per launch
    names = ["factor_kernel", "gemm_all_variants", "trinv_diag_tiles_kernel", "other"]
    T_ = (b + 63) // 64
    trinv_fl = n * T_ * (64.0 ** 3) / 3.0
    per_step_flops = {"factor_kernel": fl["factor"], "gemm_all_variants": fl["selinv"] - trinv_fl,
                      "trinv_diag_tiles_kernel": trinv_fl, "other": 0.0}
    # the factorization from the timed region, the other kinds from the instrumented extra step
    kern = {}
    for k, nm in enumerate(names):
        tms, tcnt, nst = (kms[k], kcnt[k], args.steps) if k == 0 else (kms1[k], kcnt1[k], 1)
        if tcnt == 0:
            continue
        launches_per_step = tcnt / nst
        avg_ms = tms / tcnt
        fl_launch = per_step_flops[nm] / launches_per_step
        kern[nm] = {"launches_per_step": launches_per_step, "avg_ms": avg_ms, "total_ms_per_step": tms / nst,
                    "flops_per_launch": fl_launch, "tflops": fl_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0}
    # the roofline record is for the largest single kernel
    singles = [k for k in kern if k not in ("gemm_all_variants", "other")]
    dom = max(singles, key=lambda k: kern[k]["total_ms_per_step"]) if singles else None
    roofline = None
    if dom:
        ach = kern[dom]["tflops"]
        roofline = {"bound": "mfma", "kernel": dom, "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4),
                    "traffic": profiled_traffic(dom, wl.name),
                    "flops_per_launch": kern[dom]["flops_per_launch"], "avg_launch_ms": round(kern[dom]["avg_ms"], 4),
                    "frac_of_probe": round(ach / probe, 4) if probe else None}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(b, a, args.seed, args.cpu_target_s)

    line = {
        "metric": METRIC,
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": n, "b": b, "a": a, "reading": reading,
                   "diag_range": [wl.diag_lo, wl.diag_hi], "seed": args.seed,
                   "flops_per_step": fl["total"], "flops_factor": fl["factor"], "flops_selinv": fl["selinv"]},
        "pct_fp64_peak": round(100.0 * tflops / PEAK_FP64_TFLOPS, 2),
        "step_ms": st,
        "tflops_at_median_step": round(fl["total"] / (st["median"] * 1e-3) / 1e12, 3),
        "mfma_probe_tflops": probe,
        "phases": {"factor_ms": round(ms_factor, 3), "selinv_ms": round(ms_selinv, 3),
                   "factor_tflops": round(fl["factor"] / (ms_factor * 1e-3) / 1e12, 3),
                   "selinv_tflops": round(fl["selinv"] / (ms_selinv * 1e-3) / 1e12, 3)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()} for k, v in kern.items()},
        "kernels_source": "factor_kernel: HIP events of the timed steps; other kinds: one instrumented step after them",
        "timer_status": int(rd),
        "wall_s_timed": round(t_wall, 3),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
