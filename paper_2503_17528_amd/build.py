"""Build the HIP shared library ``libbta.so`` for gfx950 with hipcc.

Every call compiles from source (the sources in parallel, then one link);
``python -m
paper_2503_17528_amd.build`` does the same from the command line.  The build
fails if any kernel needs scratch memory (register spills or private arrays):
the kernels are written to run from registers and LDS alone, and spilling
builds of them have produced wrong results.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbta.so")
SOURCES = ["abi.hip", "batched.hip", "factor.hip", "gemm.hip", "selinv.hip", "solve.hip", "tune.hip"]
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden",
    "-Wno-unused-result",
    # per-kernel resource report (parsed below for scratch use)
    "-Rpass-analysis=kernel-resource-usage",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, obj: str, inc) -> subprocess.CompletedProcess:
    flags = [f for f in FLAGS if f != "-shared"] + ["-c"]
    cmd = [hipcc()] + flags + inc + [src, "-o", obj]
    return subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel, check the resource
    report for scratch use, and link libbta.so."""
    from concurrent.futures import ThreadPoolExecutor

    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    tmpdir = tempfile.mkdtemp(prefix="bta_build_", dir=HERE)
    try:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]
        jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", "8"))))
        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(lambda so: _compile(so[0], so[1], inc), zip(srcs, objs)))
        lines = []
        for src, res in zip(srcs, results):
            lines += res.stdout.splitlines()
            if res.returncode != 0:
                out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l
                                and "is not a recognized feature" not in l and "kernel-resource-usage" not in l)
                raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({res.returncode}):\n{out}")
        spills = scratch_kernels(lines)
        if spills:
            raise RuntimeError("kernels using scratch memory: " + ", ".join(f"{k} ({v} B/lane)" for k, v in spills))
        tmp = os.path.join(tmpdir, "libbta.so")
        cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed ({res.returncode}):\n{res.stdout}")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


def scratch_kernels(lines):
    """(kernel, bytes per lane) for every kernel of the resource report with scratch."""
    found, name = [], None
    for l in lines:
        m = re.search(r"remark: Function Name: (\S+)", l)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"remark:\s+ScratchSize \[bytes/lane\]: (\d+)", l)
        if m and name is not None and int(m.group(1)) > 0:
            found.append((name, int(m.group(1))))
    return found


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
