"""Build the in-tree HIP library ``libsgwls.so`` for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsgwls.so")
SOURCES = ["sgwls_pass_r1.hip", "sgwls_pass_r2.hip", "sgwls_pass_r3.hip", "sgwls_pass_r4.hip",
           "sgwls_aux.hip", "sgwls_batch.hip", "sgwls_wls2d.hip", "sgwls_delta.hip",
           "sgwls_noalloc.hip", "sgwls_plan.cpp", "sgwls_api.cpp"]
ARCH = os.environ.get("SGWLS_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions are disabled for all device code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the SG-WLS library needs ROCm's hipcc to build")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile the library (always recompiles) and return its path.  The
    translation units (one per neighbourhood radius) compile in parallel."""
    from concurrent.futures import ThreadPoolExecutor

    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmds.append([hipcc(), f"--offload-arch={ARCH}", *HIP_FLAGS, *inc, "-c",
                     os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda c: _run(c, verbose), cmds))
    for cmd, res in zip(cmds, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed on {cmd[-3]} with code {res.returncode}")
    tmp = LIB + ".tmp"
    res = _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc link failed with code {res.returncode}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
