"""Build the gfx950 shared library libkpme.so in-tree with hipcc.

Usage: python -m paper_2601_18838_amd.build   (always recompiles)
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkpme.so")
SOURCES = ["api.cpp", "factors.cpp", "quadrature.cpp", "grid_kernels.hip", "skp_kernels.hip",
           "noalloc.hip", "rect.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS_C = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every device code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


NOISE = "is not a recognized feature for this target"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host compilation pass does not know the device-only feature flag
    msgs = [l for l in (res.stdout + res.stderr).splitlines() if NOISE not in l]
    return res.returncode, msgs


def build(verbose=False):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = []
    for s in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        jobs.append(([HIPCC, *FLAGS_C, *inc, "-c", os.path.join(CSRC, s), "-o", obj], obj))
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda j: _run(j[0], verbose), jobs))
    for (rc, msgs), (cmd, _) in zip(results, jobs):
        if rc != 0:
            sys.stderr.write("\n".join(msgs) + "\n")
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
        if msgs and verbose:
            print("\n".join(msgs))
    tmp = LIB + ".tmp"
    rc, msgs = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC",
                     *[o for _, o in jobs], "-o", tmp, "-L/opt/rocm/lib", "-lrocblas",
                     "-Wl,-rpath,/opt/rocm/lib"], verbose)
    if rc != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
