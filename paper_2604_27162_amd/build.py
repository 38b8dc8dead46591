"""Build libhase.so in-tree for gfx950.

    python -m paper_2604_27162_amd.build

Kernels are compiled by hipcc for gfx950 only; the host runtime is plain C++
(g++) against the HIP runtime API; hipcc links the shared library.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libhase.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

# packed-FP32 instructions are disabled for all device code
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    p = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return p


def _run(cmd, quiet):
    if not quiet:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=ROOT)


def build(quiet: bool = False, jobs: int | None = None) -> str:
    """Compile the kernels (one hipcc per translation unit, in parallel) and
    the runtime, and link libhase.so (always rebuilds)."""
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    cmds, objs = [], []
    # the largest translation units (terrain with line of sight or radio)
    # first, so the longest compiles do not trail the pool
    def weight(src):
        name = os.path.basename(src)
        return (0 if ("radioter" in name or "terrlos" in name) else
                1 if ("radio" in name or "terr" in name or "feat" in name) else 2, name)

    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip")), key=weight):
        obj = os.path.join(bdir, os.path.basename(src)[:-4] + ".o")
        cmds.append([_hipcc(), *HIP_FLAGS, "-c", "-o", obj, src])
        objs.append(obj)
    robj = os.path.join(bdir, "hase_runtime.o")
    cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
                 f"-I{ROCM}/include", "-c", "-o", robj, os.path.join(CSRC, "hase_runtime.cpp")])
    objs.append(robj)
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c, quiet) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], quiet)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(quiet="-q" in sys.argv)
