"""Compile libgca.so (HIP for gfx950 + host C++) in-tree.

    python -m paper_1810_08429_amd.build

Every HIP source is compiled with packed-FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops).  The host tree code is
compiled with -ffp-contract=off so that box diameters and distances are
rounded exactly as written.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libgca.so")
BUILD = os.path.join(HERE, "_build")

HIP_SOURCES = ["quad.hip", "basis.hip", "h2.hip", "solve.hip", "adjoint.hip", "grad.hip", "linear.hip",
               "noalloc.hip", "multi.hip", "colloc.hip",
               "dlayer.hip", "curved.hip", "lin_h2.hip"]
HOST_SOURCES = ["host.cpp", "capi.cpp", "lin_h2.cpp"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(args):
    cmd, src = args
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return src


# MFMA results and accumulators in ordinary VGPRs: the point-pair kernels
# feed every MFMA result straight into VALU work, which AGPR results would
# first have to be copied out for
MFMA_FLAGS = ["-mllvm", "-amdgpu-mfma-vgpr-form"]


def build(verbose: bool = False, jobs: int = 4, out: str = None, defines=()) -> str:
    """Compile and link libgca.so (to `out`, default the package directory);
    `defines` are extra -D flags for tuning variants."""
    hipcc = _hipcc()
    out = out or OUT
    build_dir = BUILD if out == OUT else out + "_build"
    os.makedirs(build_dir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
              "-I" + os.path.join(HERE, "..", "include")] + ["-D" + d for d in defines]
    hip_flags = ["-x", "hip", "--offload-arch=gfx950",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *MFMA_FLAGS]
    tasks = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        tasks.append(([hipcc, *common, *hip_flags, "-c", os.path.join(CSRC, src), "-o", obj], src))
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        extra = ["-ffp-contract=off"] if src == "host.cpp" else []
        tasks.append(([hipcc, *common, *extra, "-c", os.path.join(CSRC, src), "-o", obj], src))
        objs.append(obj)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src in ex.map(_compile, tasks):
            if verbose:
                print("compiled", src, flush=True)
    tmp = out + ".tmp"
    link = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(link)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out, flush=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
