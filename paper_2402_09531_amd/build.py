"""Build libdwfmm.so (HIP for gfx950) in-tree with hipcc: one object per source, compiled in
parallel, then linked."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdwfmm.so")
OBJDIR = os.path.join(HERE, "..", "_build")
# (source, object, extra flags): kernels.hip is compiled in two parts (single-problem and
# batched entry points) so the two halves of its template instantiations build in parallel
UNITS = [("kernels.hip", "kernels_single.o", ["-DDWFMM_KERNELS_PART=1"]),
         ("kernels.hip", "kernels_batch.o", ["-DDWFMM_KERNELS_PART=2"]),
         ("api.hip", "api.o", []),
         ("setup.cpp", "setup.o", [])]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs: no accvgpr moves around the nearfield tiles
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = True) -> str:
    """Compile every source into libdwfmm.so (always recompiles)."""
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(HERE, "..", "include")]
    procs, objs = [], []
    for src, o, extra in UNITS:
        obj = os.path.join(OBJDIR, o)
        cmd = [HIPCC, *FLAGS, *extra, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    failed = [p.args for p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
