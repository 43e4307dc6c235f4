"""Build the gfx950 shared library ``libcqrrpt.so`` next to this file.

Compiles every ``csrc/*.hip`` with hipcc for gfx950 and links them into one
shared object exposing the C ABI of ``include/cqrrpt.h``.
"""

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libcqrrpt.so")

ARCH = "gfx950"
FLAGS = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    # Packed FP32 instructions stay off (set by policy for all device code).
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]
# Per-source options. In the tall kernels the matrix-core accumulators stay in
# ordinary vector registers (the instructions' VGPR form): with accumulation
# registers the compiler copied every accumulator in and out of them around
# code that reads the sums (the Gram's compensated fold).
EXTRA = {
    "tall.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
    # The directly loaded Gram: in accumulation registers every accumulator
    # was copied out and back on each trip of the K loop.
    "gram.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
    # The directly loaded Q product, for the same reason.
    "qform_dv.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
    # The throughput probe's accumulators too (in accumulation registers they
    # were copied out and back around every round of the loop).
    "probe.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
}


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return exe


def _compile(src, obj):
    cmd = [_hipcc(), *FLAGS, *EXTRA.get(os.path.basename(src), []), "-I",
           os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {os.path.basename(src)}:\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    objs = [os.path.join(BUILD, s[:-4] + ".o") for s in srcs]
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        list(ex.map(_compile, [os.path.join(CSRC, s) for s in srcs], objs))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
