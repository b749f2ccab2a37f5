"""Build libfsmi.so (HIP, gfx950) in-tree: paper_1905_02238_amd/libfsmi.so.

Each .hip source under csrc/ is compiled by hipcc for gfx950 into _build/,
then linked into one shared library.  Packed FP32 instructions are disabled
(-packed-fp32-ops) for all device code.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfsmi.so")
ARCH = os.environ.get("FSMI_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
         "-I" + os.path.join(ROOT, "include"), "-I" + SRC,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # loop heads on 64-byte boundaries: keeps the hot loops' timing
         # independent of unrelated code placed before them
         "-falign-loops=64",
         # matrix-core results in ordinary VGPRs: without it the compiler
         # shuffles loop-carried accumulators through AGPR moves every iteration
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-Wno-unused-command-line-argument"]


def _compile(src, verbose):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(SRC, "*.hip")))
    jobs = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
