"""Build the gfx950 HIP library ``libgs.so`` in-tree with hipcc.

Every ``csrc/*.hip`` file is compiled for gfx950 and linked into one shared
library exporting the C ABI of ``include/gs.h``.  Packed FP32 instruction
selection is disabled (``-packed-fp32-ops``) for all device code.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgs.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


# per-file additions: the rasterisers' work-queue atomics are issued by one
# lane and their result is read a whole tile later; the atomic optimizer would
# rewrite them into a wave-aggregated form that reads the result at once
# The projection is compiled without floating-point contraction: its one-view
# and several-view kernels differ in code shape, and the renders of a view
# must not depend on which of them produced its splats.
FILE_FLAGS = {"raster.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"],
              "project.hip": ["-ffp-contract=off"]}


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose=False, jobs=8):
    """Compile each source to an object in parallel, then link libgs.so."""
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)
    objs, procs = [], []
    for src in sources():
        obj = os.path.join(outdir, os.path.basename(src)[:-4] + ".o")
        cmd = [HIPCC] + FLAGS + FILE_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _wait(item):
    p, src = item
    _, err = p.communicate()
    lines = [l for l in (err or "").splitlines() if "packed-fp32-ops" not in l]
    if lines:
        sys.stderr.write("\n".join(lines) + "\n")
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}")


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
