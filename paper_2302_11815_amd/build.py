"""Builds libwost.so in-tree: the HIP kernels and the C-ABI for gfx950
(hipcc) plus the host tree builder (g++)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libwost.so")
ARCH = os.environ.get("WOST_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-function", "-Wno-unused-result",
               "-I", os.path.join(ROOT, "include")]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:3])} ...")
    if verbose and r.stderr.strip():
        # hipcc's host pass warns about the packed-fp32 feature; keep other output visible
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    # the walk kernels build as four translation units (dimension 2 / 3, with
    # or without double-sided primitives) so that they compile in parallel
    walks = [(d, ds) for d in (2, 3) for ds in (0, 1)]
    jobs = [
        ["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "scene_build.cpp"), "-o", os.path.join(OBJ, "scene_build.o")],
        ["hipcc", *HIPCC_FLAGS, "-c", os.path.join(CSRC, "wost_kernels.hip"), "-o", os.path.join(OBJ, "wost_kernels.o")],
        ["hipcc", *HIPCC_FLAGS, "-c", os.path.join(CSRC, "api.hip"), "-o", os.path.join(OBJ, "api.o")],
    ] + [["hipcc", *HIPCC_FLAGS, f"-DWOST_DIM={d}", f"-DWOST_DS={ds}", "-c", os.path.join(CSRC, "wost_walks.hip"),
          "-o", os.path.join(OBJ, f"wost_walks_{d}d_ds{ds}.o")] for d, ds in walks]
    with ThreadPoolExecutor(min(len(jobs), os.cpu_count() or 1)) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    objs = [os.path.join(OBJ, n) for n in ("api.o", "wost_kernels.o", "scene_build.o")]
    objs += [os.path.join(OBJ, f"wost_walks_{d}d_ds{ds}.o") for d, ds in walks]
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
