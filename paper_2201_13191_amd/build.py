"""Build libmcx.so (HIP kernels for gfx950 + host runtime) in-tree.

Floating-point flags are part of the transport's definition: no a*b+c
contraction into fma (-ffp-contract=off), no fast-math, IEEE fp32 division
and square root (hipcc's default), denormals kept, and no packed-fp32
instructions (-packed-fp32-ops).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.environ.get("MCX_BUILD_DIR", os.path.join(HERE, "_build"))
LIB = os.environ.get("MCX_LIB_OUT", os.path.join(HERE, "libmcx.so"))
ARCH = os.environ.get("MCX_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
             "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall"]

# build-time knobs, e.g. MCX_DEFINES="MCX_PREFETCH=12 MCX_EDGE_PAD=13" (steps per
# prefetch group; edge copies past the high faces, at least the group plus one),
# MCX_CELL_LOG (log2 of the uniform cells' edge in voxels), MCX_MIN_SKIP
# (shortest run of uniform steps taken at once)
HIP_FLAGS += [f"-D{d}" for d in os.environ.get("MCX_DEFINES", "").split()]
CXX_FLAGS += [f"-D{d}" for d in os.environ.get("MCX_DEFINES", "").split()]

SOURCES = [("transport.hip", "hip"), ("postproc.hip", "hip"), ("unet.hip", "hip"),
           ("recon.hip", "hip"),
           ("probes.hip", "hip"),
           ("runtime.hip", "hip"),
           ("tables.cpp", "cxx"), ("cells.cpp", "cxx"), ("autotune.cpp", "hiphost")]


def _compile(src, kind):
    out = os.path.join(BUILD, os.path.basename(src) + ".o")
    path = os.path.join(CSRC, src)
    if kind == "hip":
        cmd = ["hipcc", "-x", "hip", *HIP_FLAGS, "-c", path, "-o", out]
    elif kind == "hiphost":   # host-only C++ against the HIP runtime API
        cmd = ["hipcc", *CXX_FLAGS, "-c", path, "-o", out]
    else:
        cmd = ["g++", *CXX_FLAGS, "-c", path, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out, r.stderr


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        results = list(ex.map(lambda s: _compile(*s), SOURCES))
    if verbose:
        for _, err in results:
            lines = [l for l in err.splitlines() if "packed-fp32-ops" not in l]
            if lines:
                print("\n".join(lines))
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
