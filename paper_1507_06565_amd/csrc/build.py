"""Build libmi355lbm.so (HIP kernels for gfx950 + the C ABI) in-tree.

    python -m paper_1507_06565_amd.csrc.build
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
OUT = os.path.join(PKG, "libmi355lbm.so")
BUILD = os.path.join(HERE, "_build")
ARCH = "gfx950"

HIP_SOURCES = ["sweep.hip", "reduce.hip", "batch.hip", "gray.hip", "mlp.hip", "probe.hip"]
HOST_SOURCES = ["geometry.cpp", "images.cpp", "capi.cpp", "brick_batch.cpp"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src, verbose):
    hipcc = _hipcc()
    path = os.path.join(HERE, src)
    obj = os.path.join(BUILD, src + ".o")
    common = ["-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I", os.path.join(PKG, "..", "include")]
    if src.endswith(".hip"):
        cmd = [hipcc, "-O3", f"--offload-arch={ARCH}", "-x", "hip",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-munsafe-fp-atomics"] + common + ["-c", path, "-o", obj]
    else:
        # host code: no FP contraction, so the exact geometry arithmetic is
        # evaluated exactly as written
        cmd = [hipcc, "-O2", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__"] + common + ["-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    sources = [s for s in HIP_SOURCES + HOST_SOURCES if os.path.exists(os.path.join(HERE, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(sources))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), sources))
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", OUT + ".tmp"] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stdout}\n{r.stderr}")
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
