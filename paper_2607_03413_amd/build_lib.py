"""Build libfe.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Every translation unit is compiled in parallel, then linked into one shared
library next to this file.  The packed-FP32 instructions are disabled for
device code.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfe.so")
SOURCES = ["fe_api.cpp", "solver.cpp", "basis1d.cpp", "k_apply.hip", "k_dss.hip", "k_fdm.hip", "k_mg.hip",
           "k_general.hip", "k_mlp.hip", "k_smooth.hip", "k_fdm_fused.hip", "k_fdm_lattice.hip", "k_fdm_wave.hip",
           "fe_noalloc.hip", "adaptive.cpp", "k_adapt.hip",
           "multiblock.cpp", "k_multiblock.hip"]
ARCH = os.environ.get("FE_OFFLOAD_ARCH", "gfx950")


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found")
    return path


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(HERE, "..", "include"), "-Wno-unused-result", "-Wno-unused-command-line-argument"]


def compile_one(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + common_flags()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    workers = min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH, "-fPIC"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    try:
        build()
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
