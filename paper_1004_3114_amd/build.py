"""Build libwallace.so (HIP kernels for gfx950 + C++ host runtime) in-tree.

Usage: python -m paper_1004_3114_amd.build   (or build() from Python)

Flags that are part of the numerical contract:
  -ffp-contract=off            no fused multiply-add contraction: the pass and
                               the sum of squares are bit-exact only with the
                               stated operation order
  -fno-gpu-flush-denormals-to-zero   IEEE subnormals
  -Xclang -target-feature -Xclang -packed-fp32-ops
                               no packed FP32 (v_pk_*) instructions
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIBRARY = os.path.join(PKG, "libwallace.so")

# (source, extra defines, object name)
SOURCES = [("wallace_kernels.hip", [], "wallace_kernels"),
           ("wallace_stream.hip", [], "wallace_stream"),
           ("wallace_host.cpp", [], "wallace_host"),
           ("wallace_batch.cpp", [], "wallace_batch"),
           ("wallace_tune.cpp", [], "wallace_tune"),
           ("wallace_static.hip", [], "wallace_static")]
for _n in (2, 4, 16):
    for _rm in (0, 1, 2):
        SOURCES.append(("wallace_pool_inst.hip",
                        [f"-DWALLACE_POOL_N={_n}", f"-DWALLACE_POOL_RM={_rm}"],
                        f"wallace_pool_{_n}_{_rm}"))

# libwallace_check.so: device arithmetic checks and store-ceiling kernels,
# used only by the tests and the benchmark (include/wallace_check.h)
CHECK_SOURCES = [("wallace_check.hip", [], "wallace_check")]
CHECK_LIBRARY = os.path.join(PKG, "libwallace_check.so")

ARCH = os.environ.get("WALLACE_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            f"-I{INCLUDE}", f"-I{CSRC}", "-Wall", "-Wno-unused-function"]


def compile_one(item) -> str:
    src, defines, name = item
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc(), *common_flags(), *defines, "-c", path, "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
                    "-Xclang", "-packed-fp32-ops", "-fno-gpu-flush-denormals-to-zero",
                    "-x", "hip"]
    else:
        rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
        cmd[1:1] = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include"]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{proc.stdout}\n{proc.stderr}")
    return obj


def link(objs, library):
    tmp = library + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-lpthread"]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{proc.stdout}\n{proc.stderr}")
    os.replace(tmp, library)


def build(verbose: bool = False) -> str:
    """Compile every source and link libwallace.so and libwallace_check.so
    (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    items = SOURCES + CHECK_SOURCES
    with cf.ThreadPoolExecutor(max_workers=min(os.cpu_count() or 8, 16, len(items))) as ex:
        objs = list(ex.map(compile_one, items))
    link(objs[:len(SOURCES)], LIBRARY)
    link(objs[len(SOURCES):], CHECK_LIBRARY)
    if verbose:
        print(f"built {LIBRARY} and {CHECK_LIBRARY}")
    return LIBRARY


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
