"""Build libckks_hip.so (gfx950) in-tree with hipcc.

The kernels and the host runtime are compiled as separate translation
units in parallel, then linked into ``paper_2110_13638_amd/libckks_hip.so``.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libckks_hip.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["ckks_ntt16.hip", "ckks_ntt15.hip", "ckks_ntt15_fixed.hip", "ckks_ntt15_inv.hip", "ckks_ntt14.hip", "ckks_ntt13.hip", "ckks_ntt_small.hip", "ckks_kernels.hip", "ckks_noalloc.hip",
           "ckks_host.cpp", "ckks_eval.cpp", "ckks_linear.cpp", "ckks_graph.cpp"]
ARCH = os.environ.get("CKKS_OFFLOAD_ARCH", "gfx950")
# packed-fp32 instructions are disabled for every HIP translation unit
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + ["-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
