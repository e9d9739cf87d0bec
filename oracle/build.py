"""Compile the plain-C oracle into ``oracle/liboracle.so`` with gcc.

Test infrastructure: the oracle is built so that tests, the smoke check and
the CPU-baseline leg of the benchmark can call it; the product never does.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckks_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-function",
           SRC, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def build_timing_copy(out_dir: str) -> str:
    """The same source compiled with -O3 -march=native for the host it runs
    on (the CPU-baseline timing of the benchmark); the arithmetic is the
    same code. Returns the path of the shared object in ``out_dir``."""
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, "liboracle_native%d.so" % os.getpid())
    cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-function", SRC, "-o", path]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    return path


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
