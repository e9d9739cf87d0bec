"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the oracle (plain
C) and of the library's host C++ (parameter checks, context tables, encoder
and decoder, workspace sizing, graph planner and Algorithms 6-8, the error
paths of the device entry points), each run by a small driver under
tests/sanitize/. The device kernels are not part of these builds (GPU code
is never built with a sanitizer); the host driver never reaches a launch."""
import os
import shlex
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2110_13638_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")

# host-only sanitizer flags (each one for the host pass alone)
HIPCC_SAN = ("hipcc -O1 -g -std=c++17 --offload-arch=gfx950 -Xarch_host -fsanitize=address "
             "-Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all -fno-omit-frame-pointer")
GCC_SAN = "gcc -O1 -g -std=c11 -fsanitize=address,undefined -fno-sanitize-recover=all -fno-omit-frame-pointer"


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, "%s\n%s%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_asan")
    _run(shlex.split(GCC_SAN) + [os.path.join(HERE, "sanitize", "oracle_main.c"),
                                 os.path.join(ROOT, "oracle", "ckks_oracle.c"), "-o", exe], str(tmp_path))
    assert "oracle driver ok" in _run([exe], str(tmp_path))


def test_host_runtime_under_asan_ubsan(tmp_path):
    if not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host_asan")
    srcs = [os.path.join(HERE, "sanitize", "host_main.cpp")] + [
        os.path.join(CSRC, f) for f in ("ckks_host.cpp", "ckks_eval.cpp", "ckks_linear.cpp", "ckks_graph.cpp",
                                         "ckks_noalloc.hip")]
    _run(shlex.split(HIPCC_SAN) + srcs + ["-o", exe], str(tmp_path))
    assert "host driver ok" in _run([exe], str(tmp_path))
