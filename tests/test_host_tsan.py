"""Host code under ThreadSanitizer (CPU, no GPU): aqc_host.cpp is built with
g++ -fsanitize=thread against the CPU stand-in of the HIP runtime
(tests/hostsan/fake_hip.cpp, itself serialised by one lock) and driven from
three threads at once, with finalizers of unclosed objects running on any
thread and in any order (tests/hostsan/drive_threads.py).  A data race or a
use after free in the library's host code fails the test; among the latter, a
batch destroyed after its context (the order a reference cycle's finalizers
may take)."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _libtsan():
    gxx = shutil.which("g++")
    if gxx is None:
        return None, None
    p = subprocess.run([gxx, "-print-file-name=libtsan.so"], capture_output=True, text=True).stdout.strip()
    return gxx, (p if os.path.isabs(p) and os.path.exists(p) else None)


def test_host_code_under_tsan(tmp_path):
    gxx, tsan = _libtsan()
    if gxx is None or tsan is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ with libtsan and the HIP headers")
    so = str(tmp_path / "libaqc_tsan.so")
    build = [gxx, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-fsanitize=thread",
             "-g", "-O1", "-shared", "-fPIC", "-w",
             os.path.join(ROOT, "paper_1311_3938_amd", "csrc", "aqc_host.cpp"),
             os.path.join(HERE, "hostsan", "fake_hip.cpp"), "-o", so]
    r = subprocess.run(build, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=tsan, TSAN_OPTIONS="halt_on_error=0 report_signal_unsafe=0",
               CUDA_VISIBLE_DEVICES="", HIP_VISIBLE_DEVICES="", OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.join(HERE, "hostsan", "drive_threads.py"), so],
                       capture_output=True, text=True, timeout=900, env=env, cwd=ROOT)
    out = r.stdout + r.stderr
    assert "WARNING: ThreadSanitizer" not in out, out[-8000:]
    assert r.returncode == 0 and "threads done" in out, out[-6000:]
