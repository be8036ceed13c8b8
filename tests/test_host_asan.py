"""Host code under AddressSanitizer (CPU, no GPU): aqc_host.cpp is built with
g++ -fsanitize=address against a CPU stand-in of the HIP runtime and of the
kernel launchers (tests/hostsan/fake_hip.cpp), and the Python front end drives
every host path through it (tests/hostsan/drive.py).  Any out-of-bounds
access, use after free or double free in the host code, any free of a handle
the runtime did not hand out, and any handle left alive at the end fails the
test.  Kernels do nothing here, so only the host logic is checked."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _libasan():
    gxx = shutil.which("g++")
    if gxx is None:
        return None, None
    p = subprocess.run([gxx, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return gxx, (p if os.path.isabs(p) and os.path.exists(p) else None)


def test_host_code_under_asan(tmp_path):
    gxx, asan = _libasan()
    if gxx is None or asan is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ with libasan and the HIP headers")
    so = str(tmp_path / "libaqc_asan.so")
    build = [gxx, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-fsanitize=address",
             "-fno-omit-frame-pointer", "-g", "-O1", "-shared", "-fPIC", "-w",
             os.path.join(ROOT, "paper_1311_3938_amd", "csrc", "aqc_host.cpp"),
             os.path.join(HERE, "hostsan", "fake_hip.cpp"), "-o", so]
    r = subprocess.run(build, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               CUDA_VISIBLE_DEVICES="", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, os.path.join(HERE, "hostsan", "drive.py"), so], capture_output=True,
                       text=True, timeout=900, env=env, cwd=ROOT)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-6000:]
    assert r.returncode == 0 and "host paths done" in out, out[-6000:]
