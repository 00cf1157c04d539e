"""The field kernels' index arithmetic (voxel tiling, XCD-aware block order,
paired-row lanes, periodic neighbours, semi-Lagrangian cell wrap), the
trajectory-policy choice and the FFT plans, run on the host over every block and
thread of real launch shapes with explicit bounds checks, built with the
address and undefined-behaviour sanitizers (host code only)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_index_math_under_sanitizers(tmp_path):
    cc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "index_math_host")
    src = os.path.join(HERE, "native", "index_math_host.cpp")
    inc = os.path.join(ROOT, "paper_1807_04638_amd", "csrc")
    flags = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all"]
    subprocess.run([cc] + flags + ["-I", inc, src, "-o", exe], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert " 0 failures" in r.stdout
    assert "Sanitizer" not in r.stderr
