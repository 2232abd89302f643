"""The host runtime's threaded code under ThreadSanitizer (CPU only): the host variant's FP32 GEMM
(csrc/host_gemm.cpp, row tiles on std::threads) built with -fsanitize=thread on the host side
(hipcc, -Xarch_host before the flag) and driven by tests/tsan_host_gemm.cpp, which checks every
result exactly.  The run fails on any ThreadSanitizer report.  (The OpenMP oracle is checked
under ASan/UBSan instead: its OpenMP runtime is not built for ThreadSanitizer.)"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.skipif(hipcc() is None, reason="hipcc not found")
@pytest.mark.skipif(os.environ.get("COMPAR_SANITIZED") == "1",
                    reason="the AddressSanitizer run preloads its runtime, which ThreadSanitizer cannot share")
def test_host_gemm_threads_under_thread_sanitizer():
    csrc = os.path.join(ROOT, "paper_2311_03543_amd", "csrc")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "tsan_host_gemm")
        cmd = [hipcc(), "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=thread",
               "-I", os.path.join(ROOT, "include"), "-I", csrc,
               os.path.join(csrc, "host_gemm.cpp"), os.path.join(ROOT, "tests", "tsan_host_gemm.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0 and "mismatches 0" in r.stdout, (r.stdout, r.stderr[-2000:])
