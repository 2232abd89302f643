"""The CPU suite once more under AddressSanitizer + UBSan builds of the host runtime and the
oracle (tests/run_sanitized.py); skipped inside that run itself."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)


@pytest.mark.skipif(os.environ.get("COMPAR_SANITIZED") == "1", reason="already the sanitized run")
def test_cpu_suite_under_asan_and_ubsan():
    import run_sanitized
    env = run_sanitized.sanitized_env(run_sanitized.build())
    r = subprocess.run([sys.executable, "-m", "pytest", HERE, "-m", "not gpu", "-q", "-x",
                        "-p", "no:cacheprovider"], env=env, cwd=os.path.dirname(HERE),
                       capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
