"""Run the CPU test suite (-m "not gpu") against AddressSanitizer + UndefinedBehaviorSanitizer
builds of the host runtime (libcompar_san.so: host code instrumented, gfx950 device code as
usual) and of the C oracle (liboracle_san.so, clang).  Python itself is not instrumented, so
clang's shared ASan runtime is preloaded; leak checking is off (the interpreter's own
allocations would be reported), every UBSan finding aborts the run.

    python tests/run_sanitized.py [extra pytest arguments]
"""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def build() -> str:
    from oracle import build as obuild
    from paper_2311_03543_amd import build as lbuild
    lbuild.build(sanitize=True)
    obuild.build(sanitize=True)
    return lbuild.sanitizer_runtime()


def sanitized_env(runtime: str) -> dict:
    env = dict(os.environ)
    env.update(COMPAR_SANITIZED="1", LD_PRELOAD=runtime, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:strict_string_checks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return env


def main(argv: list[str]) -> int:
    env = sanitized_env(build())
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-q", "-x"] + argv
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
