"""Compile the C oracle into oracle/liboracle.so with gcc (binary64, no fast-math, OpenMP).

`build(sanitize=True)` compiles oracle/liboracle_san.so with clang under AddressSanitizer and
UndefinedBehaviorSanitizer instead (clang, so that one ASan runtime serves it and the
sanitized libcompar in one process); loaded when COMPAR_SANITIZED=1.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(verbose: bool = False, sanitize: bool = False) -> str:
    lib = LIB_SAN if sanitize else LIB
    tmp = lib + ".tmp"
    if sanitize:
        cmd = [CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-shared-libsan", "-mavx2", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    else:
        cmd = ["gcc", "-O3", "-mavx2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
