"""Build libcompar.so (the C-ABI library: host runtime + gfx950 HIP kernels) in-tree with hipcc.

`build(sanitize=True)` builds libcompar_san.so instead: the same sources with AddressSanitizer
and UndefinedBehaviorSanitizer on the host code only (every -fsanitize= behind -Xarch_host;
the gfx950 device code is built as usual).  It needs clang's ASan runtime loaded first
(LD_PRELOAD=`sanitizer_runtime()`); the binding loads it when COMPAR_SANITIZED=1
(tests/run_sanitized.py runs the CPU test suite that way).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcompar.so")
LIB_SAN = os.path.join(HERE, "libcompar_san.so")
SOURCES = ["runtime.cpp", "gemm_f32_simt.hip", "gemm_mfma.hip", "prepass.hip", "mx6.hip", "freivalds.hip",
           "mlp.hip", "host_gemm.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def common_flags() -> list[str]:
    # Packed FP32 instructions are disabled on purpose: the FP32 kernels use
    # plain v_fma_f32 only.
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-result"]


SAN_HOST = ["address", "undefined"]


def sanitize_flags() -> list[str]:
    """Host-only sanitizer flags for hipcc: each -fsanitize= directly after -Xarch_host."""
    f = []
    for s in SAN_HOST:
        f += ["-Xarch_host", f"-fsanitize={s}"]
    return f + ["-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                "-Xarch_host", "-g"]


def sanitizer_runtime() -> str:
    """Path of clang's shared ASan runtime (to preload into an uninstrumented python)."""
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True,
                       check=True)
    return r.stdout.strip()


def _compile(src: str, out: str, sanitize: bool = False) -> tuple[str, str]:
    cmd = [hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out] + common_flags()
    if sanitize:
        cmd += sanitize_flags()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return src, warn


def build(verbose: bool = False, jobs: int = 6, sanitize: bool = False) -> str:
    lib = LIB_SAN if sanitize else LIB
    tmp = tempfile.mkdtemp(prefix="compar_build_")
    try:
        objs = [os.path.join(tmp, s + ".o") for s in SOURCES]
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            for src, warn in ex.map(lambda so: _compile(so[0], so[1], sanitize), zip(SOURCES, objs)):
                if verbose:
                    print(f"compiled {src}")
                if warn and verbose:
                    print(warn)
        out = lib + ".tmp"
        cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", out] + objs
        if sanitize:
            cmd += ["-Xarch_host", "-shared-libsan"] + sanitize_flags()
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(out, lib)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
