"""Build libcompar.so (the C-ABI library: host runtime + gfx950 HIP kernels) in-tree with hipcc."""
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


def _compile(src: str, out: str) -> tuple[str, str]:
    cmd = [hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out] + common_flags()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return src, warn


def build(verbose: bool = False, jobs: int = 6) -> str:
    tmp = tempfile.mkdtemp(prefix="compar_build_")
    try:
        objs = [os.path.join(tmp, s + ".o") for s in SOURCES]
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            for src, warn in ex.map(_compile, SOURCES, objs):
                if verbose:
                    print(f"compiled {src}")
                if warn and verbose:
                    print(warn)
        out = LIB + ".tmp"
        cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", out] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(out, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
