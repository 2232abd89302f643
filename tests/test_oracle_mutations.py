"""Planted mistakes: copies of the oracle with one plausible error each (a transposed operand, a
flipped sign, a dropped term, a wrong tie rule, a wrong format maximum) are compiled on the CPU and must fail the same
independent pins that the real oracle passes (exact rational arithmetic, torch's E4M3 codes)."""
import ctypes as C
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest
import torch

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = {
    "transposed_B": ("                    s += (double)A[i * lda + k] * (double)B[k * ldb + j];",
                     "                    s += (double)A[i * lda + k] * (double)B[j * ldb + k];"),
    "beta_sign": ("r += b * (double)C0[i * ldc + j];", "r -= b * (double)C0[i * ldc + j];"),
    "dropped_last_k": ("                for (int64_t k = 0; k < K; ++k)\n                    s += (double)A[i * lda + k]",
                       "                for (int64_t k = 0; k < K - 1; ++k)\n                    s += (double)A[i * lda + k]"),
    "e4m3_ties_away": ("if (rem > 0.5 * step || (rem == 0.5 * step && fmod(lowm, 2.0) != 0.0)) m = lowm + 1.0;\n"
                       "    const double v = m * step;\n    if (v > 448.0)",
                       "if (rem >= 0.5 * step) m = lowm + 1.0;\n    const double v = m * step;\n    if (v > 448.0)"),
    "e2m3_ties_away": ("if (rem > 0.5 * step || (rem == 0.5 * step && fmod(lowm, 2.0) != 0.0)) m = lowm + 1.0;\n"
                       "    const double v = m * step;                    /* <= 7.5",
                       "if (rem >= 0.5 * step) m = lowm + 1.0;\n"
                       "    const double v = m * step;                    /* <= 7.5"),
    "mx6_scale_to_8": ("while (ldexp(a, e) > 7.5) --e;\n    while (ldexp(a, e + 1) <= 7.5) ++e;",
                       "while (ldexp(a, e) > 8.0) --e;\n    while (ldexp(a, e + 1) <= 8.0) ++e;"),
    "relfro_list_no_sqrt": ("        den += r[t] * r[t];\n    }\n    return den > 0.0 ? sqrt(num) / sqrt(den) : sqrt(num);",
                            "        den += r[t] * r[t];\n    }\n    return den > 0.0 ? num / den : num;"),
    "relfro_list_no_nan_check": ("        if (!isfinite(cv)) return INFINITY;\n", ""),
}


def build_mutant(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", "-o", str(so),
                    str(path), "-lm"], check=True)
    return C.CDLL(str(so))


def gemm_pin_holds(L):
    """The exact-rational pin of the plain GEMM on one small non-square case."""
    g = synth.rng(77)
    M, N, K = 3, 4, 5
    A = g.uniform(-1, 1, (M, K)).astype(np.float32)
    B = g.uniform(-1, 1, (K, N)).astype(np.float32)
    C0 = g.uniform(-1, 1, (M, N)).astype(np.float32)
    out = np.empty((M, N), np.float64)
    fp = C.POINTER(C.c_float)
    L.oracle_gemm_f64.argtypes = [C.c_int64] * 3 + [C.c_float, fp, C.c_int64, fp, C.c_int64, C.c_float, fp,
                                                    C.c_int64, C.POINTER(C.c_double), C.c_int64]
    L.oracle_gemm_f64(M, N, K, 1.0, A.ctypes.data_as(fp), K, B.ctypes.data_as(fp), N, 0.5,
                      C0.ctypes.data_as(fp), N, out.ctypes.data_as(C.POINTER(C.c_double)), N)
    for i in range(M):
        for j in range(N):
            ex = sum((Fraction(float(A[i, k])) * Fraction(float(B[k, j])) for k in range(K)), Fraction(0)) \
                + Fraction(1, 2) * Fraction(float(C0[i, j]))
            if abs(Fraction(out[i, j]) - ex) > Fraction(1, 2 ** 40):
                return False
    return True


def e4m3_pin_holds(L):
    pos = np.array([float(v) for v in torch.arange(0, 0x7F, dtype=torch.uint8).view(torch.float8_e4m3fn)
                    .to(torch.float32)])
    pos.sort()
    mids = ((pos[1:] + pos[:-1]) / 2).astype(np.float32)
    L.oracle_e4m3_rne.argtypes = [C.c_float]
    L.oracle_e4m3_rne.restype = C.c_uint8
    ours = np.array([L.oracle_e4m3_rne(float(v)) for v in mids], np.uint8)
    ref = torch.from_numpy(mids).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    return np.array_equal(ours, ref)


def e2m3_pin_holds(L):
    """E2M3 rounding of the midpoints of its grid: torch's E4M3 on [1, 7.5], half-to-even
    multiples of 1/8 below 1."""
    L.oracle_e2m3_rne.argtypes = [C.c_float]
    L.oracle_e2m3_rne.restype = C.c_uint8
    L.oracle_e2m3_to_float.argtypes = [C.c_uint8]
    L.oracle_e2m3_to_float.restype = C.c_float
    val = lambda x: float(L.oracle_e2m3_to_float(L.oracle_e2m3_rne(float(x))))
    pos = np.array([float(v) for v in torch.arange(0, 0x7F, dtype=torch.uint8).view(torch.float8_e4m3fn)
                    .to(torch.float32)])
    grid = np.sort(pos[(pos >= 1.0) & (pos <= 7.5)])
    mids = ((grid[1:] + grid[:-1]) / 2).astype(np.float32)
    ref = torch.from_numpy(mids).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    if any(val(m) != float(r) for m, r in zip(mids, ref)):
        return False
    sub = (np.arange(16) + 0.5) / 16
    return all(val(x) == float(np.round(x * 8) / 8) for x in sub)


def mx6_scale_pin_holds(L):
    L.oracle_mx6_scale_exp.argtypes = [C.c_float]
    L.oracle_mx6_scale_exp.restype = C.c_int
    return all(L.oracle_mx6_scale_exp(a) == e for a, e in [(7.5, 0), (1.0, 2), (3.75, 1), (7.6, -1)])


def relfro_list_pin_holds(L):
    """The sampled-entry metric on hand values: 1/5 for a 3-4-5 triangle, infinity for a NaN."""
    fp, dp = C.POINTER(C.c_float), C.POINTER(C.c_double)
    L.oracle_relfro_list.argtypes = [C.c_int64, fp, dp]
    L.oracle_relfro_list.restype = C.c_double
    f = lambda c, r: L.oracle_relfro_list(len(c), np.array(c, np.float32).ctypes.data_as(fp),
                                          np.array(r, np.float64).ctypes.data_as(dp))
    return f([3.0, 5.0], [3.0, 4.0]) == 0.2 and f([1.0, np.nan], [1.0, 1.0]) == float("inf")


def test_real_oracle_passes_the_pins(tmp_path):
    import oracle
    assert gemm_pin_holds(oracle.lib())
    assert e4m3_pin_holds(oracle.lib())
    assert e2m3_pin_holds(oracle.lib())
    assert mx6_scale_pin_holds(oracle.lib())
    assert relfro_list_pin_holds(oracle.lib())


@pytest.mark.parametrize("name", ["transposed_B", "beta_sign", "dropped_last_k"])
def test_gemm_mutants_are_caught(name, tmp_path):
    assert not gemm_pin_holds(build_mutant(name, tmp_path))


def test_e4m3_mutant_is_caught(tmp_path):
    assert not e4m3_pin_holds(build_mutant("e4m3_ties_away", tmp_path))


def test_e2m3_mutant_is_caught(tmp_path):
    assert not e2m3_pin_holds(build_mutant("e2m3_ties_away", tmp_path))


def test_mx6_scale_mutant_is_caught(tmp_path):
    assert not mx6_scale_pin_holds(build_mutant("mx6_scale_to_8", tmp_path))


@pytest.mark.parametrize("name", ["relfro_list_no_sqrt", "relfro_list_no_nan_check"])
def test_relfro_list_mutants_are_caught(name, tmp_path):
    assert not relfro_list_pin_holds(build_mutant(name, tmp_path))
