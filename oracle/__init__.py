"""CPU oracle for the GEMM component and its selector (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2311_03543_amd``) and never imports it; the two meet only through the
seeded inputs of the ``synth`` module.

* GEMM, operand encodings (bfloat16, E4M3 with tile scales, MX E2M3 with
  block scales) and the Freivalds probe: ``oracle.c`` (binary64 C),
  wrapped here with numpy arrays.
* Selector network (forward, gradient, Adam): ``oracle.mlp`` (numpy binary64).
* Selection rules (admissibility, exhaustive best, nearest neighbour, regret):
  ``oracle.selection`` (plain Python).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# COMPAR_SANITIZED=1: the AddressSanitizer/UBSan build (oracle/build.py, sanitize=True)
_LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if os.environ.get("COMPAR_SANITIZED") == "1"
                         else "liboracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")
_i64 = C.c_int64


def lib():
    """Load liboracle.so, compiling it first only if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build(sanitize=os.environ.get("COMPAR_SANITIZED") == "1")
    L = C.CDLL(_LIB_PATH)
    gemm_args = [_i64, _i64, _i64, C.c_float, _f32p, _i64, _f32p, _i64, C.c_float,
                 C.c_void_p, _i64, _f64p, _i64]
    for name in ("oracle_gemm_f64", "oracle_gemm_f64_blocked"):
        fn = getattr(L, name)
        fn.argtypes = gemm_args
        fn.restype = None
    L.oracle_absgemm_f64.argtypes = [_i64, _i64, _i64, _f32p, _i64, _f32p, _i64, _f64p, _i64]
    L.oracle_absgemm_f64.restype = None
    L.oracle_gemm_f64_entries.argtypes = [_i64, _i64, _i64, C.c_float, _f32p, _i64, _f32p, _i64,
                                          C.c_float, C.c_void_p, _i64, _i64, _i64p, _f64p]
    L.oracle_gemm_f64_entries.restype = None
    L.oracle_relfro.argtypes = [_i64, _i64, _f32p, _i64, _f64p, _i64]
    L.oracle_relfro.restype = C.c_double
    L.oracle_relfro_list.argtypes = [_i64, _f32p, _f64p]
    L.oracle_relfro_list.restype = C.c_double
    L.oracle_bf16_rne.argtypes = [C.c_float]
    L.oracle_bf16_rne.restype = C.c_uint16
    L.oracle_bf16_to_float.argtypes = [C.c_uint16]
    L.oracle_bf16_to_float.restype = C.c_float
    L.oracle_split_bf16.argtypes = [_i64, _i64, _f32p, _i64, _u16p, _u16p]
    L.oracle_split_bf16.restype = None
    L.oracle_e4m3_rne.argtypes = [C.c_float]
    L.oracle_e4m3_rne.restype = C.c_uint8
    L.oracle_e4m3_to_float.argtypes = [C.c_uint8]
    L.oracle_e4m3_to_float.restype = C.c_float
    L.oracle_scale_exp.argtypes = [C.c_float]
    L.oracle_scale_exp.restype = C.c_int
    L.oracle_quant_fp8.argtypes = [_i64, _i64, _f32p, _i64, _u8p, _u8p, _u8p, _u8p, _f32p]
    L.oracle_quant_fp8.restype = None
    L.oracle_e2m3_rne.argtypes = [C.c_float]
    L.oracle_e2m3_rne.restype = C.c_uint8
    L.oracle_e2m3_to_float.argtypes = [C.c_uint8]
    L.oracle_e2m3_to_float.restype = C.c_float
    L.oracle_mx6_scale_exp.argtypes = [C.c_float]
    L.oracle_mx6_scale_exp.restype = C.c_int
    L.oracle_quant_mx6.argtypes = [_i64, _i64, _f32p, _i64, _u8p, _u8p, _u8p, _u8p]
    L.oracle_quant_mx6.restype = None
    L.oracle_freivalds.argtypes = [_i64, _i64, _i64, C.c_float, _f32p, _i64, _f32p, _i64,
                                   C.c_float, C.c_void_p, _f32p, _i64, _f64p]
    L.oracle_freivalds.restype = C.c_double
    L.oracle_threads.argtypes = []
    L.oracle_threads.restype = C.c_int
    _lib = L
    return L


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def gemm(A, B, alpha=1.0, beta=0.0, C0=None, blocked=True) -> np.ndarray:
    """C = alpha*A@B + beta*C0 in binary64 from float32 A (M x K), B (K x N), C0 (M x N).

    ``blocked`` selects the cache-blocked loop nest, bit-identical to the plain
    triple loop (``blocked=False``).
    """
    A, B = _f32(A), _f32(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    out = np.empty((M, N), dtype=np.float64)
    c0 = None
    if beta != 0.0:
        c0 = _f32(C0)
        assert c0.shape == (M, N)
    fn = lib().oracle_gemm_f64_blocked if blocked else lib().oracle_gemm_f64
    fn(M, N, K, alpha, A, max(K, 1), B, max(N, 1), beta,
       None if c0 is None else c0.ctypes.data, max(N, 1), out, max(N, 1))
    return out


def gemm_entries(A, B, ij, alpha=1.0, beta=0.0, C0=None) -> np.ndarray:
    """The definition at listed entries; ij is an int64 (count x 2) array of (i, j)."""
    A, B = _f32(A), _f32(B)
    M, K = A.shape
    N = B.shape[1]
    ij = np.ascontiguousarray(ij, dtype=np.int64)
    out = np.empty(ij.shape[0], dtype=np.float64)
    c0 = _f32(C0) if beta != 0.0 else None
    lib().oracle_gemm_f64_entries(M, N, K, alpha, A, max(K, 1), B, max(N, 1), beta,
                                  None if c0 is None else c0.ctypes.data, max(N, 1),
                                  ij.shape[0], ij, out)
    return out


def absgemm(A, B) -> np.ndarray:
    """|A| @ |B| in binary64."""
    A, B = _f32(A), _f32(B)
    M, K = A.shape
    N = B.shape[1]
    out = np.empty((M, N), dtype=np.float64)
    lib().oracle_absgemm_f64(M, N, K, A, max(K, 1), B, max(N, 1), out, max(N, 1))
    return out


def relfro(Cgpu, R) -> float:
    """||C - R||_F / ||R||_F (absolute when ||R|| = 0; +inf if C has NaN/inf)."""
    Cg = _f32(Cgpu)
    R = np.ascontiguousarray(R, dtype=np.float64)
    if Cg.ndim == 1:
        return float(lib().oracle_relfro_list(Cg.shape[0], Cg, R))
    M, N = Cg.shape
    return float(lib().oracle_relfro(M, N, Cg, max(N, 1), R, max(N, 1)))


def bf16_rne(x) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of float32 values, round-to-nearest-even."""
    f = lib().oracle_bf16_rne
    x = _f32(x)
    return np.fromiter((f(float(v)) for v in x.ravel()), dtype=np.uint16, count=x.size).reshape(x.shape)


def bf16_to_float(h) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.uint16)
    return (h.astype(np.uint32) << 16).view(np.float32)


def split_bf16(X):
    """(hi, lo) bfloat16 bit patterns with hi = bf16(x), lo = bf16(x - hi)."""
    X = _f32(X)
    r, c = X.shape
    hi = np.empty((r, c), dtype=np.uint16)
    lo = np.empty((r, c), dtype=np.uint16)
    lib().oracle_split_bf16(r, c, X, max(c, 1), hi, lo)
    return hi, lo


def e4m3_rne(x) -> np.ndarray:
    """OCP E4M3 codes (uint8), round-to-nearest-even, saturating to +-448."""
    f = lib().oracle_e4m3_rne
    x = _f32(x)
    return np.fromiter((f(float(v)) for v in x.ravel()), dtype=np.uint8, count=x.size).reshape(x.shape)


def e4m3_to_float(q) -> np.ndarray:
    f = lib().oracle_e4m3_to_float
    q = np.ascontiguousarray(q, dtype=np.uint8)
    return np.fromiter((f(int(v)) for v in q.ravel()), dtype=np.float32, count=q.size).reshape(q.shape)


def scale_exp(amax: float) -> int:
    return int(lib().oracle_scale_exp(float(amax)))


def quant_fp8(X):
    """Tile-scaled E4M3 quantisation with one residual pass (128 x 128 tiles).

    Returns dict(q, qscale, rq, rscale, resid): codes row-major (rows x cols),
    E8M0 scale bytes per tile (tile-row-major), and the float32 residual.
    """
    X = _f32(X)
    r, c = X.shape
    tr, tc = (r + 127) // 128, (c + 127) // 128
    q = np.empty((r, c), dtype=np.uint8)
    rq = np.empty((r, c), dtype=np.uint8)
    qs = np.empty((tr, tc), dtype=np.uint8)
    rs = np.empty((tr, tc), dtype=np.uint8)
    res = np.empty((r, c), dtype=np.float32)
    lib().oracle_quant_fp8(r, c, X, max(c, 1), q, qs, rq, rs, res)
    return dict(q=q, qscale=qs, rq=rq, rscale=rs, resid=res)


_E4M3_TABLE = None


def e4m3_values(q) -> np.ndarray:
    """Vectorised decode of E4M3 codes to float64 (table built from oracle_e4m3_to_float)."""
    global _E4M3_TABLE
    if _E4M3_TABLE is None:
        f = lib().oracle_e4m3_to_float
        _E4M3_TABLE = np.array([f(i) for i in range(256)], dtype=np.float64)
    return _E4M3_TABLE[np.asarray(q, dtype=np.uint8)]


def dequant_fp8(q, scale_bytes, rows, cols) -> np.ndarray:
    """float64 values q * 2^(byte - 127) with one scale byte per 128 x 128 tile."""
    v = e4m3_values(q)
    sb = np.asarray(scale_bytes, dtype=np.int64)
    srow = np.repeat(np.repeat(sb, 128, axis=0), 128, axis=1)[:rows, :cols]
    return np.ldexp(v, srow - 127)


def e2m3_rne(x) -> np.ndarray:
    """OCP MX FP6 E2M3 codes (uint8, low 6 bits), round-to-nearest-even, saturating to +-7.5."""
    f = lib().oracle_e2m3_rne
    x = _f32(x)
    return np.fromiter((f(float(v)) for v in x.ravel()), dtype=np.uint8, count=x.size).reshape(x.shape)


def e2m3_to_float(q) -> np.ndarray:
    f = lib().oracle_e2m3_to_float
    q = np.ascontiguousarray(q, dtype=np.uint8)
    return np.fromiter((f(int(v)) for v in q.ravel()), dtype=np.float32, count=q.size).reshape(q.shape)


def mx6_scale_exp(amax: float) -> int:
    return int(lib().oracle_mx6_scale_exp(float(amax)))


def quant_mx6(X):
    """MX E2M3 quantisation with one residual level, blocks of 32 along each row.

    Returns dict(q, qscale, rq, rscale): codes row-major (rows x cols) and E8M0
    scale bytes (rows x ceil(cols / 32)); 0xff marks a block with a non-finite value.
    """
    X = _f32(X)
    r, c = X.shape
    nb = (c + 31) // 32
    q = np.empty((r, c), dtype=np.uint8)
    rq = np.empty((r, c), dtype=np.uint8)
    qs = np.empty((r, nb), dtype=np.uint8)
    rs = np.empty((r, nb), dtype=np.uint8)
    lib().oracle_quant_mx6(r, c, X, max(c, 1), q, qs, rq, rs)
    return dict(q=q, qscale=qs, rq=rq, rscale=rs)


_E2M3_TABLE = None


def dequant_mx6(q, scale_bytes) -> np.ndarray:
    """float64 values e2m3(q) * 2^(byte - 127), one scale byte per 32 elements of a row
    (NaN for the 0xff byte)."""
    global _E2M3_TABLE
    if _E2M3_TABLE is None:
        f = lib().oracle_e2m3_to_float
        _E2M3_TABLE = np.array([f(i) for i in range(64)], dtype=np.float64)
    q = np.asarray(q, dtype=np.uint8)
    v = _E2M3_TABLE[q & 63]
    sb = np.repeat(np.asarray(scale_bytes, dtype=np.int64), 32, axis=1)[:, :q.shape[1]]
    out = np.ldexp(v, np.where(sb == 0xff, 0, sb) - 127)
    return np.where(sb == 0xff, np.nan, out)


def freivalds(A, B, Cout, x, alpha=1.0, beta=0.0, C0=None) -> float:
    """||C x - (alpha A (B x) + beta C0 x)|| / ||alpha A (B x) + beta C0 x|| in binary64."""
    A, B, Cout = _f32(A), _f32(B), _f32(Cout)
    M, K = A.shape
    N = B.shape[1]
    x = np.ascontiguousarray(x, dtype=np.float64)
    c0 = _f32(C0) if beta != 0.0 else None
    return float(lib().oracle_freivalds(M, N, K, alpha, A, max(K, 1), B, max(N, 1), beta,
                                        None if c0 is None else c0.ctypes.data,
                                        Cout, max(N, 1), x))


# ---------------------------------------------------------------------------
# splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
# generators", 2014): output j of the generator seeded with s is
# mix(s + (j + 1) * 0x9e3779b97f4a7c15) with the 64-bit finaliser below.
_GOLDEN = 0x9E3779B97F4A7C15
_MASK = (1 << 64) - 1


def splitmix64(seed: int, j: int) -> int:
    z = (seed + (j + 1) * _GOLDEN) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def rademacher_splitmix(n: int, seed: int) -> np.ndarray:
    """Probe vector x[j] = -1 if the top bit of splitmix64(seed, j) is set, else +1."""
    return np.array([-1.0 if splitmix64(seed, j) >> 63 else 1.0 for j in range(n)])
