"""GPU parity of every gemm variant against the FP64 CPU oracle, through the C ABI.

Bars:
  * small-integer operands: bit-exact for all four variants (every product and
    partial sum is exact in each variant's arithmetic);
  * random operands: relative Frobenius error within the variant's stated bound,
    and every entry within the rigorous a-priori rounding bound of its arithmetic
    (gamma_n times the absolute product of the operands the variant multiplies,
    which the oracle computes from its own encodings of A and B; for fp8r also the
    truncation of products inside the scaled FP8 MFMA, fp8_mfma_truncation);
  * BLAS edge cases (beta == 0 ignores C, alpha == 0 ignores A and B, empty
    and ragged shapes, padded and misaligned leading dimensions);
  * bitwise repeatability of each variant.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, gamma, host, say

pytestmark = pytest.mark.gpu

VARIANTS = ["f32_simt", "bf16x3", "fp8r", "bf16", "fp6x3"]
BOUND = {"f32_simt": 1e-5, "bf16x3": 1e-5, "fp8r": 1e-3, "bf16": 1e-2, "fp6x3": 1e-2}


@pytest.fixture(scope="module")
def cx():
    import paper_2311_03543_amd as pa
    c = pa.Compar(0)
    assert c.device()["arch"].startswith("gfx950")
    assert c.register_builtin("fp6x3") == 4
    yield c
    c.close()


def run(cx, name, A, B, C0=None, alpha=1.0, beta=0.0):
    import torch
    M, N = A.shape[0], B.shape[1]
    dA, dB = dev(A), dev(B)
    dC = dev(C0) if C0 is not None else torch.zeros((M, N), dtype=torch.float32, device="cuda")
    say(f"  gemm {name} M={M} N={N} K={A.shape[1]} alpha={alpha} beta={beta}")
    cx.gemm_variant(cx.variant_find(name), dA, dB, dC, alpha, beta)
    return host(dC)


# ---- config: single FP32 GEMM, 256^3, uniform[-1, 1], seed 0 ------------------

def test_f32_simt_256_uniform(cx):
    A, B = synth.gemm_operands(256, 256, 256, seed=0, dist="uniform")
    C = run(cx, "f32_simt", A, B)
    ref = oracle.gemm(A, B)
    err = oracle.relfro(C, ref)
    assert err <= 1e-5, err
    assert np.all(np.abs(C - ref) <= gamma(256) * oracle.absgemm(A, B))


# ---- exactness on small integers ---------------------------------------------

INT_SHAPES = [(1, 1, 1), (7, 5, 3), (256, 256, 256), (300, 520, 200), (257, 255, 129),
              (64, 1000, 33), (513, 130, 640),
              # extreme aspect ratios: one tile over a long K (many pipeline stages),
              # a single row or column over several tiles, K just past a block boundary
              (64, 64, 16384), (1, 4096, 1000), (4096, 1, 1000), (33, 65, 8200),
              # many 256 x 256 tiles in both M and N: the XCD renumbering and the
              # grouped tile walk of the MFMA kernels cover a 9 x 10 tile grid
              (2304, 2560, 384),
              # the FP32 SIMT kernel's 128 x 128 tile (fewer than 512 tiles of 128 x 256)
              (2048, 4096, 72)]


@pytest.mark.parametrize("name", VARIANTS)
@pytest.mark.parametrize("M,N,K", INT_SHAPES)
def test_integer_exact(cx, name, M, N, K):
    A = synth.int_matrix(M, K, M * 7 + K)
    B = synth.int_matrix(K, N, N * 11 + K)
    C = run(cx, name, A, B)
    # entries are small integers and every partial sum is below 2^53: exact in float64
    ref = A.astype(np.float64) @ B.astype(np.float64)
    assert np.array_equal(C.astype(np.float64), ref)


# Unsplit K over many operand-image blocks: each workgroup of an MFMA kernel then
# copies K blocks far past its first one, which automatic split-K (at least four
# blocks per slice on shapes with few tiles) never reaches on the shapes above.
UNSPLIT_SHAPES = [(256, 256, 2048), (300, 520, 1000), (512, 768, 777)]


@pytest.mark.parametrize("name", ["bf16x3", "fp8r", "bf16", "fp6x3"])
@pytest.mark.parametrize("M,N,K", UNSPLIT_SHAPES)
def test_integer_exact_unsplit_long_k(cx, name, M, N, K):
    A = synth.int_matrix(M, K, M * 13 + K)
    B = synth.int_matrix(K, N, N * 17 + K)
    cx.set_split_k(1)
    try:
        C = run(cx, name, A, B)
    finally:
        cx.set_split_k(0)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    assert np.array_equal(C.astype(np.float64), ref)


# ---- random operands: stated bound and entrywise rounding bound ----------------

def e4m3_place(codes, scale_bytes):
    """Exponent of the leading binary place of each E4M3 code's dequantised value (normal
    codes: field - 7; subnormal codes: -6, the place of 0.m; zero: -inf), plus its 128 x 128
    tile's scale exponent (E8M0 byte - 127)."""
    field = (codes >> 3) & 15
    e = np.where(field == 0, -6.0, field.astype(np.float64) - 7.0)
    e = np.where((codes & 0x7f) == 0, -np.inf, e)
    s = np.repeat(np.repeat(scale_bytes.astype(np.float64) - 127.0, 128, 0), 128, 1)
    return e + s[:codes.shape[0], :codes.shape[1]]


def fp8_mfma_truncation(ca, sa, xa, cb, sb, xb):
    """Bound on what the scaled FP8 MFMA loses on X_a X_b (codes ca / cb, scale bytes sa / sb,
    dequantised values xa (M x K) and xb (K x N)).  Measured on gfx950 with in-bounds probes of
    v_mfma_scale_f32_32x32x64_f8f6f4: a single product plus the accumulator is rounded once,
    but within one instruction every product is truncated toward zero to a multiple of
    2^(E - 13), E the largest sum of the two operands' leading-place exponents among its 64
    products (exact cancellation of the large products still leaves the small ones
    truncated).  Per 64-value K block each entry therefore loses at most
    min(sum |products|, 64 * 2^(Ea + Eb - 12)), with Ea, Eb the row's and the column's largest
    leading-place exponents in the block (twice the measured grid, as a margin)."""
    M, K = xa.shape
    N = xb.shape[1]
    ea, eb = e4m3_place(ca, sa), e4m3_place(cb, sb)
    out = np.zeros((M, N))
    for k0 in range(0, K, 64):
        k1 = min(k0 + 64, K)
        emax_a = ea[:, k0:k1].max(axis=1)
        emax_b = eb[k0:k1, :].max(axis=0)
        with np.errstate(invalid="ignore"):
            grid = np.exp2(emax_a[:, None] + emax_b[None, :] - 12.0)
        grid = np.nan_to_num(grid, nan=0.0, posinf=0.0)
        absblk = np.abs(xa[:, k0:k1]).astype(np.float64) @ np.abs(xb[k0:k1, :]).astype(np.float64)
        out += np.minimum(absblk, (k1 - k0) * grid)
    return out


def variant_reference(name, A, B):
    """(product of the operands the variant multiplies, entrywise rounding bound)."""
    M, K = A.shape
    if name == "f32_simt":
        return oracle.gemm(A, B), gamma(K) * oracle.absgemm(A, B)
    if name == "bf16":
        a = oracle.bf16_to_float(oracle.bf16_rne(A))
        b = oracle.bf16_to_float(oracle.bf16_rne(B))
        return oracle.gemm(a, b), gamma(K) * oracle.absgemm(a, b)
    if name == "bf16x3":
        ah, al = (oracle.bf16_to_float(x) for x in oracle.split_bf16(A))
        bh, bl = (oracle.bf16_to_float(x) for x in oracle.split_bf16(B))
        prod = oracle.gemm(ah, bh) + oracle.gemm(ah, bl) + oracle.gemm(al, bh)
        mag = oracle.absgemm(ah, bh) + oracle.absgemm(ah, bl) + oracle.absgemm(al, bh)
        return prod, gamma(3 * K) * mag
    if name == "fp8r":
        qa, qb = oracle.quant_fp8(A), oracle.quant_fp8(B)
        a1 = oracle.dequant_fp8(qa["q"], qa["qscale"], *A.shape)
        a2 = oracle.dequant_fp8(qa["rq"], qa["rscale"], *A.shape)
        b1 = oracle.dequant_fp8(qb["q"], qb["qscale"], *B.shape)
        b2 = oracle.dequant_fp8(qb["rq"], qb["rscale"], *B.shape)
        # dequantised values are exact binary32 numbers (power-of-two scaling)
        f = [x.astype(np.float32) for x in (a1, a2, b1, b2)]
        assert all(np.array_equal(x.astype(np.float64), y) for x, y in zip(f, (a1, a2, b1, b2)))
        prod = sum(oracle.gemm(x, y) for x in f[:2] for y in f[2:])
        mag = sum(oracle.absgemm(x, y) for x in f[:2] for y in f[2:])
        # FP32 roundings: at most one per 16 K values of each of the four products, plus the
        # split-K reduction; and the scaled FP8 MFMA's own truncation (fp8_mfma_truncation)
        nkb = -(-K // 64)
        trunc = sum(fp8_mfma_truncation(ca, sa, xa, cb, sb, xb)
                    for ca, sa, xa in ((qa["q"], qa["qscale"], f[0]), (qa["rq"], qa["rscale"], f[1]))
                    for cb, sb, xb in ((qb["q"], qb["qscale"], f[2]), (qb["rq"], qb["rscale"], f[3])))
        return prod, gamma(16 * nkb + 8) * mag + trunc
    if name == "fp6x3":
        qa, qb = oracle.quant_mx6(A), oracle.quant_mx6(np.ascontiguousarray(B.T))
        ah = oracle.dequant_mx6(qa["q"], qa["qscale"])
        al = oracle.dequant_mx6(qa["rq"], qa["rscale"])
        bh = np.ascontiguousarray(oracle.dequant_mx6(qb["q"], qb["qscale"]).T)
        bl = np.ascontiguousarray(oracle.dequant_mx6(qb["rq"], qb["rscale"]).T)
        f = [x.astype(np.float32) for x in (ah, al, bh, bl)]
        assert all(np.array_equal(x.astype(np.float64), y) for x, y in zip(f, (ah, al, bh, bl)))
        pairs = [(f[0], f[2]), (f[0], f[3]), (f[1], f[2])]         # hi.hi + hi.lo + lo.hi
        prod = sum(oracle.gemm(x, y) for x, y in pairs)
        mag = sum(oracle.absgemm(x, y) for x, y in pairs)
        return prod, gamma(3 * K) * mag
    raise ValueError(name)


RAND_SHAPES = [(256, 256, 256), (384, 640, 512), (1000, 300, 777), (129, 1031, 260), (512, 512, 2048)]


@pytest.mark.parametrize("name", VARIANTS)
@pytest.mark.parametrize("M,N,K", RAND_SHAPES)
def test_random_within_bounds(cx, name, M, N, K):
    A, B = synth.gemm_operands(M, N, K, seed=M + 3 * N + 7 * K)
    C = run(cx, name, A, B)
    ref = oracle.gemm(A, B)
    err = oracle.relfro(C, ref)
    assert err <= BOUND[name], (name, err)
    prod, bnd = variant_reference(name, A, B)
    viol = np.abs(C.astype(np.float64) - prod) - bnd
    assert np.all(viol <= 0), (name, float(viol.max()))


# expected error levels for normal(0,1) operands: a kernel far off these has a
# rounding bug (for instance truncation instead of round-to-nearest-even)
LEVEL = {"f32_simt": (1e-8, 2e-6), "bf16x3": (1e-6, 8e-6), "fp8r": (5e-4, 9.6e-4), "bf16": (1.5e-3, 3.5e-3),
         "fp6x3": (8e-4, 2.5e-3)}


@pytest.mark.parametrize("name", VARIANTS)
def test_error_levels_1024(cx, name):
    A, B = synth.gemm_operands(1024, 1024, 1024, seed=1010)
    C = run(cx, name, A, B)
    err = oracle.relfro(C, oracle.gemm(A, B))
    lo, hi = LEVEL[name]
    say(f"  {name} 1024^3 rel-Frobenius {err:.3e}")
    assert lo <= err <= hi, err


# ---- BLAS semantics and edge cases -------------------------------------------

@pytest.mark.parametrize("name", VARIANTS)
def test_alpha_beta(cx, name):
    A, B = synth.gemm_operands(200, 300, 150, seed=4)
    C0 = synth.normal_matrix(200, 300, 5)
    C = run(cx, name, A, B, C0, alpha=-0.5, beta=2.0)
    ref = oracle.gemm(A, B, -0.5, 2.0, C0)
    assert oracle.relfro(C, ref) <= BOUND[name]


@pytest.mark.parametrize("name", VARIANTS)
def test_beta_zero_ignores_nan_c(cx, name):
    A, B = synth.gemm_operands(130, 140, 150, seed=6)
    C0 = np.full((130, 140), np.nan, np.float32)
    C = run(cx, name, A, B, C0, beta=0.0)
    assert np.all(np.isfinite(C))
    assert oracle.relfro(C, oracle.gemm(A, B)) <= BOUND[name]


@pytest.mark.parametrize("name", VARIANTS)
def test_alpha_zero_and_k_zero(cx, name):
    A = np.full((50, 60), np.nan, np.float32)
    B = np.full((60, 70), np.nan, np.float32)
    C0 = synth.normal_matrix(50, 70, 7)
    C = run(cx, name, A, B, C0, alpha=0.0, beta=0.5)
    assert np.array_equal(C, (0.5 * C0.astype(np.float64)).astype(np.float32))
    C = run(cx, name, np.zeros((50, 0), np.float32), np.zeros((0, 70), np.float32), C0, beta=3.0)
    assert np.array_equal(C, (3.0 * C0.astype(np.float64)).astype(np.float32))


@pytest.mark.parametrize("name", VARIANTS)
def test_empty_shapes(cx, name):
    import torch
    vid = cx.variant_find(name)
    for M, N, K in [(0, 5, 5), (5, 0, 5)]:
        A = torch.zeros((M, K), device="cuda")
        B = torch.zeros((K, N), device="cuda")
        C = torch.zeros((M, N), device="cuda")
        cx.gemm_variant(vid, A, B, C)
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", VARIANTS)
def test_padded_and_misaligned_leading_dims(cx, name):
    import torch
    M, N, K = 150, 170, 131        # K % 4 != 0: rows of A are not 16-byte aligned
    A, B = synth.gemm_operands(M, N, K, seed=8)
    Abig = np.zeros((M, K + 5), np.float32)
    Abig[:, :K] = A
    Bbig = np.zeros((K, N + 3), np.float32)
    Bbig[:, :N] = B
    dA, dB = dev(Abig), dev(Bbig)
    dC = torch.zeros((M, N + 9), device="cuda")
    vid = cx.variant_find(name)
    say(f"  gemm {name} with lda={K + 5} ldb={N + 3} ldc={N + 9}")
    cx.gemm_variant(vid, dA[:, :K], dB[:, :N], dC[:, :N])
    C = host(dC)
    assert np.all(C[:, N:] == 0.0)
    assert oracle.relfro(C[:, :N], oracle.gemm(A, B)) <= BOUND[name]


@pytest.mark.parametrize("name", VARIANTS)
def test_bitwise_repeatable(cx, name):
    A, B = synth.gemm_operands(300, 400, 500, seed=9)
    c1 = run(cx, name, A, B)
    c2 = run(cx, name, A, B)
    assert np.array_equal(c1.view(np.uint32), c2.view(np.uint32))


@pytest.mark.parametrize("name", VARIANTS)
def test_nan_in_a_propagates(cx, name):
    A, B = synth.gemm_operands(64, 64, 64, seed=10)
    A[3, 5] = np.nan
    C = run(cx, name, A, B)
    assert np.all(np.isnan(C[3])) and np.all(np.isfinite(np.delete(C, 3, axis=0)))


def test_optional_builtin_registration(cx):
    import paper_2311_03543_amd as pa
    assert cx.variant_find("fp6x3") == 4 and cx.variant_count() == 5
    for name, st in (("fp6x3", pa.CMP_EDUP), ("fp4x9", pa.CMP_ENOTFOUND)):
        with pytest.raises(pa.ComparError) as e:
            cx.register_builtin(name)
        assert e.value.status == st
    assert cx.variant_count() == 5


# ---- split-K: few output tiles over a long K ----------------------------------------

MFMA_VARIANTS = ["bf16x3", "fp8r", "bf16", "fp6x3"]


def run_split(cx, name, splits, A, B, C0=None, alpha=1.0, beta=0.0):
    """One call with the slice count forced; returns (C, whether the reduction ran)."""
    cx.set_split_k(splits)
    cx.kernel_stats(reset=True)
    cx.kernel_timing(True)
    try:
        say(f"  split-K {splits}")
        C = run(cx, name, A, B, C0, alpha, beta)
    finally:
        cx.kernel_timing(False)
        cx.set_split_k(0)
    return C, "splitk_reduce" in cx.kernel_stats(reset=True)


@pytest.mark.parametrize("name", VARIANTS)
def test_split_k_count_choice(cx, name):
    vid = cx.variant_find(name)
    assert cx.split_k(vid, 8192, 8192, 8192) == 1          # 1024 tiles fill the CUs
    assert cx.split_k(vid, 512, 512, 64) == 1              # too few K blocks to cut
    if name == "f32_simt":
        assert cx.split_k(vid, 512, 512, 8192) == 1
        return
    s = cx.split_k(vid, 512, 512, 8192)                    # 4 tiles over a long K
    assert 2 <= s <= 64
    cx.set_split_k(7)
    try:
        assert cx.split_k(vid, 512, 512, 8192) == 7
        assert cx.split_k(vid, 512, 512, 128) <= 4         # at most one slice per K block
    finally:
        cx.set_split_k(0)
    with pytest.raises(Exception):
        cx.set_split_k(65)


# K = 2000: bf16 images hold 64 K blocks of 64 bytes, fp8 images 32; a count of 7
# gives the fp8 kernel slices of 5 blocks (odd first blocks, so each slice starts
# half way through a 128-wide scale tile) and a shorter last slice; 64 gives
# one-block slices.
@pytest.mark.parametrize("name", MFMA_VARIANTS)
@pytest.mark.parametrize("splits", [1, 2, 3, 7, 64])
def test_split_k_integer_exact(cx, name, splits):
    M, N, K = 300, 520, 2000
    A = synth.int_matrix(M, K, 101)
    B = synth.int_matrix(K, N, 202)
    C, reduced = run_split(cx, name, splits, A, B)
    assert reduced == (splits > 1)
    ref = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(C.astype(np.float64), ref)


@pytest.mark.parametrize("name", MFMA_VARIANTS)
@pytest.mark.parametrize("splits", [3, 7])
def test_split_k_random_alpha_beta(cx, name, splits):
    M, N, K = 384, 640, 3000
    A, B = synth.gemm_operands(M, N, K, seed=303)
    C0 = synth.normal_matrix(M, N, 304)
    C, reduced = run_split(cx, name, splits, A, B, C0, alpha=-0.5, beta=2.0)
    assert reduced
    assert oracle.relfro(C, oracle.gemm(A, B, -0.5, 2.0, C0)) <= BOUND[name]
    # the partial sums reorder the K sum only: the entrywise bound still holds
    C1, _ = run_split(cx, name, splits, A, B)
    prod, bnd = variant_reference(name, A, B)
    viol = np.abs(C1.astype(np.float64) - prod) - bnd
    assert np.all(viol <= 0), (name, float(viol.max()))


@pytest.mark.parametrize("name", MFMA_VARIANTS)
def test_split_k_beta_zero_ignores_nan_c_and_nan_propagates(cx, name):
    M, N, K = 200, 300, 2500
    A, B = synth.gemm_operands(M, N, K, seed=305)
    C0 = np.full((M, N), np.nan, np.float32)
    C, reduced = run_split(cx, name, 5, A, B, C0, beta=0.0)
    assert reduced and np.all(np.isfinite(C))
    assert oracle.relfro(C, oracle.gemm(A, B)) <= BOUND[name]
    A[7, K - 1] = np.nan                                   # only the last slice sees it
    C, _ = run_split(cx, name, 5, A, B)
    assert np.all(np.isnan(C[7])) and np.all(np.isfinite(np.delete(C, 7, axis=0)))


@pytest.mark.parametrize("name", MFMA_VARIANTS)
def test_split_k_automatic_repeatable(cx, name):
    M, N, K = 512, 512, 8192
    vid = cx.variant_find(name)
    assert cx.split_k(vid, M, N, K) > 1
    A, B = synth.gemm_operands(M, N, K, seed=306)
    c1 = run(cx, name, A, B)
    c2 = run(cx, name, A, B)
    assert np.array_equal(c1.view(np.uint32), c2.view(np.uint32))
    ij = synth.sample_entries(M, N, 2048, 307)
    err = oracle.relfro(c1[ij[:, 0], ij[:, 1]], oracle.gemm_entries(A, B, ij))
    assert err <= BOUND[name], err


# ---- full-size square sweep point, sampled entries --------------------------------

@pytest.mark.parametrize("name", VARIANTS)
def test_square_8192_sampled(cx, name):
    n = 8192
    A, B = synth.gemm_operands(n, n, n, seed=synth.square_sweep_seed(n))
    C = run(cx, name, A, B)
    ij = synth.sample_entries(n, n, 4096, 77)
    ref = oracle.gemm_entries(A, B, ij)
    got = C[ij[:, 0], ij[:, 1]]
    err = oracle.relfro(got, ref)
    say(f"  {name} 8192^3 sampled rel-Frobenius {err:.3e}")
    assert err <= BOUND[name], err


@pytest.mark.parametrize("name", VARIANTS)
@pytest.mark.parametrize("M,N,K", [(8192, 8192, 8192), (8191, 8189, 8190)])
def test_full_size_integer_sampled_exact(cx, name, M, N, K):
    """At the measured size (and one short of it in every dimension: ragged last tiles, a
    ragged last K block) small-integer operands make every variant exact.  The expected
    entries are int64 dot products of the sampled rows and columns; the sample holds the
    four corners and the last row and column of every tile edge it can reach."""
    A = synth.int_matrix(M, K, 8001 + M)
    B = synth.int_matrix(K, N, 8002 + N)
    C = run(cx, name, A, B)
    ij = synth.sample_entries(M, N, 4096, 8003)
    edge = np.array([(0, 0), (0, N - 1), (M - 1, 0), (M - 1, N - 1), (255, 256), (256, 255),
                     (M - 1, N // 2), (M // 2, N - 1)], np.int64)
    ij = np.concatenate([ij, edge])
    want = np.einsum("ik,ki->i", A[ij[:, 0]].astype(np.int64), B[:, ij[:, 1]].astype(np.int64))
    got = C[ij[:, 0], ij[:, 1]].astype(np.float64)
    assert np.array_equal(got, want.astype(np.float64)), (name, int(np.sum(got != want)))


# ---- operands whose magnitude changes from tile to tile ----------------------------
# Tile (i, j) of 128 x 128 entries of A and of B^T is scaled by 2^((3 i + 5 j) mod 23 - 11):
# every FP8 tile scale and MX block scale differs from its neighbours, so a swapped or
# shifted scale index (A tile, transposed-B tile, K block of a split-K slice that starts
# inside a tile) breaks the entrywise bound.

def tile_operands(M, N, K, seed):
    A = synth.tile_scaled_matrix(M, K, seed)
    B = np.ascontiguousarray(synth.tile_scaled_matrix(N, K, seed + 1).T)
    return A, B


@pytest.mark.parametrize("name", VARIANTS)
@pytest.mark.parametrize("M,N,K", [(640, 768, 1024), (385, 300, 260), (1000, 129, 520)])
def test_tile_scaled_within_entrywise_bound(cx, name, M, N, K):
    A, B = tile_operands(M, N, K, M + N + K)
    C = run(cx, name, A, B)
    prod, bnd = variant_reference(name, A, B)
    viol = np.abs(C.astype(np.float64) - prod) - bnd
    assert np.all(viol <= 0), (name, float(viol.max()))


@pytest.mark.parametrize("name", MFMA_VARIANTS)
def test_tile_scaled_split_k_3(cx, name):
    """Forced split-K 3 over K = 896: the fp8 and fp6 images hold 14 K blocks of 64 values,
    cut into slices of 5, 5 and 4 blocks, so the second slice starts half way through a
    128-wide FP8 scale tile."""
    M, N, K = 640, 768, 896
    A, B = tile_operands(M, N, K, 11)
    C, reduced = run_split(cx, name, 3, A, B)
    assert reduced
    prod, bnd = variant_reference(name, A, B)
    viol = np.abs(C.astype(np.float64) - prod) - bnd
    assert np.all(viol <= 0), (name, float(viol.max()))
