"""Pins of the FP64 GEMM oracle against exact arithmetic, closed forms and a library routine."""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
import synth



def exact_gemm(A, B, alpha, beta, C0):
    """Exact rational alpha*A@B + beta*C0 (brute force, tiny shapes)."""
    M, K = A.shape
    N = B.shape[1]
    out = [[None] * N for _ in range(M)]
    fa, fb = Fraction(float(alpha)), Fraction(float(beta))
    for i in range(M):
        for j in range(N):
            s = sum((Fraction(float(A[i, k])) * Fraction(float(B[k, j])) for k in range(K)), Fraction(0))
            r = fa * s if alpha != 0 else Fraction(0)
            if beta != 0:
                r += fb * Fraction(float(C0[i, j]))
            out[i][j] = r
    return out


TINY = [(1, 1, 1), (2, 3, 4), (3, 1, 5), (5, 7, 2), (9, 8, 9), (4, 4, 0), (1, 9, 17), (7, 3, 33)]


@pytest.mark.parametrize("M,N,K", TINY)
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-0.75, 0.5), (2.5, -1.25)])
def test_bruteforce_exact(M, N, K, alpha, beta):
    g = synth.rng(M * 100 + N * 10 + K)
    A = g.uniform(-1, 1, (M, K)).astype(np.float32)
    B = g.uniform(-1, 1, (K, N)).astype(np.float32)
    C0 = g.uniform(-1, 1, (M, N)).astype(np.float32)
    ex = exact_gemm(A, B, alpha, beta, C0)
    for blocked in (False, True):
        got = oracle.gemm(A, B, alpha, beta, C0, blocked=blocked)
        u = 2.0 ** -53
        for i in range(M):
            for j in range(N):
                # products exact; K-1 additions, one multiply by alpha, one fma-free add of beta*C0
                mag = abs(alpha) * sum(abs(float(A[i, k]) * float(B[k, j])) for k in range(K)) \
                    + abs(beta) * abs(float(C0[i, j]))
                bound = (K + 3) * u * mag * 1.01
                assert abs(Fraction(got[i, j]) - ex[i][j]) <= Fraction(bound) + Fraction(0), (i, j)


def test_integer_inputs_exact():
    """Small-integer operands: every partial sum is an integer < 2^53, so the result is exact."""
    A = synth.int_matrix(37, 53, 1)
    B = synth.int_matrix(53, 29, 2)
    got = oracle.gemm(A, B)
    ref = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(got, ref.astype(np.float64))


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 300, 33), (64, 257, 513), (300, 31, 260), (129, 129, 129)])
def test_blocked_bit_identical(M, N, K):
    A, B = synth.gemm_operands(M, N, K, seed=M + N + K)
    C0 = synth.normal_matrix(M, N, 7)
    for alpha, beta in [(1.0, 0.0), (0.5, 2.0), (0.0, 1.5)]:
        a = oracle.gemm(A, B, alpha, beta, C0, blocked=False)
        b = oracle.gemm(A, B, alpha, beta, C0, blocked=True)
        assert np.array_equal(a.view(np.int64), b.view(np.int64))


def test_identity_closed_form():
    M = 45
    A = np.eye(M, dtype=np.float32)
    B = synth.normal_matrix(M, 38, 3)
    C0 = synth.normal_matrix(M, 38, 4)
    got = oracle.gemm(A, B, 1.5, -0.25, C0)
    assert np.array_equal(got, 1.5 * B.astype(np.float64) + (-0.25) * C0.astype(np.float64))


@pytest.mark.parametrize("K", [1, 7, 256, 1000])
def test_all_ones_closed_form(K):
    A = np.ones((13, K), np.float32)
    B = np.ones((K, 21), np.float32)
    assert np.all(oracle.gemm(A, B, 0.5) == 0.5 * K)


def test_rank1_closed_forms():
    g = synth.rng(11)
    u = g.integers(-5, 6, 19).astype(np.float32)
    v = g.integers(-5, 6, 23).astype(np.float32)
    # K = 1: C = alpha u v^T
    got = oracle.gemm(u[:, None], v[None, :], 3.0)
    assert np.array_equal(got, 3.0 * np.outer(u.astype(np.float64), v.astype(np.float64)))
    # A = u a^T, B = b v^T: C = (a . b) u v^T
    a = g.integers(-3, 4, 31).astype(np.float32)
    b = g.integers(-3, 4, 31).astype(np.float32)
    A = np.outer(u, a).astype(np.float32)
    B = np.outer(b, v).astype(np.float32)
    got = oracle.gemm(A, B)
    assert np.array_equal(got, float(a.astype(np.float64) @ b.astype(np.float64)) * np.outer(u, v).astype(np.float64))


def test_numpy_matmul_agrees():
    A, B = synth.gemm_operands(200, 150, 333, seed=5)
    got = oracle.gemm(A, B)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-13


def test_transpose_duality():
    A, B = synth.gemm_operands(31, 47, 19, seed=9)
    c1 = oracle.gemm(A, B)
    c2 = oracle.gemm(B.T.copy(), A.T.copy())
    assert np.array_equal(c1, c2.T)


def test_blas_semantics_nan_not_read():
    A, B = synth.gemm_operands(9, 11, 13, seed=1)
    C0 = np.full((9, 11), np.nan, np.float32)
    assert np.all(np.isfinite(oracle.gemm(A, B, 1.0, 0.0, C0)))
    An = np.full_like(A, np.nan)
    Bn = np.full_like(B, np.nan)
    C1 = synth.normal_matrix(9, 11, 2)
    got = oracle.gemm(An, Bn, 0.0, 2.0, C1)
    assert np.array_equal(got, 2.0 * C1.astype(np.float64))


def test_k_zero():
    A = np.zeros((5, 0), np.float32)
    B = np.zeros((0, 6), np.float32)
    C0 = synth.normal_matrix(5, 6, 3)
    assert np.array_equal(oracle.gemm(A, B, 1.0, 0.5, C0), 0.5 * C0.astype(np.float64))
    assert np.all(oracle.gemm(A, B, 1.0, 0.0) == 0.0)


def test_k_split_additivity():
    A, B = synth.gemm_operands(40, 50, 96, seed=2)
    full = oracle.gemm(A, B)
    p1 = oracle.gemm(A[:, :40].copy(), B[:40].copy())
    p2 = oracle.gemm(A[:, 40:].copy(), B[40:].copy())
    assert np.max(np.abs(full - (p1 + p2))) <= 1e-12 * np.max(np.abs(full))


def test_entries_match_full():
    A, B = synth.gemm_operands(70, 90, 110, seed=3)
    C0 = synth.normal_matrix(70, 90, 4)
    full = oracle.gemm(A, B, 1.25, -0.5, C0)
    ij = synth.sample_entries(70, 90, 500, 6)
    got = oracle.gemm_entries(A, B, ij, 1.25, -0.5, C0)
    assert np.array_equal(got, full[ij[:, 0], ij[:, 1]])


def test_absgemm():
    A, B = synth.gemm_operands(33, 44, 55, seed=8)
    ab = oracle.absgemm(A, B)
    assert np.array_equal(ab, oracle.gemm(np.abs(A), np.abs(B)))
    assert np.all(ab >= np.abs(oracle.gemm(A, B)))


def test_relfro_metric():
    R = synth.normal_matrix(20, 30, 1).astype(np.float64)
    C = R.astype(np.float32)
    C2 = C.copy()
    C2[3, 4] += 1.0
    d = C2.astype(np.float64) - R
    assert math.isclose(oracle.relfro(C2, R), np.linalg.norm(d) / np.linalg.norm(R), rel_tol=1e-12)
    Z = np.zeros((4, 4))
    E = np.zeros((4, 4), np.float32)
    E[0, 0] = 3.0
    E[1, 1] = 4.0
    assert oracle.relfro(E, Z) == 5.0
    E[2, 2] = np.nan
    assert oracle.relfro(E, Z) == math.inf


def test_relfro_list_metric():
    """The sampled-entry form of the metric (a 1-D list of values against their references),
    pinned by hand values: a 3-4-5 triangle, a zero reference (absolute norm), a NaN or an
    infinity anywhere in the list (infinity), and the 2-D form over the same entries."""
    f32 = lambda v: np.array(v, np.float32)
    f64 = lambda v: np.array(v, np.float64)
    # ||(0, 1)|| / ||(3, 4)|| = 1/5: a dropped square root would give 1/25
    assert oracle.relfro(f32([3.0, 5.0]), f64([3.0, 4.0])) == 0.2
    # ||(3, 4)|| against a zero reference is the absolute norm 5
    assert oracle.relfro(f32([3.0, 4.0]), f64([0.0, 0.0])) == 5.0
    # an exact match is 0; a one-element list
    assert oracle.relfro(f32([1.5, -2.0, 8.0]), f64([1.5, -2.0, 8.0])) == 0.0
    assert oracle.relfro(f32([2.0]), f64([4.0])) == 0.5
    for bad in (np.nan, np.inf, -np.inf):
        for pos in (0, 2, 4):
            c = f32([1.0, 2.0, 3.0, 4.0, 5.0])
            c[pos] = bad
            assert oracle.relfro(c, f64([1.0, 2.0, 3.0, 4.0, 5.0])) == math.inf
    # the list form over sampled entries equals the 2-D form over the same entries
    R = synth.normal_matrix(40, 50, 3).astype(np.float64)
    C = (R + 1e-3 * synth.normal_matrix(40, 50, 4)).astype(np.float32)
    assert math.isclose(oracle.relfro(C.ravel(), R.ravel()), oracle.relfro(C, R), rel_tol=1e-13)
    rng = np.random.default_rng(5)
    ij = rng.integers(0, 40, size=(300, 2))
    ij[:, 1] = rng.integers(0, 50, size=300)
    c, r = C[ij[:, 0], ij[:, 1]], R[ij[:, 0], ij[:, 1]]
    d = c.astype(np.float64) - r
    assert math.isclose(oracle.relfro(c, r), math.sqrt(np.sum(d * d) / np.sum(r * r)), rel_tol=1e-13)
