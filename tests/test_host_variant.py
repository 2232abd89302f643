"""The optional host variant "host_f32" (FP32 GEMM on the CPU) in a host-only context, where the
operands are host memory used in place: parity against the FP64 oracle (integer operands exact,
random operands within the FP32 entrywise rounding bound), BLAS semantics, leading dimensions,
and independence from the thread split.  The same variant on device operands is covered by the
GPU tests."""
import numpy as np
import pytest
import torch

import oracle
import synth

pa = pytest.importorskip("paper_2311_03543_amd")

U = 2.0 ** -24


def gamma(n):
    return n * U / (1 - n * U)


@pytest.fixture(scope="module")
def cx():
    c = pa.Compar(device=-1)
    vid = c.register_builtin("host_f32")
    assert c.variant_info(vid)[0] == "host_f32"
    yield c, vid
    c.close()


def run(cx, A, B, C0=None, alpha=1.0, beta=0.0):
    c, vid = cx
    M, N = A.shape[0], B.shape[1]
    tA, tB = torch.from_numpy(np.ascontiguousarray(A)), torch.from_numpy(np.ascontiguousarray(B))
    tC = torch.from_numpy(C0.copy()) if C0 is not None else torch.zeros((M, N), dtype=torch.float32)
    c.gemm_variant(vid, tA, tB, tC, alpha, beta, stream=0)      # host-only context: no stream
    return tC.numpy()


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (7, 5, 3), (33, 65, 129), (300, 520, 200), (64, 1000, 33)])
def test_integer_exact(cx, M, N, K):
    A = synth.int_matrix(M, K, M + K)
    B = synth.int_matrix(K, N, N + 2 * K)
    C = run(cx, A, B)
    assert np.array_equal(C.astype(np.float64), (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))


@pytest.mark.parametrize("M,N,K", [(256, 256, 256), (129, 1031, 260), (1000, 300, 777)])
def test_random_within_rounding_bound(cx, M, N, K):
    A, B = synth.gemm_operands(M, N, K, seed=M + N + K)
    C = run(cx, A, B)
    ref = oracle.gemm(A, B)
    assert oracle.relfro(C, ref) <= 1e-5
    assert np.all(np.abs(C.astype(np.float64) - ref) <= gamma(K) * oracle.absgemm(A, B))


def test_alpha_beta_and_beta_zero_ignores_nan(cx):
    A, B = synth.gemm_operands(70, 90, 50, seed=3)
    C0 = synth.normal_matrix(70, 90, 4)
    C = run(cx, A, B, C0, alpha=-0.5, beta=2.0)
    assert oracle.relfro(C, oracle.gemm(A, B, -0.5, 2.0, C0)) <= 1e-5
    C = run(cx, A, B, np.full((70, 90), np.nan, np.float32), beta=0.0)
    assert np.all(np.isfinite(C))


def test_alpha_zero_and_k_zero_do_not_read_a_or_b(cx):
    A = np.full((20, 30), np.nan, np.float32)
    B = np.full((30, 40), np.nan, np.float32)
    C0 = synth.normal_matrix(20, 40, 7)
    C = run(cx, A, B, C0, alpha=0.0, beta=0.5)
    assert np.array_equal(C, (0.5 * C0.astype(np.float64)).astype(np.float32))
    C = run(cx, np.zeros((20, 0), np.float32), np.zeros((0, 40), np.float32), C0, beta=3.0)
    assert np.array_equal(C, (3.0 * C0.astype(np.float64)).astype(np.float32))


def test_leading_dimensions(cx):
    c, vid = cx
    M, N, K = 40, 50, 30
    A, B = synth.gemm_operands(M, N, K, seed=5)
    Abig = torch.zeros((M, K + 3))
    Abig[:, :K] = torch.from_numpy(A)
    Bbig = torch.zeros((K, N + 5))
    Bbig[:, :N] = torch.from_numpy(B)
    Cbig = torch.zeros((M, N + 7))
    c.gemm_variant(vid, Abig[:, :K], Bbig[:, :N], Cbig[:, :N], stream=0)
    assert oracle.relfro(Cbig[:, :N].numpy(), oracle.gemm(A, B)) <= 1e-5
    assert torch.all(Cbig[:, N:] == 0)


def test_result_does_not_depend_on_the_thread_split(cx):
    # 2 Mflop per thread: 96^3 runs on one thread, 512^3 on several; the k order is the same
    A, B = synth.gemm_operands(512, 512, 512, seed=6)
    C1 = run(cx, A, B)
    C2 = run(cx, A[:96], B)                 # the first 96 rows alone: fewer threads
    assert np.array_equal(C1[:96].view(np.uint32), C2.view(np.uint32))
