"""The optional host variant "host_f32" in a GPU context: device operands are copied to the host
after the stream's earlier work, multiplied on the CPU, and C is copied back before the call
returns.  Parity against the FP64 oracle, BLAS semantics, leading dimensions, and selection
through cmp_gemm like any other variant."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, gamma, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cx():
    import paper_2311_03543_amd as pa
    c = pa.Compar(0)
    vid = c.register_builtin("host_f32")
    assert c.variant_info(vid)[0] == "host_f32" and vid == c.variant_count() - 1
    yield c, vid
    c.close()


@pytest.mark.parametrize("M,N,K", [(33, 65, 129), (300, 520, 200), (1000, 300, 777)])
def test_device_operands_within_rounding_bound(cx, M, N, K):
    import torch
    c, vid = cx
    A, B = synth.gemm_operands(M, N, K, seed=M + 2 * N + K)
    dC = torch.zeros((M, N), device="cuda")
    say(f"  host_f32 M={M} N={N} K={K}")
    c.gemm_variant(vid, dev(A), dev(B), dC)
    C = host(dC)
    ref = oracle.gemm(A, B)
    assert oracle.relfro(C, ref) <= 1e-5
    assert np.all(np.abs(C.astype(np.float64) - ref) <= gamma(K) * oracle.absgemm(A, B))


def test_alpha_beta_and_leading_dimensions(cx):
    import torch
    c, vid = cx
    M, N, K = 150, 170, 131
    A, B = synth.gemm_operands(M, N, K, seed=8)
    C0 = synth.normal_matrix(M, N, 9)
    Abig = np.zeros((M, K + 5), np.float32)
    Abig[:, :K] = A
    Bbig = np.zeros((K, N + 3), np.float32)
    Bbig[:, :N] = B
    Cbig = np.zeros((M, N + 9), np.float32)
    Cbig[:, :N] = C0
    dA, dB, dC = dev(Abig), dev(Bbig), dev(Cbig)
    say("  host_f32 with alpha/beta and padded leading dimensions")
    c.gemm_variant(vid, dA[:, :K], dB[:, :N], dC[:, :N], -0.5, 2.0)
    C = host(dC)
    assert oracle.relfro(C[:, :N], oracle.gemm(A, B, -0.5, 2.0, C0)) <= 1e-5
    assert np.all(C[:, N:] == 0.0)


def test_selected_through_cmp_gemm_when_forced(cx):
    import torch
    c, vid = cx
    A, B = synth.gemm_operands(64, 96, 80, seed=10)
    dC = torch.zeros((64, 96), device="cuda")
    c.force_variant(vid)
    try:
        chosen = c.gemm(dev(A), dev(B), dC, tol=1e-5)
    finally:
        c.force_variant(-1)
    assert chosen == vid
    assert oracle.relfro(host(dC), oracle.gemm(A, B)) <= 1e-5
