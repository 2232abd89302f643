"""cmp_gemm_variant_static: the allocation-free form of cmp_gemm_variant, its workspace taken from
the library's fixed device array.  Checked against cmp_gemm_variant (bit-identical: the same
kernels) and against the FP64 oracle, on two calls in a row per variant, the second with a
smaller input whose images and padding overwrite less of the shared array; then its errors."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu
GPU_VARIANTS = ["f32_simt", "bf16x3", "fp8r", "bf16", "fp6x3"]
BOUND = {"f32_simt": 1e-5, "bf16x3": 1e-5, "fp8r": 1e-3, "bf16": 1e-2, "fp6x3": 1e-2}


@pytest.fixture(scope="module")
def cx():
    import paper_2311_03543_amd as pa
    c = pa.Compar(0)
    c.register_builtin("fp6x3")
    yield c
    c.close()


@pytest.mark.parametrize("name", GPU_VARIANTS)
def test_static_workspace_matches_gemm_variant(cx, name):
    import torch
    vid = cx.variant_find(name)
    # a split-K shape (few tiles, long K) first, then a smaller ragged one
    for (M, N, K), alpha, beta in (((700, 520, 3000), 1.0, 0.0), ((300, 257, 129), -0.5, 2.0)):
        say(f"  static workspace {name} M={M} N={N} K={K} alpha={alpha} beta={beta}")
        A, B = synth.gemm_operands(M, N, K, seed=M + N + K)
        C0 = synth.normal_matrix(M, N, M * N)
        dA, dB = dev(A), dev(B)
        c_static, c_ref = dev(C0), dev(C0)
        cx.gemm_variant_static(vid, dA, dB, c_static, alpha, beta)
        cx.gemm_variant(vid, dA, dB, c_ref, alpha, beta)
        torch.cuda.synchronize()
        got, ref = host(c_static), host(c_ref)
        assert np.array_equal(got, ref)
        assert oracle.relfro(got, oracle.gemm(A, B, alpha, beta, C0)) <= BOUND[name]


def test_static_workspace_errors(cx):
    import torch
    import paper_2311_03543_amd as pa
    # bf16x3 at 8192 x 8192 x 4096 needs 256 MiB of images: more than the fixed array holds;
    # the call fails before any launch and C is left as it was
    M = N = 8192
    K = 4096
    dA = torch.zeros((M, K), device="cuda")
    dB = torch.zeros((K, N), device="cuda")
    dC = torch.full((M, N), 3.0, device="cuda")
    with pytest.raises(pa.ComparError) as e:
        cx.gemm_variant_static(cx.variant_find("bf16x3"), dA, dB, dC)
    assert e.value.status == pa.CMP_ENOMEM
    torch.cuda.synchronize()
    assert bool((dC == 3.0).all())
    del dA, dB, dC
    # a host-target variant has no GPU workspace to take
    small = [torch.ones((8, 8), device="cuda") for _ in range(3)]
    hv = cx.register_builtin("host_f32")
    with pytest.raises(pa.ComparError) as e:
        cx.gemm_variant_static(hv, *small)
    assert e.value.status == pa.CMP_EUNSUPPORTED
