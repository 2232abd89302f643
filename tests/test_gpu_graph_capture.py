"""cmp_gemm captured into a graph: after one eager call of the shape (which sizes the workspace
and fills the decision cache), the selected variant's launches — pre-passes on the caller's and
the auxiliary stream, the GEMM, the split-K reduction — are recorded by a stream capture and
replayed.  Every replay follows eager work that changes the operands, and is checked against
the FP64 oracle on the operands it saw."""
import pytest

import oracle
import synth
from gpu_util import host, say

pytestmark = pytest.mark.gpu
BOUND = {"f32_simt": 1e-5, "bf16x3": 1e-5, "fp8r": 1e-3, "bf16": 1e-2, "fp6x3": 1e-2}


@pytest.mark.parametrize("name", list(BOUND))
@pytest.mark.parametrize("M,N,K", [(512, 384, 1000), (300, 260, 4000)])   # the second splits K
def test_captured_gemm_replays(name, M, N, K):
    import torch
    import paper_2311_03543_amd as pa
    cx = pa.Compar(0)
    try:
        cx.register_builtin("fp6x3")
        cx.force_variant(cx.variant_find(name))
        tol = BOUND[name]
        A0, B0 = synth.gemm_operands(M, N, K, seed=M + K)
        dA = torch.from_numpy(A0).cuda()
        dB = torch.from_numpy(B0).cuda()
        dC = torch.zeros((M, N), device="cuda")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            say(f"  eager warm-up {name} M={M} N={N} K={K}")
            vid = cx.gemm(dA, dB, dC, tol=tol, stream=s)
            s.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                cx.gemm(dA, dB, dC, tol=tol, stream=s)
        torch.cuda.synchronize()
        assert cx.variant_info(vid)[0] == name
        for r in range(3):
            # eager work between replays: new operand values in place
            dA.mul_(-0.5 if r % 2 else 1.5)
            dB.add_(0.25)
            dC.zero_()
            torch.cuda.synchronize()
            say(f"  replay {r} of {name}")
            g.replay()
            torch.cuda.synchronize()
            A, B = host(dA), host(dB)
            err = oracle.relfro(host(dC), oracle.gemm(A, B))
            assert err <= tol, (name, r, err)
        del g
    finally:
        cx.close()


def test_reserved_workspace_keeps_captured_graph_valid():
    """cmp_reserve pins the shared workspace: a later eager call that would need more fails
    with CMP_ENOMEM instead of freeing the buffer a captured graph replays into; releasing
    the pin lets the workspace grow again."""
    import torch
    import paper_2311_03543_amd as pa
    cx = pa.Compar(0)
    try:
        M, N, K = 512, 384, 640
        cx.force_variant(cx.variant_find("bf16x3"))
        cx.reserve(M, N, K)
        A0, B0 = synth.gemm_operands(M, N, K, seed=77)
        dA, dB = torch.from_numpy(A0).cuda(), torch.from_numpy(B0).cuda()
        dC = torch.zeros((M, N), device="cuda")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            say("  reserved workspace: eager warm-up and capture of bf16x3 512x384x640")
            cx.gemm(dA, dB, dC, tol=1e-5, stream=s)
            s.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                cx.gemm(dA, dB, dC, tol=1e-5, stream=s)
        torch.cuda.synchronize()
        big = [torch.zeros((2048, 2048), device="cuda") for _ in range(3)]
        bf16x3 = cx.variant_find("bf16x3")
        with pytest.raises(pa.ComparError) as e:
            cx.gemm_variant(bf16x3, big[0], big[1], big[2])
        assert e.value.status == pa.CMP_ENOMEM
        # the selected call falls back to the best other admissible variant, which needs no
        # workspace (f32_simt at 1e-5), and still runs
        fb0 = cx.last_verify()[1]
        assert cx.gemm(big[0], big[1], big[2], tol=1e-5) == cx.variant_find("f32_simt")
        assert cx.last_verify()[1] == fb0 + 1
        dA.mul_(0.5)
        dC.zero_()
        torch.cuda.synchronize()
        g.replay()
        err = oracle.relfro(host(dC), oracle.gemm(host(dA), B0))
        assert err <= 1e-5
        cx.reserve(0, 0, 0)                       # pin released: the workspace may grow again
        assert cx.gemm(big[0], big[1], big[2], tol=1e-5) == bf16x3
        torch.cuda.synchronize()
        del g
    finally:
        cx.close()
