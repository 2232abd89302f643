"""Request stream through cmp_gemm: every request's output is checked against the full FP64
oracle within that request's tolerance, ill-conditioned operands included (served in
verify mode), and the chosen variant is always admissible for the request's tolerance."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import host, say

pytestmark = pytest.mark.gpu
BOUNDS = [1e-5, 1e-5, 1e-3, 1e-2]


def test_request_stream_outputs_within_tolerance():
    import paper_2311_03543_amd as pa
    from paper_2311_03543_amd import stream as st
    req = st.make_stream(nshapes=12, nreq=240, lo=64, hi=1024, seed=21)
    pool = st.build_pool(req["shapes"], seed=3, host_arrays=True)
    cx = pa.Compar(0)
    try:
        import torch
        A = torch.randn(1024 * 1024, device="cuda")
        B = torch.randn(1024 * 1024, device="cuda")
        C = torch.zeros(1024 * 1024, device="cuda")
        cx.calibrate([tuple(map(int, s)) for s in req["shapes"]], A, B, C, warmup=1, reps=3)
        errors = []

        def check(i, Cdev):
            sh = int(req["ranks"][i]) - 1
            kind = "ill" if req["ill"][i] else "well"
            Ah, Bh = pool[sh]["host"][kind][i % 2]
            errors.append((i, oracle.relfro(host(Cdev), oracle.gemm(Ah, Bh)), float(req["tols"][i])))

        say("  serving 240 requests")
        lat, chosen, fallbacks = st.run_stream(cx, req, pool, verify_ill=True, on_result=check)
    finally:
        cx.close()
    for i, c in enumerate(chosen):
        assert BOUNDS[c] <= req["tols"][i]
    bad = [(i, e, t) for i, e, t in errors if not e <= t]
    assert not bad, bad[:5]
    assert np.all(lat > 0)


def test_native_request_stream_outputs_within_tolerance():
    """The same kind of stream served by the library's executor (cmp_gemm_stream) in one call,
    every request with an output of its own so that all of them can be checked afterwards;
    the ids chosen for requests outside verify mode equal those of one cmp_select per request
    (a verify-mode request may fall back to a tighter variant)."""
    import torch
    import paper_2311_03543_amd as pa
    from paper_2311_03543_amd import stream as st
    req = st.make_stream(nshapes=10, nreq=200, lo=64, hi=768, seed=23)
    pool = st.build_pool(req["shapes"], seed=4, host_arrays=True)
    cx = pa.Compar(0)
    try:
        A = torch.randn(768 * 768, device="cuda")
        B = torch.randn(768 * 768, device="cuda")
        C = torch.zeros(768 * 768, device="cuda")
        shapes = [tuple(map(int, s)) for s in req["shapes"]]
        cx.calibrate(shapes, A, B, C, warmup=1, reps=3)
        outs = []
        for r in req["ranks"]:
            M, N, _ = shapes[int(r) - 1]
            outs.append(torch.zeros((M, N), device="cuda"))
        say("  serving 200 requests natively")
        lat, chosen, _ = st.run_stream_native(cx, req, pool, verify_ill=True, outputs=outs)
        want = [cx.select(*shapes[int(r) - 1], float(t)) for r, t in zip(req["ranks"], req["tols"])]
        first = [host(o) for o in outs]
        # the same stream only enqueued (sync = 0, no verify mode): the requests that ran
        # without verify mode before get the same variants and the same bits
        for o in outs:
            o.zero_()
        say("  serving 200 requests natively, enqueue only")
        chosen2, lat2 = cx.gemm_stream(st.requests_of(req, pool, outs), np.asarray(req["tols"], np.float64),
                                       verify=np.zeros(len(outs), bool), sync=False)
        torch.cuda.synchronize()
        assert lat2 is None
        for i, o in enumerate(outs):
            if not req["ill"][i]:
                assert chosen2[i] == chosen[i]
                assert np.array_equal(first[i].view(np.uint32), host(o).view(np.uint32))
    finally:
        cx.close()
    assert all(c == w for c, w, ill in zip(chosen, want, req["ill"]) if not ill)
    assert np.all(lat > 0)
    for i in range(len(chosen)):
        assert BOUNDS[chosen[i]] <= req["tols"][i]
        sh = int(req["ranks"][i]) - 1
        kind = "ill" if req["ill"][i] else "well"
        Ah, Bh = pool[sh]["host"][kind][i % 2]
        err = oracle.relfro(host(outs[i]), oracle.gemm(Ah, Bh))
        assert err <= req["tols"][i], (i, err, req["tols"][i])
