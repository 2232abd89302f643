"""Grouped launches of many GEMMs of uneven shapes: every configuration gives results
bit-identical to one launch per problem of the variant whose arithmetic it uses (the FP32 SIMT
tiles: f32_simt, each entry the same chain of FP32 FMAs over k; the MFMA configuration: an
unsplit bf16x3 call, the same pre-pass images and the same tile code), the autotuned plan is
within 1e-5 of the FP64 oracle per problem, and the captured graph replays correctly several
times with eager work in between."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cx():
    import paper_2311_03543_amd as pa
    c = pa.Compar(0)
    yield c
    c.close()


def _problems(count, seed, lo=32, hi=1024):
    shapes = synth.log_uniform_shapes(count, lo, hi, seed)
    g = synth.rng(seed + 100)
    probs = []
    for s, (M, N, K) in enumerate(shapes):
        A = g.standard_normal((M, K), dtype=np.float32)
        B = g.standard_normal((K, N), dtype=np.float32)
        probs.append((A, B))
    return probs


def _run_separate(cx, dprobs, variant=0):
    """One launch per problem of built-in variant `variant` (unsplit: the grouped MFMA
    configuration runs every problem's whole K range in one tile)."""
    import torch
    outs = []
    cx.set_split_k(1)
    try:
        for dA, dB in dprobs:
            dC = torch.zeros((dA.shape[0], dB.shape[1]), device="cuda")
            cx.gemm_variant(variant, dA, dB, dC)
            outs.append(dC)
    finally:
        cx.set_split_k(0)
    return [host(o) for o in outs]


def test_every_config_bit_identical_to_separate(cx):
    import torch
    import paper_2311_03543_amd as pa
    probs = _problems(40, 1, 32, 600)
    dprobs = [(dev(A), dev(B)) for A, B in probs]
    refs = {}
    assert sorted({pa.grouped_config_variant(c) for c in range(len(pa.grouped_configs()))}) == [0, 1]
    for cfg in range(len(pa.grouped_configs())):
        v = pa.grouped_config_variant(cfg)
        if v not in refs:
            refs[v] = _run_separate(cx, dprobs, v)
        ref = refs[v]
        outs = [torch.zeros((A.shape[0], B.shape[1]), device="cuda") for A, B in probs]
        say(f"  grouped config {cfg} {pa.grouped_configs()[cfg]} (variant {v})")
        plan = cx.grouped_plan([(a, b, o) for (a, b), o in zip(dprobs, outs)], config=cfg)
        try:
            plan.launch()
            got = [host(o) for o in outs]
        finally:
            plan.destroy()
        for g_, r in zip(got, ref):
            assert np.array_equal(g_.view(np.uint32), r.view(np.uint32))


def test_autotuned_plan_matches_oracle_and_graph_replays(cx):
    import torch
    probs = _problems(64, 2)
    dprobs = [(dev(A), dev(B)) for A, B in probs]
    outs = [torch.zeros((A.shape[0], B.shape[1]), device="cuda") for A, B in probs]
    say("  grouped autotune over 64 problems")
    plan = cx.grouped_plan([(a, b, o) for (a, b), o in zip(dprobs, outs)], config=-1, reps=3)
    try:
        info = plan.info()
        assert 0 <= info["config"] < len(info["config_ms"])
        assert all(v is not None and v > 0 for v in info["config_ms"])
        assert info["config_ms"][info["config"]] == min(info["config_ms"])
        plan.launch()
        first = [host(o) for o in outs]
        for (A, B), C in zip(probs, first):
            assert oracle.relfro(C, oracle.gemm(A, B)) <= 1e-5
        for rep in range(3):
            for o in outs:
                o.zero_()                       # eager work between replays
            torch.cuda.synchronize()
            say(f"  graph replay {rep}")
            plan.graph_launch()
            again = [host(o) for o in outs]
            for a_, b_ in zip(again, first):
                assert np.array_equal(a_.view(np.uint32), b_.view(np.uint32))
    finally:
        plan.destroy()


def test_degenerate_problems_in_a_group(cx):
    import torch
    A, B = synth.gemm_operands(70, 90, 50, seed=3)
    C0 = synth.normal_matrix(70, 90, 4)
    dA, dB = dev(A), dev(B)
    c1 = dev(C0)                                            # alpha = 0: C = beta C
    c2 = torch.zeros((70, 90), device="cuda")               # ordinary
    c3 = dev(C0)                                            # K = 0: C = beta C
    c4 = dev(C0)                                            # alpha, beta general
    e1 = torch.zeros((0, 90), device="cuda")                # M = 0
    z = torch.zeros((70, 0), device="cuda")
    zb = torch.zeros((0, 90), device="cuda")
    plan = cx.grouped_plan([(dA, dB, c1, 0.0, 2.0), (dA, dB, c2), (z, zb, c3, 1.0, 0.5),
                            (dA, dB, c4, -1.5, 0.25), (torch.zeros((0, 50), device="cuda"), dB, e1)],
                           config=0)
    try:
        say("  grouped degenerate problems")
        plan.launch()
        assert np.array_equal(host(c1), (2.0 * C0.astype(np.float64)).astype(np.float32))
        assert oracle.relfro(host(c2), oracle.gemm(A, B)) <= 1e-5
        assert np.array_equal(host(c3), (0.5 * C0.astype(np.float64)).astype(np.float32))
        assert oracle.relfro(host(c4), oracle.gemm(A, B, -1.5, 0.25, C0)) <= 1e-5
    finally:
        plan.destroy()


@pytest.mark.parametrize("cfg", [0, 4, 7, 10])
def test_tile_queue_with_many_more_tiles_than_workgroups(cx, cfg):
    """A group with several times more tiles than resident workgroups, so that most tiles are
    claimed from the plan's counter: every problem bit-identical to its own launch of the
    configuration's variant, on an eager launch, a second eager launch (the counter is zeroed
    again) and a graph replay."""
    import torch
    import paper_2311_03543_amd as pa
    probs = _problems(300, 7, 192, 1024)
    dprobs = [(dev(A), dev(B)) for A, B in probs]
    ref = _run_separate(cx, dprobs, pa.grouped_config_variant(cfg))
    outs = [torch.zeros((A.shape[0], B.shape[1]), device="cuda") for A, B in probs]
    plan = cx.grouped_plan([(a, b, o) for (a, b), o in zip(dprobs, outs)], config=cfg)
    try:
        info = plan.info()
        say(f"  grouped config {cfg}: {info['tiles']} tiles on {info['grid']} workgroups")
        assert info["tiles"] >= 3 * info["grid"]
        for how in ("launch", "launch", "graph"):
            for o in outs:
                o.fill_(float("nan"))
            torch.cuda.synchronize()
            plan.launch() if how == "launch" else plan.graph_launch()
            got = [host(o) for o in outs]
            for g_, r in zip(got, ref):
                assert np.array_equal(g_.view(np.uint32), r.view(np.uint32)), how
    finally:
        plan.destroy()


def test_mfma_configuration_needs_operands_read(cx):
    """The bf16x3 configuration reads A and B of every problem, so a group holding a problem
    with alpha = 0 or K = 0 (C = beta C, operands never read) is refused for it, and the
    autotuner leaves it out; the SIMT configurations serve such a group."""
    import torch
    import paper_2311_03543_amd as pa
    mfma = [c for c in range(len(pa.grouped_configs())) if pa.grouped_config_variant(c) == 1]
    assert len(mfma) == 1
    A, B = synth.gemm_operands(70, 90, 50, seed=5)
    C0 = synth.normal_matrix(70, 90, 6)
    dA, dB = dev(A), dev(B)
    for extra in ((dA, dB, dev(C0), 0.0, 2.0),
                  (torch.zeros((70, 0), device="cuda"), torch.zeros((0, 90), device="cuda"), dev(C0), 1.0, 0.5)):
        group = [(dA, dB, torch.zeros((70, 90), device="cuda")), extra]
        with pytest.raises(pa.ComparError) as err:
            cx.grouped_plan(group, config=mfma[0])
        assert err.value.status == pa.CMP_EUNSUPPORTED
        plan = cx.grouped_plan(group, config=-1, reps=2)
        try:
            info = plan.info()
            assert info["config_ms"][mfma[0]] is None and info["config"] != mfma[0]
            assert all(v is not None for i, v in enumerate(info["config_ms"]) if i != mfma[0])
        finally:
            plan.destroy()


def test_mfma_configuration_unaligned_operands(cx):
    """The bf16x3 configuration on operands that are column slices of wider tensors (leading
    dimensions that are not multiples of 4, first elements off 16-byte alignment), with alpha and
    beta general: the pre-pass takes its element-wise load paths, and every problem stays
    bit-identical to its own unsplit bf16x3 call."""
    import torch
    import paper_2311_03543_amd as pa
    mfma = next(c for c in range(len(pa.grouped_configs())) if pa.grouped_config_variant(c) == 1)
    g = synth.rng(31)
    shapes = [(77, 130, 45), (300, 257, 129), (5, 600, 70), (513, 33, 300)]
    group, refs, outs = [], [], []
    for i, (M, N, K) in enumerate(shapes):
        Aw = dev(g.standard_normal((M, K + 3), dtype=np.float32))
        Bw = dev(g.standard_normal((K, N + 5), dtype=np.float32))
        C0 = g.standard_normal((M, N), dtype=np.float32)
        A, B = Aw[:, 1:K + 1], Bw[:, 3:N + 3]          # lda = K + 3, ldb = N + 5, misaligned starts
        alpha, beta = (1.0, 0.0) if i % 2 == 0 else (-0.75, 0.5)
        ref = dev(C0)
        cx.set_split_k(1)
        try:
            cx.gemm_variant(1, A, B, ref, alpha, beta)
        finally:
            cx.set_split_k(0)
        refs.append(host(ref))
        out = dev(C0)
        outs.append(out)
        group.append((A, B, out, alpha, beta))
    plan = cx.grouped_plan(group, config=mfma)
    try:
        say("  grouped bf16x3 on sliced operands")
        plan.launch()
        for o, r in zip(outs, refs):
            assert np.array_equal(host(o).view(np.uint32), r.view(np.uint32))
    finally:
        plan.destroy()
