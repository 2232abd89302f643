"""GPU tests of the runtime around the kernels: selection through cmp_gemm, timing and
calibration, verify mode with its FP64 probe, and the learned selector's kernels against the
binary64 network oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, say
from oracle import mlp as omlp
from oracle import selection as S

pytestmark = pytest.mark.gpu
BOUNDS = [1e-5, 1e-5, 1e-3, 1e-2]


@pytest.fixture()
def cx():
    import paper_2311_03543_amd as pa
    c = pa.Compar(0)
    yield c
    c.close()


def test_builtin_registration(cx):
    import paper_2311_03543_amd as pa
    assert [cx.variant_info(i)[0] for i in range(cx.variant_count())] == list(pa.BUILTIN_VARIANTS)
    assert [cx.variant_info(i)[2] for i in range(4)] == BOUNDS


@pytest.mark.parametrize("tol", [1e-5, 1e-3, 1e-2])
def test_cmp_gemm_selected_variant_is_admissible_and_accurate(cx, tol):
    import torch
    A, B = synth.gemm_operands(512, 384, 640, seed=21)
    dC = torch.zeros((512, 384), device="cuda")
    say(f"  cmp_gemm tol={tol}")
    chosen = cx.gemm(dev(A), dev(B), dC, tol=tol)
    assert BOUNDS[chosen] <= tol
    assert oracle.relfro(host(dC), oracle.gemm(A, B)) <= tol


def test_timing_and_calibration_feed_selection(cx):
    import torch
    shapes = [(256, 256, 256), (1024, 1024, 1024), (64, 4096, 128)]
    A = torch.randn(1024 * 4096, device="cuda")
    B = torch.randn(4096 * 4096, device="cuda")
    C = torch.zeros(4096 * 1024, device="cuda")
    say("  calibrate 3 shapes x 4 variants")
    cx.calibrate(shapes, A, B, C, warmup=1, reps=5)
    rows = cx.history()
    assert len(rows) == 12
    for (M, N, K, vid, reps, med, mn, mean) in rows:
        assert reps == 5 and 0 < mn <= med
    # a second calibration of the same shapes is skipped (resumable)
    cx.calibrate(shapes, A, B, C, warmup=1, reps=5)
    assert len(cx.history()) == 12
    # nearest-neighbour selection on recorded shapes = exhaustive best of the table
    T = np.zeros((3, 4))
    for (M, N, K, vid, reps, med, mn, mean) in rows:
        T[shapes.index((M, N, K)), vid] = med
    for s, (M, N, K) in enumerate(shapes):
        for tol in synth.TOL_CLASSES:
            assert cx.select(M, N, K, tol) == S.exhaustive_best(list(T[s]), BOUNDS, tol)


def test_verify_mode_probe_matches_oracle(cx):
    import torch
    import paper_2311_03543_amd as pa
    A, B = synth.gemm_operands(300, 260, 200, seed=22)
    C0 = synth.normal_matrix(300, 260, 23)
    dC = dev(C0)
    cx.set_flags(pa.CMP_FLAG_VERIFY)
    say("  verify-mode cmp_gemm tol=1e-2, beta=0.5")
    chosen = cx.gemm(dev(A), dev(B), dC, alpha=1.0, beta=0.5, tol=1e-2)
    est, fallbacks = cx.last_verify()
    C = host(dC)
    assert fallbacks == 0
    # the library's probe vector is splitmix64-Rademacher with seed 0x5eed (first call)
    x = oracle.rademacher_splitmix(260, 0x5EED)
    ref = oracle.freivalds(A, B, C, x, alpha=1.0, beta=0.5, C0=C0)
    assert abs(est - ref) <= 1e-9 * max(ref, 1e-300), (est, ref)
    assert oracle.relfro(C, oracle.gemm(A, B, 1.0, 0.5, C0)) <= BOUNDS[chosen]


@pytest.mark.parametrize("name", ["f32_simt", "bf16", "fp8r"])
def test_verify_mode_with_a_column_slice_of_c(name):
    """Verify mode with beta != 0 and C a column slice of a wider matrix (ldc > N): the probe
    reads the kept old C at its own packed pitch, so it equals the oracle's probe of the same
    C, no fallback is taken, and the columns of the wide matrix outside the slice are untouched.
    cmp_freivalds itself takes the caller's old C at ldc: a strided slice there too."""
    import paper_2311_03543_amd as pa
    c = pa.Compar(0)
    try:
        M, N, K, W, off = 300, 200, 250, 333, 71
        A, B = synth.gemm_operands(M, N, K, seed=26)
        wide0 = synth.normal_matrix(M, W, 27)
        dwide = dev(wide0)
        dC = dwide[:, off:off + N]
        assert dC.stride(0) == W
        vid = c.variant_find(name)
        c.force_variant(vid)
        c.set_flags(pa.CMP_FLAG_VERIFY)
        say(f"  verify-mode cmp_gemm {name} beta=0.5 on a column slice (ldc {W}, N {N})")
        chosen = c.gemm(dev(A), dev(B), dC, alpha=1.0, beta=0.5, tol=1e-2)
        est, fallbacks = c.last_verify()
        wide = host(dwide)
        assert chosen == vid and fallbacks == 0
        C0 = np.ascontiguousarray(wide0[:, off:off + N])
        Cout = np.ascontiguousarray(wide[:, off:off + N])
        x = oracle.rademacher_splitmix(N, 0x5EED)
        ref = oracle.freivalds(A, B, Cout, x, alpha=1.0, beta=0.5, C0=C0)
        assert abs(est - ref) <= 1e-9 * max(ref, 1e-300), (est, ref)
        assert oracle.relfro(Cout, oracle.gemm(A, B, 1.0, 0.5, C0)) <= BOUNDS[vid]
        assert np.array_equal(wide[:, :off], wide0[:, :off])
        assert np.array_equal(wide[:, off + N:], wide0[:, off + N:])
        # the probe entry point with a strided old C (ld = ldc of the product's C)
        say("  cmp_freivalds with strided C and old C")
        dC0 = dev(wide0)[:, off:off + N]
        got = c.freivalds(dev(A), dev(B), dC, x, alpha=1.0, beta=0.5, C0=dC0)
        assert abs(got - ref) <= 1e-9 * max(ref, 1e-300), (got, ref)
    finally:
        c.close()


@pytest.mark.parametrize("name", ["bf16x3", "fp8r", "bf16"])
def test_verify_mode_on_a_split_k_call(name):
    """Verify mode over a split-K launch (4 output tiles over K = 4000): the FP64 probe sees the
    reduced C, agrees with the oracle's probe of the same C, and no fallback is taken."""
    import paper_2311_03543_amd as pa
    c = pa.Compar(0)
    try:
        M, N, K = 300, 260, 4000
        vid = c.variant_find(name)
        assert c.split_k(vid, M, N, K) > 1
        A, B = synth.gemm_operands(M, N, K, seed=24)
        C0 = synth.normal_matrix(M, N, 25)
        dC = dev(C0)
        c.force_variant(vid)
        c.set_flags(pa.CMP_FLAG_VERIFY)
        say(f"  verify-mode split-K cmp_gemm {name} beta=0.5")
        chosen = c.gemm(dev(A), dev(B), dC, alpha=1.0, beta=0.5, tol=1e-2)
        est, fallbacks = c.last_verify()
        C = host(dC)
        assert chosen == vid and fallbacks == 0
        x = oracle.rademacher_splitmix(N, 0x5EED)            # the context's first call
        ref = oracle.freivalds(A, B, C, x, alpha=1.0, beta=0.5, C0=C0)
        assert abs(est - ref) <= 1e-9 * max(ref, 1e-300), (est, ref)
        assert oracle.relfro(C, oracle.gemm(A, B, 1.0, 0.5, C0)) <= BOUNDS[vid]
    finally:
        c.close()


def test_mlp_selector_estimates_optional_variants_from_history():
    """With the learned selector, the four default variants are predicted by the network and any
    other variant by the ln(us) of its nearest timed history shape; the choice is the argmin over
    both, admissible variants only."""
    import math
    import paper_2311_03543_amd as pa
    c = pa.Compar(0)
    try:
        f6, hv = c.register_builtin("fp6x3"), c.register_builtin("host_f32")
        assert (f6, hv) == (4, 5)
        p = np.zeros(synth.mlp_param_count(), np.float32)
        p[-4:] = [3.0, 2.0, 1.0, 0.5]                       # constant ln(us) per default variant
        c.mlp_set_params(p)
        c.mlp_set_norm(np.zeros(4), np.ones(4), np.zeros(4), np.ones(4))
        c.selector_set(pa.CMP_SEL_MLP)
        ms = lambda ln_us: math.exp(ln_us) / 1000.0
        c.history_add(1024, 1024, 1024, f6, 1, ms(0.2))
        c.history_add(1024, 1024, 1024, hv, 1, ms(0.3))
        c.history_add(64, 64, 64, hv, 1, ms(9.0))           # farther from the query below
        q = (1000, 1000, 1000)
        assert c.select(*q, 1e-2) == f6                     # 0.2 beats 0.5 (bf16) and 0.3
        assert c.select(*q, 1e-3) == hv                     # fp6x3 inadmissible: 0.3 beats 1.0
        assert c.select(*q, 1e-5) == hv                     # 0.3 beats 2.0 (bf16x3)
        c.history_add(1024, 1024, 1024, hv, 1, ms(5.0))     # the later record of a shape counts
        assert c.select(*q, 1e-5) == 1 and c.select(*q, 1e-3) == 2
        assert c.select(70, 70, 70, 1e-5) == 1              # nearest host record: 9.0
    finally:
        c.close()


def test_split_k_prices_k_blocks_from_this_device_history(cx):
    """The split-K cost model prices a K block at the per-block time the context's own history
    implies (a timed shape whose tiles fill every CU), within [0.75, 1.33] of the built-in
    constant: a slow record means more slices, a fast one fewer, no record the constant."""
    vid = cx.variant_find("bf16")
    shapes = [(m, m, k) for m in (256, 512, 768, 1024, 1536, 2048) for k in (2048, 4096, 8192, 16384)]
    cx.history_clear()
    s0 = [cx.split_k(vid, *s) for s in shapes]
    cx.history_add(8192, 8192, 8192, vid, 1, 10.0)        # far slower than the constant implies
    s1 = [cx.split_k(vid, *s) for s in shapes]
    cx.history_clear()
    cx.history_add(8192, 8192, 8192, vid, 1, 0.3)         # far faster
    s2 = [cx.split_k(vid, *s) for s in shapes]
    cx.history_clear()
    assert [cx.split_k(vid, *s) for s in shapes] == s0
    assert all(a >= b for a, b in zip(s1, s0)) and any(a > b for a, b in zip(s1, s0))
    assert all(a <= b for a, b in zip(s2, s0)) and any(a < b for a, b in zip(s2, s0))
    # shapes too small to fill the CUs, or with a short K, do not inform the price
    cx.history_add(1024, 1024, 8192, vid, 1, 10.0)
    cx.history_add(8192, 8192, 512, vid, 1, 10.0)
    assert [cx.split_k(vid, *s) for s in shapes] == s0
    cx.history_clear()


def test_injected_failure_falls_back(monkeypatch):
    """COMPAR_FAULT=bf16:1 makes every bf16 call fail; cmp_gemm must fall back once to the
    best other admissible variant (fp8r by the recorded times) and still meet tol."""
    import torch
    import paper_2311_03543_amd as pa
    monkeypatch.setenv("COMPAR_FAULT", "bf16:1")      # read by cmp_init
    c = pa.Compar(0)
    try:
        A, B = synth.gemm_operands(256, 256, 256, seed=5)
        C = torch.zeros((256, 256), device="cuda")
        for i, t in enumerate([4.0, 3.0, 2.0, 1.0]):
            c.history_add(256, 256, 256, i, 1, t)
        say("  cmp_gemm with injected bf16 failure")
        chosen = c.gemm(dev(A), dev(B), C, tol=1e-2)
        assert chosen == 2 and c.last_verify()[1] == 1
        assert oracle.relfro(host(C), oracle.gemm(A, B)) <= 1e-3
    finally:
        c.close()


# ---- learned selector kernels vs the binary64 oracle ------------------------------

def _mlp_data(n, seed):
    shapes = synth.log_uniform_shapes(n, 64, 8192, seed)
    tols = synth.tol_classes(n, seed + 1)
    X = omlp.features(shapes[:, 0], shapes[:, 1], shapes[:, 2], tols)
    # a smooth synthetic log-time surface per variant (stand-in targets)
    flops = np.log(2.0 * shapes.prod(axis=1))
    Y = np.stack([flops - 24.0 + 0.1 * X[:, 0], flops - 26.0 + 0.2 * X[:, 1],
                  flops - 26.5 + 0.05 * X[:, 2], flops - 27.0], axis=1)
    return X, Y


def test_mlp_gradient_matches_oracle(cx):
    X, Y = _mlp_data(2000, 31)
    mx, sx = omlp.standardize_stats(X)
    my, sy = omlp.standardize_stats(Y)
    Xs, Ys = (X - mx) / sx, (Y - my) / sy
    p0 = synth.mlp_init(7)
    cx.mlp_set_params(p0)
    say("  mlp gradient n=2000")
    loss, g = cx.mlp_grad(Xs.astype(np.float32), Ys.astype(np.float32))
    rl, rg = omlp.loss_and_grad(p0.astype(np.float64), Xs.astype(np.float32).astype(np.float64),
                                Ys.astype(np.float32).astype(np.float64))
    assert abs(loss - rl) <= 1e-5 * abs(rl)
    assert np.linalg.norm(g - rg) <= 1e-4 * np.linalg.norm(rg)


def test_mlp_training_trajectory_matches_oracle(cx):
    X, Y = _mlp_data(2000, 33)
    p0 = synth.mlp_init(8)
    cx.mlp_set_params(p0)
    say("  mlp train 50 steps")
    trace = cx.mlp_train(X.astype(np.float32), Y.astype(np.float32), steps=50, lr=1e-3)
    p_gpu = cx.mlp_get_params()
    mx, sx, my, sy = cx.mlp_get_norm()
    Xf, Yf = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    omx, osx = omlp.standardize_stats(Xf)
    omy, osy = omlp.standardize_stats(Yf)
    assert np.allclose(mx, omx, rtol=1e-6) and np.allclose(sx, osx, rtol=1e-5)
    p_ref, losses = omlp.train(p0.astype(np.float64), (Xf - omx) / osx, (Yf - omy) / osy, 50, 1e-3)
    assert np.allclose(trace, losses, rtol=1e-4)
    assert np.linalg.norm(p_gpu - p_ref) <= 1e-3 * np.linalg.norm(p_ref)


def test_mlp_inference_matches_oracle(cx):
    X, _ = _mlp_data(3000, 35)
    p = synth.mlp_init(9)
    cx.mlp_set_params(p)
    Xs = ((X - X.mean(0)) / X.std(0)).astype(np.float32)
    say("  mlp inference n=3000")
    got = cx.mlp_infer(Xs)
    ref, _ = omlp.forward(p.astype(np.float64), Xs.astype(np.float64))
    assert np.max(np.abs(got - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))


def test_mlp_selector_uses_network(cx):
    import paper_2311_03543_amd as pa
    # a network whose output favours variant 3 everywhere (output bias), zero weights
    p = np.zeros(synth.mlp_param_count(), np.float32)
    p[-4:] = [3.0, 2.0, 1.0, 0.0]
    cx.mlp_set_params(p)
    cx.mlp_set_norm(np.zeros(4), np.ones(4), np.zeros(4), np.ones(4))
    cx.selector_set(pa.CMP_SEL_MLP)
    assert cx.select_batch([(100, 200, 300, 1e-2), (100, 200, 300, 1e-3), (5000, 5000, 64, 1e-5)]) == [3, 2, 1]


def test_mlp_checkpoint_restores_selection(tmp_path):
    """A network trained on this device, saved and loaded into a fresh context, infers the same
    ln-times bit for bit and makes the same choices over a batch of shapes."""
    import paper_2311_03543_amd as pa
    X, Y = _mlp_data(400, 36)
    a = pa.Compar(0)
    b = pa.Compar(0)
    try:
        mx, sx, my, sy = X.mean(0), X.std(0), Y.mean(0), Y.std(0)
        a.mlp_set_params(synth.mlp_init(10))
        a.mlp_set_norm(mx, sx, my, sy)
        a.mlp_train(((X - mx) / sx).astype(np.float32), ((Y - my) / sy).astype(np.float32), 200, 1e-2)
        p = str(tmp_path / "net.txt")
        a.mlp_save(p)
        b.mlp_load(p)
        Xs = ((X[:64] - mx) / sx).astype(np.float32)
        assert a.mlp_infer(Xs).tobytes() == b.mlp_infer(Xs).tobytes()
        a.selector_set(pa.CMP_SEL_MLP)
        b.selector_set(pa.CMP_SEL_MLP)
        rng = np.random.default_rng(11)
        qs = [(int(m), int(n), int(k), t) for (m, n, k), t in
              zip(rng.integers(16, 9000, (60, 3)), rng.choice([1e-5, 1e-3, 1e-2], 60))]
        say("  mlp checkpoint: 60 selections")
        assert a.select_batch(qs) == b.select_batch(qs)
    finally:
        a.close()
        b.close()


def test_call_log_gpu(cx, tmp_path):
    """CMP_FLAG_LOG on the GPU: measured time from the call's HIP event pair, the selector's
    predicted time from the history, the verify-mode residual, and no measurement for a call
    made during stream capture."""
    import json
    import torch
    import paper_2311_03543_amd as pa
    M, N, K = 320, 256, 384
    A, B = synth.gemm_operands(M, N, K, seed=5)
    dA, dB = dev(A), dev(B)
    dC = torch.zeros((M, N), device="cuda")
    for vid in range(4):
        med, mn, mean = cx.time_variant(vid, dA, dB, dC, warmup=1, reps=3)
        cx.history_add(M, N, K, vid, 3, med, mn, mean)
    path = str(tmp_path / "gpu_calls.jsonl")
    cx.set_log_file(path)
    cx.set_flags(pa.CMP_FLAG_LOG)
    say("  logged cmp_gemm x3 (plain, verify)")
    for tol in (1e-2, 1e-5):
        cx.gemm(dA, dB, dC, tol=tol)
    cx.set_flags(pa.CMP_FLAG_LOG | pa.CMP_FLAG_VERIFY)
    vchosen = cx.gemm(dA, dB, dC, tol=1e-3)
    cx.set_flags(pa.CMP_FLAG_LOG)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        cx.gemm(dA, dB, dC, tol=1e-2)          # warm: the capture only enqueues kernels
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            cx.gemm(dA, dB, dC, tol=1e-2)
    g.replay()
    torch.cuda.synchronize()
    cx.log_flush()
    recs = [json.loads(l) for l in open(path).read().splitlines()]
    assert [r["call"] for r in recs] == [1, 2, 3, 4, 5]
    T = {r[3]: r[5] for r in cx.history()}
    for r in recs[:4]:
        assert r["selector"] == "nn" and r["measured_us"] > 0 and (r["M"], r["N"], r["K"]) == (M, N, K)
        assert r["predicted_us"] == pytest.approx(1e3 * T[r["id"]], rel=1e-6)
    assert recs[0]["residual"] is None and recs[1]["residual"] is None
    assert recs[2]["id"] == vchosen and 0 <= recs[2]["residual"] <= 1e-3
    assert recs[4]["measured_us"] is None and recs[4]["variant"] == recs[3]["variant"]
    assert oracle.relfro(host(dC), oracle.gemm(A, B)) <= 1e-2
