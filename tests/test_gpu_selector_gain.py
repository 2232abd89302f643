"""What the trained network gains over selection without it (paper Sec. 3.2: StarPU's
history-based choice picks the wrong mmul variant at several sizes; Sec. 5: better-trained
performance models as the remedy).

The learned selector (a 4-64-64-4 network trained on the GPU by the library's own kernels from
the timing history, cmp_mlp_fit_history) is compared with the two selectors that need no
network: the history nearest neighbour and the static best-per-tolerance choice.  Regret is
judged against exhaustive timing of every variant on held-out shapes, with the selection rules of
oracle/selection.py.  The history is sparse (150 timed shapes spread over [64, 8192]^3), the
setting where a fitted model has the most to add over a table lookup.

Two tables:
  * a synthetic cost table (roofline-style times with tile-quantised MFMA work and seeded
    measurement noise): deterministic, so the gain over nearest neighbour is asserted;
  * times measured on this GPU with cmp_calibrate: the network must stay within 5 % of the
    exhaustive best; its gain over nearest neighbour and static is reported, and asserted
    against static.
"""
import math

import numpy as np
import pytest

import synth
from gpu_util import say
from oracle import selection as S

pytestmark = pytest.mark.gpu
BOUNDS = [1e-5, 1e-5, 1e-3, 1e-2]      # f32_simt, bf16x3, fp8r, bf16
N_TRAIN, N_HELD = 150, 200


def synthetic_times(shapes, seed):
    """ms per variant from a cost model of the four built-ins (launch cost, operand pre-pass
    traffic, MFMA or vector work on 256 x 256 tiles with wave quantisation over 256 CUs), each
    time multiplied by a seeded log-normal factor (3 % spread) standing in for timing noise."""
    g = synth.rng(seed)
    out = []
    for M, N, K in shapes:
        M, N, K = float(M), float(N), float(K)
        ops = M * K + K * N
        tiles = math.ceil(M / 256) * math.ceil(N / 256)
        waves = math.ceil(tiles / 256)
        mfma = waves * 256 * 256 * 256          # padded tile work per K element, all waves
        f32 = 4e-3 + 2 * M * N * K / 80e12 * 1e3 + 4 * (ops + M * N) / 5e12 * 1e3
        bf16x3 = 12e-3 + 8 * ops / 4e12 * 1e3 + 6 * mfma * math.ceil(K / 32) * 32 / 1.5e15 * 1e3
        fp8r = 16e-3 + 6 * ops / 2.5e12 * 1e3 + 8 * mfma * math.ceil(K / 128) * 128 / 3.0e15 * 1e3
        bf16 = 10e-3 + 6 * ops / 4e12 * 1e3 + 2 * mfma * math.ceil(K / 32) * 32 / 1.3e15 * 1e3
        t = np.array([f32, bf16x3, fp8r, bf16])
        out.append(t * np.exp(0.03 * g.standard_normal(4)))
    return np.array(out)


def compare(c, pa, train, Ttr, held, Tho, tols, steps=5000):
    """Regret of the nearest-neighbour, static and learned selectors on the held-out rows."""
    c.history_clear()
    for (M, N, K), row in zip(train, Ttr):
        for v in range(4):
            c.history_add(int(M), int(N), int(K), v, 1, float(row[v]))
    q = [(int(m), int(n), int(k), float(t)) for (m, n, k), t in zip(held, tols)]
    res = {}
    for kind, label in [(pa.CMP_SEL_NN, "nn"), (pa.CMP_SEL_STATIC, "static")]:
        c.selector_set(kind)
        res[label] = S.regret(Tho, c.select_batch(q), list(tols), BOUNDS)
    loss = c.mlp_fit_history(steps=steps, lr=1e-3, seed=0)
    c.selector_set(pa.CMP_SEL_MLP)
    res["mlp"] = S.regret(Tho, c.select_batch(q), list(tols), BOUNDS)
    say("  regret (aggregate / mean / p95 %): " + ", ".join(
        f"{k} {100 * v['aggregate']:.2f} / {100 * v['mean']:.2f} / {100 * v['p95']:.2f}" for k, v in res.items())
        + f"; final training loss {loss:.4f}")
    return res


def test_network_gain_on_a_sparse_synthetic_table():
    import paper_2311_03543_amd as pa
    train = synth.log_uniform_shapes(N_TRAIN, 64, 8192, 50)
    held = synth.log_uniform_shapes(N_HELD, 64, 8192, 51, avoid={tuple(r) for r in train})
    tols = synth.tol_classes(N_HELD, 52)
    Ttr, Tho = synthetic_times(train, 53), synthetic_times(held, 54)
    # the held-out optimum is not one variant per tolerance: there is something to select
    best = {S.exhaustive_best(list(Tho[s]), BOUNDS, tols[s]) for s in range(N_HELD)}
    assert len(best) >= 3
    c = pa.Compar(0)
    try:
        res = compare(c, pa, train, Ttr, held, Tho, tols)
    finally:
        c.close()
    assert res["mlp"]["aggregate"] <= 0.05
    assert res["mlp"]["aggregate"] < res["nn"]["aggregate"]
    assert res["mlp"]["aggregate"] < res["static"]["aggregate"]


def test_network_gain_on_a_sparse_measured_history():
    import torch
    import paper_2311_03543_amd as pa
    train = synth.log_uniform_shapes(N_TRAIN, 64, 8192, 40)
    held = synth.log_uniform_shapes(N_HELD, 64, 8192, 41, avoid={tuple(r) for r in train})
    tols = synth.tol_classes(N_HELD, 42)
    shapes = np.vstack([train, held])
    g = torch.Generator(device="cuda").manual_seed(7)
    dA = torch.randn(int(max(s[0] * s[2] for s in shapes)), device="cuda", generator=g)
    dB = torch.randn(int(max(s[2] * s[1] for s in shapes)), device="cuda", generator=g)
    dC = torch.zeros(int(max(s[0] * s[1] for s in shapes)), device="cuda")
    c = pa.Compar(0)
    try:
        for i in range(0, len(shapes), 50):
            say(f"  calibrate shapes {i}..{min(i + 50, len(shapes))} of {len(shapes)}")
            c.calibrate([tuple(map(int, s)) for s in shapes[i:i + 50]], dA, dB, dC, warmup=2, reps=10)
        T = {}
        for (M, N, K, vid, reps, med, mn, mean) in c.history():
            T.setdefault((M, N, K), [math.nan] * 4)[vid] = med
        Ttr = np.array([T[tuple(map(int, s))] for s in train])
        Tho = np.array([T[tuple(map(int, s))] for s in held])
        assert np.all(np.isfinite(Ttr)) and np.all(np.isfinite(Tho))
        res = compare(c, pa, train, Ttr, held, Tho, tols)
    finally:
        c.close()
    assert res["mlp"]["aggregate"] <= 0.05
    assert res["mlp"]["aggregate"] < res["static"]["aggregate"]
