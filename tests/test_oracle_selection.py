"""Pins of the selection rules and of the Freivalds probe oracle."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import selection as S

BOUNDS = [1e-5, 1e-5, 1e-3, 1e-2]      # f32_simt, bf16x3, fp8r, bf16


def test_admissible_sets():
    assert S.admissible(BOUNDS, 1e-5) == [0, 1]
    assert S.admissible(BOUNDS, 1e-3) == [0, 1, 2]
    assert S.admissible(BOUNDS, 1e-2) == [0, 1, 2, 3]
    assert S.admissible(BOUNDS, 1e-8) == []


def test_tiebreak_prefers_tighter_then_lower_id():
    assert S.argmin_tiebreak([1.0, 1.0, 1.0, 1.0], [0, 1, 2, 3], BOUNDS) == 0
    assert S.argmin_tiebreak([2.0, 1.0, 1.0, 1.0], [0, 1, 2, 3], BOUNDS) == 1
    assert S.argmin_tiebreak([2.0, 2.0, 1.0, 1.0], [0, 1, 2, 3], BOUNDS) == 2


def test_exhaustive_best():
    t = [5.0, 3.0, 2.0, 1.0]
    assert S.exhaustive_best(t, BOUNDS, 1e-5) == 1
    assert S.exhaustive_best(t, BOUNDS, 1e-3) == 2
    assert S.exhaustive_best(t, BOUNDS, 1e-2) == 3


def test_nearest_row_and_ties():
    shapes = [(64, 64, 64), (128, 128, 128), (64, 64, 64), (4096, 4096, 4096)]
    assert S.nearest_row(shapes, 64, 64, 64) == 0          # exact match, earliest of duplicates
    assert S.nearest_row(shapes, 90, 91, 92) == 0 or S.nearest_row(shapes, 90, 91, 92) == 1
    assert S.nearest_row(shapes, 3000, 5000, 4096) == 3
    # equidistant in log2 space between 64^3 and 256^3 -> earliest row
    assert S.nearest_row([(256, 256, 256), (64, 64, 64)], 128, 128, 128) == 0


def test_regret_perfect_predictor_is_zero():
    g = synth.rng(3)
    T = g.uniform(1, 10, (50, 4))
    tols = synth.tol_classes(50, 4)
    best = [S.exhaustive_best(list(T[s]), BOUNDS, tols[s]) for s in range(50)]
    r = S.regret(T, best, tols, BOUNDS)
    assert r["aggregate"] == 0.0 and r["mean"] == 0.0


def test_nn_on_training_shapes_is_exact():
    g = synth.rng(5)
    shapes = synth.log_uniform_shapes(40, 64, 8192, 6)
    T = g.uniform(1, 10, (40, 4))
    tols = synth.tol_classes(40, 7)
    choices = [S.nn_select(shapes, T, BOUNDS, *shapes[s], tols[s]) for s in range(40)]
    assert S.regret(T, choices, tols, BOUNDS)["aggregate"] == 0.0


def test_regret_known_value():
    T = np.array([[1.0, 2.0, 3.0, 4.0], [4.0, 1.0, 1.0, 1.0]])
    tols = [1e-2, 1e-2]
    r = S.regret(T, [1, 1], tols, BOUNDS)             # best: 0 (1.0) and 1 (1.0)
    assert math.isclose(r["aggregate"], (2.0 + 1.0) / (1.0 + 1.0) - 1.0)


def test_static_choice():
    T = [[1.0, 5.0, 5.0, 5.0], [9.0, 2.0, 1.0, 0.5]]
    assert S.static_choice(T, BOUNDS, 1e-2) == 3   # totals 10, 7, 6, 5.5
    assert S.static_choice(T, BOUNDS, 1e-5) == 1   # admissible {0,1}: 10 vs 7
    assert S.static_choice([], BOUNDS, 1e-3) == 0


def test_log_uniform_shapes_range_and_distinct():
    s = synth.log_uniform_shapes(500, 64, 8192, 2)
    assert s.min() >= 64 and s.max() <= 8192
    assert len({tuple(r) for r in s}) == 500
    h = synth.log_uniform_shapes(100, 64, 8192, 3, avoid={tuple(r) for r in s})
    assert not ({tuple(r) for r in h} & {tuple(r) for r in s})


# --- Freivalds probe ---------------------------------------------------------

def test_freivalds_exact_product_is_tiny():
    A, B = synth.gemm_operands(60, 70, 80, seed=1)
    C = oracle.gemm(A, B).astype(np.float32)
    x = synth.rademacher(70, 2)
    assert oracle.freivalds(A, B, C, x) < 1e-6


def test_freivalds_bruteforce_tiny():
    A, B = synth.gemm_operands(3, 4, 5, seed=3)
    C0 = synth.normal_matrix(3, 4, 4)
    Cout = synth.normal_matrix(3, 4, 5)
    x = synth.rademacher(4, 6)
    Ad, Bd, C0d, Cd = (m.astype(np.float64) for m in (A, B, C0, Cout))
    z = [0.75 * sum(Ad[i, k] * sum(Bd[k, j] * x[j] for j in range(4)) for k in range(5))
         - 0.25 * sum(C0d[i, j] * x[j] for j in range(4)) for i in range(3)]
    w = [sum(Cd[i, j] * x[j] for j in range(4)) for i in range(3)]
    ref = math.sqrt(sum((w[i] - z[i]) ** 2 for i in range(3))) / math.sqrt(sum(v * v for v in z))
    got = oracle.freivalds(A, B, Cout, x, alpha=0.75, beta=-0.25, C0=C0)
    assert math.isclose(got, ref, rel_tol=1e-12)


def test_freivalds_estimates_relative_frobenius():
    """E||E x||^2 = ||E||_F^2: averaged over probes the estimate matches the true error."""
    A, B = synth.gemm_operands(128, 96, 64, seed=7)
    R = oracle.gemm(A, B)
    E = 1e-3 * synth.normal_matrix(128, 96, 8).astype(np.float64) * np.abs(R)
    C = (R + E).astype(np.float32)
    true = oracle.relfro(C, R)
    ests = [oracle.freivalds(A, B, C, synth.rademacher(96, s)) ** 2 for s in range(40)]
    assert abs(math.sqrt(np.mean(ests)) / true - 1.0) < 0.15
