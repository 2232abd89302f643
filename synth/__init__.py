"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This module only draws numbers: matrices, shapes, request streams, probe vectors
and initial network weights.  It holds none of the arithmetic of the GEMM
component or of its selector, so that the CPU oracle and the HIP library can
both consume it without sharing any computation.

All generators are numpy ``Generator(PCG64(seed))``; the same seed always yields
the same bits on every machine.
"""
from __future__ import annotations

import math

import numpy as np

# Tolerance classes a caller can attach to a request (relative Frobenius error).
TOL_CLASSES = (1e-5, 1e-3, 1e-2)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_matrix(rows: int, cols: int, seed: int, lo: float = -1.0, hi: float = 1.0,
                   gen: np.random.Generator | None = None) -> np.ndarray:
    """rows x cols float32, i.i.d. uniform[lo, hi), row-major."""
    g = gen if gen is not None else rng(seed)
    return g.uniform(lo, hi, size=(rows, cols)).astype(np.float32)


def normal_matrix(rows: int, cols: int, seed: int, gen: np.random.Generator | None = None) -> np.ndarray:
    """rows x cols float32, i.i.d. normal(0, 1), row-major."""
    g = gen if gen is not None else rng(seed)
    return g.standard_normal(size=(rows, cols), dtype=np.float32)


def int_matrix(rows: int, cols: int, seed: int, lo: int = -4, hi: int = 4) -> np.ndarray:
    """rows x cols float32 holding small integers drawn uniformly from [lo, hi]."""
    return rng(seed).integers(lo, hi + 1, size=(rows, cols)).astype(np.float32)


def ill_conditioned_matrix(rows: int, cols: int, seed: int, umax: int = 20) -> np.ndarray:
    """normal(0,1) * 2**u with u an integer drawn per entry, uniform in [-umax, umax]."""
    g = rng(seed)
    x = g.standard_normal(size=(rows, cols), dtype=np.float32)
    u = g.integers(-umax, umax + 1, size=(rows, cols))
    return np.ldexp(x, u).astype(np.float32)


def tile_scaled_matrix(rows: int, cols: int, seed: int, tile: int = 128) -> np.ndarray:
    """normal(0,1) entries with tile (i, j) of `tile` x `tile` entries scaled by
    2^((3 i + 5 j) mod 23 - 11), so neighbouring tiles (and blocks inside them) have different
    magnitudes and therefore different scale exponents."""
    X = normal_matrix(rows, cols, seed).astype(np.float64)
    i = (np.arange(rows) // tile)[:, None]
    j = (np.arange(cols) // tile)[None, :]
    return (X * np.exp2((3 * i + 5 * j) % 23 - 11)).astype(np.float32)


def gemm_operands(M: int, N: int, K: int, seed: int, dist: str = "normal"):
    """A (M x K) then B (K x N) from one stream, as float32 row-major arrays."""
    g = rng(seed)
    if dist == "normal":
        A = g.standard_normal(size=(M, K), dtype=np.float32)
        B = g.standard_normal(size=(K, N), dtype=np.float32)
    elif dist == "uniform":
        A = g.uniform(-1.0, 1.0, size=(M, K)).astype(np.float32)
        B = g.uniform(-1.0, 1.0, size=(K, N)).astype(np.float32)
    else:
        raise ValueError(dist)
    return A, B


def square_sweep_sizes() -> list[int]:
    """Square sizes of the exhaustive sweep: powers of two from 128 to 8192."""
    return [1 << p for p in range(7, 14)]


def square_sweep_seed(n: int) -> int:
    return 1000 + int(round(math.log2(n)))


def log_uniform_shapes(n: int, lo: int, hi: int, seed: int, avoid: set | None = None) -> np.ndarray:
    """n distinct (M, N, K) triples, each dimension round(2**U(log2 lo, log2 hi)) clamped to [lo, hi].

    Triples already in ``avoid`` (or drawn earlier in this call) are redrawn.
    """
    g = rng(seed)
    seen = set(avoid) if avoid else set()
    out = []
    a, b = math.log2(lo), math.log2(hi)
    while len(out) < n:
        t = tuple(int(min(hi, max(lo, round(2.0 ** g.uniform(a, b))))) for _ in range(3))
        if t in seen:
            continue
        seen.add(t)
        out.append(t)
    return np.asarray(out, dtype=np.int64)


def tol_classes(n: int, seed: int) -> np.ndarray:
    """n tolerance classes drawn uniformly from TOL_CLASSES."""
    idx = rng(seed).integers(0, len(TOL_CLASSES), size=n)
    return np.asarray(TOL_CLASSES, dtype=np.float64)[idx]


def zipf_ranks(n: int, s: float, nranks: int, seed: int) -> np.ndarray:
    """n ranks in 1..nranks with P(r) proportional to r**-s (finite Zipf)."""
    w = np.arange(1, nranks + 1, dtype=np.float64) ** (-s)
    w /= w.sum()
    return rng(seed).choice(np.arange(1, nranks + 1), size=n, p=w)


def rademacher(n: int, seed: int) -> np.ndarray:
    """n entries of +1.0 / -1.0 (float64), equiprobable."""
    return np.where(rng(seed).integers(0, 2, size=n) == 0, -1.0, 1.0)


def sample_entries(M: int, N: int, count: int, seed: int) -> np.ndarray:
    """count (i, j) index pairs (int64, shape count x 2) drawn uniformly with replacement."""
    g = rng(seed)
    i = g.integers(0, M, size=count)
    j = g.integers(0, N, size=count)
    return np.stack([i, j], axis=1).astype(np.int64)


# ---------------------------------------------------------------------------
# Selector network: 4 inputs -> 64 -> 64 -> 4 outputs.
MLP_SIZES = (4, 64, 64, 4)


def mlp_param_count(sizes=MLP_SIZES) -> int:
    return sum(sizes[i] * sizes[i + 1] + sizes[i + 1] for i in range(len(sizes) - 1))


def mlp_init(seed: int, sizes=MLP_SIZES) -> np.ndarray:
    """Initial parameters, float32, packed layer by layer as [W (out x in, row-major), b (out)].

    Weights are Kaiming-uniform for ReLU fan-in, U(-sqrt(6/fan_in), +sqrt(6/fan_in));
    biases are U(-1/sqrt(fan_in), +1/sqrt(fan_in)).
    """
    g = rng(seed)
    parts = []
    for i in range(len(sizes) - 1):
        fi, fo = sizes[i], sizes[i + 1]
        wb = math.sqrt(6.0 / fi)
        bb = 1.0 / math.sqrt(fi)
        parts.append(g.uniform(-wb, wb, size=fo * fi))
        parts.append(g.uniform(-bb, bb, size=fo))
    return np.concatenate(parts).astype(np.float32)
