"""Pins of the oracle's MX FP6 (E2M3) encoding and its block-scaled two-level quantisation.

Independent references: torch's float8_e4m3fn (its grid coincides with E2M3's on [1, 7.5],
three fraction bits in the same binades, and E2M3's subnormals are the E4M3 values below 1
that are multiples of 1/8), numpy's half-to-even rounding on the uniform subnormal grid, and
a vectorised nearest-grid-point quantiser written here from the format's value set."""
import numpy as np
import pytest
import torch

import oracle
import synth

E4M3_POS = np.array(sorted(float(v) for v in torch.arange(0, 0x7F, dtype=torch.uint8)
                           .view(torch.float8_e4m3fn).to(torch.float32)))


def test_e2m3_value_set_from_e4m3():
    pos = oracle.e2m3_to_float(np.arange(32, dtype=np.uint8)).astype(np.float64)
    expect = E4M3_POS[(E4M3_POS <= 7.5) & (np.floor(E4M3_POS * 8) == E4M3_POS * 8)]
    assert np.array_equal(np.sort(pos), expect)
    assert np.all(np.diff(pos) > 0)                     # codes 0..31 increase with value
    neg = oracle.e2m3_to_float(np.arange(32, 64, dtype=np.uint8)).astype(np.float64)
    assert np.array_equal(neg[1:], -pos[1:]) and neg[0] == 0.0
    assert pos[-1] == 7.5 and pos[8] == 1.0 and pos[1] == 0.125


def _e2m3_value(x):
    return oracle.e2m3_to_float(oracle.e2m3_rne(x)).astype(np.float64)


def test_e2m3_encode_matches_e4m3_on_normal_range():
    g = synth.rng(11)
    grid = E4M3_POS[(E4M3_POS >= 1.0) & (E4M3_POS <= 7.5)]
    mids = (grid[1:] + grid[:-1]) / 2
    x = np.concatenate([g.uniform(1.0, 7.5, 50_000), mids, grid]).astype(np.float32)
    x = np.concatenate([x, -x])
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(_e2m3_value(x), ref)


def test_e2m3_encode_subnormal_range_half_to_even():
    g = synth.rng(12)
    x = np.concatenate([g.uniform(0.0, 1.0, 50_000), (np.arange(16) + 0.5) / 16]).astype(np.float32)
    ref = np.round(x.astype(np.float64) * 8.0) / 8.0     # numpy rounds halves to even
    assert np.array_equal(_e2m3_value(x), ref)
    assert np.array_equal(_e2m3_value(-x), -ref)


def test_e2m3_saturates_and_non_finite():
    x = np.array([7.5, 7.6, 7.75, 8.0, 1e30, -7.75, -1e30], np.float32)
    assert np.array_equal(_e2m3_value(x), [7.5, 7.5, 7.5, 7.5, 7.5, -7.5, -7.5])
    assert np.array_equal(oracle.e2m3_rne(np.array([np.nan, np.inf, -np.inf], np.float32)), [0, 0, 0])


@pytest.mark.parametrize("amax,e", [(7.5, 0), (7.5 * 2 ** 5, -5), (7.5 * 2 ** -7, 7), (1.0, 2),
                                    (4.0, 0), (3.75, 1), (3.7500002, 0), (0.0, 0), (2.0 ** -140, 127)])
def test_mx6_scale_exp_values(amax, e):
    assert oracle.mx6_scale_exp(amax) == e


def test_mx6_scale_exp_defining_inequality():
    g = synth.rng(13)
    for a in np.exp(g.uniform(-80, 80, 2000)).astype(np.float32):
        e = oracle.mx6_scale_exp(float(a))
        assert np.ldexp(float(a), e) <= 7.5 < np.ldexp(float(a), e + 1)


def _nearest_on_grid(v):
    """Round |v| to the E2M3 magnitude grid by search: nearest point, ties to the even code."""
    grid = np.concatenate([np.arange(8) / 8.0, E4M3_POS[(E4M3_POS >= 1.0) & (E4M3_POS <= 7.5)]])
    a = np.minimum(np.abs(v), 7.5)
    hi = np.clip(np.searchsorted(grid, a), 1, len(grid) - 1)
    lo = hi - 1
    dlo, dhi = a - grid[lo], grid[hi] - a
    pick = np.where((dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0)), hi, lo)
    return np.sign(v) * grid[pick]


def _quant_mx6_reference(X):
    """Two-level MX E2M3 quantisation written with numpy from the format's value set."""
    X = X.astype(np.float64)
    r, c = X.shape
    nb = (c + 31) // 32
    pad = np.zeros((r, nb * 32))
    pad[:, :c] = X

    def level(V):
        blocks = V.reshape(r, nb, 32)
        amax = np.abs(blocks).max(-1, keepdims=True)
        e = np.zeros_like(amax)
        nz = amax > 0
        e[nz] = np.floor(np.log2(7.5 / amax[nz]))
        # floor(log2(.)) in binary64 can be off by one near powers of two: fix by the inequality
        e = np.where(np.ldexp(amax, e.astype(int)) > 7.5, e - 1, e)
        e = np.where(np.ldexp(amax, e.astype(int) + 1) <= 7.5, e + 1, e)
        vals = _nearest_on_grid(np.ldexp(blocks, e.astype(int)))
        return np.ldexp(vals, -e.astype(int)).reshape(r, nb * 32), (127 - e[..., 0]).astype(np.uint8)

    v1, s1 = level(pad)
    res = (pad - v1).astype(np.float32).astype(np.float64)
    v2, s2 = level(res)
    return v1[:, :c], s1, v2[:, :c], s2


@pytest.mark.parametrize("rows,cols,dist", [(40, 96, "normal"), (33, 70, "normal"), (16, 64, "ill")])
def test_quant_mx6_matches_numpy_reference(rows, cols, dist):
    X = synth.normal_matrix(rows, cols, rows * cols)
    if dist == "ill":
        X = (X * np.ldexp(1.0, synth.rng(5).integers(-20, 21, X.shape))).astype(np.float32)
    o = oracle.quant_mx6(X)
    v1, s1, v2, s2 = _quant_mx6_reference(X)
    assert np.array_equal(o["qscale"], s1) and np.array_equal(o["rscale"], s2)
    assert np.array_equal(oracle.dequant_mx6(o["q"], o["qscale"]), v1)
    assert np.array_equal(oracle.dequant_mx6(o["rq"], o["rscale"]), v2)


def test_quant_mx6_integers_exact_and_empty_residual():
    X = synth.int_matrix(20, 100, 3)
    o = oracle.quant_mx6(X)
    assert np.array_equal(oracle.dequant_mx6(o["q"], o["qscale"]), X.astype(np.float64))
    assert not np.any(o["rq"] & 31)


def test_quant_mx6_error_bounds_and_levels():
    X = synth.normal_matrix(64, 256, 21)
    o = oracle.quant_mx6(X)
    v1 = oracle.dequant_mx6(o["q"], o["qscale"])
    v2 = oracle.dequant_mx6(o["rq"], o["rscale"])
    x = X.astype(np.float64)
    # one level: half a grid step of the scaled value; the step is 1/8 below 2, else 2^(floor(log2)-3)
    e = 127 - np.repeat(o["qscale"].astype(np.int64), 32, axis=1)
    xs = np.abs(np.ldexp(x, e))
    half = np.where(xs < 2, 1 / 16, np.ldexp(1.0, np.floor(np.log2(np.maximum(xs, 2))).astype(int) - 4))
    assert np.all(np.abs(x - v1) <= np.ldexp(half, -e))
    # the residual level reduces the error of every block
    blk = lambda a: np.abs(a).reshape(64, 8, 32).max(-1)
    assert np.all(blk(x - v1 - v2) <= blk(x - v1) / 4)
    # GEMM error levels of the three-product form (hi.hi + lo.hi + hi.lo), normal operands
    A, B = synth.gemm_operands(128, 128, 512, seed=22)
    qa, qb = oracle.quant_mx6(A), oracle.quant_mx6(np.ascontiguousarray(B.T))
    a1, a2 = oracle.dequant_mx6(qa["q"], qa["qscale"]), oracle.dequant_mx6(qa["rq"], qa["rscale"])
    b1, b2 = oracle.dequant_mx6(qb["q"], qb["qscale"]).T, oracle.dequant_mx6(qb["rq"], qb["rscale"]).T
    ref = A.astype(np.float64) @ B.astype(np.float64)
    rel = lambda C: np.linalg.norm(C - ref) / np.linalg.norm(ref)
    assert 2e-2 < rel(a1 @ b1) < 8e-2                    # one level: ~4e-2
    assert 8e-4 < rel(a1 @ b1 + a2 @ b1 + a1 @ b2) < 2.5e-3  # three products: ~1.4e-3


def test_quant_mx6_non_finite_block_and_ragged_tail():
    X = synth.normal_matrix(3, 70, 23)
    X[1, 40] = np.nan
    X[2, 5] = np.inf
    o = oracle.quant_mx6(X)
    assert o["qscale"].shape == (3, 3)
    assert o["qscale"][1, 1] == 0xFF and o["rscale"][1, 1] == 0xFF
    assert o["qscale"][2, 0] == 0xFF
    assert not np.any(o["q"][1, 32:64]) and not np.any(o["q"][2, :32])
    d = oracle.dequant_mx6(o["q"], o["qscale"])
    assert np.all(np.isnan(d[1, 32:64])) and np.all(np.isfinite(d[1, :32])) and np.all(np.isfinite(d[1, 64:]))
    # the 6-element tail block takes its own scale
    assert o["qscale"][0, 2] == 127 - oracle.mx6_scale_exp(float(np.abs(X[0, 64:]).max()))
