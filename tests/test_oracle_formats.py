"""Pins of the oracle's operand encodings (bfloat16, OCP E4M3, tile scales, residual split)
against torch's CPU conversions (a library special case) and against exact definitions."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth


def _edge_floats():
    vals = [0.0, -0.0, 1.0, -1.0, 1.5, 3.0e38, -3.0e38, 3.4028235e38, 1e-45, -1e-45, 1.1754944e-38,
            65504.0, 448.0, 464.0, 480.0, 1e-30, 2.0 ** -9, 2.0 ** -10, 1.5 * 2.0 ** -10, 2.0 ** -6,
            math.inf, -math.inf]
    # exact bfloat16 ties: x = bf16 value + half ulp, with even and odd last bits
    for base in (1.0, 1.0078125, 2.0, 3.0e-5, 1.0e20):
        b = np.float32(base).view(np.uint32) & np.uint32(0xFFFF0000)
        for lsb in (0, 1):
            bb = np.uint32(b | (lsb << 16))
            vals.append(float(np.uint32(bb | 0x8000).view(np.float32)))
    return np.array(vals, np.float32)


def test_bf16_matches_torch():
    g = synth.rng(123)
    bits = g.integers(0, 2 ** 32, size=200_000, dtype=np.uint64).astype(np.uint32)
    x = np.concatenate([bits.view(np.float32), _edge_floats()])
    x = x[~np.isnan(x)]
    ours = oracle.bf16_rne(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_bf16_nan_stays_nan():
    x = np.array([np.nan, -np.nan], np.float32)
    assert np.all(np.isnan(oracle.bf16_to_float(oracle.bf16_rne(x))))


def test_split_bf16_reconstructs():
    X = synth.normal_matrix(50, 70, 4)
    hi, lo = oracle.split_bf16(X)
    h = oracle.bf16_to_float(hi).astype(np.float64)
    l = oracle.bf16_to_float(lo).astype(np.float64)
    # hi is RNE of x, and x - hi is exactly representable: |x - hi - lo| <= 2^-9 |x - hi|
    r = X.astype(np.float64) - h
    assert np.all(np.abs(r) <= np.abs(X) * 2.0 ** -8)
    assert np.all(np.abs(r - l) <= np.abs(r) * 2.0 ** -8)
    assert np.array_equal(hi, oracle.bf16_rne(X))


def test_e4m3_decode_all_codes_match_torch():
    codes = np.arange(256, dtype=np.uint8)
    ours = oracle.e4m3_to_float(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float32).numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], ref[~nan])
    assert ours[0x7e] == 448.0 and ours[0x01] == 2.0 ** -9


def test_e4m3_encode_matches_torch_in_range():
    g = synth.rng(7)
    x = np.concatenate([
        g.uniform(-448, 448, 100_000).astype(np.float32),
        (g.standard_normal(100_000) * np.exp2(g.integers(-14, 9, 100_000))).astype(np.float32),
        oracle.e4m3_to_float(np.arange(256, dtype=np.uint8)),
    ])
    # all midpoints between neighbouring codes (exact ties)
    pos = np.sort(oracle.e4m3_to_float(np.arange(0, 0x7f, dtype=np.uint8)).astype(np.float64))
    mids = ((pos[1:] + pos[:-1]) / 2).astype(np.float32)
    x = np.concatenate([x, mids, -mids])
    x = x[np.isfinite(x) & (np.abs(x) <= 448)]
    ours = oracle.e4m3_rne(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)


def test_e4m3_saturates_and_nan():
    x = np.array([449.0, 464.0, 1e6, -1e30, np.inf, -np.inf, np.nan], np.float32)
    q = oracle.e4m3_rne(x)
    assert list(q[:4]) == [0x7e, 0x7e, 0x7e, 0xfe]
    assert np.all(np.isnan(oracle.e4m3_to_float(q[4:])))


@pytest.mark.parametrize("amax,e", [(448.0, 0), (1.0, 8), (1.75, 8), (1.7500001, 7), (449.0, -1),
                                    (0.0, 0), (2.0 ** -100, 108), (1e-40, 127), (3.0e38, -120)])
def test_scale_exp_values(amax, e):
    assert oracle.scale_exp(amax) == e


def test_scale_exp_defining_inequality():
    g = synth.rng(5)
    for a in (g.standard_normal(2000) * np.exp2(g.integers(-60, 60, 2000))).astype(np.float32):
        a = abs(float(a))
        if a == 0:
            continue
        e = oracle.scale_exp(a)
        assert math.ldexp(a, e) <= 448.0 < math.ldexp(a, e + 1)


def test_quant_fp8_integers_exact():
    """Entries in {-4..4}: tile amax 4 -> scale 2^6, codes exact, residual exactly zero."""
    X = synth.int_matrix(200, 300, 3)
    r = oracle.quant_fp8(X)
    assert np.all(r["resid"] == 0.0)
    assert np.array_equal(oracle.dequant_fp8(r["q"], r["qscale"], 200, 300), X.astype(np.float64))
    assert np.all(oracle.dequant_fp8(r["rq"], r["rscale"], 200, 300) == 0.0)


def test_quant_fp8_error_levels():
    X = synth.normal_matrix(256, 384, 9)
    r = oracle.quant_fp8(X)
    d1 = oracle.dequant_fp8(r["q"], r["qscale"], 256, 384)
    d2 = oracle.dequant_fp8(r["rq"], r["rscale"], 256, 384)
    x = X.astype(np.float64)
    e1 = np.linalg.norm(x - d1) / np.linalg.norm(x)
    e2 = np.linalg.norm(x - d1 - d2) / np.linalg.norm(x)
    assert np.array_equal((x - d1).astype(np.float32), r["resid"])   # residual is exact in binary32
    assert 5e-3 < e1 < 5e-2            # 3 fraction bits: ~2^-5 relative
    assert e2 < 2.0 ** -8              # one residual pass
    assert e2 < e1 / 8


def test_quant_fp8_ragged_tiles_and_scale_bytes():
    X = synth.normal_matrix(130, 257, 10)
    X[129, 256] = 1000.0               # last (partial) tile gets its own scale
    r = oracle.quant_fp8(X)
    assert r["qscale"].shape == (2, 3)
    assert r["qscale"][1, 2] == 127 - oracle.scale_exp(1000.0)
    assert r["q"][129, 256] == oracle.e4m3_rne(np.float32(1000.0 * 2.0 ** oracle.scale_exp(1000.0)))
