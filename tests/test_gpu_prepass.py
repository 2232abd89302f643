"""Bit-exact parity of the operand pre-pass kernels (bf16 split, E4M3 tile quantisation with
residual, MX E2M3 block quantisation with residual) against the oracle's encodings, and of the
FP64 Freivalds probe."""
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


def _special_values(n, seed):
    g = synth.rng(seed)
    x = (g.standard_normal(n) * np.exp2(g.integers(-30, 30, n))).astype(np.float32)
    edge = np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.4e38, 1e-40, -1e-45, 2.0 ** -126, 65504.0,
                     1.0039062, 1.0078125, 448.0, 449.0, 1e-8], np.float32)
    m = min(n, edge.size)
    x[:m] = edge[:m]
    return x


@pytest.mark.parametrize("rows,cols", [(1, 1), (37, 53), (256, 512), (129, 1000)])
def test_split_bf16_bit_exact(cx, rows, cols):
    import torch
    X = _special_values(rows * cols, rows + cols).reshape(rows, cols)
    hi = torch.empty((rows, cols), dtype=torch.int16, device="cuda")
    lo = torch.empty((rows, cols), dtype=torch.int16, device="cuda")
    say(f"  split_bf16 {rows}x{cols}")
    cx.split_bf16(dev(X), hi, lo)
    gh = host(hi).view(np.uint16)
    gl = host(lo).view(np.uint16)
    rh, rl = oracle.split_bf16(X)
    assert np.array_equal(gh, rh)
    assert np.array_equal(gl, rl)


def test_split_bf16_nan_and_inf(cx):
    import torch
    X = np.array([[np.nan, np.inf, -np.inf, 1.0]], np.float32)
    hi = torch.empty((1, 4), dtype=torch.int16, device="cuda")
    lo = torch.empty((1, 4), dtype=torch.int16, device="cuda")
    cx.split_bf16(dev(X), hi, lo)
    gh = oracle.bf16_to_float(host(hi).view(np.uint16))
    gl = host(lo).view(np.uint16)
    # NaN encodings are not unique: compare NaN-ness, and the rest exactly
    assert np.isnan(gh[0, 0]) and gh[0, 1] == np.inf and gh[0, 2] == -np.inf and gh[0, 3] == 1.0
    assert list(gl[0]) == [0, 0, 0, 0]


def _quant_gpu(cx, X):
    import torch
    r, c = X.shape
    tr, tc = (r + 127) // 128, (c + 127) // 128
    q = torch.empty((r, c), dtype=torch.uint8, device="cuda")
    rq = torch.empty((r, c), dtype=torch.uint8, device="cuda")
    qs = torch.empty((tr, tc), dtype=torch.uint8, device="cuda")
    rs = torch.empty((tr, tc), dtype=torch.uint8, device="cuda")
    say(f"  quant_fp8 {r}x{c}")
    cx.quant_fp8(dev(X), q, qs, rq, rs)
    return dict(q=host(q), qscale=host(qs), rq=host(rq), rscale=host(rs))


@pytest.mark.parametrize("rows,cols,dist", [(128, 128, "normal"), (256, 384, "normal"), (300, 257, "normal"),
                                            (1, 5, "normal"), (513, 129, "ill"), (256, 256, "special")])
def test_quant_fp8_bit_exact(cx, rows, cols, dist):
    if dist == "normal":
        X = synth.normal_matrix(rows, cols, rows * cols)
    elif dist == "ill":
        X = synth.ill_conditioned_matrix(rows, cols, 3)
    else:
        X = _special_values(rows * cols, 5).reshape(rows, cols)
    got = _quant_gpu(cx, X)
    ref = oracle.quant_fp8(X)
    for k in ("qscale", "rscale", "q", "rq"):
        assert np.array_equal(got[k], ref[k]), k


def test_quant_fp8_integers_have_zero_residual(cx):
    X = synth.int_matrix(256, 256, 4)
    got = _quant_gpu(cx, X)
    assert np.all((got["rq"] & 0x7F) == 0)
    assert np.array_equal(oracle.dequant_fp8(got["q"], got["qscale"], 256, 256), X.astype(np.float64))


# ---- MX FP6 (E2M3) block quantisation -------------------------------------------

def _quant_mx6_gpu(cx, X, transpose):
    import torch
    r, c = X.shape
    orows, K = (c, r) if transpose else (r, c)
    nb = (K + 31) // 32
    q = torch.empty((orows, K), dtype=torch.uint8, device="cuda")
    rq = torch.empty((orows, K), dtype=torch.uint8, device="cuda")
    qs = torch.empty((orows, nb), dtype=torch.uint8, device="cuda")
    rs = torch.empty((orows, nb), dtype=torch.uint8, device="cuda")
    say(f"  quant_mx6 {r}x{c} transpose={transpose}")
    cx.quant_mx6(dev(X), q, qs, rq, rs, transpose=transpose)
    return dict(q=host(q), qscale=host(qs), rq=host(rq), rscale=host(rs))


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("rows,cols,dist", [(1, 1, "normal"), (37, 53, "normal"), (256, 512, "normal"),
                                            (129, 1000, "normal"), (300, 70, "ill"), (64, 96, "special")])
def test_quant_mx6_bit_exact(cx, rows, cols, dist, transpose):
    if dist == "normal":
        X = synth.normal_matrix(rows, cols, rows * cols + 1)
    elif dist == "ill":
        X = synth.ill_conditioned_matrix(rows, cols, 6)
    else:
        X = _special_values(rows * cols, 7).reshape(rows, cols)
    got = _quant_mx6_gpu(cx, X, transpose)
    ref = oracle.quant_mx6(np.ascontiguousarray(X.T) if transpose else X)
    for k in ("qscale", "rscale", "q", "rq"):
        assert np.array_equal(got[k], ref[k]), k


@pytest.mark.parametrize("transpose", [False, True])
def test_quant_mx6_non_finite_blocks(cx, transpose):
    X = synth.normal_matrix(40, 70, 8)
    X[3, 40] = np.nan
    X[35, 2] = np.inf
    X[20, 69] = -np.inf
    got = _quant_mx6_gpu(cx, X, transpose)
    ref = oracle.quant_mx6(np.ascontiguousarray(X.T) if transpose else X)
    for k in ("qscale", "rscale", "q", "rq"):
        assert np.array_equal(got[k], ref[k]), k
    assert np.sum(got["qscale"] == 0xFF) == 3


def test_quant_mx6_integers_have_zero_residual(cx):
    X = synth.int_matrix(64, 256, 9)
    got = _quant_mx6_gpu(cx, X, False)
    assert not np.any(got["rq"] & 31)
    assert np.array_equal(oracle.dequant_mx6(got["q"], got["qscale"]), X.astype(np.float64))


# ---- Freivalds probe -----------------------------------------------------------

def test_freivalds_matches_oracle(cx):
    import torch
    A, B = synth.gemm_operands(300, 200, 250, seed=12)
    C0 = synth.normal_matrix(300, 200, 13)
    Cout = (oracle.gemm(A, B, 1.5, -0.5, C0) + 1e-3 * synth.normal_matrix(300, 200, 14)).astype(np.float32)
    x = synth.rademacher(200, 15)
    say("  freivalds 300x200x250")
    got = cx.freivalds(dev(A), dev(B), dev(Cout), x, alpha=1.5, beta=-0.5, C0=dev(C0))
    ref = oracle.freivalds(A, B, Cout, x, alpha=1.5, beta=-0.5, C0=C0)
    assert abs(got - ref) <= 1e-9 * ref, (got, ref)
