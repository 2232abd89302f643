"""Bit-exact parity of the pre-pass each MFMA variant runs on its hot path (cmp_prepass_images:
the variant's own kernels and launch configuration, writing the panel images the GEMM kernel
streams) against the oracle's encodings of A and of B transposed: bf16 hi/lo splits, E4M3 tile
quantisation with one residual pass, MX E2M3 block quantisation with one residual level
(every variant computes the same function from these encodings, Sec. 2.2.2).  The images are
mapped back to row-major arrays by index arithmetic only (tests/image_layout.py); padding must
hold the encoding of zero."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, say
from image_layout import (unpack_mx6_codes, unpack_mx6_scales, unpack_panel_bf16,
                          unpack_panel_bytes)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cx():
    import paper_2311_03543_amd as pa
    c = pa.Compar(0)
    c.register_builtin("fp6x3")
    yield c
    c.close()


def operands(M, N, K, dist, seed):
    if dist == "normal":
        return synth.gemm_operands(M, N, K, seed=seed)
    if dist == "ill":
        return synth.ill_conditioned_matrix(M, K, seed), synth.ill_conditioned_matrix(K, N, seed + 1)
    if dist == "tiles":
        return (synth.tile_scaled_matrix(M, K, seed),
                np.ascontiguousarray(synth.tile_scaled_matrix(N, K, seed + 1).T))
    if dist == "special":
        g = synth.rng(seed)
        edge = np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.4e38, 1e-40, -1e-45, 2.0 ** -126, 65504.0,
                         1.0039062, 1.0078125, 448.0, 449.0, 1e-8, 7.5, 7.75, 0.0625], np.float32)
        def mat(r, c):
            x = (g.standard_normal(r * c) * np.exp2(g.integers(-30, 30, r * c))).astype(np.float32)
            x[:edge.size] = edge[:min(edge.size, x.size)]
            return x.reshape(r, c)
        return mat(M, K), mat(K, N)
    raise ValueError(dist)


def padded(X, rows, cols):
    P = np.zeros((rows, cols), np.float32)
    P[:X.shape[0], :X.shape[1]] = X
    return P


def run_images(cx, name, A, B):
    import torch
    vid = cx.variant_find(name)
    M, K = A.shape
    N = B.shape[1]
    lay = cx.prepass_layout(vid, M, N, K)
    out = torch.full((lay["total"],), 0xA5, dtype=torch.uint8, device="cuda")   # poison
    say(f"  prepass_images {name} M={M} N={N} K={K}")
    cx.prepass_images(vid, dev(A), dev(B), out)
    img = host(out)
    return lay, [img[o:o + n] for o, n in zip(lay["offset"], lay["bytes"])]


SHAPES = [(1, 1, 1, "normal"), (300, 257, 129, "normal"), (513, 130, 700, "ill"),
          (640, 768, 1024, "tiles"), (385, 300, 260, "tiles"), (256, 384, 200, "special"),
          (2304, 2560, 384, "tiles")]


@pytest.mark.parametrize("name", ["bf16", "bf16x3"])
@pytest.mark.parametrize("M,N,K,dist", SHAPES)
def test_bf16_images_bit_exact(cx, name, M, N, K, dist):
    A, B = operands(M, N, K, dist, M + N + K)
    lay, imgs = run_images(cx, name, A, B)
    Mp, Np, Kp = lay["Mp"], lay["Np"], lay["Kp"]
    ah, al = oracle.split_bf16(padded(A, Mp, Kp))
    bh, bl = oracle.split_bf16(padded(np.ascontiguousarray(B.T), Np, Kp))
    assert np.array_equal(unpack_panel_bf16(imgs[0], Mp, Kp), ah)
    assert np.array_equal(unpack_panel_bf16(imgs[1], Np, Kp), bh)
    if name == "bf16x3":
        assert np.array_equal(unpack_panel_bf16(imgs[2], Mp, Kp), al)
        assert np.array_equal(unpack_panel_bf16(imgs[3], Np, Kp), bl)
    else:
        assert len(imgs) == 2


def _fp8_check(img_codes, img_scales, X, rows, kp):
    ref = oracle.quant_fp8(padded(X, rows, kp))
    nt = (rows // 128) * (kp // 128)
    got_q = unpack_panel_bytes(img_codes[0], rows, kp)
    got_r = unpack_panel_bytes(img_codes[1], rows, kp)
    gs_q = img_scales[0][:nt].reshape(rows // 128, kp // 128)
    gs_r = img_scales[1][:nt].reshape(rows // 128, kp // 128)
    assert np.array_equal(gs_q, ref["qscale"])
    assert np.array_equal(gs_r, ref["rscale"])
    assert np.array_equal(got_q, ref["q"])
    assert np.array_equal(got_r, ref["rq"])
    return ref


@pytest.mark.parametrize("M,N,K,dist", SHAPES)
def test_fp8r_images_bit_exact(cx, M, N, K, dist):
    A, B = operands(M, N, K, dist, M + 2 * N + K)
    lay, imgs = run_images(cx, "fp8r", A, B)
    Mp, Np, Kp = lay["Mp"], lay["Np"], lay["Kp"]
    assert Kp % 128 == 0
    ra = _fp8_check(imgs[0:2], imgs[4:6], A, Mp, Kp)
    rb = _fp8_check(imgs[2:4], imgs[6:8], np.ascontiguousarray(B.T), Np, Kp)
    if dist == "tiles":
        # the tile exponents really differ across tiles (the indexing is exercised)
        assert len(np.unique(ra["qscale"][: (M + 127) // 128, : (K + 127) // 128])) > 3
        assert len(np.unique(rb["qscale"][: (N + 127) // 128, : (K + 127) // 128])) > 3


def _mx6_check(codes_hi, codes_lo, scales, X, rows, kp):
    ref = oracle.quant_mx6(padded(X, rows, kp))
    sh, sl = unpack_mx6_scales(scales, rows, kp)
    assert np.array_equal(sh, ref["qscale"])
    assert np.array_equal(sl, ref["rscale"])
    assert np.array_equal(unpack_mx6_codes(codes_hi, rows, kp), ref["q"])
    assert np.array_equal(unpack_mx6_codes(codes_lo, rows, kp), ref["rq"])


@pytest.mark.parametrize("M,N,K,dist", SHAPES)
def test_fp6x3_images_bit_exact(cx, M, N, K, dist):
    A, B = operands(M, N, K, dist, M + 3 * N + K)
    lay, imgs = run_images(cx, "fp6x3", A, B)
    Mp, Np, Kp = lay["Mp"], lay["Np"], lay["Kp"]
    _mx6_check(imgs[0], imgs[1], imgs[4], A, Mp, Kp)
    _mx6_check(imgs[2], imgs[3], imgs[5], np.ascontiguousarray(B.T), Np, Kp)


def test_fp8r_and_fp6x3_images_non_finite(cx):
    """NaN and infinities: E4M3 encodes them as its NaN code (either sign) with a zero residual;
    an MX block holding one gets the E8M0 NaN byte at both levels and zero codes."""
    M, N, K = 200, 150, 300
    A, B = synth.gemm_operands(M, N, K, seed=41)
    A[5, 7], A[130, 290], B[17, 3], B[250, 149] = np.nan, np.inf, -np.inf, np.nan
    lay, imgs = run_images(cx, "fp8r", A, B)
    Mp, Np, Kp = lay["Mp"], lay["Np"], lay["Kp"]
    nan8 = lambda q: np.where((q & 0x7F) == 0x7F, 0x7F, q)
    for codes, scales, X, rows in ((imgs[0:2], imgs[4:6], A, Mp),
                                   (imgs[2:4], imgs[6:8], np.ascontiguousarray(B.T), Np)):
        ref = oracle.quant_fp8(padded(X, rows, Kp))
        nt = (rows // 128) * (Kp // 128)
        assert np.array_equal(scales[0][:nt].reshape(rows // 128, -1), ref["qscale"])
        assert np.array_equal(scales[1][:nt].reshape(rows // 128, -1), ref["rscale"])
        assert np.array_equal(nan8(unpack_panel_bytes(codes[0], rows, Kp)), nan8(ref["q"]))
        assert np.array_equal(nan8(unpack_panel_bytes(codes[1], rows, Kp)), nan8(ref["rq"]))
    lay, imgs = run_images(cx, "fp6x3", A, B)
    Mp, Np, Kp = lay["Mp"], lay["Np"], lay["Kp"]
    _mx6_check(imgs[0], imgs[1], imgs[4], A, Mp, Kp)
    _mx6_check(imgs[2], imgs[3], imgs[5], np.ascontiguousarray(B.T), Np, Kp)


def test_prepass_images_argument_checks(cx):
    import torch
    import paper_2311_03543_amd as pa
    A, B = synth.gemm_operands(64, 64, 64, seed=1)
    with pytest.raises(pa.ComparError) as e:
        cx.prepass_layout(cx.variant_find("f32_simt"), 64, 64, 64)
    assert e.value.status == pa.CMP_EUNSUPPORTED
    vid = cx.variant_find("bf16")
    lay = cx.prepass_layout(vid, 64, 64, 64)
    small = torch.zeros(lay["total"] - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(pa.ComparError) as e:
        cx.prepass_images(vid, dev(A), dev(B), small)
    assert e.value.status == pa.CMP_EINVAL
