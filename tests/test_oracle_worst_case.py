"""The stated bounds of the variants (f32_simt and bf16x3 1e-5, fp8r 1e-3, bf16 and fp6x3
1e-2) are the relative Frobenius errors they meet on the input distributions of the
workloads (i.i.d. normal or uniform entries, the per-entry 2^u ill-conditioned recipe), not
worst-case bounds.  Perfectly correlated operands defeat the averaging of rounding errors:
these tests pin, with the oracle's own encodings (which the pre-pass kernels match bit for
bit) and with hand-derived closed forms, constant operands whose products exceed the
stated bounds of fp8r, bf16x3 and FP32 accumulation.  Verify mode (the FP64 probe) is what
guarantees a requested tolerance."""
from fractions import Fraction

import numpy as np

import oracle


def test_fp8r_constant_operand_exceeds_its_bound():
    """A = B = c = 1.033203125 (every tile constant): c 2^8 = 264.5 lies in E4M3's binade
    [256, 512) of spacing 32 and rounds to 256, so q = 1; the residual 17/512 takes e = 13,
    17/512 * 2^13 = 272 is the midpoint of 256 and 288 and rounds to even, 256, so the
    residual code is 2^-5.  Every product then uses (1 + 2^-5)^2 for c^2."""
    c = np.float32(1.033203125)
    X = np.full((128, 128), c, np.float32)
    r = oracle.quant_fp8(X)
    assert r["qscale"][0, 0] == 127 - 8 and r["rscale"][0, 0] == 127 - 13
    a_hat = oracle.dequant_fp8(r["q"], r["qscale"], 128, 128) + oracle.dequant_fp8(r["rq"], r["rscale"], 128, 128)
    assert np.all(a_hat == 1.0 + 2.0 ** -5)
    exact = Fraction(float(c)) ** 2
    err = abs(exact - Fraction(33, 32) ** 2) / exact      # relative error of every entry of C
    assert abs(float(err) - 3.777144878698957e-3) < 1e-15
    assert float(err) > 3.7 * 1e-3                         # 3.8 x the stated 1e-3


def test_bf16x3_constant_operand_exceeds_its_bound():
    """A = B = c = 1.0039134: hi rounds up to 1 + 2^-7, lo = RNE_bf16(c - hi) keeps 8 more
    bits, and the dropped lo.lo term plus lo's own rounding leave 2.9e-5 relative."""
    c = np.float32(1.0039134)
    hi, lo = oracle.split_bf16(np.array([[c]], np.float32))
    h = Fraction(float(oracle.bf16_to_float(hi)[0, 0]))
    l = Fraction(float(oracle.bf16_to_float(lo)[0, 0]))
    assert h == 1 + Fraction(1, 128)
    exact = Fraction(float(c)) ** 2
    err = float(abs(exact - (h * h + 2 * h * l)) / exact)
    assert 2.9e-5 < err < 3.0e-5                           # 2.9 x the stated 1e-5


def test_fp32_accumulation_of_equal_terms_exceeds_1e5():
    """Any variant that sums K products in one FP32 accumulator (f32_simt's FMA chain; the
    MFMA variants' accumulators): K = 8192 equal products c^2 summed in order, each step
    rounded to binary32, drift by 9.2e-5 relative for c = 1.3333334."""
    c = float(np.float32(1.3333334))
    p = c * c                                              # exact in binary64
    acc = np.float32(0.0)
    for _ in range(8192):
        acc = np.float32(float(acc) + p)                   # one rounding per step, as an FMA chain
    err = abs(Fraction(float(acc)) - 8192 * Fraction(p)) / (8192 * Fraction(p))
    assert float(err) > 5e-5


def test_iid_operands_stay_inside_the_bounds():
    """The same representation errors on i.i.d. normal operands average out: the 4-term FP8
    product and the 3-term bf16 product of 256 x 256 x 256 normal operands, in binary64 from
    the oracle's encodings, stay inside 1e-3 and 1e-5."""
    g = np.random.default_rng(11)
    A = g.standard_normal((256, 256)).astype(np.float32)
    B = g.standard_normal((256, 256)).astype(np.float32)
    ref = A.astype(np.float64) @ B.astype(np.float64)

    def deq8(X):
        r = oracle.quant_fp8(X)
        n, m = X.shape
        return oracle.dequant_fp8(r["q"], r["qscale"], n, m) + oracle.dequant_fp8(r["rq"], r["rscale"], n, m)

    e8 = np.linalg.norm(deq8(A) @ deq8(B) - ref) / np.linalg.norm(ref)
    ah, al = (oracle.bf16_to_float(x).astype(np.float64) for x in oracle.split_bf16(A))
    bh, bl = (oracle.bf16_to_float(x).astype(np.float64) for x in oracle.split_bf16(B))
    e3 = np.linalg.norm(ah @ bh + ah @ bl + al @ bh - ref) / np.linalg.norm(ref)
    assert e8 < 1e-3 and e3 < 1e-5
