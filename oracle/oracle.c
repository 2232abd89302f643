/*
 * CPU oracle for the GEMM component (test infrastructure only).
 *
 * Only the tests, the smoke check and the bench's CPU-baseline leg may load this
 * library.  It shares no code, header, table or constant with the HIP library:
 * everything here is written from the definitions it cites, in plain C, in
 * IEEE binary64 unless a function states otherwise.
 *
 * What the component computes.  COMPAR (Sec. 2.1, the matrix-multiplication
 * interface of the sort/mmul example) exposes several implementation variants
 * of one interface, and the runtime (Sec. 2.2.2) runs exactly one of them per
 * call: every variant computes the same function, only its speed and rounding
 * differ.  The interface here is the BLAS-style product over float matrices
 *
 *     C[i][j] = alpha * sum_{k=0}^{K-1} A[i][k] * B[k][j]  +  beta * C0[i][j]
 *
 * with row-major operands and leading dimensions.  BLAS conventions: when
 * beta == 0 the old C is never read (a NaN there does not propagate), and when
 * alpha == 0 (or K == 0) A and B are never read.
 *
 * Exactness.  A product of two binary32 numbers is exact in binary64 (24+24
 * significant bits <= 53), so whether the compiler contracts s += a*b into an
 * FMA cannot change a result.  The k-sum runs in increasing k, one rounding per
 * addition; the blocked form below visits every entry's k in the same order and
 * is therefore bit-identical to the plain triple loop.  No -ffast-math.
 *
 * Precision variants.  The functions after the GEMMs define, from the formats'
 * published definitions, the operand encodings the reduced-precision variants
 * use: bfloat16 round-to-nearest-even, the OCP FP8 E4M3 ("e4m3fn") encoding
 * with round-to-nearest-even and saturation to +-448, per-tile power-of-two
 * scales stored as E8M0 exponents, the FP32 residual of a quantisation, and
 * the OCP Microscaling FP6 E2M3 encoding with one E8M0 scale per block of 32
 * consecutive elements.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* Threads                                                                    */

OR_EXPORT int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* GEMM, plain definition: triple loop, k innermost in increasing order.      */

OR_EXPORT void oracle_gemm_f64(int64_t M, int64_t N, int64_t K, float alpha,
                               const float *A, int64_t lda, const float *B, int64_t ldb,
                               float beta, const float *C0, int64_t ldc,
                               double *out, int64_t ldo)
{
    const double a = (double)alpha, b = (double)beta;
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            double s = 0.0;
            if (alpha != 0.0f)
                for (int64_t k = 0; k < K; ++k)
                    s += (double)A[i * lda + k] * (double)B[k * ldb + j];
            double r = (alpha != 0.0f) ? a * s : 0.0;
            if (beta != 0.0f)
                r += b * (double)C0[i * ldc + j];
            out[i * ldo + j] = r;
        }
    }
}

/*
 * GEMM, blocked for speed but bit-identical to oracle_gemm_f64: each output
 * tile keeps one binary64 accumulator per entry and visits k-blocks in
 * increasing order, k increasing inside a block, so every entry sees exactly
 * the same sequence of additions.  Rows of tiles are spread over OpenMP
 * threads; threads never share an accumulator.
 */
#define OB_I 32
#define OB_J 256
#define OB_K 256

static void blocked_core(int64_t M, int64_t N, int64_t K, double alpha, int use_abs,
                         const float *A, int64_t lda, const float *B, int64_t ldb,
                         double beta, const float *C0, int64_t ldc,
                         double *out, int64_t ldo)
{
    const int64_t ti = (M + OB_I - 1) / OB_I, tj = (N + OB_J - 1) / OB_J;
    const int skip_ab = (alpha == 0.0);
    #pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * OB_I * OB_J);
        double *brow = (double *)malloc(sizeof(double) * OB_K * OB_J);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < ti * tj; ++t) {
            const int64_t i0 = (t / tj) * OB_I, j0 = (t % tj) * OB_J;
            const int64_t ni = (M - i0 < OB_I) ? M - i0 : OB_I;
            const int64_t nj = (N - j0 < OB_J) ? N - j0 : OB_J;
            memset(acc, 0, sizeof(double) * OB_I * OB_J);
            for (int64_t k0 = 0; k0 < K && !skip_ab; k0 += OB_K) {
                const int64_t nk = (K - k0 < OB_K) ? K - k0 : OB_K;
                /* widen the B block once (exact), then stream it per row */
                for (int64_t kk = 0; kk < nk; ++kk) {
                    const float *bp = B + (k0 + kk) * ldb + j0;
                    double *dst = brow + kk * OB_J;
                    for (int64_t jj = 0; jj < nj; ++jj)
                        dst[jj] = use_abs ? fabs((double)bp[jj]) : (double)bp[jj];
                }
                for (int64_t ii = 0; ii < ni; ++ii) {
                    const float *ap = A + (i0 + ii) * lda + k0;
                    double *arow = acc + ii * OB_J;
                    for (int64_t kk = 0; kk < nk; ++kk) {
                        const double av = use_abs ? fabs((double)ap[kk]) : (double)ap[kk];
                        const double *bk = brow + kk * OB_J;
                        for (int64_t jj = 0; jj < nj; ++jj)
                            arow[jj] += av * bk[jj];
                    }
                }
            }
            for (int64_t ii = 0; ii < ni; ++ii)
                for (int64_t jj = 0; jj < nj; ++jj) {
                    double r = skip_ab ? 0.0 : alpha * acc[ii * OB_J + jj];
                    if (beta != 0.0)
                        r += beta * (double)C0[(i0 + ii) * ldc + (j0 + jj)];
                    out[(i0 + ii) * ldo + (j0 + jj)] = r;
                }
        }
        free(acc);
        free(brow);
    }
}

OR_EXPORT void oracle_gemm_f64_blocked(int64_t M, int64_t N, int64_t K, float alpha,
                                       const float *A, int64_t lda, const float *B, int64_t ldb,
                                       float beta, const float *C0, int64_t ldc,
                                       double *out, int64_t ldo)
{
    blocked_core(M, N, K, (double)alpha, 0, A, lda, B, ldb, (double)beta, C0, ldc, out, ldo);
}

/* |A| * |B| in binary64 (entrywise absolute values), for a-priori error bounds. */
OR_EXPORT void oracle_absgemm_f64(int64_t M, int64_t N, int64_t K,
                                  const float *A, int64_t lda, const float *B, int64_t ldb,
                                  double *out, int64_t ldo)
{
    blocked_core(M, N, K, 1.0, 1, A, lda, B, ldb, 0.0, NULL, 0, out, ldo);
}

/* The plain definition evaluated at `count` listed entries (i, j) only. */
OR_EXPORT void oracle_gemm_f64_entries(int64_t M, int64_t N, int64_t K, float alpha,
                                       const float *A, int64_t lda, const float *B, int64_t ldb,
                                       float beta, const float *C0, int64_t ldc,
                                       int64_t count, const int64_t *ij, double *out)
{
    (void)M; (void)N;
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = ij[2 * t], j = ij[2 * t + 1];
        double s = 0.0;
        if (alpha != 0.0f)
            for (int64_t k = 0; k < K; ++k)
                s += (double)A[i * lda + k] * (double)B[k * ldb + j];
        double r = (alpha != 0.0f) ? (double)alpha * s : 0.0;
        if (beta != 0.0f)
            r += (double)beta * (double)C0[i * ldc + j];
        out[t] = r;
    }
}

/*
 * Relative Frobenius error ||C - R||_F / ||R||_F in binary64, C float (ld ldc),
 * R double (ld ldr).  A zero reference norm gives the absolute norm ||C - R||_F.
 * Any NaN or infinity in C gives +infinity.
 */
OR_EXPORT double oracle_relfro(int64_t M, int64_t N, const float *C, int64_t ldc,
                               const double *R, int64_t ldr)
{
    double num = 0.0, den = 0.0;
    int bad = 0;
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            const double c = (double)C[i * ldc + j], r = R[i * ldr + j];
            if (!isfinite(c)) bad = 1;
            num += (c - r) * (c - r);
            den += r * r;
        }
    if (bad) return INFINITY;
    return den > 0.0 ? sqrt(num) / sqrt(den) : sqrt(num);
}

/* Same metric over a list of values (sampled entries). */
OR_EXPORT double oracle_relfro_list(int64_t n, const float *c, const double *r)
{
    double num = 0.0, den = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        const double cv = (double)c[t];
        if (!isfinite(cv)) return INFINITY;
        num += (cv - r[t]) * (cv - r[t]);
        den += r[t] * r[t];
    }
    return den > 0.0 ? sqrt(num) / sqrt(den) : sqrt(num);
}

/* ------------------------------------------------------------------------- */
/* bfloat16: 1 sign, 8 exponent, 7 fraction bits = the upper half of a binary32.
 * Round-to-nearest-even from binary32: of the two bfloat16 neighbours of x
 * (x truncated toward zero, and that value one bfloat16 ulp further from zero)
 * take the nearer; on a tie take the one whose last fraction bit is 0.
 * Rounding past the largest finite value gives infinity, as IEEE 754 does.
 * NaN stays NaN (quiet bit set, sign kept).                                   */

static uint32_t f2u(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }
static float u2f(uint32_t u) { float x; memcpy(&x, &u, 4); return x; }

OR_EXPORT uint16_t oracle_bf16_rne(float x)
{
    const uint32_t u = f2u(x);
    if (isnan(x))
        return (uint16_t)((u >> 16) | 0x0040u);
    const uint32_t sign = u & 0x80000000u;
    const uint32_t mag = u & 0x7fffffffu;
    const uint32_t down = mag & 0xffff0000u;          /* toward zero */
    const uint32_t up = down + 0x00010000u;           /* away from zero (may be inf) */
    const double dx = fabs((double)x);
    const double dd = (double)u2f(down);
    /* one ulp past the largest finite bfloat16 is 2^128 */
    const double dup = (up >= 0x7f800000u) ? ldexp(1.0, 128) : (double)u2f(up);
    uint32_t pick;
    if (dx - dd < dup - dx) pick = down;
    else if (dx - dd > dup - dx) pick = up;
    else pick = ((down >> 16) & 1u) ? up : down;
    if (pick >= 0x7f800000u) pick = 0x7f800000u;
    return (uint16_t)((sign | pick) >> 16);
}

OR_EXPORT float oracle_bf16_to_float(uint16_t h) { return u2f((uint32_t)h << 16); }

/* hi = bf16(x), lo = bf16(x - hi); x - hi is exact in binary32 (Sterbenz). */
OR_EXPORT void oracle_split_bf16(int64_t rows, int64_t cols, const float *X, int64_t ldx,
                                 uint16_t *hi, uint16_t *lo)
{
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t c = 0; c < cols; ++c) {
            const float x = X[r * ldx + c];
            const uint16_t h = oracle_bf16_rne(x);
            hi[r * cols + c] = h;
            const float d = isfinite(x) ? x - oracle_bf16_to_float(h) : 0.0f;
            lo[r * cols + c] = oracle_bf16_rne(d);
        }
}

/* ------------------------------------------------------------------------- */
/* OCP FP8 E4M3 ("e4m3fn"): 1 sign, 4 exponent (bias 7), 3 fraction bits.
 * Normal: (1 + f/8) * 2^(e-7), e = 1..15; subnormal: (f/8) * 2^-6; no infinity;
 * S.1111.111 is NaN, so the largest finite magnitude is S.1111.110 = 448.
 * Encoding: round-to-nearest-even onto that grid, saturating to +-448;
 * NaN and infinity encode as NaN (0x7f with the sign).                        */

OR_EXPORT float oracle_e4m3_to_float(uint8_t q)
{
    const int s = q >> 7, e = (q >> 3) & 15, f = q & 7;
    double v;
    if (e == 15 && f == 7) return NAN;
    if (e == 0) v = ldexp((double)f, -9);
    else v = ldexp(8.0 + f, e - 10);
    return (float)(s ? -v : v);
}

static uint8_t e4m3_from_double(double x)
{
    if (isnan(x) || isinf(x)) return (uint8_t)((signbit(x) ? 0x80 : 0) | 0x7f);
    const uint8_t sign = signbit(x) ? 0x80 : 0;
    double a = fabs(x);
    if (a >= 448.0) return sign | 0x7e;
    /* grid spacing where a lives: 2^-9 below 2^-6, else 2^(floor(log2 a) - 3) */
    int ex;
    if (a < ldexp(1.0, -6)) ex = -9;
    else { int e2; frexp(a, &e2); ex = (e2 - 1) - 3; }
    const double step = ldexp(1.0, ex);
    const double lowm = floor(a / step);          /* exact: a / 2^ex is exact */
    const double rem = a - lowm * step;
    double m = lowm;
    if (rem > 0.5 * step || (rem == 0.5 * step && fmod(lowm, 2.0) != 0.0)) m = lowm + 1.0;
    const double v = m * step;
    if (v > 448.0) return sign | 0x7e;            /* cannot happen below 448, kept for clarity */
    /* encode v */
    if (v == 0.0) return sign;
    if (v < ldexp(1.0, -6)) return sign | (uint8_t)(v / ldexp(1.0, -9));
    int e2; frexp(v, &e2);                        /* v = [0.5,1) * 2^e2 */
    const int E = (e2 - 1) + 7;
    const int F = (int)(v / ldexp(1.0, e2 - 1) * 8.0) - 8;
    return sign | (uint8_t)(E << 3) | (uint8_t)F;
}

OR_EXPORT uint8_t oracle_e4m3_rne(float x) { return e4m3_from_double((double)x); }

/*
 * Power-of-two tile scale: the integer e with amax * 2^e <= 448 < amax * 2^(e+1),
 * i.e. s = 2^e = 2^floor(log2(448 / amax)), computed with exact comparisons.
 * amax == 0 gives e = 0; e is clamped to [-127, 127] so that the dequantisation
 * factor 2^-e fits an E8M0 exponent byte (127 - e).  Non-finite amax gives 0.
 */
OR_EXPORT int oracle_scale_exp(float amax)
{
    if (!(amax > 0.0f) || isinf(amax)) return 0;
    int e = 0;
    const double a = (double)amax;
    while (ldexp(a, e) > 448.0) --e;
    while (ldexp(a, e + 1) <= 448.0) ++e;
    if (e > 127) e = 127;
    if (e < -127) e = -127;
    return e;
}

/*
 * Tile-scaled E4M3 quantisation with one residual pass, over 128x128 tiles of a
 * rows x cols matrix (edge tiles are partial; padding counts as zero).
 * For every tile T:
 *   e   = scale_exp(max |x|, x in T);      q  = e4m3(x * 2^e)
 *   r   = x - e4m3val(q) * 2^-e            (exact in binary32)
 *   er  = scale_exp(max |r|, r in T);      rq = e4m3(r * 2^er)
 * Outputs are row-major rows x cols bytes; scale bytes are E8M0 (127 - e) per
 * tile, tile-row-major ((rows+127)/128) x ((cols+127)/128).
 */
OR_EXPORT void oracle_quant_fp8(int64_t rows, int64_t cols, const float *X, int64_t ldx,
                                uint8_t *q, uint8_t *qscale, uint8_t *rq, uint8_t *rscale,
                                float *resid)
{
    const int64_t tr = (rows + 127) / 128, tc = (cols + 127) / 128;
    for (int64_t a = 0; a < tr; ++a)
        for (int64_t b = 0; b < tc; ++b) {
            const int64_t r0 = a * 128, c0 = b * 128;
            const int64_t r1 = (r0 + 128 < rows) ? r0 + 128 : rows;
            const int64_t c1 = (c0 + 128 < cols) ? c0 + 128 : cols;
            float amax = 0.0f;
            for (int64_t r = r0; r < r1; ++r)
                for (int64_t c = c0; c < c1; ++c) {
                    const float v = fabsf(X[r * ldx + c]);
                    if (isnan(v)) amax = NAN;          /* NaN propagates */
                    else if (v > amax) amax = v;
                }
            const int e = oracle_scale_exp(amax);
            qscale[a * tc + b] = (uint8_t)(127 - e);
            float ramax = 0.0f;
            for (int64_t r = r0; r < r1; ++r)
                for (int64_t c = c0; c < c1; ++c) {
                    const float x = X[r * ldx + c];
                    const uint8_t qq = e4m3_from_double(ldexp((double)x, e));
                    q[r * cols + c] = qq;
                    const double back = ldexp((double)oracle_e4m3_to_float(qq), -e);
                    const float rr = isfinite(x) ? (float)((double)x - back) : 0.0f;
                    resid[r * cols + c] = rr;
                    if (fabsf(rr) > ramax) ramax = fabsf(rr);
                }
            const int er = oracle_scale_exp(ramax);
            rscale[a * tc + b] = (uint8_t)(127 - er);
            for (int64_t r = r0; r < r1; ++r)
                for (int64_t c = c0; c < c1; ++c)
                    rq[r * cols + c] = e4m3_from_double(ldexp((double)resid[r * cols + c], er));
        }
}

/* ------------------------------------------------------------------------- */
/* OCP Microscaling (MX) FP6 E2M3: 1 sign, 2 exponent (bias 1), 3 fraction
 * bits, no infinity and no NaN.  Normal: (1 + f/8) * 2^(e-1), e = 1..3;
 * subnormal (e = 0): f/8.  The largest magnitude is 7.5.  Code bits: sign 5,
 * exponent 4..3, fraction 2..0.  Encoding: round-to-nearest-even onto that
 * grid, saturating to +-7.5.  Non-finite values have no code; the block
 * quantisation below marks their block with the E8M0 NaN scale instead and
 * this function returns the zero code for them.                              */

OR_EXPORT float oracle_e2m3_to_float(uint8_t q)
{
    const int s = (q >> 5) & 1, e = (q >> 3) & 3, f = q & 7;
    const double v = (e == 0) ? f / 8.0 : ldexp(8.0 + f, e - 4);
    return (float)(s ? -v : v);
}

static uint8_t e2m3_from_double(double x)
{
    if (isnan(x) || isinf(x)) return 0;
    const uint8_t sign = signbit(x) ? 0x20 : 0;
    const double a = fabs(x);
    if (a >= 7.5) return sign | 0x1f;
    /* grid spacing where a lives: 1/8 below 2 (subnormals and the first
     * binade share it), else 2^(floor(log2 a) - 3) */
    int ex;
    if (a < 2.0) ex = -3;
    else { int e2; frexp(a, &e2); ex = (e2 - 1) - 3; }
    const double step = ldexp(1.0, ex);
    const double lowm = floor(a / step);          /* exact: a / 2^ex is exact */
    const double rem = a - lowm * step;
    double m = lowm;
    if (rem > 0.5 * step || (rem == 0.5 * step && fmod(lowm, 2.0) != 0.0)) m = lowm + 1.0;
    const double v = m * step;                    /* <= 7.5: 7.5 is on the grid */
    if (v < 1.0) return sign | (uint8_t)(v * 8.0);
    int e2; frexp(v, &e2);                        /* v = [0.5,1) * 2^e2, e2 = 1..3 */
    const int F = (int)(v / ldexp(1.0, e2 - 1) * 8.0) - 8;
    return sign | (uint8_t)(e2 << 3) | (uint8_t)F;
}

OR_EXPORT uint8_t oracle_e2m3_rne(float x) { return e2m3_from_double((double)x); }

/*
 * MX block scale for E2M3: the integer e with amax * 2^e <= 7.5 < amax * 2^(e+1)
 * (the block's largest magnitude lands in the top binade of the format without
 * saturating), by exact comparisons; amax == 0 gives 0; clamped to
 * [-127, 127] so that 2^-e is an E8M0 byte (127 - e).
 */
OR_EXPORT int oracle_mx6_scale_exp(float amax)
{
    if (!(amax > 0.0f) || isinf(amax)) return 0;
    int e = 0;
    const double a = (double)amax;
    while (ldexp(a, e) > 7.5) --e;
    while (ldexp(a, e + 1) <= 7.5) ++e;
    if (e > 127) e = 127;
    if (e < -127) e = -127;
    return e;
}

/*
 * MX-style E2M3 quantisation with one residual level.  Every row of X is cut
 * into blocks of 32 consecutive elements (the last block of a row partial;
 * missing elements count as zero).  For a block B whose elements are finite:
 *   e  = mx6_scale_exp(max |x|, x in B);   q  = e2m3(x * 2^e)
 *   r  = x - e2m3val(q) * 2^-e             (exact in binary32)
 *   er = mx6_scale_exp(max |r|, r in B);   rq = e2m3(r * 2^er)
 * with E8M0 scale bytes 127 - e and 127 - er.  A block holding a NaN or an
 * infinity gets the E8M0 NaN byte 0xff at both levels and zero codes, so that
 * every product it enters is NaN.
 * Outputs: codes rows x cols (one per byte, row-major); scale bytes
 * rows x ceil(cols / 32), row-major.
 */
OR_EXPORT void oracle_quant_mx6(int64_t rows, int64_t cols, const float *X, int64_t ldx,
                                uint8_t *q, uint8_t *qscale, uint8_t *rq, uint8_t *rscale)
{
    const int64_t nb = (cols + 31) / 32;
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t c0 = b * 32, c1 = (c0 + 32 < cols) ? c0 + 32 : cols;
            int finite = 1;
            float amax = 0.0f;
            for (int64_t c = c0; c < c1; ++c) {
                const float x = X[r * ldx + c];
                if (!isfinite(x)) finite = 0;
                else if (fabsf(x) > amax) amax = fabsf(x);
            }
            if (!finite) {
                qscale[r * nb + b] = 0xff;
                rscale[r * nb + b] = 0xff;
                for (int64_t c = c0; c < c1; ++c) q[r * cols + c] = rq[r * cols + c] = 0;
                continue;
            }
            const int e = oracle_mx6_scale_exp(amax);
            qscale[r * nb + b] = (uint8_t)(127 - e);
            float res[32];
            float ramax = 0.0f;
            for (int64_t c = c0; c < c1; ++c) {
                const float x = X[r * ldx + c];
                const uint8_t qq = e2m3_from_double(ldexp((double)x, e));
                q[r * cols + c] = qq;
                const double back = ldexp((double)oracle_e2m3_to_float(qq), -e);
                res[c - c0] = (float)((double)x - back);
                if (fabsf(res[c - c0]) > ramax) ramax = fabsf(res[c - c0]);
            }
            const int er = oracle_mx6_scale_exp(ramax);
            rscale[r * nb + b] = (uint8_t)(127 - er);
            for (int64_t c = c0; c < c1; ++c)
                rq[r * cols + c] = e2m3_from_double(ldexp((double)res[c - c0], er));
        }
}

/* ------------------------------------------------------------------------- */
/*
 * Freivalds-style probe of a finished product.  With a probe vector x (here
 * Rademacher +-1), y = B x, z = alpha * A y + beta * C0 x and w = C x; for an
 * error E = C - C_exact, E[ ||E x||^2 ] = ||E||_F^2 and E[ ||C_exact x||^2 ] =
 * ||C_exact||_F^2, so ||w - z|| / ||z|| estimates the relative Frobenius error.
 * All arithmetic in binary64.  C0 may be NULL when beta == 0.
 */
OR_EXPORT double oracle_freivalds(int64_t M, int64_t N, int64_t K, float alpha,
                                  const float *A, int64_t lda, const float *B, int64_t ldb,
                                  float beta, const float *C0, const float *C, int64_t ldc,
                                  const double *x)
{
    double *y = (double *)calloc((size_t)(K > 0 ? K : 1), sizeof(double));
    for (int64_t k = 0; k < K; ++k) {
        double s = 0.0;
        for (int64_t j = 0; j < N; ++j) s += (double)B[k * ldb + j] * x[j];
        y[k] = s;
    }
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < M; ++i) {
        double z = 0.0;
        for (int64_t k = 0; k < K; ++k) z += (double)A[i * lda + k] * y[k];
        z *= (double)alpha;
        double w = 0.0, c0x = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            w += (double)C[i * ldc + j] * x[j];
            if (beta != 0.0f) c0x += (double)C0[i * ldc + j] * x[j];
        }
        z += (double)beta * c0x;
        num += (w - z) * (w - z);
        den += z * z;
    }
    free(y);
    return den > 0.0 ? sqrt(num) / sqrt(den) : sqrt(num);
}
