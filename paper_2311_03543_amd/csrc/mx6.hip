// MX FP6 pre-pass: two-level E2M3 quantisation with one E8M0 scale per block
// of 32 consecutive K values (the OCP Microscaling block size, which is also
// the K extent of one lane's operand in the scaled 32x32x64 MFMA).
//
// For a block x of 32 values (missing values count as zero):
//   e  = the largest integer with max|x| * 2^e <= 7.5 (E2M3's largest value)
//   q  = RNE_e2m3(x * 2^e),   r = x - q * 2^-e  (exact in FP32)
//   er = the same for max|r|, rq = RNE_e2m3(r * 2^er)
// with scale bytes 127 - e and 127 - er.  A block holding a NaN or an
// infinity gets the E8M0 NaN byte 0xff at both levels and zero codes; the
// MFMA then turns every product of that block into NaN.
//
// Panel images (tiled) are the MX FP6 images of common.h: hi codes, lo codes
// (48 bytes per row and 64-value K block) and one scale array holding both
// levels' E8M0 bytes per row and K half.
#include "common.h"
#include "kernels.h"

namespace cmp {
namespace {

// Largest e with amax * 2^e <= 7.5 = 1.875 * 2^2, from the bits of amax: for
// a normal amax = 1.m * 2^(E-127) that is e = 129 - E, one less when
// 1.m > 1.875 (fraction bits above 0x700000).  Zero gives 0, a subnormal
// amax 127 (the clamp), and e is clamped to [-127, 127].
__device__ __forceinline__ int mx6_scale_exp(float amax) {
    if (!(amax > 0.f)) return 0;
    const uint32_t u = __builtin_bit_cast(uint32_t, amax);
    const int E = (int)((u >> 23) & 255u);
    if (E == 0) return 127;
    const int e = 129 - E - ((u & 0x7fffffu) > 0x700000u ? 1 : 0);
    return e > 127 ? 127 : (e < -127 ? -127 : e);
}

// Four E2M3 codes, packed 6 bits each at bits 0, 6, 12, 18, of values whose
// scaled forms s_j = x_j 2^e satisfy |s_j| <= 7.5, given as t_j = s_j 2^-6.
// They come from the E4M3 converter (v_cvt_pk_fp8_f32, round to nearest
// even): on [0, 7.5 2^-6] the E4M3 grid is the E2M3 grid scaled by 2^-6 (the
// E4M3 subnormals k 2^-9 are E2M3's k / 8 there, and from 2^-6 up both keep
// three fraction bits), so rounding t_j onto one is rounding s_j onto the
// other, and the E4M3 byte, whose exponent field is at most 3, holds the E2M3
// code in its sign (bit 7 -> 5), the low two exponent bits and the fraction.
// q8 receives the four E4M3 bytes: their values times 2^6 are the codes'
// values s_j rounded.
__device__ __forceinline__ uint32_t e2m3x4(float t0, float t1, float t2, float t3, uint32_t& q8) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(t0, t1, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(t2, t3, w, true);
    q8 = (uint32_t)w;
    const uint32_t by = (q8 & 0x1f1f1f1fu) | ((q8 >> 2) & 0x20202020u);   // one code per byte
    return (by & 0x3fu) | ((by >> 2) & 0xfc0u) | ((by >> 4) & 0x3f000u) | ((by >> 6) & 0xfc0000u);
}
// First level of four values x_j of a block with exponent e (inv = 2^-e):
// their packed codes, and the residuals x - q 2^-e (one FMA, rounded once; a
// zero code leaves x, and -0 - (-0) gives +0 as the definition does), which
// replace the values.
__device__ __forceinline__ uint32_t mx6_level1(float (&x)[4], int e, float inv) {
    uint32_t q8;
    const uint32_t code = e2m3x4(__builtin_ldexpf(x[0], e - 6), __builtin_ldexpf(x[1], e - 6),
                                 __builtin_ldexpf(x[2], e - 6), __builtin_ldexpf(x[3], e - 6), q8);
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)q8, false);
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)q8, true);
    const float qv[4] = {lo[0] * 64.f, lo[1] * 64.f, hi[0] * 64.f, hi[1] * 64.f};
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = __builtin_fmaf(-qv[j], inv, x[j]);
    return code;
}
// Second level: the residuals' packed codes with their block exponent e.
__device__ __forceinline__ uint32_t mx6_level2(const float (&r)[4], int e) {
    uint32_t q8;
    return e2m3x4(__builtin_ldexpf(r[0], e - 6), __builtin_ldexpf(r[1], e - 6),
                  __builtin_ldexpf(r[2], e - 6), __builtin_ldexpf(r[3], e - 6), q8);
}

// ---------------------------------------------------------------------------
// Rows of X (blocks along X's rows, K = cols): eight lanes per block, four
// consecutive values each, so one wave reads 1 KiB of a row with each load;
// a lane takes kMx6RowsPerLane rows at a time and issues all their loads
// first.  The block's amax and NaN flag are reduced over the eight lanes; each
// lane then holds 4 codes (24 bits) and lane i < 6 assembles dword i of the
// packed 192 bits from the 24-bit words of two neighbours; lane 6 writes the
// block's two scale bytes.
constexpr int kMx6RowsPerLane = 4;
// Workgroup (bx, by) of a grid whose y extent is gy.
template <bool VEC, bool TILED>
__device__ __forceinline__ void quant_mx6_rows(
    int bx, int64_t by, int64_t gy, int64_t rows, int64_t cols, const float* __restrict__ X, int64_t ldx,
    int64_t out_rows, int64_t Kp, uint8_t* __restrict__ q, uint8_t* __restrict__ qscale,
    uint8_t* __restrict__ rq, uint8_t* __restrict__ rscale) {
    // grid: x over the 8 nb lanes of one output row (nb * 8 < 2^31), y over rows
    const int nb = (int)(TILED ? Kp / 32 : (cols + 31) / 32);   // blocks per output row
    const int64_t nrows = TILED ? out_rows : rows;
    const int64_t nkb = Kp / 64;
    const int i = bx * 256 + (int)threadIdx.x;                  // lane of the row: block i / 8
    if ((i >> 3) >= nb) return;                                 // whole 8-lane groups only
    const int lane = threadIdx.x & 63;
    const int li = lane & 7, gbase = lane & ~7;
    // source lanes of the packed dword this lane assembles (li < 6)
    const int src_lo = li < 6 ? gbase + 4 * (li / 3) + li % 3 : lane;
    const int src_hi = li < 6 ? src_lo + 1 : lane;
    const int sh = li < 6 ? 8 * (li % 3) : 0;
    const int b = i >> 3;
    const int64_t k = (int64_t)b * 32 + 4 * li;
    constexpr int RPL = kMx6RowsPerLane;
    for (int64_t r0 = by * RPL; r0 < nrows; r0 += gy * RPL) {
        float vr[RPL][4];
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int64_t r = r0 + rr;
            float* v = vr[rr];
            v[0] = v[1] = v[2] = v[3] = 0.f;
            if (r < rows) {
                const float* p = X + r * ldx + k;
                if (VEC && k + 3 < cols) {
                    const float4 a = *reinterpret_cast<const float4*>(p);
                    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (k + j < cols) v[j] = p[j];
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
            const int64_t r = r0 + rr;
            if (r >= nrows) break;                  // uniform: r depends on the workgroup only
            float (&v)[4] = vr[rr];
            float amax = 0.f;
            int bad = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (!__builtin_isfinite(v[j])) bad = 1;
                else amax = fmaxf(amax, fabsf(v[j]));
            }
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) {
                amax = fmaxf(amax, __shfl_xor(amax, off));
                bad |= __shfl_xor(bad, off);
            }
            uint32_t w0 = 0, w1 = 0, sb0 = 0xffu, sb1 = 0xffu;
            if (!bad) {
                const int e0 = mx6_scale_exp(amax);
                w0 = mx6_level1(v, e0, __builtin_ldexpf(1.f, -e0));
                float ramax = fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
#pragma unroll
                for (int off = 1; off < 8; off <<= 1) ramax = fmaxf(ramax, __shfl_xor(ramax, off));
                const int e1 = mx6_scale_exp(ramax);
                w1 = mx6_level2(v, e1);
                sb0 = (uint32_t)(127 - e0);
                sb1 = (uint32_t)(127 - e1);
            }
            if (TILED) {
                // dword li (< 6) of this block's 24 code bytes; the scales from lane 6
                const uint32_t lo0 = __shfl(w0, src_lo), hi0 = __shfl(w0, src_hi);
                const uint32_t lo1 = __shfl(w1, src_lo), hi1 = __shfl(w1, src_hi);
                if (li < 6) {
                    const int64_t o = mx6_code_offset(r, b >> 1, b & 1, 4 * li, nkb);
                    *reinterpret_cast<uint32_t*>(q + o) = (lo0 >> sh) | (hi0 << (24 - sh));
                    *reinterpret_cast<uint32_t*>(rq + o) = (lo1 >> sh) | (hi1 << (24 - sh));
                } else if (li == 6) {
                    *reinterpret_cast<uint16_t*>(qscale + mx6_scale_offset(r, b >> 1, b & 1, 0, nkb)) =
                        (uint16_t)(sb0 | (sb1 << 8));
                }
            } else {
                // one code per byte, row-major rows x cols; the scales from lane 0
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (k + j < cols) {
                        q[r * cols + k + j] = (uint8_t)((w0 >> (6 * j)) & 63u);
                        rq[r * cols + k + j] = (uint8_t)((w1 >> (6 * j)) & 63u);
                    }
                if (li == 0) {
                    qscale[r * nb + b] = (uint8_t)sb0;
                    rscale[r * nb + b] = (uint8_t)sb1;
                }
            }
        }
    }
}

template <bool VEC, bool TILED>
__global__ __launch_bounds__(256) void quant_mx6_rows_kernel(
    int64_t rows, int64_t cols, const float* __restrict__ X, int64_t ldx, int64_t out_rows,
    int64_t Kp, uint8_t* __restrict__ q, uint8_t* __restrict__ qscale, uint8_t* __restrict__ rq,
    uint8_t* __restrict__ rscale) {
    quant_mx6_rows<VEC, TILED>((int)blockIdx.x, blockIdx.y, gridDim.y, rows, cols, X, ldx, out_rows, Kp,
                               q, qscale, rq, rscale);
}

// ---------------------------------------------------------------------------
// Columns of X (X is K x N; output row n = column n of X, blocks along K):
// one lane per pair of blocks (64 K values, one 48-byte image row and its 4
// scale bytes), consecutive lanes on consecutive columns, so each load of a
// lane is one coalesced row segment of X and a wave's stores fill contiguous
// 3 KiB of each code image.  The lane packs its 32 codes per block itself.
// Workgroup (bx, by) of a grid whose y extent is gy; stage_h / stage_l are the
// LDS staging blocks (kMx6Block bytes each when TILED).
template <bool TILED>
__device__ __forceinline__ void quant_mx6_cols(
    int64_t bx, int64_t by, int64_t gy, int64_t K, int64_t N, const float* __restrict__ X, int64_t ldx,
    int64_t out_rows, int64_t Kp, uint8_t* __restrict__ q, uint8_t* __restrict__ qscale,
    uint8_t* __restrict__ rq, uint8_t* __restrict__ rscale, uint4* stage_h, uint4* stage_l) {
    // grid: x over output rows (columns of X), y over pairs of blocks.  Tiled:
    // a workgroup's 256 rows are one 256-row image block, staged in LDS so that
    // its two 12 KiB code blocks leave as whole coalesced lines.
    static_assert(kMx6Block % (16 * 256) == 0, "a staged block is whole 16-byte stores per lane");
    const int64_t nb = TILED ? Kp / 32 : (K + 31) / 32;
    const int64_t npairs = (nb + 1) / 2;
    const int64_t nrows = TILED ? out_rows : N;
    const int64_t nkb = Kp / 64;
    const int t = threadIdx.x;
    const int64_t n = bx * 256 + t;
    if (!TILED && n >= nrows) return;        // tiled: out_rows % 256 == 0, every lane has a row
    for (int64_t pr = by; pr < npairs; pr += gy) {
        uint32_t scales = 0;                    // (h0 hi, h0 lo, h1 hi, h1 lo) of this row segment
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            const int64_t b = 2 * pr + h;
            if (b >= nb) break;
            const int64_t k0 = b * 32;
            float v[32];
            float amax = 0.f;
            bool bad = false;
            // out-of-range lanes load X[0] (in bounds) and keep 0: no branch per load
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                const bool in = n < N && k0 + j < K;
                const float x = X[in ? (k0 + j) * ldx + n : 0];
                v[j] = in ? x : 0.f;
            }
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                if (!__builtin_isfinite(v[j])) bad = true;
                else amax = fmaxf(amax, fabsf(v[j]));
            }
            // codes packed as they are made: code j at bit 6 j of p0 / p1, four
            // codes (24 bits) at a time
            uint32_t p0[6] = {0, 0, 0, 0, 0, 0}, p1[6] = {0, 0, 0, 0, 0, 0};
            auto put24 = [](uint32_t (&p)[6], int m, uint32_t c) {
                const int bit = 24 * m, d = bit >> 5, sh = bit & 31;
                p[d] |= c << sh;
                if (sh > 8) p[d + 1] |= c >> (32 - sh);
            };
            uint32_t sb0 = 0xffu, sb1 = 0xffu;
            if (!bad) {
                const int e0 = mx6_scale_exp(amax);
                const float inv = __builtin_ldexpf(1.f, -e0);
                float ramax = 0.f;
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    float x4[4] = {v[4 * m], v[4 * m + 1], v[4 * m + 2], v[4 * m + 3]};
                    put24(p0, m, mx6_level1(x4, e0, inv));
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        v[4 * m + j] = x4[j];
                        ramax = fmaxf(ramax, fabsf(x4[j]));
                    }
                }
                const int e1 = mx6_scale_exp(ramax);
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const float r4[4] = {v[4 * m], v[4 * m + 1], v[4 * m + 2], v[4 * m + 3]};
                    put24(p1, m, mx6_level2(r4, e1));
                }
                sb0 = (uint32_t)(127 - e0);
                sb1 = (uint32_t)(127 - e1);
            }
            if (TILED) {
                // this row's 48 bytes at 48 t of the staged block (the image's row layout)
                uint8_t* sh8 = reinterpret_cast<uint8_t*>(stage_h) + t * kMx6RowBytes;
                uint8_t* sl8 = reinterpret_cast<uint8_t*>(stage_l) + t * kMx6RowBytes;
                *reinterpret_cast<uint4*>(sh8 + 16 * h) = make_uint4(p0[0], p0[1], p0[2], p0[3]);
                *reinterpret_cast<uint2*>(sh8 + 32 + 8 * h) = make_uint2(p0[4], p0[5]);
                *reinterpret_cast<uint4*>(sl8 + 16 * h) = make_uint4(p1[0], p1[1], p1[2], p1[3]);
                *reinterpret_cast<uint2*>(sl8 + 32 + 8 * h) = make_uint2(p1[4], p1[5]);
                scales |= (sb0 | (sb1 << 8)) << (16 * h);
            } else {
#pragma unroll
                for (int j = 0; j < 32; ++j) {
                    const int bit = 6 * j, d = bit >> 5, sh = bit & 31;
                    const uint32_t c0 = ((p0[d] >> sh) | (sh > 26 ? p0[d + 1] << (32 - sh) : 0u)) & 63u;
                    const uint32_t c1 = ((p1[d] >> sh) | (sh > 26 ? p1[d + 1] << (32 - sh) : 0u)) & 63u;
                    if (k0 + j < K) {
                        q[n * K + k0 + j] = (uint8_t)c0;
                        rq[n * K + k0 + j] = (uint8_t)c1;
                    }
                }
                qscale[n * nb + b] = (uint8_t)sb0;
                rscale[n * nb + b] = (uint8_t)sb1;
            }
        }
        if (TILED) {
            *reinterpret_cast<uint32_t*>(qscale + mx6_scale_offset(n, pr, 0, 0, nkb)) = scales;
            __syncthreads();
            const int64_t base = (bx * nkb + pr) * kMx6Block;
#pragma unroll
            for (int c = 0; c < kMx6Block / 16 / 256; ++c) {
                reinterpret_cast<uint4*>(q + base)[t + 256 * c] = stage_h[t + 256 * c];
                reinterpret_cast<uint4*>(rq + base)[t + 256 * c] = stage_l[t + 256 * c];
            }
            __syncthreads();                     // the stage is rewritten by the next pair
        }
    }
}

template <bool TILED>
__global__ __launch_bounds__(256) void quant_mx6_cols_kernel(
    int64_t K, int64_t N, const float* __restrict__ X, int64_t ldx, int64_t out_rows, int64_t Kp,
    uint8_t* __restrict__ q, uint8_t* __restrict__ qscale, uint8_t* __restrict__ rq,
    uint8_t* __restrict__ rscale) {
    __shared__ uint4 stage_h[TILED ? kMx6Block / 16 : 1], stage_l[TILED ? kMx6Block / 16 : 1];
    quant_mx6_cols<TILED>(blockIdx.x, blockIdx.y, gridDim.y, K, N, X, ldx, out_rows, Kp, q, qscale, rq,
                          rscale, stage_h, stage_l);
}

// Both operands' MX FP6 images in one launch: A by rows (a.gx x a.gy
// workgroups of quant_mx6_rows) and B by columns (b.gx x b.gy workgroups of
// quant_mx6_cols), interleaved by paired_kind.
struct Mx6Operand {
    int64_t rows, cols, ldx, out_rows, Kp, gx, gy;
    const float* X;
    uint8_t *q, *qscale, *rq;
};
template <bool VA>
__global__ __launch_bounds__(256) void quant_mx6_pair_kernel(Mx6Operand a, Mx6Operand b) {
    __shared__ uint4 stage_h[kMx6Block / 16], stage_l[kMx6Block / 16];
    int64_t w;
    const int kind = paired_kind(blockIdx.x, a.gx * a.gy, b.gx * b.gy, &w);
    if (kind < 0) return;
    if (kind == 1)
        quant_mx6_cols<true>(w % b.gx, w / b.gx, b.gy, b.rows, b.cols, b.X, b.ldx, b.out_rows, b.Kp, b.q,
                             b.qscale, b.rq, nullptr, stage_h, stage_l);
    else
        quant_mx6_rows<VA, true>((int)(w % a.gx), w / a.gx, a.gy, a.rows, a.cols, a.X, a.ldx, a.out_rows,
                                 a.Kp, a.q, a.qscale, a.rq, nullptr);
}

unsigned cap(int64_t v, int64_t m) { return (unsigned)(v < 1 ? 1 : (v > m ? m : v)); }

}  // namespace

hipError_t launch_quant_mx6_pair(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                                const float* B, int64_t ldb, int64_t Mp, int64_t Np, int64_t Kp,
                                uint8_t* aq, uint8_t* ar, uint8_t* as, uint8_t* bq, uint8_t* br,
                                uint8_t* bs, hipStream_t stream) {
    if (M <= 0 || N <= 0 || K <= 0 || !A || !B || !aq || !ar || !as || !bq || !br || !bs ||
        Mp % kPanelRows || Np % kPanelRows || Mp < M || Np < N || Kp % 64 || Kp < K)
        return hipErrorInvalidValue;
    const int64_t nb = Kp / 32;
    if (nb * 8 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    Mx6Operand a{M, K, lda, Mp, Kp, (int64_t)cap((nb * 8 + 255) / 256, 1 << 30),
                 (int64_t)cap((Mp + kMx6RowsPerLane - 1) / kMx6RowsPerLane, 65535), A, aq, as, ar};
    Mx6Operand b{K, N, ldb, Np, Kp, Np / 256, (int64_t)cap((nb + 1) / 2, 65535), B, bq, bs, br};
    const int64_t blocks = paired_blocks(a.gx * a.gy, b.gx * b.gy);
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const bool va = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
    if (va)
        hipLaunchKernelGGL(quant_mx6_pair_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, stream, a, b);
    else
        hipLaunchKernelGGL(quant_mx6_pair_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, stream, a, b);
    return hipGetLastError();
}

hipError_t launch_quant_mx6(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                            bool transpose, bool tiled, int64_t out_rows, int64_t Kp, uint8_t* q,
                            uint8_t* qscale, uint8_t* rq, uint8_t* rscale, hipStream_t stream) {
    if (rows <= 0 || cols <= 0 || !X || !q || !rq) return hipErrorInvalidValue;
    const int64_t orows = transpose ? cols : rows, K = transpose ? rows : cols;
    if (tiled) {
        if (out_rows % kPanelRows || out_rows < orows || Kp % 64 || Kp < K || !qscale)
            return hipErrorInvalidValue;
    } else if (!qscale || !rscale) {
        return hipErrorInvalidValue;
    }
    if (!transpose) {
        const int64_t nb = tiled ? Kp / 32 : (cols + 31) / 32;
        if (nb * 8 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
        const int64_t nr = tiled ? out_rows : rows;
        const dim3 g(cap((nb * 8 + 255) / 256, 1 << 30), cap((nr + kMx6RowsPerLane - 1) / kMx6RowsPerLane, 65535));
        const bool vec = (ldx % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
        auto go = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, g, dim3(256), 0, stream, rows, cols, X, ldx, out_rows, Kp, q,
                               qscale, rq, rscale);
        };
        if (vec) tiled ? go(quant_mx6_rows_kernel<true, true>) : go(quant_mx6_rows_kernel<true, false>);
        else tiled ? go(quant_mx6_rows_kernel<false, true>) : go(quant_mx6_rows_kernel<false, false>);
    } else {
        const int64_t nb = tiled ? Kp / 32 : (rows + 31) / 32;
        const dim3 g(cap(((tiled ? out_rows : cols) + 255) / 256, 1 << 30), cap((nb + 1) / 2, 65535));
        if (tiled)
            hipLaunchKernelGGL(quant_mx6_cols_kernel<true>, g, dim3(256), 0, stream, rows, cols, X, ldx,
                               out_rows, Kp, q, qscale, rq, rscale);
        else
            hipLaunchKernelGGL(quant_mx6_cols_kernel<false>, g, dim3(256), 0, stream, rows, cols, X, ldx,
                               out_rows, Kp, q, qscale, rq, rscale);
    }
    return hipGetLastError();
}

}  // namespace cmp
