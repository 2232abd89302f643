// Operand pre-pass kernels for the MFMA variants.  They read the FP32
// operands once and write K-contiguous, zero-padded panel images (layout in
// common.h) the GEMM kernels stream without bounds checks:
//
//   bf16 split:   hi = RNE_bf16(x), lo = RNE_bf16(x - hi)   (x - hi is exact in FP32)
//   E4M3 quant:   per 128 x 128 tile, e = the largest integer with
//                 amax * 2^e <= 448 (OCP E4M3's largest finite value),
//                 q = RNE_e4m3(x * 2^e), r = x - q * 2^-e (exact in FP32),
//                 then the same with r's own tile exponent: rq = RNE_e4m3(r * 2^er).
//                 Scale bytes are E8M0 exponents 127 - e, the dequantisation
//                 factor the scaled MFMA applies.
//
// All kernels are HBM-bound (4 bytes read, 2 or 4 written per element); the
// B operand is transposed through LDS so that the written image is N x K.
#include "common.h"
#include "kernels.h"

namespace cmp {
namespace {

__device__ __forceinline__ uint16_t bf16_bits(float x) {
    const __bf16 h = (__bf16)x;  // v_cvt_pk_bf16_f32: round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float bf16_val(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}
// (hi, lo) pair for one value; lo is 0 for non-finite x.
__device__ __forceinline__ void split1(float x, uint16_t& hi, uint16_t& lo) {
    hi = bf16_bits(x);
    lo = __builtin_isfinite(x) ? bf16_bits(x - bf16_val(hi)) : (uint16_t)0;
}

// ---------------------------------------------------------------------------
// A (M x K, lda) -> hi/lo panel images (Mp rows, Kp bf16 per row).  One lane
// per 16-byte image chunk (8 consecutive k), lanes in image order: the writes
// are contiguous and each group of 4 lanes reads 32 consecutive floats of a row.
template <bool VEC>
__global__ void split_a_kernel(int64_t M, int64_t K, const float* __restrict__ A, int64_t lda,
                               int64_t Mp, int64_t Kp, uint16_t* __restrict__ hi,
                               uint16_t* __restrict__ lo) {
    const int64_t nkb = Kp * 2 / kPanelRowBytes;
    const int64_t total = Mp * (Kp / 8);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t blk = e >> 10;            // 1024 chunks per 16 KiB block
        const int w = (int)(e & 1023), rr = w >> 2, pos = w & 3;
        const int64_t rb = blk / nkb, kb = blk - rb * nkb;
        const int64_t r = rb * kPanelRows + rr;
        const int64_t k = kb * 32 + (int64_t)((pos ^ ((rr >> 2) & 3)) * 8);
        float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (r < M) {
            const float* p = A + r * lda + k;
            if (VEC && k + 7 < K) {
                const float4 a0 = *reinterpret_cast<const float4*>(p);
                const float4 a1 = *reinterpret_cast<const float4*>(p + 4);
                v[0] = a0.x; v[1] = a0.y; v[2] = a0.z; v[3] = a0.w;
                v[4] = a1.x; v[5] = a1.y; v[6] = a1.z; v[7] = a1.w;
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (k + i < K) v[i] = p[i];
            }
        }
        uint16_t h[8], l[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) split1(v[i], h[i], l[i]);
        uint4 hv, lv;
        hv.x = h[0] | ((uint32_t)h[1] << 16); hv.y = h[2] | ((uint32_t)h[3] << 16);
        hv.z = h[4] | ((uint32_t)h[5] << 16); hv.w = h[6] | ((uint32_t)h[7] << 16);
        *reinterpret_cast<uint4*>(hi + e * 8) = hv;
        if (lo) {
            lv.x = l[0] | ((uint32_t)l[1] << 16); lv.y = l[2] | ((uint32_t)l[3] << 16);
            lv.z = l[4] | ((uint32_t)l[5] << 16); lv.w = l[6] | ((uint32_t)l[7] << 16);
            *reinterpret_cast<uint4*>(lo + e * 8) = lv;
        }
    }
}

// B (K x N, ldb) -> hi/lo transposed panel images (Np rows, Kp bf16 per row);
// one 64 x 64 tile per workgroup.
template <bool VEC>
__global__ __launch_bounds__(256) void split_bt_kernel(int64_t K, int64_t N,
                                                       const float* __restrict__ B, int64_t ldb,
                                                       int64_t Kp, uint16_t* __restrict__ hi,
                                                       uint16_t* __restrict__ lo) {
    __shared__ float T[64][65];
    const int t = threadIdx.x;
    const int64_t tiles_k = Kp / 64;
    const int64_t k0 = (blockIdx.x % tiles_k) * 64;
    const int64_t n0 = (blockIdx.x / tiles_k) * 64;
    // load: rows k0 + t/16 + 16 i, columns n0 + 4 (t % 16) .. +3
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int kl = (t >> 4) + 16 * i;
        const int nl = (t & 15) * 4;
        const int64_t k = k0 + kl, n = n0 + nl;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k < K) {
            const float* p = B + k * ldb + n;
            if (VEC && n + 3 < N) {
                v = *reinterpret_cast<const float4*>(p);
            } else {
                if (n + 0 < N) v.x = p[0];
                if (n + 1 < N) v.y = p[1];
                if (n + 2 < N) v.z = p[2];
                if (n + 3 < N) v.w = p[3];
            }
        }
        T[kl][nl + 0] = v.x;
        T[kl][nl + 1] = v.y;
        T[kl][nl + 2] = v.z;
        T[kl][nl + 3] = v.w;
    }
    __syncthreads();
    // store: row n0 + t/4 of the image, k0 + 16 (t % 4) .. +15
    const int nl = t >> 2;
    const int kb = (t & 3) * 16;
    uint16_t h[16], l[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) split1(T[kb + i][nl], h[i], l[i]);
    const int64_t nkb = Kp * 2 / kPanelRowBytes;
    // image byte offsets of this lane's two 8-k chunks
    const int64_t o0 = panel_offset(n0 + nl, (k0 + kb) * 2, nkb);
    const int64_t o1 = panel_offset(n0 + nl, (k0 + kb + 8) * 2, nkb);
    uint8_t* ph = reinterpret_cast<uint8_t*>(hi);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        uint4 hv;
        hv.x = h[8 * q + 0] | ((uint32_t)h[8 * q + 1] << 16);
        hv.y = h[8 * q + 2] | ((uint32_t)h[8 * q + 3] << 16);
        hv.z = h[8 * q + 4] | ((uint32_t)h[8 * q + 5] << 16);
        hv.w = h[8 * q + 6] | ((uint32_t)h[8 * q + 7] << 16);
        *reinterpret_cast<uint4*>(ph + (q ? o1 : o0)) = hv;
    }
    if (lo) {
        uint8_t* pl = reinterpret_cast<uint8_t*>(lo);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            uint4 lv;
            lv.x = l[8 * q + 0] | ((uint32_t)l[8 * q + 1] << 16);
            lv.y = l[8 * q + 2] | ((uint32_t)l[8 * q + 3] << 16);
            lv.z = l[8 * q + 4] | ((uint32_t)l[8 * q + 5] << 16);
            lv.w = l[8 * q + 6] | ((uint32_t)l[8 * q + 7] << 16);
            *reinterpret_cast<uint4*>(pl + (q ? o1 : o0)) = lv;
        }
    }
}

__global__ void split_plain_kernel(int64_t rows, int64_t cols, const float* __restrict__ X,
                                   int64_t ldx, uint16_t* __restrict__ hi,
                                   uint16_t* __restrict__ lo) {
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / cols, c = e - r * cols;
        uint16_t h, l;
        split1(X[r * ldx + c], h, l);
        hi[e] = h;
        if (lo) lo[e] = l;
    }
}

// ---------------------------------------------------------------------------
// E4M3 tile quantisation.

// Largest e with amax * 2^e <= 448, from the bits of amax (exact): for a
// normal amax = 1.m * 2^(E-127), amax * 2^e <= 448 = 1.75 * 2^8 holds up to
// e = 135 - E, one less when 1.m > 1.75.  Zero, NaN and infinity give 0;
// e is clamped to [-127, 127] (subnormal amax lands on 127).
__device__ __forceinline__ int scale_exp(float amax) {
    if (!(amax > 0.f) || __builtin_isinf(amax)) return 0;
    const uint32_t u = __builtin_bit_cast(uint32_t, amax);
    const int E = (int)((u >> 23) & 255u);
    if (E == 0) return 127;
    int e = 135 - E - ((u & 0x7fffffu) > 0x600000u ? 1 : 0);
    return e > 127 ? 127 : (e < -127 ? -127 : e);
}

// Encoding rule at the ends of the range: finite values beyond +-448
// saturate, infinities and NaN become the NaN code.
__device__ __forceinline__ float e4m3_sat(float s) {
    if (__builtin_isinf(s)) return __builtin_nanf("");
    return fabsf(s) > 448.f ? copysignf(448.f, s) : s;
}
// Four floats -> four E4M3 bytes (v_cvt_pk_fp8_f32, round to nearest even).
__device__ __forceinline__ uint32_t e4m3x4(float a, float b, float c, float d) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_sat(a), e4m3_sat(b), 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_sat(c), e4m3_sat(d), w, true);
    return (uint32_t)w;
}
__device__ __forceinline__ float e4m3_byte_val(uint32_t word, int byte) {
    switch (byte) {
        case 0: return __builtin_amdgcn_cvt_f32_fp8((int)word, 0);
        case 1: return __builtin_amdgcn_cvt_f32_fp8((int)word, 1);
        case 2: return __builtin_amdgcn_cvt_f32_fp8((int)word, 2);
        default: return __builtin_amdgcn_cvt_f32_fp8((int)word, 3);
    }
}

__device__ __forceinline__ float block_max(float v, float* red, bool& any_nan_inout) {
    // NaN propagates: any NaN in the block makes the result NaN.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int nan_flag = any_nan_inout ? 1 : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v = fmaxf(v, __shfl_xor(v, off));
        nan_flag |= __shfl_xor(nan_flag, off);
    }
    __syncthreads();
    if (lane == 0) {
        red[wave] = v;
        red[4 + wave] = nan_flag ? 1.f : 0.f;
    }
    __syncthreads();
    float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    const bool nan_any = (red[4] + red[5] + red[6] + red[7]) > 0.f;
    any_nan_inout = nan_any;
    return nan_any ? __builtin_nanf("") : m;
}

// One 128 x 128 output tile per workgroup of 256 lanes.  Lane t holds rows
// 8 i + t/32 (i = 0..15) and columns 4 (t % 32) .. +3 of the X tile.  The
// code images are row-major out_rows x out_cols (TILED false) or panel images
// with out_cols bytes of K per row (TILED true).
template <bool VEC, bool TRANS, bool TILED>
__global__ __launch_bounds__(256) void quant_fp8_kernel(
    int64_t rows, int64_t cols, const float* __restrict__ X, int64_t ldx, int64_t out_cols,
    uint8_t* __restrict__ q, uint8_t* __restrict__ qscale, uint8_t* __restrict__ rq,
    uint8_t* __restrict__ rscale) {
    __shared__ float red[8];
    __shared__ uint32_t tq[128][33];   // transposed staging: [col][row/4] words
    __shared__ uint32_t tr[128][33];
    const int t = threadIdx.x;
    const int64_t ot_cols = out_cols / 128;
    const int64_t nkb = out_cols / kPanelRowBytes;
    auto out_off = [&](int64_t orow, int64_t ocol) -> int64_t {
        return TILED ? panel_offset(orow, ocol, nkb) : orow * out_cols + ocol;
    };
    const int64_t ot_r = blockIdx.x / ot_cols, ot_c = blockIdx.x % ot_cols;
    // tile origin in X coordinates
    const int64_t x_r0 = TRANS ? ot_c * 128 : ot_r * 128;
    const int64_t x_c0 = TRANS ? ot_r * 128 : ot_c * 128;
    const int cl = (t & 31) * 4;

    float v[16][4];
    float amax = 0.f;
    bool nan_seen = false;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t r = x_r0 + 8 * i + (t >> 5);
        const int64_t c = x_c0 + cl;
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < rows) {
            const float* p = X + r * ldx + c;
            if (VEC && c + 3 < cols) {
                a = *reinterpret_cast<const float4*>(p);
            } else {
                if (c + 0 < cols) a.x = p[0];
                if (c + 1 < cols) a.y = p[1];
                if (c + 2 < cols) a.z = p[2];
                if (c + 3 < cols) a.w = p[3];
            }
        }
        v[i][0] = a.x; v[i][1] = a.y; v[i][2] = a.z; v[i][3] = a.w;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float m = fabsf(v[i][j]);
            if (__builtin_isnan(m)) nan_seen = true;
            else amax = fmaxf(amax, m);
        }
    }
    amax = block_max(amax, red, nan_seen);
    const int e = scale_exp(amax);

    // Residual r = x - q * 2^-e, rounded once to FP32.  In the scaled domain
    // s - q is exact (s = x * 2^e is exact whenever q != 0), and scaling it
    // back rounds once; this also avoids q * 2^-e overflowing FP32 when x is
    // within rounding distance of FLT_MAX.  A zero code leaves r = x - (+-0),
    // which is x except that -0 - (-0) = +0.
    uint32_t qw[16];
    float ramax = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        float s[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) s[j] = ldexpf(v[i][j], e);
        qw[i] = e4m3x4(s[0], s[1], s[2], s[3]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float qv = e4m3_byte_val(qw[i], j);
            float r = 0.f;
            if (__builtin_isfinite(v[i][j])) r = (qv == 0.f) ? v[i][j] - qv : ldexpf(s[j] - qv, -e);
            v[i][j] = r;
            ramax = fmaxf(ramax, fabsf(r));
        }
    }
    bool no_nan = false;
    ramax = block_max(ramax, red, no_nan);
    const int er = scale_exp(ramax);
    uint32_t rw[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        rw[i] = e4m3x4(ldexpf(v[i][0], er), ldexpf(v[i][1], er), ldexpf(v[i][2], er),
                       ldexpf(v[i][3], er));

    if (t == 0) {
        qscale[blockIdx.x] = (uint8_t)(127 - e);
        rscale[blockIdx.x] = (uint8_t)(127 - er);
    }
    if (!TRANS) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t orow = ot_r * 128 + 8 * i + (t >> 5);
            const int64_t ocol = ot_c * 128 + cl;
            const int64_t o = out_off(orow, ocol);
            *reinterpret_cast<uint32_t*>(q + o) = qw[i];
            *reinterpret_cast<uint32_t*>(rq + o) = rw[i];
        }
    } else {
        // out[x_col][x_row]: stage bytes by column, then write rows of 128 bytes
        uint8_t* sq = reinterpret_cast<uint8_t*>(&tq[0][0]);
        uint8_t* sr = reinterpret_cast<uint8_t*>(&tr[0][0]);
        constexpr int stride = 33 * 4;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int xr = 8 * i + (t >> 5);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                sq[(cl + j) * stride + xr] = (uint8_t)(qw[i] >> (8 * j));
                sr[(cl + j) * stride + xr] = (uint8_t)(rw[i] >> (8 * j));
            }
        }
        __syncthreads();
        const int oc = t >> 1;            // output row within the tile (= X column)
        const int half = (t & 1) * 64;    // 64 bytes of that row
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            uint4 a, b;
            const uint32_t* srcq = &tq[oc][(half + 16 * w) / 4];
            const uint32_t* srcr = &tr[oc][(half + 16 * w) / 4];
            a.x = srcq[0]; a.y = srcq[1]; a.z = srcq[2]; a.w = srcq[3];
            b.x = srcr[0]; b.y = srcr[1]; b.z = srcr[2]; b.w = srcr[3];
            const int64_t o = out_off(ot_r * 128 + oc, ot_c * 128 + half + 16 * w);
            *reinterpret_cast<uint4*>(q + o) = a;
            *reinterpret_cast<uint4*>(rq + o) = b;
        }
    }
}

unsigned grid_for(int64_t work, int64_t per_block) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_split_a_bf16(int64_t M, int64_t K, const float* A, int64_t lda, int64_t Mp,
                               int64_t Kp, uint16_t* hi, uint16_t* lo, hipStream_t stream) {
    const bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
    const unsigned g = grid_for(Mp * (Kp / 8), 256);
    if (vec)
        hipLaunchKernelGGL(split_a_kernel<true>, dim3(g), dim3(256), 0, stream, M, K, A, lda, Mp,
                           Kp, hi, lo);
    else
        hipLaunchKernelGGL(split_a_kernel<false>, dim3(g), dim3(256), 0, stream, M, K, A, lda, Mp,
                           Kp, hi, lo);
    return hipGetLastError();
}

hipError_t launch_split_bt_bf16(int64_t K, int64_t N, const float* B, int64_t ldb, int64_t Np,
                                int64_t Kp, uint16_t* hi, uint16_t* lo, hipStream_t stream) {
    const bool vec = (ldb % 4 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
    const unsigned g = (unsigned)((Np / 64) * (Kp / 64));
    if (vec)
        hipLaunchKernelGGL(split_bt_kernel<true>, dim3(g), dim3(256), 0, stream, K, N, B, ldb, Kp,
                           hi, lo);
    else
        hipLaunchKernelGGL(split_bt_kernel<false>, dim3(g), dim3(256), 0, stream, K, N, B, ldb,
                           Kp, hi, lo);
    return hipGetLastError();
}

hipError_t launch_split_bf16_plain(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                                   uint16_t* hi, uint16_t* lo, hipStream_t stream) {
    hipLaunchKernelGGL(split_plain_kernel, dim3(grid_for(rows * cols, 256)), dim3(256), 0, stream,
                       rows, cols, X, ldx, hi, lo);
    return hipGetLastError();
}

hipError_t launch_quant_fp8(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                            bool transpose, bool tiled, int64_t out_rows, int64_t out_cols,
                            uint8_t* q, uint8_t* qscale, uint8_t* rq, uint8_t* rscale,
                            hipStream_t stream) {
    if ((out_rows % 128) || (out_cols % 128)) return hipErrorInvalidValue;
    if (tiled && (out_rows % kPanelRows)) return hipErrorInvalidValue;
    if (transpose ? (out_rows < cols || out_cols < rows) : (out_rows < rows || out_cols < cols))
        return hipErrorInvalidValue;
    const bool vec = (ldx % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
    const unsigned g = (unsigned)((out_rows / 128) * (out_cols / 128));
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(g), dim3(256), 0, stream, rows, cols, X, ldx, out_cols, q,
                           qscale, rq, rscale);
    };
    const int sel = (vec ? 4 : 0) | (transpose ? 2 : 0) | (tiled ? 1 : 0);
    switch (sel) {
        case 0: go(quant_fp8_kernel<false, false, false>); break;
        case 1: go(quant_fp8_kernel<false, false, true>); break;
        case 2: go(quant_fp8_kernel<false, true, false>); break;
        case 3: go(quant_fp8_kernel<false, true, true>); break;
        case 4: go(quant_fp8_kernel<true, false, false>); break;
        case 5: go(quant_fp8_kernel<true, false, true>); break;
        case 6: go(quant_fp8_kernel<true, true, false>); break;
        default: go(quant_fp8_kernel<true, true, true>); break;
    }
    return hipGetLastError();
}

}  // namespace cmp
