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
// All kernels are HBM-bound (4 bytes read, 2 or 4 written per element).  The
// written B images are N x K: the bf16 split transposes B through LDS, the
// E4M3 quantisation in registers (each lane loads the K values of its own
// output rows).
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
// Workgroup bx of gx (256 lanes each, grid-stride over the chunks).  Rows at
// or past Mw are not written (Mw = Mp: the whole image, padding rows zero).
template <bool VEC>
__device__ __forceinline__ void split_a(int64_t bx, int64_t gx, int64_t M, int64_t K,
                                        const float* __restrict__ A, int64_t lda, int64_t Mp, int64_t Kp,
                                        uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int64_t Mw) {
    const int64_t nkb = Kp * 2 / kPanelRowBytes;
    const int64_t total = Mp * (Kp / 8);
    for (int64_t e = bx * 256 + threadIdx.x; e < total; e += gx * 256) {
        const int64_t blk = e >> 10;            // 1024 chunks per 16 KiB block
        const int w = (int)(e & 1023), rr = w >> 2, pos = w & 3;
        const int64_t rb = blk / nkb, kb = blk - rb * nkb;
        const int64_t r = rb * kPanelRows + rr;
        if (r >= Mw) continue;
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
// one 64 x 64 tile per workgroup (tile `tile`), transposed through T.
template <bool VEC>
__device__ __forceinline__ void split_bt(int64_t tile, int64_t K, int64_t N, const float* __restrict__ B,
                                         int64_t ldb, int64_t Kp, uint16_t* __restrict__ hi,
                                         uint16_t* __restrict__ lo, float (*T)[65]) {
    const int t = threadIdx.x;
    const int64_t tiles_k = Kp / 64;
    const int64_t k0 = (tile % tiles_k) * 64;
    const int64_t n0 = (tile / tiles_k) * 64;
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

// Both operands' bf16 images in one launch: ga grid-stride workgroups of
// split_a and gb tiles of split_bt, interleaved by paired_kind.
struct SplitPair {
    int64_t M, N, K, lda, ldb, Mp, Kp, ga, gb;
    const float* A;
    const float* B;
    uint16_t *ah, *al, *bh, *bl;
};
template <bool VA, bool VB>
__global__ __launch_bounds__(256) void split_pair_kernel(SplitPair p) {
    __shared__ float T[64][65];
    int64_t w;
    const int kind = paired_kind(blockIdx.x, p.ga, p.gb, &w);
    if (kind == 0) split_a<VA>(w, p.ga, p.M, p.K, p.A, p.lda, p.Mp, p.Kp, p.ah, p.al, p.Mp);
    else if (kind == 1) split_bt<VB>(w, p.K, p.N, p.B, p.ldb, p.Kp, p.bh, p.bl, T);
}

// The hi / lo images of every problem of a grouped bf16x3 plan in one launch:
// workgroup w belongs to the problem p with desc[p].pre_start <= w (problems
// in list order, each A's ga workgroups then B's gb), one split_a chunk pass
// or one split_bt tile per workgroup.  Only rows below M (A, whose idle
// 64-row quarters get no workgroup) and the 64-row tiles that start below N
// (B^T) are written: padding rows of an image feed
// only output rows and columns past the problem, which the GEMM never stores,
// while padding K inside the written rows is zero as the products need.
__global__ __launch_bounds__(256) void split_grouped_kernel(const GroupedMfmaDesc* __restrict__ desc,
                                                            int count) {
    __shared__ float T[64][65];
    typedef const __attribute__((address_space(1))) GroupedMfmaDesc* gdesc;
    const gdesc dg = (gdesc)desc;
    const int w = (int)blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (dg[mid].pre_start <= w) lo = mid;
        else hi = mid - 1;
    }
    const __attribute__((address_space(1))) GroupedMfmaDesc& d = dg[lo];
    const int local = w - d.pre_start;
    if (local < d.ga) {
        // split_a workgroup bx covers rows 64 (bx % 4) .. + 63 of block bx / 4 (block =
        // row panel x K block): the ga workgroups here are those whose rows start below M,
        // the full panels' (four quarters per block) and then the last panel's nq quarters
        const int64_t nkb = d.Kp * 2 / kPanelRowBytes;
        const int64_t full = d.M / kPanelRows, nq = ((d.M % kPanelRows) + 63) / 64;
        int64_t bx = local;
        if (bx >= full * nkb * 4) {
            const int64_t c = bx - full * nkb * 4;
            bx = (full * nkb + c / nq) * 4 + c % nq;
        }
        const int64_t gx = d.Mp * (d.Kp / 8) / 256;   // every chunk pass: one iteration each
        if (d.vec & 1) split_a<true>(bx, gx, d.M, d.K, d.A, d.lda, d.Mp, d.Kp, d.ah, d.al, d.M);
        else split_a<false>(bx, gx, d.M, d.K, d.A, d.lda, d.Mp, d.Kp, d.ah, d.al, d.M);
    } else if (local - d.ga < d.gb) {
        if (d.vec & 2) split_bt<true>(local - d.ga, d.K, d.N, d.B, d.ldb, d.Kp, d.bh, d.bl, T);
        else split_bt<false>(local - d.ga, d.K, d.N, d.B, d.ldb, d.Kp, d.bh, d.bl, T);
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
// Four floats -> four E4M3 bytes, byte j = value j (v_cvt_pk_fp8_f32, round
// to nearest even; the inputs are already within the finite range or NaN).
__device__ __forceinline__ uint32_t e4m3x4(float a, float b, float c, float d) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
    return (uint32_t)w;
}

// Workgroup maximum of a 32-bit key; `slot` holds 4 words of LDS used by this
// call site only, so consecutive calls need no barrier between them.
__device__ __forceinline__ uint32_t block_umax(uint32_t v, uint32_t* slot) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off));
    if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = v;
    __syncthreads();
    return max(max(slot[0], slot[1]), max(slot[2], slot[3]));
}
__device__ __forceinline__ uint32_t mag_bits(float x) { return __builtin_bit_cast(uint32_t, x) & 0x7fffffffu; }

// First level of one output row's 16 values: q codes (4 words) and the
// residuals x - q 2^-e (rounded once, by the fused multiply-add), which
// replace the values.  SPECIAL: the tile holds an infinity or NaN (then
// e = 0): out-of-range values saturate, non-finite ones encode as NaN and
// leave a zero residual.  Returns the row's largest residual magnitude bits.
template <bool SPECIAL>
__device__ __forceinline__ uint32_t level1(float (&v)[16], uint32_t (&qw)[4], int e, float inv) {
    uint32_t rmax = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        float s[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s[j] = ldexpf(v[4 * m + j], e);
            if (SPECIAL) s[j] = e4m3_sat(s[j]);
        }
        qw[m] = e4m3x4(s[0], s[1], s[2], s[3]);
        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)qw[m], false);
        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)qw[m], true);
        const float qv[4] = {lo[0], lo[1], hi[0], hi[1]};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float x = v[4 * m + j];
            float r = __builtin_fmaf(-qv[j], inv, x);
            if (SPECIAL && !__builtin_isfinite(x)) r = 0.f;
            v[4 * m + j] = r;
            rmax = max(rmax, mag_bits(r));
        }
    }
    return rmax;
}

// One 128 x 128 tile per workgroup of 256 lanes; each lane ends up holding 16
// consecutive K values of 4 output rows, so every image write is one 16-byte
// store per row and level, in the image's final order (no LDS staging):
//   TRANS false (X = A, rows x cols = M x K): lane t takes output rows
//     t/8 + 32 i (i = 0..3), K values 16 (t % 8) .. +15 of each (four float4
//     loads per row);
//   TRANS true (X = B, rows x cols = K x N; output row = column of X): lane t
//     takes X rows 16 (t % 8) .. +15 (its K values) of X columns 4 (t / 8)
//     .. +3 (one float4 load per X row); eight consecutive lanes cover the
//     128 K values of one output row.
// The tile exponents come from integer maxima of the magnitudes' bit patterns:
// non-negative floats order like their bits, and infinities and NaN sit above
// every finite value, so the same maximum tells a non-finite tile (then
// scale_exp gives e = 0, as for a NaN or infinite amax).  In a finite tile
// |x 2^e| <= 448, so the encoder needs no saturation; x 2^e is exact whenever
// its code is non-zero, and the residual x - q 2^-e is one FMA rounded once
// (for a zero code it is x itself, and -0 - (-0) gives +0 as the definition
// does).  The code images are row-major out_rows x out_cols (TILED false) or
// panel images with out_cols bytes of K per row (TILED true).
template <bool VEC, bool TRANS, bool TILED>
__device__ __forceinline__ void quant_tile(int64_t tile, int64_t rows, int64_t cols,
                                           const float* __restrict__ X, int64_t ldx, int64_t out_cols,
                                           uint8_t* __restrict__ q, uint8_t* __restrict__ qscale,
                                           uint8_t* __restrict__ rq, uint8_t* __restrict__ rscale,
                                           uint32_t* red) {
    const int t = threadIdx.x;
    const int64_t ot_cols = out_cols / 128;
    const int64_t nkb = out_cols / kPanelRowBytes;
    const int64_t ot_r = tile / ot_cols, ot_c = tile % ot_cols;
    // tile origin in X coordinates
    const int64_t x_r0 = TRANS ? ot_c * 128 : ot_r * 128;
    const int64_t x_c0 = TRANS ? ot_r * 128 : ot_c * 128;
    const int g = t & 7, h = t >> 3;

    float v[4][16];                // [output row][K value]
    // whole tile inside X with 16-byte aligned rows: unguarded float4 loads
    const bool interior = VEC && x_r0 + 128 <= rows && x_c0 + 128 <= cols;
    auto load4 = [&](const float* __restrict__ X, int64_t r, int64_t c, bool guard) -> float4 {
        if (!guard) return *reinterpret_cast<const float4*>(X + r * ldx + c);
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
        return a;
    };
    auto load_tile = [&](const float* __restrict__ X, bool guard) {
        if (!TRANS) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float4 a = load4(X, x_r0 + h + 32 * i, x_c0 + 16 * g + 4 * u, guard);
                    v[i][4 * u + 0] = a.x; v[i][4 * u + 1] = a.y;
                    v[i][4 * u + 2] = a.z; v[i][4 * u + 3] = a.w;
                }
        } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const float4 a = load4(X, x_r0 + 16 * g + j, x_c0 + 4 * h, guard);
                v[0][j] = a.x; v[1][j] = a.y; v[2][j] = a.z; v[3][j] = a.w;
            }
        }
    };
    if (interior) load_tile(X, false);
    else load_tile(X, true);
    uint32_t amax = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 16; ++j) amax = max(amax, mag_bits(v[i][j]));
    amax = block_umax(amax, red);
    const int e = scale_exp(__builtin_bit_cast(float, amax));
    const float inv = ldexpf(1.f, -e);          // 2^-e, exact for e in [-127, 127]

    uint32_t qw[4][4], ramax = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) ramax = max(ramax, level1<false>(v[i], qw[i], e, inv));
    if (amax >= 0x7f800000u) {                  // uniform: a tile with an infinity or NaN (rare)
        // start again from x with the element-wise rules; the opaque copy of
        // the base pointer keeps the compiler from holding the first pass's
        // addresses live over the whole tile for this rare reload
        const float* X2 = X;
        asm volatile("" : "+s"(X2));
        load_tile(X2, true);
        ramax = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) ramax = max(ramax, level1<true>(v[i], qw[i], e, inv));
    }
    ramax = block_umax(ramax, red + 4);
    const int er = scale_exp(__builtin_bit_cast(float, ramax));
    uint32_t rw[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int m = 0; m < 4; ++m)
            rw[i][m] = e4m3x4(ldexpf(v[i][4 * m + 0], er), ldexpf(v[i][4 * m + 1], er),
                              ldexpf(v[i][4 * m + 2], er), ldexpf(v[i][4 * m + 3], er));

    if (t == 0) {
        qscale[tile] = (uint8_t)(127 - e);
        rscale[tile] = (uint8_t)(127 - er);
    }
    const int64_t ocol = ot_c * 128 + 16 * g;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t orow = ot_r * 128 + (TRANS ? 4 * h + i : h + 32 * i);
        const int64_t o = TILED ? panel_offset(orow, ocol, nkb) : orow * out_cols + ocol;
        *reinterpret_cast<uint4*>(q + o) = make_uint4(qw[i][0], qw[i][1], qw[i][2], qw[i][3]);
        *reinterpret_cast<uint4*>(rq + o) = make_uint4(rw[i][0], rw[i][1], rw[i][2], rw[i][3]);
    }
}

template <bool VEC, bool TRANS, bool TILED>
__global__ __launch_bounds__(256) void quant_fp8_kernel(
    int64_t rows, int64_t cols, const float* __restrict__ X, int64_t ldx, int64_t out_cols,
    uint8_t* __restrict__ q, uint8_t* __restrict__ qscale, uint8_t* __restrict__ rq,
    uint8_t* __restrict__ rscale) {
    __shared__ uint32_t red[8];    // the two reductions
    quant_tile<VEC, TRANS, TILED>(blockIdx.x, rows, cols, X, ldx, out_cols, q, qscale, rq, rscale, red);
}

// The images of both operands of a GEMM in one launch: A (M x K, a.tiles
// tiles) and B (K x N, transposed into its N x K image, b.tiles tiles), the
// tiles of the two interleaved by paired_kind, so the two halves stream from
// HBM side by side and one launch replaces two kernels on two streams with
// their event fork and join.
struct QuantOperand {
    int64_t rows, cols, ldx, out_cols, tiles;
    const float* X;
    uint8_t *q, *qscale, *rq, *rscale;
};
template <bool VA, bool VB>
__global__ __launch_bounds__(256) void quant_fp8_pair_kernel(QuantOperand a, QuantOperand b) {
    __shared__ uint32_t red[8];
    int64_t tile;
    const int kind = paired_kind(blockIdx.x, a.tiles, b.tiles, &tile);
    if (kind < 0) return;
    if (kind == 1)
        quant_tile<VB, true, true>(tile, b.rows, b.cols, b.X, b.ldx, b.out_cols, b.q, b.qscale, b.rq,
                                   b.rscale, red);
    else
        quant_tile<VA, false, true>(tile, a.rows, a.cols, a.X, a.ldx, a.out_cols, a.q, a.qscale, a.rq,
                                    a.rscale, red);
}

unsigned grid_for(int64_t work, int64_t per_block) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_quant_fp8_pair(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                                const float* B, int64_t ldb, int64_t Mp, int64_t Np, int64_t Kp,
                                uint8_t* aq, uint8_t* aqs, uint8_t* ar, uint8_t* ars, uint8_t* bq,
                                uint8_t* bqs, uint8_t* br, uint8_t* brs, hipStream_t stream) {
    if (M <= 0 || N <= 0 || K <= 0 || Kp % 128 || Mp % kPanelRows || Np % kPanelRows || Mp < M ||
        Np < N || Kp < K)
        return hipErrorInvalidValue;
    const QuantOperand a{M, K, lda, Kp, (Mp / 128) * (Kp / 128), A, aq, aqs, ar, ars};
    const QuantOperand b{K, N, ldb, Kp, (Np / 128) * (Kp / 128), B, bq, bqs, br, brs};
    const bool va = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
    const bool vb = (ldb % 4 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
    const dim3 g((unsigned)paired_blocks(a.tiles, b.tiles));
    auto go = [&](auto kernel) { hipLaunchKernelGGL(kernel, g, dim3(256), 0, stream, a, b); };
    if (va && vb) go(quant_fp8_pair_kernel<true, true>);
    else if (va) go(quant_fp8_pair_kernel<true, false>);
    else if (vb) go(quant_fp8_pair_kernel<false, true>);
    else go(quant_fp8_pair_kernel<false, false>);
    return hipGetLastError();
}

hipError_t launch_split_grouped(const GroupedMfmaDesc* desc, int count, int64_t pre_total,
                                hipStream_t stream) {
    if (pre_total <= 0) return hipSuccess;
    if (!desc || count < 1 || pre_total >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(split_grouped_kernel, dim3((unsigned)pre_total), dim3(256), 0, stream, desc, count);
    return hipGetLastError();
}

hipError_t launch_split_bf16_pair(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                                 const float* B, int64_t ldb, int64_t Mp, int64_t Np, int64_t Kp,
                                 uint16_t* ah, uint16_t* al, uint16_t* bh, uint16_t* bl,
                                 hipStream_t stream) {
    if (M <= 0 || N <= 0 || K <= 0 || !ah || !bh || (!al) != (!bl) || Mp % kPanelRows ||
        Np % kPanelRows || Mp < M || Np < N || Kp % 64 || Kp < K)
        return hipErrorInvalidValue;
    const SplitPair p{M, N, K, lda, ldb, Mp, Kp, grid_for(Mp * (Kp / 8), 256), (Np / 64) * (Kp / 64),
                      A, B, ah, al, bh, bl};
    const int64_t blocks = paired_blocks(p.ga, p.gb);
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const bool va = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
    const bool vb = (ldb % 4 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
    auto go = [&](auto kernel) { hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p); };
    if (va && vb) go(split_pair_kernel<true, true>);
    else if (va) go(split_pair_kernel<true, false>);
    else if (vb) go(split_pair_kernel<false, true>);
    else go(split_pair_kernel<false, false>);
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
