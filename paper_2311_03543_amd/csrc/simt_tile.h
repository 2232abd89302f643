// FP32 SIMT GEMM tile, shared by the single-problem kernel and the grouped
// (batched) kernel: one workgroup of 256 lanes computes a BM x BN tile of
// C = alpha * A * B + beta * C, walking K in steps of BK.
//
// Each step's A tile (BM x BK) and B tile (BK x BN) come from global memory
// with 16-byte loads where alignment allows and are staged in LDS (A stored
// k-major so a lane's TM row values are two TM/2-wide LDS reads), double
// buffered: the next step's global loads are in flight in registers while the
// current step computes.  Lane (tx, ty) owns rows ty*TM/2 + [0, TM/2) and
// BM/2 + ty*TM/2 + [0, TM/2), and the TN columns g*BN*4/TN + tx*4 + [0, 4)
// for g < TN/4: the lanes of a wave that share ty read one broadcast address
// of A, and each 16-byte B read of the 16 lanes that share ty covers 256
// contiguous bytes, so LDS reads are conflict-free.
//
// Every output entry is one lane's chain of FP32 FMAs over k in increasing
// order, whatever the tile shape, so all configurations give bit-identical C.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cmp {

struct SimtProblem {
    int64_t M, N, K, lda, ldb, ldc;
    float alpha, beta;
    const float* A;
    const float* B;
    float* C;
};

// Global-address-space views of the operand pointers: pointers that arrive
// through memory (the grouped descriptors) are generic to the compiler and
// would otherwise turn every access into a FLAT instruction.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) float* gcfloat;
typedef __attribute__((address_space(1))) float* gfloat;
typedef const __attribute__((address_space(1))) f32x4* gcf32x4;
typedef __attribute__((address_space(1))) f32x4* gf32x4;

template <int BM_, int BN_, int BK_, int TM_, int TN_>
struct SimtCfg {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, TM = TM_, TN = TN_;
    static constexpr int THREADS = 256;
    static constexpr int TX = BN / TN, TY = BM / TM;     // lane grid
    static_assert(TX * TY == THREADS, "256 lanes per tile");
    static constexpr int APITCH = BM + 4;                // k-major A rows, 16-byte aligned
    static constexpr int LA = BM * BK / 4 / THREADS;     // float4 loads of A per lane per step
    static constexpr int LB = BK * BN / 4 / THREADS;     // float4 loads of B per lane per step
    static_assert(LA >= 1 && LB >= 1, "tile too small for 256 lanes");
    static constexpr int SMEM_FLOATS = 2 * BK * APITCH + 2 * BK * BN;
};

template <typename Cfg, bool VEC>
__device__ __forceinline__ void simt_load(const SimtProblem& p, int64_t m0, int64_t n0,
                                          int64_t k0, int t, f32x4 (&ra)[Cfg::LA],
                                          f32x4 (&rb)[Cfg::LB]) {
    constexpr int AQ = Cfg::BK / 4;   // float4 per A row
#pragma unroll
    for (int h = 0; h < Cfg::LA; ++h) {
        const int f = t + h * Cfg::THREADS;
        const int64_t row = m0 + f / AQ;
        const int64_t k = k0 + (f % AQ) * 4;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (row < p.M) {
            gcfloat src = (gcfloat)p.A + row * p.lda + k;
            if (VEC && k + 3 < p.K) {
                v = *(gcf32x4)src;
            } else {
                if (k + 0 < p.K) v.x = src[0];
                if (k + 1 < p.K) v.y = src[1];
                if (k + 2 < p.K) v.z = src[2];
                if (k + 3 < p.K) v.w = src[3];
            }
        }
        ra[h] = v;
    }
    constexpr int BQ = Cfg::BN / 4;   // float4 per B row
#pragma unroll
    for (int h = 0; h < Cfg::LB; ++h) {
        const int f = t + h * Cfg::THREADS;
        const int64_t k = k0 + f / BQ;
        const int64_t col = n0 + (f % BQ) * 4;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (k < p.K) {
            gcfloat src = (gcfloat)p.B + k * p.ldb + col;
            if (VEC && col + 3 < p.N) {
                v = *(gcf32x4)src;
            } else {
                if (col + 0 < p.N) v.x = src[0];
                if (col + 1 < p.N) v.y = src[1];
                if (col + 2 < p.N) v.z = src[2];
                if (col + 3 < p.N) v.w = src[3];
            }
        }
        rb[h] = v;
    }
}

template <typename Cfg>
__device__ __forceinline__ void simt_store(float* As, float* Bs, int t,
                                           const f32x4 (&ra)[Cfg::LA],
                                           const f32x4 (&rb)[Cfg::LB]) {
    constexpr int AQ = Cfg::BK / 4;
#pragma unroll
    for (int h = 0; h < Cfg::LA; ++h) {
        const int f = t + h * Cfg::THREADS;
        const int r = f / AQ, kq = (f % AQ) * 4;
        As[(kq + 0) * Cfg::APITCH + r] = ra[h].x;
        As[(kq + 1) * Cfg::APITCH + r] = ra[h].y;
        As[(kq + 2) * Cfg::APITCH + r] = ra[h].z;
        As[(kq + 3) * Cfg::APITCH + r] = ra[h].w;
    }
    constexpr int BQ = Cfg::BN / 4;
#pragma unroll
    for (int h = 0; h < Cfg::LB; ++h) {
        const int f = t + h * Cfg::THREADS;
        *reinterpret_cast<f32x4*>(&Bs[(f / BQ) * Cfg::BN + (f % BQ) * 4]) = rb[h];
    }
}

// Reads `n` consecutive floats (n = 2, 4 or 8) from LDS into dst.
template <int n>
__device__ __forceinline__ void lds_vec(const float* src, float* dst) {
    if constexpr (n == 8) {
        const float4 v = *reinterpret_cast<const float4*>(src);
        const float4 w = *reinterpret_cast<const float4*>(src + 4);
        dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
        dst[4] = w.x; dst[5] = w.y; dst[6] = w.z; dst[7] = w.w;
    } else if constexpr (n == 4) {
        const float4 v = *reinterpret_cast<const float4*>(src);
        dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
    } else if constexpr (n == 2) {
        const float2 v = *reinterpret_cast<const float2*>(src);
        dst[0] = v.x; dst[1] = v.y;
    } else {
#pragma unroll
        for (int i = 0; i < n; ++i) dst[i] = src[i];
    }
}

// The whole tile at (m0, n0): main loop and epilogue.  `smem` holds
// Cfg::SMEM_FLOATS floats.  alpha == 0 or K == 0 never reads A or B.
template <typename Cfg, bool VEC>
__device__ __forceinline__ void simt_tile(const SimtProblem& p, int64_t m0, int64_t n0,
                                          float* smem) {
    constexpr int BK = Cfg::BK, TM = Cfg::TM, TN = Cfg::TN;
    constexpr int HM = TM / 2;
    // A lane's TN columns are NG groups of 4, GS columns apart: one 16-byte
    // LDS read per group, and the 16 lanes of a wave that share ty read 256
    // contiguous bytes (all 64 banks once).
    constexpr int NG = TN / 4, GS = Cfg::BN / NG;
    static_assert(TN % 4 == 0 && GS == 4 * Cfg::TX, "column groups of four");
    // buffer b of A at smem + b * ASZ, of B at smem + 2 * ASZ + b * BSZ (plain
    // offsets keep the pointers in the LDS address space: ds_read, not flat)
    constexpr int ASZ = BK * Cfg::APITCH, BSZ = BK * Cfg::BN;
    const int t = threadIdx.x;
    const int tx = t % Cfg::TX, ty = t / Cfg::TX;

    float acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = 0.f;

    const int nk = (p.alpha == 0.f) ? 0 : (int)((p.K + BK - 1) / BK);
    f32x4 ra[Cfg::LA], rb[Cfg::LB];
    if (nk > 0) {
        simt_load<Cfg, VEC>(p, m0, n0, 0, t, ra, rb);
        simt_store<Cfg>(smem, smem + 2 * ASZ, t, ra, rb);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) simt_load<Cfg, VEC>(p, m0, n0, (int64_t)(kt + 1) * BK, t, ra, rb);
        const float* a_s = smem + cur * ASZ;
        const float* b_s = smem + 2 * ASZ + cur * BSZ;
#pragma unroll 2
        for (int k = 0; k < BK; ++k) {
            float av[TM], bv[TN];
            lds_vec<HM>(a_s + k * Cfg::APITCH + ty * HM, av);
            lds_vec<HM>(a_s + k * Cfg::APITCH + Cfg::BM / 2 + ty * HM, av + HM);
#pragma unroll
            for (int g = 0; g < NG; ++g) lds_vec<4>(b_s + k * Cfg::BN + g * GS + tx * 4, bv + 4 * g);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_fmaf(av[i], bv[j], acc[i][j]);
        }
        if (more) simt_store<Cfg>(smem + (cur ^ 1) * ASZ, smem + 2 * ASZ + (cur ^ 1) * BSZ, t, ra, rb);
        __syncthreads();
    }

    // Epilogue: C = alpha * acc + beta * C (C not read when beta == 0).
    const bool cvec = ((p.ldc & 3) == 0) && ((reinterpret_cast<uintptr_t>(p.C) & 15) == 0);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int64_t row = m0 + (i < HM ? ty * HM + i : Cfg::BM / 2 + ty * HM + (i - HM));
        if (row >= p.M) continue;
        gfloat crow = (gfloat)p.C + row * p.ldc;
#pragma unroll
        for (int h = 0; h < NG; ++h) {
            const int64_t col = n0 + h * GS + tx * 4;
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = p.alpha * acc[i][4 * h + j];
            if (cvec && col + 3 < p.N) {
                gf32x4 q = (gf32x4)(crow + col);
                if (p.beta != 0.f) {
                    const f32x4 o = *q;
                    v[0] = __builtin_fmaf(p.beta, o.x, v[0]);
                    v[1] = __builtin_fmaf(p.beta, o.y, v[1]);
                    v[2] = __builtin_fmaf(p.beta, o.z, v[2]);
                    v[3] = __builtin_fmaf(p.beta, o.w, v[3]);
                }
                *q = f32x4{v[0], v[1], v[2], v[3]};
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (col + j < p.N) {
                        float o = v[j];
                        if (p.beta != 0.f) o = __builtin_fmaf(p.beta, crow[col + j], o);
                        crow[col + j] = o;
                    }
                }
            }
        }
    }
}

}  // namespace cmp
