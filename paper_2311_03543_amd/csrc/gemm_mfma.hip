// MFMA GEMM kernels for gfx950 over the pre-pass images (both operands
// K-contiguous: A image Mp x Kp, B image Np x Kp = B transposed).
//
//   bf16 / bf16x3:  C = alpha * sum_t A_t B_t^T + beta * C with one (bf16) or
//                   three (hi.hi + hi.lo + lo.hi, the split-precision product)
//                   operand pairs, v_mfma_f32_32x32x16_bf16, FP32 accumulation.
//   fp8 refined:    C = alpha * (Aq.Bq + Ar.Bq + Aq.Br + Ar.Br) + beta * C over
//                   E4M3 images with one E8M0 scale byte per 128 x 128 tile,
//                   v_mfma_scale_f32_32x32x64_f8f6f4, FP32 accumulation.
//
// The extra products are K-concatenated: the main loop walks nterms * Kp / BK
// steps and each step picks its operand pair, so one accumulator set and one
// pipeline serve every term.
//
// Tiling: 256 x 256 C tile per workgroup of 4 wave64 (2 x 2 waves, 128 x 128
// per wave = 4 x 4 MFMA blocks of 32 x 32, 256 FP32 accumulators per lane).
// Each K step stages a 256-row A slab and a 256-row B slab (128 bytes of K per
// row) in LDS with direct global->LDS loads (global_load_lds_dwordx4), so the
// next step's tiles stream into the other buffer while the current step's
// MFMAs run without occupying any registers.  Inside a slab row, 16-byte chunks
// are XOR-swizzled by row (see swz) so fragment reads are bank-conflict free.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace cmp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx4 __attribute__((ext_vector_type(4)));

constexpr int TM = 256, TN = 256;
constexpr int ROWB = 128;           // bytes of K per row per step
constexpr int THREADS = 256;
constexpr int SLAB = TM * ROWB;     // bytes per operand slab (32 KiB)

typedef const __attribute__((address_space(1))) void* gptr_t;
typedef __attribute__((address_space(3))) void* lptr_t;

// LDS slab layout: row r holds 128 bytes = 8 chunks of 16 bytes, and chunk c
// of row r sits at position c ^ f(r), f(r) = (r / 2) % 8.  gfx950's LDS serves
// a 16-byte-per-lane read 16 lanes per cycle over 64 banks (256 bytes); rows
// alternate between the two 128-byte bank halves, so the 16 rows one lane
// group of a fragment read touches ((r % 2), c ^ f(r)) are all distinct: no
// bank conflicts.  (With f(r) = r % 8, rows r and r + 8 collide: 2-way.)
__device__ __forceinline__ int swz_f(int r) { return (r >> 1) & 7; }

// Byte address of 16-byte chunk c of slab row r.
__device__ __forceinline__ int swz(int r, int c) { return r * ROWB + ((c ^ swz_f(r)) << 4); }

// Stage rows [row0, row0 + 256) x bytes [kbyte, kbyte + 128) of an image with
// row pitch ld_bytes into `slab`.  One wave instruction fills 1 KiB = 8 rows;
// wave w issues instructions q = 8 w .. 8 w + 7.  Lane l of instruction q
// lands at slab + 1024 q + 16 l, i.e. row 8 q + l / 8, position l % 8, which
// must hold global chunk (l % 8) ^ f(8 q + l / 8) = (l % 8) ^ ((4 q + l / 16) % 8).
__device__ __forceinline__ void stage(const uint8_t* __restrict__ img, int64_t ld_bytes,
                                      int64_t row0, int64_t kbyte, uint8_t* slab, int wave,
                                      int lane) {
    const int c_even = (lane & 7) ^ ((lane >> 4) & 7);          // q even: 4 q % 8 = 0
    const int c_odd = (lane & 7) ^ ((4 + (lane >> 4)) & 7);     // q odd:  4 q % 8 = 4
    const uint8_t* src = img + (row0 + wave * 64 + (lane >> 3)) * ld_bytes + kbyte;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int q = wave * 8 + i;
        const int chunk = (i & 1) ? c_odd : c_even;              // q has the parity of i
        __builtin_amdgcn_global_load_lds((gptr_t)(src + (int64_t)i * 8 * ld_bytes + chunk * 16),
                                         (lptr_t)(slab + q * 1024), 16, 0, 0);
    }
}

// Wait for this wave's outstanding global->LDS loads (vmcnt = 0).
__device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Wait for this wave's outstanding LDS reads (lgkmcnt = 0).
__device__ __forceinline__ void wait_lds_reads() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Scheduling pattern for one sub-step of 16 MFMAs: the `reads` LDS fragment
// reads of the next sub-step are interleaved one-for-one with the first MFMAs,
// so their latency hides behind the matrix pipe instead of stalling it.
template <int READS, int MFMAS = 16>
__device__ __forceinline__ void mfma_schedule() {
    constexpr int kMfma = 0x008, kDsRead = 0x100;
#pragma unroll
    for (int r = 0; r < READS; ++r) {
        __builtin_amdgcn_sched_group_barrier(kMfma, 1, 0);
        __builtin_amdgcn_sched_group_barrier(kDsRead, 1, 0);
    }
    if constexpr (MFMAS > READS) __builtin_amdgcn_sched_group_barrier(kMfma, MFMAS - READS, 0);
}

// Pattern for the first sub-step of a stage: the next stage's 16 direct
// global->LDS loads (two per MFMA) and the 8 LDS fragment reads of the next
// sub-step ride under the first 8 MFMAs.
__device__ __forceinline__ void mfma_schedule_with_stage() {
    constexpr int kMfma = 0x008, kVmemRead = 0x020, kDsRead = 0x100;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        __builtin_amdgcn_sched_group_barrier(kMfma, 1, 0);
        __builtin_amdgcn_sched_group_barrier(kVmemRead, 2, 0);
        __builtin_amdgcn_sched_group_barrier(kDsRead, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(kMfma, 8, 0);
}

// 32 x 32 accumulator block layout: lane l holds column l % 32 and rows
// 8 (r / 4) + 4 (l / 32) + (r % 4), r = 0..15.
__device__ __forceinline__ void epilogue(const floatx16 (&acc)[4][4], int64_t M, int64_t N,
                                         int64_t m0, int64_t n0, int wm, int wn, int lane,
                                         float alpha, float beta, float* __restrict__ C,
                                         int64_t ldc) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t col = n0 + wn * 128 + j * 32 + (lane & 31);
            if (col >= N) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = m0 + wm * 128 + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                if (row < M) {
                    float* p = C + row * ldc + col;
                    float v = alpha * acc[i][j][r];
                    if (beta != 0.f) v = __builtin_fmaf(beta, *p, v);
                    *p = v;
                }
            }
        }
}

__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int& tm, int& tn) {
    grouped_tile(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
}

// ---------------------------------------------------------------------------
template <int NTERMS>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_bf16_tn_kernel(int64_t M, int64_t N, int64_t Kp, float alpha,
                         const uint16_t* __restrict__ Ah, const uint16_t* __restrict__ Al,
                         const uint16_t* __restrict__ Bh, const uint16_t* __restrict__ Bl,
                         float beta, float* __restrict__ C, int64_t ldc, int tiles_m,
                         int tiles_n) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    // LDS: [A slab 0 | A slab 1 | B slab 0 | B slab 1]

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform (SGPR)
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TN;
    const int64_t ldb = Kp * 2;                 // row pitch of both images in bytes
    const int nk = (int)(Kp / 64);              // 64 bf16 = 128 bytes per step
    const int steps = NTERMS * nk;

    floatx16 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    auto a_img = [&](int s) -> const uint8_t* {
        return reinterpret_cast<const uint8_t*>((s / nk) == 2 ? Al : Ah);
    };
    auto b_img = [&](int s) -> const uint8_t* {
        return reinterpret_cast<const uint8_t*>((s / nk) == 1 ? Bl : Bh);
    };

    stage(a_img(0), ldb, m0, 0, smem, wave, lane);
    stage(b_img(0), ldb, n0, 0, smem + 2 * SLAB, wave, lane);
    wait_loads();
    __syncthreads();

    const int frag_row = lane & 31;
    const int frag_c = lane >> 5;               // chunk (8 bf16) within a 16-k sub-step
    auto load_frags = [&](const uint8_t* sa, const uint8_t* sb, int ks, bf16x8 (&a)[4],
                          bf16x8 (&b)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a[i] = *reinterpret_cast<const bf16x8*>(sa + swz(wm * 128 + i * 32 + frag_row, 2 * ks + frag_c));
#pragma unroll
        for (int j = 0; j < 4; ++j)
            b[j] = *reinterpret_cast<const bf16x8*>(sb + swz(wn * 128 + j * 32 + frag_row, 2 * ks + frag_c));
    };
    auto mfma16 = [&](const bf16x8 (&a)[4], const bf16x8 (&b)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    };

    // Fragments are double-buffered in registers (sub-step ks + 1 is read
    // while sub-step ks multiplies).  One stage = 4 sub-steps of 16 MFMAs:
    //   ks 0: next stage's global->LDS loads + reads of ks 1 under the MFMAs
    //   ks 1, 2: reads of ks 2, 3
    //   ks 3: wait for the next stage (own loads landed, own reads of this
    //         stage done, workgroup barrier), then its ks-0 reads under the
    //         last 16 MFMAs of this stage.
    // A buffer is overwritten only by the stage after the barrier that
    // follows every wave's last read of it.
    bf16x8 fa[2][4], fb[2][4];
    load_frags(smem, smem + 2 * SLAB, 0, fa[0], fb[0]);
    __builtin_amdgcn_sched_barrier(0);
    auto one_stage = [&](int s, auto more_tag) {
        constexpr bool MORE = decltype(more_tag)::value;
        const int cur = s & 1;
        const uint8_t* sa = smem + cur * SLAB;
        const uint8_t* sb = smem + (2 + cur) * SLAB;
        // ks 0
        if constexpr (MORE) {
            const int64_t kb = (int64_t)((s + 1) % nk) * ROWB;
            stage(a_img(s + 1), ldb, m0, kb, smem + (cur ^ 1) * SLAB, wave, lane);
            stage(b_img(s + 1), ldb, n0, kb, smem + (2 + (cur ^ 1)) * SLAB, wave, lane);
        }
        load_frags(sa, sb, 1, fa[1], fb[1]);
        mfma16(fa[0], fb[0]);
        if constexpr (MORE) mfma_schedule_with_stage();
        else mfma_schedule<8>();
        __builtin_amdgcn_sched_barrier(0);
        // ks 1
        load_frags(sa, sb, 2, fa[0], fb[0]);
        mfma16(fa[1], fb[1]);
        mfma_schedule<8>();
        __builtin_amdgcn_sched_barrier(0);
        // ks 2
        load_frags(sa, sb, 3, fa[1], fb[1]);
        mfma16(fa[0], fb[0]);
        mfma_schedule<8>();
        __builtin_amdgcn_sched_barrier(0);
        // ks 3
        if constexpr (MORE) {
            wait_lds_reads();
            wait_loads();
            __syncthreads();
            load_frags(smem + (cur ^ 1) * SLAB, smem + (2 + (cur ^ 1)) * SLAB, 0, fa[0], fb[0]);
        }
        mfma16(fa[1], fb[1]);
        if constexpr (MORE) mfma_schedule<8>();
        else mfma_schedule<0>();
        __builtin_amdgcn_sched_barrier(0);
    };
    for (int s = 0; s + 1 < steps; ++s) one_stage(s, std::true_type{});
    one_stage(steps - 1, std::false_type{});
    epilogue(acc, M, N, m0, n0, wm, wn, lane, alpha, beta, C, ldc);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_fp8r_tn_kernel(int64_t M, int64_t N, int64_t Kp, float alpha,
                         const uint8_t* __restrict__ Aq, const uint8_t* __restrict__ Ar,
                         const uint8_t* __restrict__ Asq, const uint8_t* __restrict__ Asr,
                         const uint8_t* __restrict__ Bq, const uint8_t* __restrict__ Br,
                         const uint8_t* __restrict__ Bsq, const uint8_t* __restrict__ Bsr,
                         float beta, float* __restrict__ C, int64_t ldc, int tiles_m,
                         int tiles_n) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    // LDS: [A slab 0 | A slab 1 | B slab 0 | B slab 1]

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform (SGPR)
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TN;
    const int nk = (int)(Kp / 128);             // 128 E4M3 bytes per step
    const int steps = 4 * nk;
    // this wave's 128 rows of A (and columns of C) lie in one 128-row scale tile
    const int64_t a_tile = m0 / 128 + wm, b_tile = n0 / 128 + wn;

    floatx16 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // term s / nk: 0 = q.q, 1 = r.q, 2 = q.r, 3 = r.r
    auto a_img = [&](int s) { return ((s / nk) & 1) ? Ar : Aq; };
    auto b_img = [&](int s) { return ((s / nk) & 2) ? Br : Bq; };

    // E8M0 scale bytes of step s for this wave's A rows and B columns; read
    // one step ahead (through the scalar cache: every index is wave-uniform)
    // (a byte is fetched as its aligned 32-bit word so the load is scalar)
    auto byte_at = [](const uint8_t* p, int64_t idx) -> int {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(p + (idx & ~(int64_t)3));
        return (int)((w >> ((idx & 3) * 8)) & 0xffu);
    };
    auto scale_a = [&](int s) -> int {
        const int kt = s % nk;
        return byte_at(((s / nk) & 1) ? Asr : Asq, a_tile * nk + kt);
    };
    auto scale_b = [&](int s) -> int {
        const int kt = s % nk;
        return byte_at(((s / nk) & 2) ? Bsr : Bsq, b_tile * nk + kt);
    };
    stage(a_img(0), Kp, m0, 0, smem, wave, lane);
    stage(b_img(0), Kp, n0, 0, smem + 2 * SLAB, wave, lane);
    wait_loads();
    __syncthreads();

    const int frag_row = lane & 31;
    const int frag_c = (lane >> 5) * 2;         // this lane's 2 chunks (32 bytes) of a 64-k sub-step
    auto load_frags = [&](const uint8_t* sa, const uint8_t* sb, int ks, intx8 (&a)[4],
                          intx8 (&b)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = wm * 128 + i * 32 + frag_row;
            const intx4 lo = *reinterpret_cast<const intx4*>(sa + swz(r, 4 * ks + frag_c));
            const intx4 hi = *reinterpret_cast<const intx4*>(sa + swz(r, 4 * ks + frag_c + 1));
            a[i] = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = wn * 128 + j * 32 + frag_row;
            const intx4 lo = *reinterpret_cast<const intx4*>(sb + swz(r, 4 * ks + frag_c));
            const intx4 hi = *reinterpret_cast<const intx4*>(sb + swz(r, 4 * ks + frag_c + 1));
            b[j] = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        }
    };
    auto mfma16 = [&](const intx8 (&a)[4], const intx8 (&b)[4], int sca, int scb) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[i], b[j], acc[i][j], 0, 0,
                                                                            0, sca, 0, scb);
    };

    // Same stage pipeline as the bf16 kernel with two 64-k sub-steps per
    // stage: ks 0 carries the next stage's loads and the ks-1 reads; ks 1
    // waits for the next stage and reads its ks-0 fragments under the MFMAs.
    intx8 fa[2][4], fb[2][4];
    load_frags(smem, smem + 2 * SLAB, 0, fa[0], fb[0]);
    int sca_next = scale_a(0), scb_next = scale_b(0);
    __builtin_amdgcn_sched_barrier(0);
    auto one_stage = [&](int s, auto more_tag) {
        constexpr bool MORE = decltype(more_tag)::value;
        const int cur = s & 1;
        const uint8_t* sa = smem + cur * SLAB;
        const uint8_t* sb = smem + (2 + cur) * SLAB;
        const int sca = sca_next, scb = scb_next;
        // ks 0
        if constexpr (MORE) {
            sca_next = scale_a(s + 1);
            scb_next = scale_b(s + 1);
            const int64_t kb = (int64_t)((s + 1) % nk) * ROWB;
            stage(a_img(s + 1), Kp, m0, kb, smem + (cur ^ 1) * SLAB, wave, lane);
            stage(b_img(s + 1), Kp, n0, kb, smem + (2 + (cur ^ 1)) * SLAB, wave, lane);
        }
        load_frags(sa, sb, 1, fa[1], fb[1]);
        mfma16(fa[0], fb[0], sca, scb);
        mfma_schedule<16>();
        __builtin_amdgcn_sched_barrier(0);
        // ks 1
        if constexpr (MORE) {
            wait_lds_reads();
            wait_loads();
            __syncthreads();
            load_frags(smem + (cur ^ 1) * SLAB, smem + (2 + (cur ^ 1)) * SLAB, 0, fa[0], fb[0]);
        }
        mfma16(fa[1], fb[1], sca, scb);
        if constexpr (MORE) mfma_schedule<16>();
        else mfma_schedule<0>();
        __builtin_amdgcn_sched_barrier(0);
    };
    for (int s = 0; s + 1 < steps; ++s) one_stage(s, std::true_type{});
    one_stage(steps - 1, std::false_type{});
    epilogue(acc, M, N, m0, n0, wm, wn, lane, alpha, beta, C, ldc);
}

constexpr size_t kSmem = 4 * (size_t)SLAB;   // 131072 bytes

template <int NTERMS>
hipError_t launch_bf16_terms(int64_t M, int64_t N, int64_t Kp, float alpha, const uint16_t* Ah,
                             const uint16_t* Al, const uint16_t* Bh, const uint16_t* Bl, float beta,
                             float* C, int64_t ldc, hipStream_t stream) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)gemm_bf16_tn_kernel<NTERMS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int tiles_m = (int)((M + TM - 1) / TM), tiles_n = (int)((N + TN - 1) / TN);
    hipLaunchKernelGGL(gemm_bf16_tn_kernel<NTERMS>, dim3(tiles_m * tiles_n), dim3(THREADS), kSmem,
                       stream, M, N, Kp, alpha, Ah, Al, Bh, Bl, beta, C, ldc, tiles_m, tiles_n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_bf16_tn(int64_t M, int64_t N, int64_t Kp, int nterms, float alpha,
                               const uint16_t* Ah, const uint16_t* Al, const uint16_t* Bh,
                               const uint16_t* Bl, float beta, float* C, int64_t ldc,
                               hipStream_t stream) {
    if (Kp % 64 || Kp <= 0 || (nterms != 1 && nterms != 3) || (nterms == 3 && (!Al || !Bl)))
        return hipErrorInvalidValue;
    if (nterms == 1) return launch_bf16_terms<1>(M, N, Kp, alpha, Ah, Al, Bh, Bl, beta, C, ldc, stream);
    return launch_bf16_terms<3>(M, N, Kp, alpha, Ah, Al, Bh, Bl, beta, C, ldc, stream);
}

hipError_t launch_gemm_fp8r_tn(int64_t M, int64_t N, int64_t Kp, float alpha, const uint8_t* Aq,
                               const uint8_t* Ar, const uint8_t* Asq, const uint8_t* Asr,
                               const uint8_t* Bq, const uint8_t* Br, const uint8_t* Bsq,
                               const uint8_t* Bsr, float beta, float* C, int64_t ldc,
                               hipStream_t stream) {
    if (Kp % 128 || Kp <= 0) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)gemm_fp8r_tn_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int tiles_m = (int)((M + TM - 1) / TM), tiles_n = (int)((N + TN - 1) / TN);
    hipLaunchKernelGGL(gemm_fp8r_tn_kernel, dim3(tiles_m * tiles_n), dim3(THREADS), kSmem, stream,
                       M, N, Kp, alpha, Aq, Ar, Asq, Asr, Bq, Br, Bsq, Bsr, beta, C, ldc, tiles_m,
                       tiles_n);
    return hipGetLastError();
}

}  // namespace cmp
