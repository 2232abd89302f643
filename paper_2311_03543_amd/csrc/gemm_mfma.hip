// MFMA GEMM kernels for gfx950 over the pre-pass panel images (both operands
// K-contiguous, A image of Mp rows, B image of Np rows = B transposed, in the
// panel layout of common.h).
//
//   bf16 / bf16x3:  C = alpha * sum_t A_t B_t^T + beta * C with one (bf16) or
//                   three (hi.hi + hi.lo + lo.hi, the split-precision product)
//                   operand pairs, v_mfma_f32_32x32x16_bf16, FP32 accumulation.
//   fp8 refined:    C = alpha * (Aq.Bq + Ar.Bq + Aq.Br + Ar.Br) + beta * C over
//                   E4M3 images with one E8M0 scale byte per 128 x 128 tile,
//                   v_mfma_scale_f32_32x32x64_f8f6f4, FP32 accumulation.
//   MX fp6 x3:      C = alpha * (Ah.Bh + Ah.Bl + Al.Bh) + beta * C over packed
//                   E2M3 images with one E8M0 scale per 32 K values of a row
//                   (the OCP MX block), the same MFMA at the FP6 rate.
//
// Tiling: 256 x 256 C tile per workgroup of 4 wave64 (2 x 2 waves, 128 x 128
// per wave = 4 x 4 MFMA blocks of 32 x 32, 256 FP32 accumulators per lane).
// Operands move in 16 KiB slabs (256 rows x 64 bytes of K, each one
// contiguous panel-image block) through an LDS ring.  The multi-product
// variants stage the four slabs of one K block that feed all their products
// (bf16x3: Ah Bh Al Bl; fp8: Aq Bq Ar Br) in a 2-slot ring; one-term bf16
// stages the A and B slabs of one K block in a 4-slot ring.  Direct
// global->LDS loads (global_load_lds_dwordx4) copy the slabs as linear 1 KiB
// pieces whose immediate offset advances the global and the LDS address
// together; a stage's copies go out right after the barrier that frees their
// slot.  The instruction order of every main loop is pinned: each MFMA is
// followed by the copy and fragment reads that ride under it.
#include <atomic>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace cmp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx2 __attribute__((ext_vector_type(2)));

constexpr int TM = 256, TN = 256;
constexpr int THREADS = 256;
constexpr int SLAB = kPanelBlock;          // 16 KiB: 256 rows x 64 bytes
constexpr int STAGE4 = 4 * SLAB;           // four slabs per pipeline stage
constexpr int NBUF4 = 2;                   // LDS ring depth (stages)
constexpr size_t kSmem = (size_t)NBUF4 * STAGE4;   // 128 KiB

typedef const __attribute__((address_space(1))) void* gptr_t;
typedef __attribute__((address_space(3))) void* lptr_t;

// Byte offset of 16-byte chunk c of slab row r (the panel swizzle).  gfx950's
// LDS serves a 16-byte-per-lane read 16 lanes at a time over 64 banks (256
// bytes = 4 slab rows); the 16 rows one lane group of a fragment read touches
// then occupy (r % 4, c ^ (r / 4) % 4): 16 distinct bank quads, no conflicts.
__device__ __forceinline__ int slab_off(int r, int c) { return r * 64 + ((c ^ ((r >> 2) & 3)) << 4); }

// s_waitcnt immediate: vmcnt <= vm (0..63), lgkmcnt <= lgkm (0..15), expcnt free.
constexpr int waitcnt_imm(int vm, int lgkm) {
    return (vm & 15) | ((vm >> 4) << 14) | (7 << 4) | (lgkm << 8);
}

// Stage barrier: this wave's LDS reads done, at most VM of its copies still
// in flight (copies complete in issue order), then the workgroup barrier:
// afterwards every wave's copies of the awaited stage have landed and every
// wave's reads of the slot about to be refilled are complete.  The empty asm
// statements keep the compiler from moving memory accesses across.
template <int VM>
__device__ __forceinline__ void stage_barrier() {
    static_assert(VM >= 0 && VM <= 63, "vmcnt range");
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(VM, 0));
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// One 1 KiB linear copy, part P (0..3) of this wave's quarter (4 KiB) of a
// slab.  `src` already holds the wave's and the lane's offset (wave * 4 KiB +
// 16 lane), `dst` the wave's slab quarter; lane l lands at dst + 1024 P + 16 l.
template <int P>
__device__ __forceinline__ void dma_part(const uint8_t* src, uint8_t* dst) {
    static_assert(P >= 0 && P < 4, "part of a 4 KiB quarter");
    __builtin_amdgcn_global_load_lds((gptr_t)src, (lptr_t)dst, 16, P * 1024, 0);
}

// The main loops pin their instruction order explicitly: each MFMA is
// followed by the memory instructions that ride under it, and a
// sched_barrier after each group keeps the scheduler from clustering them.
__device__ __forceinline__ void pin() { __builtin_amdgcn_sched_barrier(0); }

// f(integral_constant<int, I>) for I = B .. E - 1, unrolled at compile time.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// 32 x 32 accumulator block layout: lane l holds column l % 32 and rows
// 8 (r / 4) + 4 (l / 32) + (r % 4), r = 0..15.
template <bool FULL>
__device__ __forceinline__ void store_block(const floatx16& acc, int64_t M, int64_t N, int64_t row0,
                                            int64_t col, float alpha, float beta,
                                            float* __restrict__ C, int64_t ldc) {
    if (!FULL && col >= N) return;
    float old[16];
    if (beta != 0.f) {
        // all 16 loads in flight before the first use
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t row = row0 + (r >> 2) * 8 + (r & 3);
            old[r] = (FULL || row < M) ? C[row * ldc + col] : 0.f;
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t row = row0 + (r >> 2) * 8 + (r & 3);
        if (FULL || row < M) {
            float v = alpha * acc[r];
            if (beta != 0.f) v = __builtin_fmaf(beta, old[r], v);
            C[row * ldc + col] = v;
        }
    }
}

__device__ __forceinline__ void epilogue(const floatx16 (&acc)[4][4], int64_t M, int64_t N,
                                         int64_t m0, int64_t n0, int wm, int wn, int lane,
                                         float alpha, float beta, float* __restrict__ C,
                                         int64_t ldc) {
    const bool full = m0 + TM <= M && n0 + TN <= N;   // interior tile: no bounds checks
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t col = n0 + wn * 128 + j * 32 + (lane & 31);
            const int64_t row0 = m0 + wm * 128 + i * 32 + (lane >> 5) * 4;
            if (full) store_block<true>(acc[i][j], M, N, row0, col, alpha, beta, C, ldc);
            else store_block<false>(acc[i][j], M, N, row0, col, alpha, beta, C, ldc);
        }
}

__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int& tm, int& tn) {
    grouped_tile(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
}

// ---------------------------------------------------------------------------
// One-term bf16: a stage is one 64-byte K block of A and B (16 KiB slabs),
// NRING = 4 stages in the LDS ring.  The copies of stage s + 4 go out right
// after the barrier of stage s that frees its slot, so a copy has three stages
// (96 MFMAs) to land; the barrier waits only for stage s + 1
// (vmcnt(16): the two younger stages stay in flight).  With a single product
// the deeper ring beats the four-slab stage: its copies get one and a half
// times the cover for the price of one barrier per 32 MFMAs.
constexpr int NRING = 4;
constexpr int RSTAGE = 2 * SLAB;
static_assert((size_t)NRING * RSTAGE <= kSmem, "ring fits the LDS allocation");
static_assert(kKBlockBytes == kPanelRowBytes, "split-K counts K in operand-image blocks");
static_assert(kMx6CodeBlockBytes == kMx6Block && kMx6ScaleBlockBytes == kMx6ScaleBlock, "MX FP6 image blocks");

__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_bf16_ring_kernel(int64_t M, int64_t N, int nkb, float alpha, const uint8_t* __restrict__ Ah,
                           const uint8_t* __restrict__ Bh, float beta, float* __restrict__ C,
                           int64_t ldc, int tiles_m, int tiles_n, int kb_split,
                           float* __restrict__ P) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    // LDS ring: slot i = [A slab | B slab] at i * RSTAGE

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform (SGPR)
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TN;
    const int64_t panel = (int64_t)nkb * SLAB;        // bytes of one 256-row panel
    const int src_off = wave * 4096 + lane * 16;
    // split-K: this workgroup's K blocks [kb0, kb0 + steps) (blockIdx.y = split)
    const int kb0 = (int)blockIdx.y * kb_split;
    const int steps = nkb - kb0 < kb_split ? nkb - kb0 : kb_split;
    const int64_t koff = (int64_t)kb0 * SLAB;
    const uint8_t* a_src = Ah + tm * panel + koff + src_off;
    const uint8_t* b_src = Bh + tn * panel + koff + src_off;

    floatx16 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // Load cursor (K block, slot); past the last block it re-reads the last
    // one into the freed slot, so every stage issues the same 8 copies and the
    // in-flight count the barriers wait on stays constant.
    int ld_kb = 0, ld_left = steps, ld_slot = 0;
    int64_t kofs = 0;
    uint8_t* dd = nullptr;
    auto prepare = [&]() {
        kofs = (int64_t)ld_kb * SLAB;
        dd = smem + ld_slot * RSTAGE + wave * 4096;
        const int go = ld_left > 1 ? 1 : 0;
        ld_left -= go;
        ld_kb += go;
        ld_slot = ld_slot + 1 == NRING ? 0 : ld_slot + 1;
    };
    auto copy = [&](auto part_tag) {            // copy P: A (P < 4) or B slab, part P % 4
        constexpr int P = decltype(part_tag)::value;
        static_assert(P >= 0 && P < 8, "a stage is 8 copies");
        if constexpr (P < 4) dma_part<P>(a_src + kofs, dd);
        else dma_part<P - 4>(b_src + kofs, dd + SLAB);
    };

    // lane l feeds row l % 32 of each 32-row block, k-chunk 2 ks + l / 32;
    // fragment f < 4 is A block f, f >= 4 is B block f - 4
    const int frag_row = lane & 31;
    const int frag_c = lane >> 5;
    auto read = [&](int slot, int ks, int f, bf16x8 (&a)[4], bf16x8 (&b)[4]) {
        const uint8_t* base = smem + slot * RSTAGE;
        if (f < 4)
            a[f] = *reinterpret_cast<const bf16x8*>(base + slab_off(wm * 128 + f * 32 + frag_row, 2 * ks + frag_c));
        else
            b[f - 4] = *reinterpret_cast<const bf16x8*>(base + SLAB + slab_off(wn * 128 + (f - 4) * 32 + frag_row, 2 * ks + frag_c));
    };
    auto mfma = [&](int idx, const bf16x8 (&a)[4], const bf16x8 (&b)[4]) {
        const int i = idx >> 2, j = idx & 3;
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    };

    // prologue: the first NRING stages in flight, wait for stage 0
#pragma unroll
    for (int p = 0; p < NRING; ++p) {
        prepare();
        static_for<0, 8>(copy);
    }
    stage_barrier<8 * (NRING - 1)>();

    // One stage = two 16-MFMA sub-steps over slot `cur`:
    //   ks 0: MFMA q on fa[0], then (q < 8) read fragment q of ks 1 into fa[1]
    //   ks 1: PRE MFMAs on fa[1]; stage barrier (stage s + 1 landed, slot
    //         `cur` free); then MFMA q, copy q - PRE of stage s + NRING into
    //         slot `cur`, read fragment q - PRE of stage s + 1's ks 0 into fa[0].
    constexpr int PRE = 2;
    static_assert(PRE >= 1 && PRE + 8 <= 16, "the 8 copies and reads ride under MFMAs PRE .. PRE + 7");
    bf16x8 fa[2][4], fb[2][4];
#pragma unroll
    for (int f = 0; f < 8; ++f) read(0, 0, f, fa[0], fb[0]);
    int cur = 0;
    pin();
    auto one_stage = [&](auto more_tag) {
        constexpr bool MORE = decltype(more_tag)::value;
        const int nxt = cur + 1 == NRING ? 0 : cur + 1;
        // ks 0
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            mfma(q, fa[0], fb[0]);
            if (q < 8) read(cur, 1, q, fa[1], fb[1]);
            pin();
        }
        // ks 1
#pragma unroll
        for (int q = 0; q < PRE; ++q) mfma(q, fa[1], fb[1]);
        pin();
        if constexpr (MORE) {
            stage_barrier<8 * (NRING - 2)>();
            prepare();
        }
        pin();
        static_for<PRE, 16>([&](auto q_tag) {
            constexpr int Q = decltype(q_tag)::value;
            mfma(Q, fa[1], fb[1]);
            if constexpr (MORE && Q - PRE < 8) {
                copy(std::integral_constant<int, Q - PRE>{});
                read(nxt, 0, Q - PRE, fa[0], fb[0]);
            }
            pin();
        });
        cur = nxt;
    };
    for (int s = 0; s + 1 < steps; ++s) one_stage(std::true_type{});
    one_stage(std::false_type{});
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));   // drain the trailing copies
    if (P)   // split-K: raw partial sums of this split, reduced by splitk_reduce_kernel
        epilogue(acc, M, N, m0, n0, wm, wn, lane, 1.f, 0.f, P + (size_t)blockIdx.y * M * N, N);
    else
        epilogue(acc, M, N, m0, n0, wm, wn, lane, alpha, beta, C, ldc);
}

// ---------------------------------------------------------------------------
// bf16x3 over four-slab stages: a stage holds the slabs [Ah | Bh | Al | Bl]
// of one 64-byte K block (64 KiB), two stages in the LDS ring.  Per 16-k
// sub-step (two per stage) the 16 fragments of the four slabs (4 blocks of 32
// rows each) feed 3 x 16 MFMAs, hi.hi, then hi.lo, then lo.hi, so an
// accumulator is reused every 16 MFMAs.  Every operand block is copied once
// and feeds all the products that use it.  The copies of stage s + 2 are
// issued right after the barrier of stage s that frees its slot and must land
// by the next barrier, one stage (96 MFMAs) later.

// Slabs (A side, B side) of product p: hi.hi, hi.lo, lo.hi.
constexpr int prod_a(int p) { return p == 2 ? 2 : 0; }
constexpr int prod_b(int p) { return p == 1 ? 3 : 1; }

// Fragment read order of a sub-step (fragment f: slab f / 4, block f % 4):
// the order the next sub-step's MFMAs use them (Ah0, Bh0-3, Ah1-3 for
// hi.hi, then Bl for hi.lo, then Al for lo.hi).
constexpr int read_order(int k) {
    constexpr int order[16] = {0, 4, 5, 6, 7, 1, 2, 3, 12, 13, 14, 15, 8, 9, 10, 11};
    return order[k];
}

// One 256 x 256 tile (tm, tn) of the bf16x3 product over the K blocks
// [kb0, kb0 + steps) of images with nkb blocks per panel; `smem` is the
// 128 KiB LDS ring.  P != nullptr: the raw partial sums go to P (a split-K
// slice, row pitch N); otherwise C = alpha * acc + beta * C.  Every copy has
// landed when it returns (the ring may be reused after a workgroup barrier).
__device__ __forceinline__ void bf16x3_tile(uint8_t* smem, int64_t M, int64_t N, int nkb, float alpha,
                                            const uint8_t* __restrict__ Ah, const uint8_t* __restrict__ Al,
                                            const uint8_t* __restrict__ Bh, const uint8_t* __restrict__ Bl,
                                            float beta, float* __restrict__ C, int64_t ldc, int tm, int tn,
                                            int kb0, int steps, float* __restrict__ P) {
    // LDS ring: slot i = four slabs at i * STAGE4
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform (SGPR)
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TN;
    const int64_t panel = (int64_t)nkb * SLAB;
    const int src_off = wave * 4096 + lane * 16;
    const int64_t koff = (int64_t)kb0 * SLAB;
    const uint8_t* a_hi = Ah + tm * panel + koff + src_off;
    const uint8_t* b_hi = Bh + tn * panel + koff + src_off;
    const uint8_t* a_lo = Al + tm * panel + koff + src_off;
    const uint8_t* b_lo = Bl + tn * panel + koff + src_off;

    floatx16 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // Load cursor (stage, slot); past the last stage it re-reads the last one
    // into the freed slot, so every stage issues the same 16 copies.
    int ld_st = 0, ld_left = steps, ld_slot = 0;
    int64_t kofs = 0;
    uint8_t* dd = nullptr;
    auto prepare = [&]() {
        kofs = (int64_t)ld_st * SLAB;
        dd = smem + ld_slot * STAGE4 + wave * 4096;
        const int go = ld_left > 1 ? 1 : 0;
        ld_left -= go;
        ld_st += go;
        ld_slot ^= 1;
    };
    auto copy = [&](auto part_tag) {            // copy P: slab P / 4, part P % 4
        constexpr int P = decltype(part_tag)::value;
        static_assert(P >= 0 && P < 16, "a stage is 16 copies");
        constexpr int S = P / 4;
        const uint8_t* src = S == 0 ? a_hi : (S == 1 ? b_hi : (S == 2 ? a_lo : b_lo));
        dma_part<P % 4>(src + kofs, dd + S * SLAB);
    };

    // fragment f of a sub-step: slab f / 4 (even slabs are A sides, odd B
    // sides), 32-row block f % 4; lane l feeds row l % 32, k-chunk 2 ks + l / 32
    const int frag_row = lane & 31;
    const int frag_c = lane >> 5;
    auto read = [&](int slot, int ks, auto f_tag, bf16x8 (&F)[16]) {
        constexpr int f = decltype(f_tag)::value;
        constexpr int S = f / 4, blk = f % 4;
        const int r = ((S & 1) ? wn : wm) * 128 + blk * 32 + frag_row;
        F[f] = *reinterpret_cast<const bf16x8*>(smem + slot * STAGE4 + S * SLAB + slab_off(r, 2 * ks + frag_c));
    };
    // MFMA q of a sub-step: product q / 16, block q % 16
    auto mfma = [&](auto q_tag, const bf16x8 (&F)[16]) {
        constexpr int q = decltype(q_tag)::value;
        constexpr int p = q / 16, i = (q % 16) / 4, j = q % 4;
        constexpr int fa = 4 * prod_a(p) + i, fb = 4 * prod_b(p) + j;
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F[fa], F[fb], acc[i][j], 0, 0, 0);
    };

    // prologue: stages 0 and 1 in flight, wait for stage 0
#pragma unroll
    for (int p = 0; p < NBUF4; ++p) {
        prepare();
        static_for<0, 16>(copy);
    }
    stage_barrier<16>();                        // stage 1 (16 copies) may stay in flight

    constexpr int NM = 48;                      // MFMAs per sub-step
    // the 16 fragment reads and (after the barrier) the 16 copies go one
    // every ST = 2 MFMAs over the first 32 MFMAs of a sub-step, leaving the
    // last 16 for the reads to land before the next sub-step's first MFMA
    constexpr int ST = 2;
    static_assert(1 + 16 * ST <= NM, "reads and copies fit the sub-step");
    bf16x8 F0[16], F1[16];
    static_for<0, 16>([&](auto k) {
        read(0, 0, std::integral_constant<int, read_order(decltype(k)::value)>{}, F0);
    });
    int cur = 0;
    pin();
    // One stage = two sub-steps of NM MFMAs over slot `cur`:
    //   ks 0: MFMA q on F0; after MFMA ST k, read fragment read_order(k) of ks 1 into F1
    //   ks 1: one MFMA on F1; stage barrier (stage s + 1 landed, slot `cur`
    //         free); then MFMA q = 1 + m on F1 with, for m = ST k, the read
    //         of fragment read_order(k) of stage s + 1's ks 0 into F0 and
    //         copy k of stage s + 2 into slot `cur`.
    auto one_stage = [&](auto more_tag) {
        constexpr bool MORE = decltype(more_tag)::value;
        const int nxt = cur ^ 1;
        static_for<0, NM>([&](auto q) {
            constexpr int Q = decltype(q)::value;
            mfma(q, F0);
            if constexpr (Q % ST == 0 && Q / ST < 16)
                read(cur, 1, std::integral_constant<int, read_order(Q / ST)>{}, F1);
            pin();
        });
        mfma(std::integral_constant<int, 0>{}, F1);
        pin();
        if constexpr (MORE) {
            stage_barrier<0>();
            prepare();
        }
        pin();
        static_for<1, NM>([&](auto q) {
            constexpr int m = decltype(q)::value - 1;
            mfma(q, F1);
            if constexpr (MORE && m % ST == 0 && m / ST < 16) {
                read(nxt, 0, std::integral_constant<int, read_order(m / ST)>{}, F0);
                copy(std::integral_constant<int, m / ST>{});
            }
            pin();
        });
        cur = nxt;
    };
    for (int s = 0; s + 1 < steps; ++s) one_stage(std::true_type{});
    one_stage(std::false_type{});
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));   // drain the trailing copies
    if (P)   // split-K: raw partial sums of this split, reduced by splitk_reduce_kernel
        epilogue(acc, M, N, m0, n0, wm, wn, lane, 1.f, 0.f, P, N);
    else
        epilogue(acc, M, N, m0, n0, wm, wn, lane, alpha, beta, C, ldc);
}

__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_bf16x3_slab4_kernel(int64_t M, int64_t N, int nkb, float alpha,
                              const uint8_t* __restrict__ Ah, const uint8_t* __restrict__ Al,
                              const uint8_t* __restrict__ Bh, const uint8_t* __restrict__ Bl,
                              float beta, float* __restrict__ C, int64_t ldc, int tiles_m,
                              int tiles_n, int kb_split, float* __restrict__ P) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    int tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    // split-K: this workgroup's K blocks [kb0, kb0 + steps) (blockIdx.y = split)
    const int kb0 = (int)blockIdx.y * kb_split;
    const int steps = nkb - kb0 < kb_split ? nkb - kb0 : kb_split;
    bf16x3_tile(smem, M, N, nkb, alpha, Ah, Al, Bh, Bl, beta, C, ldc, tm, tn, kb0, steps,
                P ? P + (size_t)blockIdx.y * M * N : nullptr);
}

// Many bf16x3 problems in one persistent launch (the grouped plan's MFMA
// configuration): the tile list is the concatenation of every problem's
// 256 x 256 tiles (desc[p].tile_start = first tile of problem p, problems in
// decreasing order of K).  Workgroup b starts with tile b and each workgroup
// that finishes a tile claims the next unclaimed one from `counter` (zeroed
// by grouped_mfma_reset_kernel right before, on the same stream).  The tile
// index lives in the 16 bytes past the ring, so the LDS request is kSmem + 16.
__global__ void grouped_mfma_reset_kernel(unsigned* counter) {
    if (threadIdx.x == 0) *counter = 0u;
}

__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_bf16x3_grouped_kernel(const GroupedMfmaDesc* __restrict__ desc, int count, int total_tiles,
                                unsigned* __restrict__ counter) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    int* next_tile = reinterpret_cast<int*>(smem + kSmem);
    typedef const __attribute__((address_space(1))) GroupedMfmaDesc* gdesc;
    const gdesc dg = (gdesc)desc;
    for (int tile = blockIdx.x; tile < total_tiles;) {
        int lo = 0, hi = count - 1;            // last problem whose first tile is <= tile
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (dg[mid].tile_start <= tile) lo = mid;
            else hi = mid - 1;
        }
        const int local = tile - dg[lo].tile_start;
        const int tn_count = dg[lo].tiles_n;
        const int tm = local / tn_count, tn = local - tm * tn_count;
        const int nkb = (int)(dg[lo].Kp * 2 / kPanelRowBytes);
        bf16x3_tile(smem, dg[lo].M, dg[lo].N, nkb, dg[lo].alpha, (const uint8_t*)dg[lo].ah,
                    (const uint8_t*)dg[lo].al, (const uint8_t*)dg[lo].bh, (const uint8_t*)dg[lo].bl,
                    dg[lo].beta, dg[lo].C, dg[lo].ldc, tm, tn, 0, nkb, nullptr);
        __syncthreads();                       // every wave is done with the ring and next_tile
        if (threadIdx.x == 0) {
            const unsigned ticket = atomicAdd(counter, 1u);
            const unsigned left = (unsigned)total_tiles - gridDim.x;   // grid <= total_tiles
            *next_tile = ticket < left ? (int)(gridDim.x + ticket) : total_tiles;
        }
        __syncthreads();
        tile = __builtin_amdgcn_readfirstlane(*next_tile);
    }
}

// ---------------------------------------------------------------------------
// fp8 refined with the four products fused per K block.  A stage holds the
// four slabs [Aq | Bq | Ar | Br] of one 64-byte K block (one 64-k MFMA step),
// two stages in the ring.  The products run in the order q.q, q.r, r.q, r.r
// (16 MFMAs each), and the operand registers are reused as soon as their last
// product has issued, so one register set suffices:
//   q.q  (Aq, Bq)  under it: read Br, then Ar of this stage
//   --- stage barrier: stage s + 1 landed, every read of slot s done ---
//   q.r  (Aq, Br)  under it: the 16 copies of stage s + 2 into slot s
//   r.q  (Ar, Bq)  under it: read Aq of stage s + 1
//   r.r  (Ar, Br)  under it: read Bq of stage s + 1
// Copies get 64 MFMAs (one stage) to land; one barrier per 64 MFMAs.  Each
// product has its own pair of E8M0 tile scales (q or r of A, q or r of B).
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_fp8r_fused_kernel(int64_t M, int64_t N, int nkb, float alpha,
                            const uint8_t* __restrict__ Aq, const uint8_t* __restrict__ Ar,
                            const uint8_t* __restrict__ Asq, const uint8_t* __restrict__ Asr,
                            const uint8_t* __restrict__ Bq, const uint8_t* __restrict__ Br,
                            const uint8_t* __restrict__ Bsq, const uint8_t* __restrict__ Bsr,
                            float beta, float* __restrict__ C, int64_t ldc, int tiles_m,
                            int tiles_n, int kb_split, float* __restrict__ P) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    // LDS ring: slot i = [Aq slab | Bq slab | Ar slab | Br slab] at i * STAGE4

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform (SGPR)
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TN;
    const int64_t panel = (int64_t)nkb * SLAB;
    const int src_off = wave * 4096 + lane * 16;
    // split-K: this workgroup's K blocks [kb0, kb0 + steps) (blockIdx.y = split),
    // one 64-k MFMA step per stage
    const int kb0 = (int)blockIdx.y * kb_split;
    const int steps = nkb - kb0 < kb_split ? nkb - kb0 : kb_split;
    const int64_t koff = (int64_t)kb0 * SLAB;
    const uint8_t* a_q = Aq + tm * panel + koff + src_off;
    const uint8_t* b_q = Bq + tn * panel + koff + src_off;
    const uint8_t* a_r = Ar + tm * panel + koff + src_off;
    const uint8_t* b_r = Br + tn * panel + koff + src_off;
    const int nkt = nkb / 2;                    // 128-k scale tiles per row
    // this wave's 128 rows of A (and columns of C) lie in one 128-row scale tile
    const int64_t a_tile = m0 / 128 + wm, b_tile = n0 / 128 + wn;

    floatx16 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // Load cursor (K block, slot); past the last block it re-reads the last
    // one into the freed slot, so every stage issues the same 16 copies.
    int ld_kb = 0, ld_left = steps, ld_slot = 0;
    int64_t kofs = 0;
    uint8_t* dd = nullptr;
    auto prepare = [&]() {
        kofs = (int64_t)ld_kb * SLAB;
        dd = smem + ld_slot * STAGE4 + wave * 4096;
        const int go = ld_left > 1 ? 1 : 0;
        ld_left -= go;
        ld_kb += go;
        ld_slot ^= 1;
    };
    auto copy = [&](auto part_tag) {            // copy P: slab P / 4, part P % 4
        constexpr int P = decltype(part_tag)::value;
        static_assert(P >= 0 && P < 16, "a fused stage is 16 copies");
        constexpr int S = P / 4;
        const uint8_t* src = S == 0 ? a_q : (S == 1 ? b_q : (S == 2 ? a_r : b_r));
        dma_part<P % 4>(src + kofs, dd + S * SLAB);
    };

    // Scale bytes of a K block: E8M0 of this wave's A tile (q, r) and B tile
    // (q, r); scalar loads of the aligned words, issued one stage ahead.
    int sc_kb = 0;
    uint32_t w_aq = 0, w_ar = 0, w_bq = 0, w_br = 0;
    int sh_a = 0, sh_b = 0;
    auto load_scale_words = [&]() {
        const int64_t ia = a_tile * nkt + ((kb0 + sc_kb) >> 1), ib = b_tile * nkt + ((kb0 + sc_kb) >> 1);
        const int64_t oa = ia & ~(int64_t)3, ob = ib & ~(int64_t)3;
        w_aq = *reinterpret_cast<const uint32_t*>(Asq + oa);
        w_ar = *reinterpret_cast<const uint32_t*>(Asr + oa);
        w_bq = *reinterpret_cast<const uint32_t*>(Bsq + ob);
        w_br = *reinterpret_cast<const uint32_t*>(Bsr + ob);
        sh_a = (int)(ia & 3) * 8;
        sh_b = (int)(ib & 3) * 8;
        sc_kb = __builtin_amdgcn_readfirstlane(sc_kb + 1 < steps ? sc_kb + 1 : sc_kb);
    };
    int s_aq, s_ar, s_bq, s_br;                 // scales of the stage being multiplied
    int n_aq = 0, n_ar = 0, n_bq = 0, n_br = 0; // scales of the next stage
    auto unpack_next = [&]() {
        n_aq = (int)((w_aq >> sh_a) & 0xffu);
        n_ar = (int)((w_ar >> sh_a) & 0xffu);
        n_bq = (int)((w_bq >> sh_b) & 0xffu);
        n_br = (int)((w_br >> sh_b) & 0xffu);
    };
    auto advance_scales = [&]() {
        s_aq = n_aq;
        s_ar = n_ar;
        s_bq = n_bq;
        s_br = n_br;
    };

    // Operand registers: image X in {Aq, Bq, Ar, Br} (X = 0..3), 32-row block
    // b, half h (16 of the 32 bytes a lane feeds): R[X][2 b + h].  Lane l
    // feeds row l % 32 of a block, bytes 32 (l / 32) .. +31 of the K block.
    intx4 R[4][8];
    const int frag_row = lane & 31;
    const int frag_c = (lane >> 5) * 2;
    auto read = [&](int slot, auto x_tag, auto h_tag) {
        constexpr int X = decltype(x_tag)::value, H = decltype(h_tag)::value;
        constexpr int blk = H / 2, half = H % 2;
        const int r = ((X & 1) ? wn : wm) * 128 + blk * 32 + frag_row;
        R[X][H] = *reinterpret_cast<const intx4*>(smem + slot * STAGE4 + X * SLAB + slab_off(r, frag_c + half));
    };
    // MFMA q (0..15) of product P (0 q.q, 1 q.r, 2 r.q, 3 r.r)
    auto mfma = [&](auto p_tag, auto q_tag) {
        constexpr int P = decltype(p_tag)::value, q = decltype(q_tag)::value;
        constexpr int i = q / 4, j = q % 4;
        constexpr int XA = (P == 2 || P == 3) ? 2 : 0, XB = (P == 1 || P == 3) ? 3 : 1;
        const intx8 av = __builtin_shufflevector(R[XA][2 * i], R[XA][2 * i + 1], 0, 1, 2, 3, 4, 5, 6, 7);
        const intx8 bv = __builtin_shufflevector(R[XB][2 * j], R[XB][2 * j + 1], 0, 1, 2, 3, 4, 5, 6, 7);
        const int sa = XA == 0 ? s_aq : s_ar, sb = XB == 1 ? s_bq : s_br;
        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc[i][j], 0, 0, 0, sa, 0, sb);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;

    // prologue: stages 0 and 1 in flight, stage 0's scales, wait for stage 0,
    // read Aq and Bq of stage 0
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        prepare();
        static_for<0, 16>(copy);
    }
    load_scale_words();
    unpack_next();
    advance_scales();                            // stage 0's scales
    load_scale_words();                          // stage 1's words
    stage_barrier<16>();                         // stage 1 (16 copies) may stay in flight
    static_for<0, 8>([&](auto h) { read(0, I0{}, h); });
    static_for<0, 8>([&](auto h) { read(0, I1{}, h); });
    int cur = 0;
    pin();

    auto one_stage = [&](auto more_tag) {
        constexpr bool MORE = decltype(more_tag)::value;
        const int nxt = cur ^ 1;
        // q.q; read Br then Ar of this stage under it
        static_for<0, 16>([&](auto q) {
            mfma(I0{}, q);
            constexpr int k = decltype(q)::value;
            if constexpr (k < 8) read(cur, I3{}, std::integral_constant<int, k>{});
            else read(cur, I2{}, std::integral_constant<int, k - 8>{});
            pin();
        });
        if constexpr (MORE) {
            stage_barrier<0>();                 // stage s + 1 landed, slot `cur` free
            prepare();
        }
        pin();
        // q.r; the copies of stage s + 2 under it
        static_for<0, 16>([&](auto q) {
            mfma(I1{}, q);
            if constexpr (MORE) copy(q);
            pin();
        });
        if constexpr (MORE) {
            unpack_next();                      // stage s + 1's scales (words loaded a stage ago)
            load_scale_words();                 // stage s + 2's words
        }
        pin();
        // r.q; read Aq of stage s + 1 under it
        static_for<0, 16>([&](auto q) {
            mfma(I2{}, q);
            constexpr int k = decltype(q)::value;
            if constexpr (MORE && k < 8) read(nxt, I0{}, std::integral_constant<int, k>{});
            pin();
        });
        // r.r; read Bq of stage s + 1 under it
        static_for<0, 16>([&](auto q) {
            mfma(I3{}, q);
            constexpr int k = decltype(q)::value;
            if constexpr (MORE && k < 8) read(nxt, I1{}, std::integral_constant<int, k>{});
            pin();
        });
        if constexpr (MORE) advance_scales();
        pin();
        cur = nxt;
    };
    for (int s = 0; s + 1 < steps; ++s) one_stage(std::true_type{});
    one_stage(std::false_type{});
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));   // drain the trailing copies
    if (P)   // split-K: raw partial sums of this split, reduced by splitk_reduce_kernel
        epilogue(acc, M, N, m0, n0, wm, wn, lane, 1.f, 0.f, P + (size_t)blockIdx.y * M * N, N);
    else
        epilogue(acc, M, N, m0, n0, wm, wn, lane, alpha, beta, C, ldc);
}

// ---------------------------------------------------------------------------
// MX FP6 with one residual level, three products fused per K block.  A stage
// holds one 64-value K block: the code slabs [Ah | Bh | Al | Bl] (12 KiB each,
// 48 bytes per row: E2M3 codes packed 6 bits each) and the A and B scale
// blocks (1 KiB each: per row and K half the E8M0 bytes of both levels);
// F6NBUF stages in the ring.  Products, 16 MFMAs each:
//   h.h  (Ah, Bh)  B block major; under it: read Bl, then Al of this stage
//   --- stage barrier: stage s + 1 landed, every read of slot s done ---
//   h.l  (Ah, Bl)  under it: the 13 copies of stage s + F6NBUF into slot s
//   l.h  (Al, Bh)  B block major; under it: read Ah of stage s + 1, each Bh
//                  block and B scale of stage s + 1 as soon as the last MFMA
//                  using the current one has issued, and the A scales of stage
//                  s + 1 over the last four MFMAs, one per A block as it retires
// A lane's fragment is one 16-byte and one 8-byte LDS read (its 24 code
// bytes); the scaled MFMA takes each lane's own scale (its row, its K half):
// one 16-bit read per 32-row block gives both levels, and op_sel picks the
// byte.  Per stage each wave copies 3 KiB of each code slab and one 1 KiB
// scale piece (waves 2 and 3 a spare copy of the A piece, so that every wave
// issues the same 13 copies and the wait counts stay constants).
constexpr int F6SLAB = kMx6Block;                       // 12 KiB
constexpr int F6STAGE = 4 * F6SLAB + 4 * kMx6ScaleBlock; // codes, A and B scales, 2 spare KiB
// Two slots: copies get one stage (32 MFMAs) to land.  A third slot (156 KiB,
// two stages of cover) measured no faster at 8192^3.
constexpr int F6NBUF = 2;
constexpr size_t kSmemF6 = (size_t)F6NBUF * F6STAGE;     // 104 KiB
static_assert(kSmemF6 <= 160 * 1024, "fp6 ring fits the 160 KiB of LDS");

__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(1, 1)))
void gemm_fp6x3_fused_kernel(int64_t M, int64_t N, int nkb, float alpha,
                             const uint8_t* __restrict__ Ah, const uint8_t* __restrict__ Al,
                             const uint8_t* __restrict__ As, const uint8_t* __restrict__ Bh,
                             const uint8_t* __restrict__ Bl, const uint8_t* __restrict__ Bs,
                             float beta, float* __restrict__ C, int64_t ldc, int tiles_m,
                             int tiles_n, int kb_split, float* __restrict__ P) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform (SGPR)
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_coords(tiles_m, tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TN;
    // split-K: this workgroup's K blocks [kb0, kb0 + steps) (blockIdx.y = split)
    const int kb0 = (int)blockIdx.y * kb_split;
    const int steps = nkb - kb0 < kb_split ? nkb - kb0 : kb_split;
    const int64_t a_blk = (int64_t)tm * nkb + kb0, b_blk = (int64_t)tn * nkb + kb0;
    const int src_off = wave * 3072 + lane * 16;              // this wave's 3 KiB of a code slab
    const uint8_t* a_h = Ah + a_blk * F6SLAB + src_off;
    const uint8_t* b_h = Bh + b_blk * F6SLAB + src_off;
    const uint8_t* a_l = Al + a_blk * F6SLAB + src_off;
    const uint8_t* b_l = Bl + b_blk * F6SLAB + src_off;
    // scale piece: wave 1 the B block, the others the A block
    const uint8_t* s_src = (wave == 1 ? Bs + b_blk * kMx6ScaleBlock : As + a_blk * kMx6ScaleBlock) + lane * 16;
    const int s_dst = 4 * F6SLAB + wave * kMx6ScaleBlock;   // A at +0, B at +1 KiB, spares after

    floatx16 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // Load cursor (K block, slot); past the last block it re-reads the last
    // one into the freed slot, so every stage issues the same 13 copies.
    int ld_kb = 0, ld_left = steps, ld_slot = 0;
    int64_t kofs = 0, sofs = 0;
    uint8_t* dd = nullptr;
    uint8_t* sd = nullptr;
    auto prepare = [&]() {
        kofs = (int64_t)ld_kb * F6SLAB;
        sofs = (int64_t)ld_kb * kMx6ScaleBlock;
        dd = smem + ld_slot * F6STAGE + wave * 3072;
        sd = smem + ld_slot * F6STAGE + s_dst;
        const int go = ld_left > 1 ? 1 : 0;
        ld_left -= go;
        ld_kb += go;
        ld_slot = ld_slot == F6NBUF - 1 ? 0 : ld_slot + 1;
    };
    auto copy = [&](auto part_tag) {            // copy P < 12: slab P / 3, part P % 3; 12: scales
        constexpr int P = decltype(part_tag)::value;
        static_assert(P >= 0 && P < 13, "a stage is 13 copies");
        if constexpr (P == 12) {
            dma_part<0>(s_src + sofs, sd);
        } else {
            constexpr int S = P / 3;
            const uint8_t* src = S == 0 ? a_h : (S == 1 ? b_h : (S == 2 ? a_l : b_l));
            dma_part<P % 3>(src + kofs, dd + S * F6SLAB);
        }
    };

    // Operand registers of image X in {Ah, Bh, Al, Bl} (X = 0..3), 32-row block
    // b: code bytes 0-15 in R4[X][b], 16-23 in R2[X][b].  Lane l feeds row
    // l % 32 of a block, K half l / 32.  Scales: SA[b] / SB[b] hold (hi, lo)
    // of A / B block b, replaced by the next stage's as each retires.
    intx4 R4[4][4];
    intx2 R2[4][4];
    int SA[4], SB[4];
    const int frag_row = lane & 31;
    const int half = lane >> 5;
    // H = 2 b + p: p = 0 the 16-byte read, p = 1 the 8-byte read of block b
    auto read = [&](int slot, auto x_tag, auto h_tag) {
        constexpr int X = decltype(x_tag)::value, H = decltype(h_tag)::value;
        constexpr int blk = H / 2, part = H % 2;
        const int r = ((X & 1) ? wn : wm) * 128 + blk * 32 + frag_row;
        const uint8_t* row = smem + slot * F6STAGE + X * F6SLAB + r * kMx6RowBytes;
        if constexpr (part == 0) R4[X][blk] = *reinterpret_cast<const intx4*>(row + 16 * half);
        else R2[X][blk] = *reinterpret_cast<const intx2*>(row + 32 + 8 * half);
    };
    auto read_scale = [&](int slot, int side, int blk) -> int {
        const int r = (side ? wn : wm) * 128 + blk * 32 + frag_row;
        return *reinterpret_cast<const uint16_t*>(smem + slot * F6STAGE + 4 * F6SLAB + side * kMx6ScaleBlock +
                                                  4 * r + 2 * half);
    };
    // MFMA q (0..15) of product P (0 h.h, 1 h.l, 2 l.h); h.h and l.h run B
    // block major (j = q / 4) so that a B block is finished after 4 MFMAs.
    auto mfma = [&](auto p_tag, auto q_tag) {
        constexpr int P = decltype(p_tag)::value, q = decltype(q_tag)::value;
        constexpr int i = P == 1 ? q / 4 : q % 4, j = P == 1 ? q % 4 : q / 4;
        constexpr int XA = P == 2 ? 2 : 0, XB = P == 1 ? 3 : 1;
        constexpr int LA = XA == 0 ? 0 : 1, LB = XB == 1 ? 0 : 1;   // scale byte: hi 0, lo 1
        const intx8 av = __builtin_shufflevector(R4[XA][i], __builtin_shufflevector(R2[XA][i], R2[XA][i], 0, 1, 0, 1),
                                                 0, 1, 2, 3, 4, 5, 6, 7);
        const intx8 bv = __builtin_shufflevector(R4[XB][j], __builtin_shufflevector(R2[XB][j], R2[XB][j], 0, 1, 0, 1),
                                                 0, 1, 2, 3, 4, 5, 6, 7);
        // operand format 2 = FP6 E2M3 for both (dwords 0-5 used)
        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc[i][j], 2, 2, LA, SA[i], LB,
                                                                    SB[j]);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;

    // prologue: stages 0 .. F6NBUF - 1 in flight, wait for stage 0, read its Ah, Bh and scales
#pragma unroll
    for (int p = 0; p < F6NBUF; ++p) {
        prepare();
        static_for<0, 13>(copy);
    }
    stage_barrier<13 * (F6NBUF - 1)>();          // the later stages may stay in flight
    static_for<0, 8>([&](auto h) { read(0, I0{}, h); });
    static_for<0, 8>([&](auto h) { read(0, I1{}, h); });
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        SA[b] = read_scale(0, 0, b);
        SB[b] = read_scale(0, 1, b);
    }
    int cur = 0;
    pin();

    auto one_stage = [&](auto more_tag) {
        constexpr bool MORE = decltype(more_tag)::value;
        const int nxt = cur == F6NBUF - 1 ? 0 : cur + 1;
        // h.h; read Bl then Al of this stage under it
        static_for<0, 16>([&](auto q) {
            mfma(I0{}, q);
            constexpr int k = decltype(q)::value;
            if constexpr (k < 8) read(cur, I3{}, std::integral_constant<int, k>{});
            else read(cur, I2{}, std::integral_constant<int, k - 8>{});
            pin();
        });
        if constexpr (MORE) {
            stage_barrier<13 * (F6NBUF - 2)>(); // stage s + 1 landed, slot `cur` free
            prepare();
        }
        pin();
        // h.l; the copies of stage s + F6NBUF under it
        static_for<0, 16>([&](auto q) {
            mfma(I1{}, q);
            constexpr int k = decltype(q)::value;
            if constexpr (MORE && k < 13) copy(q);
            pin();
        });
        pin();
        // l.h; Ah of stage s + 1 under the first 8 MFMAs; Bh block j and B
        // scale j of stage s + 1 once MFMA 4 j + 3 (the last one reading them)
        // has issued; A scale i of stage s + 1 once MFMA 12 + i has issued
        static_for<0, 16>([&](auto q) {
            mfma(I2{}, q);
            constexpr int k = decltype(q)::value;
            if constexpr (MORE && k < 8) read(nxt, I0{}, std::integral_constant<int, k>{});
            if constexpr (MORE && k % 4 == 3) {
                read(nxt, I1{}, std::integral_constant<int, 2 * (k / 4)>{});
                read(nxt, I1{}, std::integral_constant<int, 2 * (k / 4) + 1>{});
                SB[k / 4] = read_scale(nxt, 1, k / 4);
            }
            if constexpr (MORE && k >= 12) SA[k - 12] = read_scale(nxt, 0, k - 12);
            pin();
        });
        pin();
        cur = nxt;
    };
    for (int s = 0; s + 1 < steps; ++s) one_stage(std::true_type{});
    one_stage(std::false_type{});
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));   // drain the trailing copies
    if (P)   // split-K: raw partial sums of this split, reduced by splitk_reduce_kernel
        epilogue(acc, M, N, m0, n0, wm, wn, lane, 1.f, 0.f, P + (size_t)blockIdx.y * M * N, N);
    else
        epilogue(acc, M, N, m0, n0, wm, wn, lane, alpha, beta, C, ldc);
}

// The kernels use more than the default 64 KiB of dynamic LDS; the limit is a
// per-device function attribute, set once on each device the library runs on.
template <class Kernel>
hipError_t allow_lds(Kernel kernel, std::atomic<uint64_t>& done, size_t bytes = kSmem) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = dev < 64 ? (uint64_t)1 << dev : 0;
    if (bit && (done.load(std::memory_order_relaxed) & bit)) return hipSuccess;
    e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done.fetch_or(bit, std::memory_order_relaxed);
    return e;
}

// Split-K: `splits` > 1 runs the K range in that many slices (grid y), each
// writing raw partial sums to partial[split] (M x N, tight), which
// splitk_reduce_kernel then sums in fixed order into C = alpha * sum + beta * C.
// Returns the K blocks per slice (the kernels' kb_split) for nkb blocks.
int kb_per_split(int nkb, int splits) { return (nkb + splits - 1) / splits; }

// Partials summed in slice order 0, 1, ..., splits - 1 for every element, so
// the result does not depend on which slice finished first.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(int64_t M, int64_t N, int splits,
                                                            const float* __restrict__ P, float alpha,
                                                            float beta, float* __restrict__ C,
                                                            int64_t ldc) {
    const int64_t plane = M * N;
    for (int64_t i = blockIdx.y; i < M; i += gridDim.y) {
        const float* p = P + i * N;
        float* c = C + i * ldc;
        for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (int64_t)gridDim.x * 256) {
            float sum = 0.f;
            for (int k = 0; k < splits; ++k) sum += p[(size_t)k * plane + j];
            float v = alpha * sum;
            if (beta != 0.f) v = __builtin_fmaf(beta, c[j], v);
            c[j] = v;
        }
    }
}

}  // namespace

hipError_t launch_splitk_reduce(int64_t M, int64_t N, int splits, const float* partial, float alpha,
                                float beta, float* C, int64_t ldc, hipStream_t stream) {
    if (splits < 2 || !partial || M <= 0 || N <= 0) return hipErrorInvalidValue;
    const int64_t bx = (N + 255) / 256 < 64 ? (N + 255) / 256 : 64;
    const int64_t by = M < 4096 ? M : 4096;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)bx, (unsigned)by), dim3(256), 0, stream, M,
                       N, splits, partial, alpha, beta, C, ldc);
    return hipGetLastError();
}

hipError_t launch_gemm_bf16_tn(int64_t M, int64_t N, int64_t Kp, int nterms, float alpha,
                               const uint16_t* Ah, const uint16_t* Al, const uint16_t* Bh,
                               const uint16_t* Bl, float beta, float* C, int64_t ldc, int splits,
                               float* partial, hipStream_t stream) {
    if (Kp % kBf16TileK || Kp <= 0 || (nterms != 1 && nterms != 3) || (nterms == 3 && (!Al || !Bl)))
        return hipErrorInvalidValue;
    const int tiles_m = (int)((M + TM - 1) / TM), tiles_n = (int)((N + TN - 1) / TN);
    const int nkb = (int)(Kp * 2 / kPanelRowBytes);
    if (splits < 1 || (splits > 1 && !partial)) return hipErrorInvalidValue;
    const int kbs = kb_per_split(nkb, splits);
    if ((int64_t)(splits - 1) * kbs >= nkb) return hipErrorInvalidValue;   // every slice non-empty
    float* P = splits > 1 ? partial : nullptr;
    const dim3 grid(tiles_m * tiles_n, splits);
    if (nterms == 3) {
        static std::atomic<uint64_t> lds_x3{0};
        if (hipError_t e = allow_lds(gemm_bf16x3_slab4_kernel, lds_x3)) return e;
        hipLaunchKernelGGL(gemm_bf16x3_slab4_kernel, grid, dim3(THREADS), kSmem, stream, M, N, nkb,
                           alpha, (const uint8_t*)Ah, (const uint8_t*)Al, (const uint8_t*)Bh,
                           (const uint8_t*)Bl, beta, C, ldc, tiles_m, tiles_n, kbs, P);
    } else {
        static std::atomic<uint64_t> lds_x1{0};
        if (hipError_t e = allow_lds(gemm_bf16_ring_kernel, lds_x1)) return e;
        hipLaunchKernelGGL(gemm_bf16_ring_kernel, grid, dim3(THREADS), kSmem, stream, M, N, nkb,
                           alpha, (const uint8_t*)Ah, (const uint8_t*)Bh, beta, C, ldc, tiles_m,
                           tiles_n, kbs, P);
    }
    return hipGetLastError();
}

hipError_t launch_gemm_bf16x3_grouped(const GroupedMfmaDesc* desc, int count, int total_tiles, int grid,
                                      unsigned* counter, hipStream_t stream) {
    if (total_tiles <= 0) return hipSuccess;
    if (grid < 1 || grid > total_tiles || !counter || !desc || count < 1) return hipErrorInvalidValue;
    static std::atomic<uint64_t> lds_g{0};
    if (hipError_t e = allow_lds(gemm_bf16x3_grouped_kernel, lds_g, kSmem + 16)) return e;
    hipLaunchKernelGGL(grouped_mfma_reset_kernel, dim3(1), dim3(64), 0, stream, counter);
    hipLaunchKernelGGL(gemm_bf16x3_grouped_kernel, dim3(grid), dim3(THREADS), kSmem + 16, stream, desc, count,
                       total_tiles, counter);
    return hipGetLastError();
}

hipError_t launch_gemm_fp8r_tn(int64_t M, int64_t N, int64_t Kp, float alpha, const uint8_t* Aq,
                               const uint8_t* Ar, const uint8_t* Asq, const uint8_t* Asr,
                               const uint8_t* Bq, const uint8_t* Br, const uint8_t* Bsq,
                               const uint8_t* Bsr, float beta, float* C, int64_t ldc, int splits,
                               float* partial, hipStream_t stream) {
    if (Kp % kFp8TileK || Kp <= 0) return hipErrorInvalidValue;
    static std::atomic<uint64_t> lds_f8{0};
    if (hipError_t e = allow_lds(gemm_fp8r_fused_kernel, lds_f8)) return e;
    const int tiles_m = (int)((M + TM - 1) / TM), tiles_n = (int)((N + TN - 1) / TN);
    const int nkb = (int)(Kp / kPanelRowBytes);
    if (splits < 1 || (splits > 1 && !partial)) return hipErrorInvalidValue;
    const int kbs = kb_per_split(nkb, splits);
    if ((int64_t)(splits - 1) * kbs >= nkb) return hipErrorInvalidValue;   // every slice non-empty
    float* P = splits > 1 ? partial : nullptr;
    hipLaunchKernelGGL(gemm_fp8r_fused_kernel, dim3(tiles_m * tiles_n, splits), dim3(THREADS), kSmem,
                       stream, M, N, nkb, alpha, Aq, Ar, Asq, Asr, Bq, Br, Bsq, Bsr, beta, C, ldc,
                       tiles_m, tiles_n, kbs, P);
    return hipGetLastError();
}

hipError_t launch_gemm_fp6x3_tn(int64_t M, int64_t N, int64_t Kp, float alpha, const uint8_t* Ah,
                                const uint8_t* Al, const uint8_t* As, const uint8_t* Bh,
                                const uint8_t* Bl, const uint8_t* Bs, float beta, float* C,
                                int64_t ldc, int splits, float* partial, hipStream_t stream) {
    if (Kp % 64 || Kp <= 0) return hipErrorInvalidValue;
    static std::atomic<uint64_t> lds_f6{0};
    if (hipError_t e = allow_lds(gemm_fp6x3_fused_kernel, lds_f6, kSmemF6)) return e;
    const int tiles_m = (int)((M + TM - 1) / TM), tiles_n = (int)((N + TN - 1) / TN);
    const int nkb = (int)(Kp / 64);               // one image block per 64 K values
    if (splits < 1 || (splits > 1 && !partial)) return hipErrorInvalidValue;
    const int kbs = kb_per_split(nkb, splits);
    if ((int64_t)(splits - 1) * kbs >= nkb) return hipErrorInvalidValue;   // every slice non-empty
    float* P = splits > 1 ? partial : nullptr;
    hipLaunchKernelGGL(gemm_fp6x3_fused_kernel, dim3(tiles_m * tiles_n, splits), dim3(THREADS), kSmemF6,
                       stream, M, N, nkb, alpha, Ah, Al, As, Bh, Bl, Bs, beta, C, ldc, tiles_m, tiles_n, kbs,
                       P);
    return hipGetLastError();
}

}  // namespace cmp
