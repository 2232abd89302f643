// Internal launch interface between the host runtime (runtime.cpp) and the
// gfx950 kernels.  Every launch_* function only enqueues work on `stream` and
// returns the hipError_t of the launch; shapes are validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace cmp {

// ---- FP32 GEMM on the host CPU (host_gemm.cpp) ------------------------------
// C = alpha * A * B + beta * C over host arrays (beta == 0: C not read), row
// tiles over at most max_threads threads.  Synchronous.
void host_gemm_f32(int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                   const float* B, int64_t ldb, float beta, float* C, int64_t ldc, int max_threads);

// ---- FP32 SIMT GEMM (vector-ALU FMA, LDS-staged tiles) -------------------
hipError_t launch_gemm_f32_simt(int64_t M, int64_t N, int64_t K, float alpha,
                                const float* A, int64_t lda, const float* B, int64_t ldb,
                                float beta, float* C, int64_t ldc, hipStream_t stream);

// Grouped FP32 SIMT launch over many problems of uneven shapes.  The
// descriptor array (device memory) lists the problems in launch order with
// the first tile index of each (prefix sum of tiles_m * tiles_n); `grid`
// persistent workgroups stride over all `total_tiles`.  `vec` marks problems
// whose A and B allow 16-byte loads (lda, ldb multiples of 4, 16-byte aligned).
struct GroupedDesc {
    int64_t M, N, K, lda, ldb, ldc;
    float alpha, beta;
    const float* A;
    const float* B;
    float* C;
    int tiles_n, tile_start, vec, pad;
};
struct GroupedConfig {
    int bm, bn, bk;
};
// One problem of a grouped bf16x3 launch: the operands, the problem's
// bf16 hi / lo panel images (Mp x Kp of A, Np x Kp of B^T, in the plan's
// workspace), the pre-pass workgroups of A (ga) and B (gb) from pre_start on,
// and the problem's 256 x 256 tiles from tile_start on.  vec: bit 0 A, bit 1 B
// can be read with 16-byte loads.
struct GroupedMfmaDesc {
    int64_t M, N, K, lda, ldb, ldc, Mp, Np, Kp;
    float alpha, beta;
    const float* A;
    const float* B;
    float* C;
    uint16_t *ah, *al, *bh, *bl;
    int ga, gb, pre_start, tile_start, tiles_n, vec;
};
constexpr int kNumGroupedConfigs = 10;
extern const GroupedConfig kGroupedConfigs[kNumGroupedConfigs];
// One persistent launch over the problems of `desc` (tile list in desc order,
// 1 <= grid <= total_tiles workgroups), preceded by a one-lane kernel that
// zeroes `counter` (device, 4 bytes), the tile queue the workgroups claim from;
// launches of one counter must not overlap.
// Grouped bf16x3: the hi / lo images of every problem in one launch (pre_total
// workgroups), then every problem's tiles in one persistent launch.
hipError_t launch_split_grouped(const GroupedMfmaDesc* desc, int count, int64_t pre_total,
                                hipStream_t stream);
hipError_t launch_gemm_bf16x3_grouped(const GroupedMfmaDesc* desc, int count, int total_tiles, int grid,
                                      unsigned* counter, hipStream_t stream);
hipError_t launch_gemm_f32_grouped(int config, const GroupedDesc* desc, int count, int total_tiles,
                                   int grid, unsigned* counter, hipStream_t stream);
// Resident workgroups per CU of the grouped kernel for a configuration.
int grouped_blocks_per_cu(int config);

// C = beta * C (or 0 when beta == 0) for the alpha == 0 / K == 0 cases.
hipError_t launch_scale_c(int64_t M, int64_t N, float beta, float* C, int64_t ldc,
                          hipStream_t stream);

// ---- operand pre-pass -------------------------------------------------------
// Padded, K-contiguous operand images used by the MFMA kernels, in the panel
// layout of common.h (Mp, Np multiples of 256, Kp a multiple of 64):
//   A  (M x K, ld lda)  ->  Ah / Al  (Mp rows x Kp bf16)
//   B  (K x N, ld ldb)  ->  Bh / Bl  (Np rows x Kp bf16, i.e. B transposed)
// Padding rows / columns are zero.  Both operands' images come from one
// launch (al and bl both null: hi images only, the one-term bf16 variant).
hipError_t launch_split_bf16_pair(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                                 const float* B, int64_t ldb, int64_t Mp, int64_t Np, int64_t Kp,
                                 uint16_t* ah, uint16_t* al, uint16_t* bh, uint16_t* bl,
                                 hipStream_t stream);
// Plain bf16 split of a row-major matrix, tight output (bit-exact checking).
hipError_t launch_split_bf16_plain(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                                   uint16_t* hi, uint16_t* lo, hipStream_t stream);

// E4M3 tile quantisation with one residual pass, 128 x 128 tiles.
//   transpose = false: X is rows x cols (ld ldx); q/rq are out_rows x out_cols with
//                      out_rows >= rows, out_cols >= cols (row-major, ld out_cols,
//                      or with tiled = true a panel image, out_rows % 256 == 0);
//                      scales are indexed [row_tile * (out_cols/128) + col_tile].
//   transpose = true:  q/rq receive X transposed (out_rows >= cols, out_cols >= rows),
//                      scales indexed [col_tile_of_X * (out_cols/128) + row_tile_of_X].
// Padding in q/rq is written as zero codes (scale bytes of all-padding tiles 127).
hipError_t launch_quant_fp8(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                            bool transpose, bool tiled, int64_t out_rows, int64_t out_cols,
                            uint8_t* q, uint8_t* qscale, uint8_t* rq, uint8_t* rscale,
                            hipStream_t stream);

// Both operands' tiled FP8 images in one launch, as launch_quant_fp8 with
// tiled = true gives them: A (M x K, lda) into Mp x Kp codes, B (K x N, ldb)
// transposed into Np x Kp codes, with their scale arrays.
hipError_t launch_quant_fp8_pair(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                                const float* B, int64_t ldb, int64_t Mp, int64_t Np, int64_t Kp,
                                uint8_t* aq, uint8_t* aqs, uint8_t* ar, uint8_t* ars, uint8_t* bq,
                                uint8_t* bqs, uint8_t* br, uint8_t* brs, hipStream_t stream);

// MX E2M3 quantisation with one residual level, one E8M0 scale per 32 K values.
//   transpose = false: X is rows x cols, blocks along its rows (K = cols), one
//                      output row per row of X.
//   transpose = true:  X is rows x cols = K x N, blocks along its columns
//                      (K = rows), one output row per column of X.
//   tiled = true:  q / rq / qscale are the hi-code, lo-code and scale arrays
//                  of an MX FP6 image (common.h) of out_rows rows (>= the
//                  output rows, a multiple of 256) and Kp K values (>= K, a
//                  multiple of 64); rscale unused.
//   tiled = false: one code per byte, row-major (output rows x K), scale
//                  bytes output rows x ceil(K / 32); out_rows, Kp unused.
// Both operands' tiled MX FP6 images in one launch, as launch_quant_mx6 with
// tiled = true gives them: A (M x K, lda) into Mp rows (codes aq / ar, scales
// as), B (K x N, ldb) transposed into Np rows (bq / br / bs), Kp K values.
hipError_t launch_quant_mx6_pair(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                                const float* B, int64_t ldb, int64_t Mp, int64_t Np, int64_t Kp,
                                uint8_t* aq, uint8_t* ar, uint8_t* as, uint8_t* bq, uint8_t* br,
                                uint8_t* bs, hipStream_t stream);
hipError_t launch_quant_mx6(int64_t rows, int64_t cols, const float* X, int64_t ldx,
                            bool transpose, bool tiled, int64_t out_rows, int64_t Kp, uint8_t* q,
                            uint8_t* qscale, uint8_t* rq, uint8_t* rscale, hipStream_t stream);

// ---- MFMA GEMMs over pre-pass images -------------------------------------
// bf16: C = alpha * sum_t A_t * B_t^T + beta * C over `nterms` (1 or 3) operand
// pairs (t = 0: hi*hi, 1: hi*lo, 2: lo*hi); Ah/Al are Mp x Kp, Bh/Bl Np x Kp.
// splits > 1 cuts K into that many slices (split-K, every slice non-empty:
// splits <= Kp / 32 and splits_for() below gives such a count): slice s then
// writes its raw sum (alpha and beta not applied, C untouched) to
// partial + s * M * N (M x N, row-major), and launch_splitk_reduce finishes C.
hipError_t launch_gemm_bf16_tn(int64_t M, int64_t N, int64_t Kp, int nterms, float alpha,
                               const uint16_t* Ah, const uint16_t* Al,
                               const uint16_t* Bh, const uint16_t* Bl,
                               float beta, float* C, int64_t ldc, int splits, float* partial,
                               hipStream_t stream);
// fp8 with refinement: C = alpha * (Aq.Bq + Ar.Bq + Aq.Br + Ar.Br) + beta * C,
// each operand dequantised by its 128 x 128 tile's E8M0 scale byte; splits and
// partial as above (K slices of 64-byte blocks, splits <= Kp / 64).
hipError_t launch_gemm_fp8r_tn(int64_t M, int64_t N, int64_t Kp, float alpha,
                               const uint8_t* Aq, const uint8_t* Ar,
                               const uint8_t* Asq, const uint8_t* Asr,
                               const uint8_t* Bq, const uint8_t* Br,
                               const uint8_t* Bsq, const uint8_t* Bsr,
                               float beta, float* C, int64_t ldc, int splits, float* partial,
                               hipStream_t stream);

// MX FP6 with one residual level: C = alpha * (Ah.Bh + Ah.Bl + Al.Bh) + beta * C
// over the MX FP6 images of launch_quant_mx6 (codes Ah / Al and scales As of
// Mp rows, Bh / Bl / Bs of Np rows, Kp K values, Kp % 64 == 0); splits and
// partial as above (splits <= Kp / 64).
hipError_t launch_gemm_fp6x3_tn(int64_t M, int64_t N, int64_t Kp, float alpha, const uint8_t* Ah,
                                const uint8_t* Al, const uint8_t* As, const uint8_t* Bh,
                                const uint8_t* Bl, const uint8_t* Bs, float beta, float* C,
                                int64_t ldc, int splits, float* partial, hipStream_t stream);

// C = alpha * (partial[0] + ... + partial[splits - 1]) + beta * C, summed in
// that order (beta == 0 never reads C); splits >= 2.
hipError_t launch_splitk_reduce(int64_t M, int64_t N, int splits, const float* partial, float alpha,
                                float beta, float* C, int64_t ldc, hipStream_t stream);

// Split-K count for an M x N product over nkb K blocks of kKBlockBytes.
// A workgroup owns one 256 x 256 tile and spends `step_ns` per K block; with
// fewer tiles than CUs, cutting K into s slices shortens the longest
// workgroup from nkb to ceil(nkb / s) blocks (while tiles * s still fits the
// CUs) but costs 2 (s - 1) M N floats of partial-sum traffic plus one
// reduction launch.  The count minimises that estimate, keeps at least 4 K
// blocks per slice (the copy ring is 4 stages deep) and every slice
// non-empty.  1 = no split.
inline int splits_for(int64_t M, int64_t N, int nkb, double step_ns, int cus = 256) {
    const int64_t tiles = ((M + 255) / 256) * ((N + 255) / 256);
    if (tiles >= cus || nkb < 8) return 1;
    const double bytes_per_ns = 4000.0;         // partial sums, mostly L2 / MALL resident
    const double launch_ns = 3000.0;
    auto cost = [&](int64_t s) {
        const int64_t kbs = (nkb + s - 1) / s;
        const int64_t waves = (tiles * s + cus - 1) / cus;
        double t = (double)(waves * kbs) * step_ns;
        if (s > 1) t += 2.0 * (double)(s - 1) * (double)M * (double)N * 4.0 / bytes_per_ns + launch_ns;
        return t;
    };
    int64_t best = 1;
    double best_t = cost(1);
    for (int64_t s = 2; s * tiles <= cus && s <= nkb / 4; ++s) {
        const double t = cost(s);
        if (t < best_t) best = s, best_t = t;
    }
    const int kbs = (int)((nkb + best - 1) / best);
    return (nkb + kbs - 1) / kbs;
}
// Measured K-block step of one workgroup on MI355X at 8192^3 (ns): one
// bf16 product, three bf16 products, four fp8 products.
constexpr double kStepNsBf16 = 790.0, kStepNsBf16x3 = 2100.0, kStepNsFp8r = 2500.0;
// three FP6 products per 64 K values: the MFMA work of 1.5 bf16 K blocks
constexpr double kStepNsFp6x3 = 1.5 * kStepNsBf16;

// Tile sizes the MFMA kernels assume for padding.
constexpr int kMfmaTileM = 256;
constexpr int kMfmaTileN = 256;
constexpr int kBf16TileK = 64;
constexpr int kFp8TileK = 128;
constexpr int kKBlockBytes = 64;   // bytes of K per operand-image block (split-K unit)
// MX FP6 image blocks (256 rows x 64 K values): codes per level, scales (both levels)
constexpr int kMx6CodeBlockBytes = 256 * 48, kMx6ScaleBlockBytes = 1024;

// ---- FP64 Freivalds probe -------------------------------------------------
// out[0] = ||C x - (alpha A (B x) + beta C0 x)||^2, out[1] = ||alpha A(Bx) + beta C0 x||^2.
// x: N doubles on the device; ws: at least (K + 2) doubles; out: 2 doubles (device).
hipError_t launch_freivalds(int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                            int64_t lda, const float* B, int64_t ldb, float beta,
                            const float* C0, int64_t ldc0, const float* C, int64_t ldc,
                            const double* x, double* ws, double* out, hipStream_t stream);
// x[j] = +-1 from splitmix64(seed + j): the top bit set gives -1.
hipError_t launch_rademacher(int64_t n, uint64_t seed, double* x, hipStream_t stream);

// ---- selector network -------------------------------------------------------
// Parameters are 4740 floats (see compar.h).  Training runs `steps` Adam steps
// in one resident workgroup; X, Y standardised (n x 4) device arrays.
constexpr int kMlpParams = 4 * 64 + 64 + 64 * 64 + 64 + 64 * 4 + 4;
constexpr int kMlpMaxRows = 8192;
// partial-gradient scratch: one (params + loss) record per 32-row workgroup
constexpr int kMlpPartFloats = (kMlpMaxRows / 32) * (kMlpParams + 1);
hipError_t launch_mlp_train(int n, const float* X, const float* Y, float* params, float* m,
                            float* v, float* part, int steps, int t0, float lr, float* loss_trace,
                            float* grad_out, hipStream_t stream);
hipError_t launch_mlp_infer(int n, const float* X, const float* params, float* Y,
                            hipStream_t stream);

}  // namespace cmp
