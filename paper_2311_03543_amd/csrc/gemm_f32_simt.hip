// FP32 SIMT GEMM for gfx950: C = alpha * A * B + beta * C, row-major, any
// shape and leading dimension.  The plain-precision variant of the "gemm"
// interface: every product and sum is an FP32 FMA on the vector ALUs.
//
// Two launch forms share the tile code of simt_tile.h:
//   - one problem: a tile per workgroup, tiles renumbered so each XCD works
//     on a contiguous, L2-friendly block of C.  The tile is the largest of
//     128 x 256, 128 x 128, 64 x 128 and 64 x 64 (K step 16) that still gives
//     every CU two tiles (the smallest when none does): on MI355X a 128 x 256
//     tile streams 91-93 TFLOP/s at 4096^2..8192^2 against 81-87 for
//     128 x 128, and at 2048^2 64 x 128 tiles (512 of them) 58 against 42;
//   - a group of problems of uneven shapes: one persistent launch whose
//     workgroups claim tiles of the concatenated tile list of all problems
//     from a counter as they go (problems sorted by decreasing K, so the
//     longest tiles go first and the tail is short), with the tile shape
//     picked per group by the autotuner from kGroupedConfigs.
#include "common.h"
#include "kernels.h"
#include "simt_tile.h"

namespace cmp {
namespace {

using CfgL = SimtCfg<128, 256, 16, 8, 16>;
using Cfg128 = SimtCfg<128, 128, 16, 8, 8>;
using CfgM = SimtCfg<64, 128, 16, 4, 8>;
using CfgS = SimtCfg<64, 64, 16, 4, 4>;

template <typename Cfg, bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_f32_simt_kernel(
    SimtProblem p, int tiles_m, int tiles_n) {
    __shared__ __attribute__((aligned(16))) float smem[Cfg::SMEM_FLOATS];
    int tm, tn;
    grouped_tile(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
    simt_tile<Cfg, VEC>(p, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN, smem);
}

// Persistent grouped kernel over the concatenated tile list (tile_start[p] is
// the first tile of problem p; problems come in decreasing order of per-tile
// work).  Workgroup b starts with tile b; each workgroup that finishes a tile
// takes the next unclaimed one from the counter (tile grid + ticket), so the
// list is served greedily in order, longest tiles first.  Every workgroup
// leaves once a claim passes the end of the list.  The counter must be zero
// at launch (grouped_reset_kernel runs right before on the same stream).
__global__ void grouped_reset_kernel(unsigned* counter) {
    if (threadIdx.x == 0) *counter = 0u;
}

template <typename Cfg>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_f32_grouped_kernel(
    const GroupedDesc* __restrict__ desc, int count, int total_tiles, unsigned* __restrict__ counter) {
    __shared__ __attribute__((aligned(16))) float smem[Cfg::SMEM_FLOATS];
    __shared__ int next_tile;
    for (int tile = blockIdx.x; tile < total_tiles;) {
        // last problem whose first tile is <= tile (binary search, wave-uniform)
        typedef const __attribute__((address_space(1))) GroupedDesc* gdesc;
        const gdesc dg = (gdesc)desc;
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (dg[mid].tile_start <= tile) lo = mid;
            else hi = mid - 1;
        }
        const int tiles_n = dg[lo].tiles_n;
        const int local = tile - dg[lo].tile_start;
        const int tm = local / tiles_n, tn = local - (local / tiles_n) * tiles_n;
        const SimtProblem p{dg[lo].M, dg[lo].N, dg[lo].K, dg[lo].lda, dg[lo].ldb, dg[lo].ldc,
                            dg[lo].alpha, dg[lo].beta, dg[lo].A, dg[lo].B, dg[lo].C};
        const bool vec = dg[lo].vec != 0;
        if (vec)
            simt_tile<Cfg, true>(p, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN, smem);
        else
            simt_tile<Cfg, false>(p, (int64_t)tm * Cfg::BM, (int64_t)tn * Cfg::BN, smem);
        __syncthreads();  // LDS is reused by the next tile; next_tile read by every lane
        if (threadIdx.x == 0) {
            const unsigned ticket = atomicAdd(counter, 1u);
            const unsigned left = (unsigned)total_tiles - gridDim.x;   // grid <= total_tiles
            next_tile = ticket < left ? (int)(gridDim.x + ticket) : total_tiles;
        }
        __syncthreads();
        tile = next_tile;
    }
}

__global__ void scale_c_kernel(int64_t M, int64_t N, float beta, float* __restrict__ C,
                               int64_t ldc) {
    const int64_t total = M * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / N, j = e - i * N;
        float* p = C + i * ldc + j;
        *p = (beta == 0.f) ? 0.f : beta * *p;
    }
}

template <typename Cfg>
hipError_t launch_grouped_cfg(const GroupedDesc* desc, int count, int total_tiles, int grid,
                              unsigned* counter, hipStream_t stream) {
    hipLaunchKernelGGL(grouped_reset_kernel, dim3(1), dim3(64), 0, stream, counter);
    hipLaunchKernelGGL(gemm_f32_grouped_kernel<Cfg>, dim3(grid), dim3(256), 0, stream, desc, count,
                       total_tiles, counter);
    return hipGetLastError();
}

}  // namespace

const GroupedConfig kGroupedConfigs[kNumGroupedConfigs] = {
    {64, 64, 16}, {64, 64, 32}, {64, 128, 16}, {128, 64, 16},
    {128, 128, 16}, {128, 128, 32}, {256, 128, 16}, {128, 256, 16},
    {64, 64, 64}, {64, 128, 64},
};

hipError_t launch_gemm_f32_grouped(int config, const GroupedDesc* desc, int count, int total_tiles,
                                   int grid, unsigned* counter, hipStream_t stream) {
    if (total_tiles <= 0) return hipSuccess;
    if (grid < 1 || grid > total_tiles || !counter) return hipErrorInvalidValue;
    switch (config) {
        case 0: return launch_grouped_cfg<SimtCfg<64, 64, 16, 4, 4>>(desc, count, total_tiles, grid, counter, stream);
        case 1: return launch_grouped_cfg<SimtCfg<64, 64, 32, 4, 4>>(desc, count, total_tiles, grid, counter, stream);
        case 2: return launch_grouped_cfg<SimtCfg<64, 128, 16, 4, 8>>(desc, count, total_tiles, grid, counter, stream);
        case 3: return launch_grouped_cfg<SimtCfg<128, 64, 16, 8, 4>>(desc, count, total_tiles, grid, counter, stream);
        case 4: return launch_grouped_cfg<SimtCfg<128, 128, 16, 8, 8>>(desc, count, total_tiles, grid, counter, stream);
        case 5: return launch_grouped_cfg<SimtCfg<128, 128, 32, 8, 8>>(desc, count, total_tiles, grid, counter, stream);
        case 6: return launch_grouped_cfg<SimtCfg<256, 128, 16, 16, 8>>(desc, count, total_tiles, grid, counter, stream);
        case 7: return launch_grouped_cfg<SimtCfg<128, 256, 16, 8, 16>>(desc, count, total_tiles, grid, counter, stream);
        case 8: return launch_grouped_cfg<SimtCfg<64, 64, 64, 4, 4>>(desc, count, total_tiles, grid, counter, stream);
        case 9: return launch_grouped_cfg<SimtCfg<64, 128, 64, 4, 8>>(desc, count, total_tiles, grid, counter, stream);
        default: return hipErrorInvalidValue;
    }
}

int grouped_blocks_per_cu(int config) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (config) {
        case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_grouped_kernel<SimtCfg<64, 64, 16, 4, 4>>, 256, 0); break;
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_grouped_kernel<SimtCfg<64, 64, 32, 4, 4>>, 256, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_grouped_kernel<SimtCfg<64, 128, 16, 4, 8>>, 256, 0); break;
        case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_grouped_kernel<SimtCfg<128, 64, 16, 8, 4>>, 256, 0); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_grouped_kernel<SimtCfg<128, 128, 16, 8, 8>>, 256, 0); break;
        case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_grouped_kernel<SimtCfg<128, 128, 32, 8, 8>>, 256, 0); break;
        case 6: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_grouped_kernel<SimtCfg<256, 128, 16, 16, 8>>, 256, 0); break;
        case 7: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_grouped_kernel<SimtCfg<128, 256, 16, 8, 16>>, 256, 0); break;
        case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_grouped_kernel<SimtCfg<64, 64, 64, 4, 4>>, 256, 0); break;
        case 9: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_f32_grouped_kernel<SimtCfg<64, 128, 64, 4, 8>>, 256, 0); break;
        default: break;
    }
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

template <typename Cfg>
hipError_t launch_simt(const SimtProblem& p, bool vec, hipStream_t stream) {
    const int tiles_m = (int)((p.M + Cfg::BM - 1) / Cfg::BM);
    const int tiles_n = (int)((p.N + Cfg::BN - 1) / Cfg::BN);
    const int nb = tiles_m * tiles_n;
    if (nb == 0) return hipSuccess;
    if (vec)
        hipLaunchKernelGGL((gemm_f32_simt_kernel<Cfg, true>), dim3(nb), dim3(256), 0, stream, p, tiles_m, tiles_n);
    else
        hipLaunchKernelGGL((gemm_f32_simt_kernel<Cfg, false>), dim3(nb), dim3(256), 0, stream, p, tiles_m, tiles_n);
    return hipGetLastError();
}

template <typename Cfg>
int64_t simt_tiles(int64_t M, int64_t N) {
    return ((M + Cfg::BM - 1) / Cfg::BM) * ((N + Cfg::BN - 1) / Cfg::BN);
}

hipError_t launch_gemm_f32_simt(int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                                int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                                int64_t ldc, hipStream_t stream) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const bool vec = (lda % 4 == 0) && (ldb % 4 == 0) &&
                     ((reinterpret_cast<uintptr_t>(A) & 15) == 0) &&
                     ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
    const SimtProblem p{M, N, K, lda, ldb, ldc, alpha, beta, A, B, C};
    constexpr int64_t kWant = 2 * 256;   // two tiles for each of the 256 CUs
    if (simt_tiles<CfgL>(M, N) >= kWant) return launch_simt<CfgL>(p, vec, stream);
    if (simt_tiles<Cfg128>(M, N) >= kWant) return launch_simt<Cfg128>(p, vec, stream);
    if (simt_tiles<CfgM>(M, N) >= kWant) return launch_simt<CfgM>(p, vec, stream);
    return launch_simt<CfgS>(p, vec, stream);
}

hipError_t launch_scale_c(int64_t M, int64_t N, float beta, float* C, int64_t ldc,
                          hipStream_t stream) {
    const int64_t total = M * N;
    if (total == 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(scale_c_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, M, N, beta,
                       C, ldc);
    return hipGetLastError();
}

}  // namespace cmp
