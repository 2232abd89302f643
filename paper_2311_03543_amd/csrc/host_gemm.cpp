// FP32 GEMM on the host CPU: the computation of the optional host variant
// "host_f32" of the gemm interface (a CPU codelet beside the GPU ones, the
// heterogeneous choice COMPAR's runtime makes between CPU and GPU
// implementations).  It is not a fallback: it runs only when registered and
// selected like any other variant.
//
// C = alpha * A * B + beta * C over row-major FP32 arrays with leading
// dimensions (beta == 0: C is not read).  Each output entry is one FP32
// accumulator over k = 0 .. K-1 in increasing order, so results do not depend
// on the thread count (they do on the CPU: the AVX-512 build may contract the
// multiply-add into an FMA, the baseline build cannot).  Tiles of 32 rows x 256 columns keep their
// accumulators (32 KiB) in the core's cache while a 1 KiB segment of a B row
// is reused by the 32 rows; the column loop is the vector loop.  Row tiles
// are spread over std::threads.
#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

#include "kernels.h"

namespace cmp {
namespace {

constexpr int kIB = 32, kJB = 256;

// One tile of C: rows [i0, i1), columns [j0, j1).  Instantiated once per ISA
// build (the template argument only keeps the two copies apart).
template <int isa>
__attribute__((always_inline)) inline void tile_body(int64_t i0, int64_t i1, int64_t j0, int64_t j1,
                                                     int64_t K, float alpha, const float* A, int64_t lda,
                                                     const float* B, int64_t ldb, float beta, float* C,
                                                     int64_t ldc) {
    alignas(64) float acc[kIB][kJB];
    const int64_t ni = i1 - i0, nj = j1 - j0;
    for (int64_t i = 0; i < ni; ++i)
        for (int64_t j = 0; j < nj; ++j) acc[i][j] = 0.f;
    for (int64_t k = 0; k < K; ++k) {
        const float* b = B + k * ldb + j0;
        for (int64_t i = 0; i < ni; ++i) {
            const float a = A[(i0 + i) * lda + k];
            float* r = acc[i];
            for (int64_t j = 0; j < nj; ++j) r[j] += a * b[j];
        }
    }
    for (int64_t i = 0; i < ni; ++i) {
        float* c = C + (i0 + i) * ldc + j0;
        if (beta != 0.f)
            for (int64_t j = 0; j < nj; ++j) c[j] = alpha * acc[i][j] + beta * c[j];
        else
            for (int64_t j = 0; j < nj; ++j) c[j] = alpha * acc[i][j];
    }
}

// The same body compiled for AVX-512 and for the baseline ISA; the caller
// picks by the running CPU's features.
__attribute__((target("avx512f"))) void tiles_avx512(int64_t t0, int64_t t1, int64_t tj, int64_t M,
                                                      int64_t N, int64_t K, float alpha, const float* A,
                                                      int64_t lda, const float* B, int64_t ldb, float beta,
                                                      float* C, int64_t ldc) {
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t ti = t / tj, j0 = (t % tj) * kJB, i0 = ti * kIB;
        tile_body<0>(i0, std::min(i0 + kIB, M), j0, std::min(j0 + kJB, N), K, alpha, A, lda, B, ldb, beta,
                     C, ldc);
    }
}
void tiles_generic(int64_t t0, int64_t t1, int64_t tj, int64_t M, int64_t N, int64_t K, float alpha,
                   const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                   int64_t ldc) {
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t ti = t / tj, j0 = (t % tj) * kJB, i0 = ti * kIB;
        tile_body<1>(i0, std::min(i0 + kIB, M), j0, std::min(j0 + kJB, N), K, alpha, A, lda, B, ldb, beta,
                     C, ldc);
    }
}

}  // namespace

void host_gemm_f32(int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                   const float* B, int64_t ldb, float beta, float* C, int64_t ldc, int max_threads) {
    if (M <= 0 || N <= 0) return;
    if (alpha == 0.f || K <= 0) {             // BLAS: A and B are not read
        for (int64_t i = 0; i < M; ++i)
            for (int64_t j = 0; j < N; ++j) C[i * ldc + j] = beta != 0.f ? beta * C[i * ldc + j] : 0.f;
        return;
    }
    const int64_t tj = (N + kJB - 1) / kJB, tiles = ((M + kIB - 1) / kIB) * tj;
    const bool wide = __builtin_cpu_supports("avx512f");
    auto run = [&](int64_t t0, int64_t t1) {
        if (wide) tiles_avx512(t0, t1, tj, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
        else tiles_generic(t0, t1, tj, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    };
    // threads only when each gets at least ~2 Mflop: spawning costs tens of microseconds
    const double flop = 2.0 * (double)M * (double)N * (double)K;
    int nt = (int)std::min<int64_t>({(int64_t)std::max(max_threads, 1), tiles, (int64_t)(flop / 2e6) + 1});
    if (nt <= 1) {
        run(0, tiles);
        return;
    }
    std::vector<std::thread> pool;
    pool.reserve(nt - 1);
    const int64_t per = (tiles + nt - 1) / nt;
    for (int w = 1; w < nt; ++w) {
        const int64_t t0 = w * per, t1 = std::min(tiles, t0 + per);
        if (t0 < t1) pool.emplace_back(run, t0, t1);
    }
    run(0, std::min(tiles, per));
    for (auto& th : pool) th.join();
}

}  // namespace cmp
