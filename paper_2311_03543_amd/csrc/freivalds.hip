// FP64 residual probe of a finished product (verify mode).  With a probe
// vector x of +-1 entries, y = B x, z = alpha A y + beta C0 x and w = C x;
// since E||E x||^2 = ||E||_F^2 for Rademacher x, ||w - z|| / ||z|| estimates
// the relative Frobenius error of C without forming A B.  Three passes, each
// reading its matrix once (HBM-bound), all arithmetic in FP64.
#include "common.h"
#include "kernels.h"

namespace cmp {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// One wave per row: y[k] = sum_j B[k][j] x[j].  Block 0 also clears out[].
__global__ __launch_bounds__(256) void bx_kernel(int64_t K, int64_t N, const float* __restrict__ B,
                                                 int64_t ldb, const double* __restrict__ x,
                                                 double* __restrict__ y, double* __restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x < 2) out[threadIdx.x] = 0.0;
    const int lane = threadIdx.x & 63;
    for (int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); k < K; k += (int64_t)gridDim.x * 4) {
        const float* row = B + k * ldb;
        double s = 0.0;
        for (int64_t j = lane; j < N; j += 64) s += (double)row[j] * x[j];
        s = wave_sum(s);
        if (lane == 0) y[k] = s;
    }
}

// One wave per row i of C: accumulates (w_i - z_i)^2 and z_i^2 into out[0..1].
__global__ __launch_bounds__(256) void rows_kernel(int64_t M, int64_t N, int64_t K, float alpha,
                                                   const float* __restrict__ A, int64_t lda,
                                                   float beta, const float* __restrict__ C0,
                                                   int64_t ldc0, const float* __restrict__ C,
                                                   int64_t ldc,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    double dd = 0.0, zz = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < M; i += (int64_t)gridDim.x * 4) {
        double za = 0.0, w = 0.0, c0 = 0.0;
        if (alpha != 0.f)
            for (int64_t k = lane; k < K; k += 64) za += (double)A[i * lda + k] * y[k];
        for (int64_t j = lane; j < N; j += 64) {
            w += (double)C[i * ldc + j] * x[j];
            if (beta != 0.f) c0 += (double)C0[i * ldc0 + j] * x[j];
        }
        za = wave_sum(za);
        w = wave_sum(w);
        c0 = wave_sum(c0);
        const double z = (double)alpha * za + (double)beta * c0;
        dd += (w - z) * (w - z);
        zz += z * z;
    }
    if (lane == 0) {
        atomicAdd(&out[0], dd);
        atomicAdd(&out[1], zz);
    }
}

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
    uint64_t z = seed + (j + 1) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ void rademacher_kernel(int64_t n, uint64_t seed, double* __restrict__ x) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        x[j] = (splitmix64_at(seed, (uint64_t)j) >> 63) ? -1.0 : 1.0;
}

unsigned waves_grid(int64_t rows) {
    int64_t b = (rows + 3) / 4;
    if (b > 8192) b = 8192;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_freivalds(int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                            int64_t lda, const float* B, int64_t ldb, float beta, const float* C0,
                            int64_t ldc0, const float* C, int64_t ldc, const double* x, double* ws,
                            double* out, hipStream_t stream) {
    double* y = ws;
    hipLaunchKernelGGL(bx_kernel, dim3(waves_grid(K)), dim3(256), 0, stream,
                       (alpha != 0.f) ? K : (int64_t)0, N, B, ldb, x, y, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rows_kernel, dim3(waves_grid(M)), dim3(256), 0, stream, M, N, K, alpha, A,
                       lda, beta, C0, ldc0, C, ldc, x, y, out);
    return hipGetLastError();
}

hipError_t launch_rademacher(int64_t n, uint64_t seed, double* x, hipStream_t stream) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(rademacher_kernel, dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, stream, n,
                       seed, x);
    return hipGetLastError();
}

}  // namespace cmp
