// FP32 SIMT GEMM for gfx950: C = alpha * A * B + beta * C, row-major, any
// shape and leading dimension.  The plain-precision variant of the "gemm"
// interface: every product and sum is an FP32 FMA on the vector ALUs.
//
// Tiling: a workgroup of 256 lanes (4 wave64) owns a 128 x 128 tile of C and
// walks K in steps of 16.  Each step's A tile (128 x 16) and B tile (16 x 128)
// are read from global memory with 16-byte loads where alignment allows,
// staged in LDS (A stored k-major so a lane's 8 row values are two 16-byte LDS
// reads), double-buffered so the next step's global loads are in flight while
// the current step computes.  Each lane accumulates an 8 x 8 block of C in
// registers (rows ty*4+{0..3} and 64+ty*4+{0..3}, columns likewise with tx),
// which keeps LDS reads conflict-free: the 16 lanes sharing ty read one
// broadcast address, and the B reads of a wave cover 256 contiguous bytes.
#include "common.h"
#include "kernels.h"

namespace cmp {
namespace {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int APAD = 4;                 // As row stride 132 floats (keeps 16-byte alignment)
constexpr int THREADS = 256;

template <bool VEC>
__device__ __forceinline__ void load_a(const float* __restrict__ A, int64_t lda, int64_t M,
                                       int64_t K, int64_t m0, int64_t k0, int t, float4 (&ra)[2]) {
    // 128 rows x 16 k = 512 float4; lane t takes rows t/4 and t/4 + 64, k-quad t%4.
    const int kq = (t & 3) * 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t row = m0 + (t >> 2) + h * 64;
        const int64_t k = k0 + kq;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < M) {
            const float* p = A + row * lda + k;
            if (VEC && k + 3 < K) {
                v = *reinterpret_cast<const float4*>(p);
            } else {
                if (k + 0 < K) v.x = p[0];
                if (k + 1 < K) v.y = p[1];
                if (k + 2 < K) v.z = p[2];
                if (k + 3 < K) v.w = p[3];
            }
        }
        ra[h] = v;
    }
}

template <bool VEC>
__device__ __forceinline__ void load_b(const float* __restrict__ B, int64_t ldb, int64_t K,
                                       int64_t N, int64_t k0, int64_t n0, int t, float4 (&rb)[2]) {
    // 16 k x 128 cols = 512 float4; lane t takes k-rows t/32 and t/32 + 8, column quad t%32.
    const int64_t col = n0 + (t & 31) * 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t k = k0 + (t >> 5) + h * 8;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k < K) {
            const float* p = B + k * ldb + col;
            if (VEC && col + 3 < N) {
                v = *reinterpret_cast<const float4*>(p);
            } else {
                if (col + 0 < N) v.x = p[0];
                if (col + 1 < N) v.y = p[1];
                if (col + 2 < N) v.z = p[2];
                if (col + 3 < N) v.w = p[3];
            }
        }
        rb[h] = v;
    }
}

__device__ __forceinline__ void store_tiles(float (*As)[BM + APAD], float (*Bs)[BN], int t,
                                            const float4 (&ra)[2], const float4 (&rb)[2]) {
    const int kq = (t & 3) * 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = (t >> 2) + h * 64;
        As[kq + 0][r] = ra[h].x;
        As[kq + 1][r] = ra[h].y;
        As[kq + 2][r] = ra[h].z;
        As[kq + 3][r] = ra[h].w;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = (t >> 5) + h * 8;
        *reinterpret_cast<float4*>(&Bs[k][(t & 31) * 4]) = rb[h];
    }
}

template <bool VEC>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(2))) void gemm_f32_simt_kernel(
    int64_t M, int64_t N, int64_t K, float alpha, const float* __restrict__ A, int64_t lda,
    const float* __restrict__ B, int64_t ldb, float beta, float* __restrict__ C, int64_t ldc,
    int tiles_m, int tiles_n) {
    __shared__ __attribute__((aligned(16))) float As[2][BK][BM + APAD];
    __shared__ __attribute__((aligned(16))) float Bs[2][BK][BN];

    const int t = threadIdx.x;
    const int nb = tiles_m * tiles_n;
    int tm, tn;
    grouped_tile(xcd_remap(blockIdx.x, nb), tiles_m, tiles_n, 8, tm, tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int tx = t & 15, ty = t >> 4;

    float acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = 0.f;

    const int nk = (int)((K + BK - 1) / BK);
    float4 ra[2], rb[2];
    if (nk > 0) {
        load_a<VEC>(A, lda, M, K, m0, 0, t, ra);
        load_b<VEC>(B, ldb, K, N, 0, n0, t, rb);
        store_tiles(As[0], Bs[0], t, ra, rb);
    }
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) {
            load_a<VEC>(A, lda, M, K, m0, (int64_t)(kt + 1) * BK, t, ra);
            load_b<VEC>(B, ldb, K, N, (int64_t)(kt + 1) * BK, n0, t, rb);
        }
#pragma unroll 2
        for (int k = 0; k < BK; ++k) {
            const float4 a0 = *reinterpret_cast<const float4*>(&As[cur][k][ty * 4]);
            const float4 a1 = *reinterpret_cast<const float4*>(&As[cur][k][64 + ty * 4]);
            const float4 b0 = *reinterpret_cast<const float4*>(&Bs[cur][k][tx * 4]);
            const float4 b1 = *reinterpret_cast<const float4*>(&Bs[cur][k][64 + tx * 4]);
            const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
            const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_fmaf(av[i], bv[j], acc[i][j]);
        }
        if (more) store_tiles(As[cur ^ 1], Bs[cur ^ 1], t, ra, rb);
        __syncthreads();
    }

    // Epilogue: C = alpha * acc + beta * C (C not read when beta == 0).
    const bool cvec = ((ldc & 3) == 0) && ((reinterpret_cast<uintptr_t>(C) & 15) == 0);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t row = m0 + (i < 4 ? ty * 4 + i : 64 + ty * 4 + (i - 4));
        if (row >= M) continue;
        float* crow = C + row * ldc;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t col = n0 + h * 64 + tx * 4;
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = alpha * acc[i][h * 4 + j];
            if (cvec && col + 3 < N) {
                float4* p = reinterpret_cast<float4*>(crow + col);
                if (beta != 0.f) {
                    const float4 o = *p;
                    v[0] = __builtin_fmaf(beta, o.x, v[0]);
                    v[1] = __builtin_fmaf(beta, o.y, v[1]);
                    v[2] = __builtin_fmaf(beta, o.z, v[2]);
                    v[3] = __builtin_fmaf(beta, o.w, v[3]);
                }
                *p = make_float4(v[0], v[1], v[2], v[3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (col + j < N) {
                        float o = v[j];
                        if (beta != 0.f) o = __builtin_fmaf(beta, crow[col + j], o);
                        crow[col + j] = o;
                    }
                }
            }
        }
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

}  // namespace

hipError_t launch_gemm_f32_simt(int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                                int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                                int64_t ldc, hipStream_t stream) {
    const int tiles_m = (int)((M + BM - 1) / BM), tiles_n = (int)((N + BN - 1) / BN);
    const int nb = tiles_m * tiles_n;
    if (nb == 0) return hipSuccess;
    const bool vec = (lda % 4 == 0) && (ldb % 4 == 0) &&
                     ((reinterpret_cast<uintptr_t>(A) & 15) == 0) &&
                     ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
    if (vec)
        hipLaunchKernelGGL(gemm_f32_simt_kernel<true>, dim3(nb), dim3(THREADS), 0, stream, M, N,
                           K, alpha, A, lda, B, ldb, beta, C, ldc, tiles_m, tiles_n);
    else
        hipLaunchKernelGGL(gemm_f32_simt_kernel<false>, dim3(nb), dim3(THREADS), 0, stream, M,
                           N, K, alpha, A, lda, B, ldb, beta, C, ldc, tiles_m, tiles_n);
    return hipGetLastError();
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
