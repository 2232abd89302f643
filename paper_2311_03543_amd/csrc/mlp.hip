// The learned selector's network on the GPU: 4 -> 64 (ReLU) -> 64 (ReLU) -> 4,
// MSE loss over all outputs, full-batch Adam.  Parameters are packed layer by
// layer as [W (out x in, row-major), b (out)] (4740 floats).
//
// Layout of the work: one wave64 evaluates one sample at a time with lane j
// owning hidden unit j of both hidden layers, so a layer's 64 x 64 product is
// 64 lane-parallel dot products whose broadcast operand comes from
// v_readlane (no LDS round trip).  Weights live in LDS (W2 both row-major and
// transposed, so both the forward and the backward product read a contiguous
// row across the wave).  Each lane accumulates its own unit's gradient row in
// registers; partial gradients are summed over the waves of a workgroup in a
// fixed order, written per workgroup, and a second kernel sums the workgroup
// partials in a fixed order and applies Adam, so results are deterministic.
#include "common.h"
#include "kernels.h"

namespace cmp {
namespace {

constexpr int H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * 4, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + 4 * H, NPAR = OFF_B3 + 4;
static_assert(NPAR == kMlpParams, "parameter packing");
constexpr int GRAD_THREADS = 256;
constexpr int ROWS_PER_WG = 32;
constexpr int MAX_WG = (kMlpMaxRows + ROWS_PER_WG - 1) / ROWS_PER_WG;

struct SParams {
    float w1[H * 4], b1[H], w2[H * H], w2t[H * H], b2[H], w3[4 * H], b3[4];
};

__device__ __forceinline__ void load_params(SParams& s, const float* __restrict__ p) {
    for (int i = threadIdx.x; i < NPAR; i += blockDim.x) {
        const float v = p[i];
        if (i < OFF_B1) s.w1[i - OFF_W1] = v;
        else if (i < OFF_W2) s.b1[i - OFF_B1] = v;
        else if (i < OFF_B2) {
            const int q = i - OFF_W2;
            s.w2[q] = v;
            s.w2t[(q % H) * H + q / H] = v;
        } else if (i < OFF_W3) s.b2[i - OFF_B2] = v;
        else if (i < OFF_B3) s.w3[i - OFF_W3] = v;
        else s.b3[i - OFF_B3] = v;
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ float bcast(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Forward pass of one sample; lane j returns its z1, z2, h2 and all 4 outputs.
struct Fwd {
    float z1, h1, z2, h2, y[4];
};
__device__ __forceinline__ Fwd forward(const SParams& s, const float x[4], int j) {
    Fwd f;
    f.z1 = s.b1[j];
#pragma unroll
    for (int c = 0; c < 4; ++c) f.z1 = __builtin_fmaf(s.w1[j * 4 + c], x[c], f.z1);
    f.h1 = fmaxf(f.z1, 0.f);
    f.z2 = s.b2[j];
#pragma unroll 16
    for (int i = 0; i < H; ++i) f.z2 = __builtin_fmaf(s.w2t[i * H + j], bcast(f.h1, i), f.z2);
    f.h2 = fmaxf(f.z2, 0.f);
#pragma unroll
    for (int o = 0; o < 4; ++o) f.y[o] = s.b3[o] + wave_sum(s.w3[o * H + j] * f.h2);
    return f;
}

// Partial gradient of the summed squared error (scaled by 2 / (4 n)) over this
// workgroup's rows; writes part[wg * (NPAR + 1) + p] and the summed squared error.
__global__ __launch_bounds__(GRAD_THREADS) void mlp_grad_kernel(int n, const float* __restrict__ X,
                                                                const float* __restrict__ Y,
                                                                const float* __restrict__ params,
                                                                float* __restrict__ part) {
    __shared__ SParams s;
    __shared__ float acc[NPAR + 1];
    load_params(s, params);
    for (int i = threadIdx.x; i < NPAR + 1; i += blockDim.x) acc[i] = 0.f;
    __syncthreads();

    const int j = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float scale = 2.f / (4.f * (float)n);
    float gw1[4] = {0.f, 0.f, 0.f, 0.f}, gb1 = 0.f, gw2[H], gb2 = 0.f, gw3[4] = {0.f, 0.f, 0.f, 0.f};
    float gb3[4] = {0.f, 0.f, 0.f, 0.f}, sq = 0.f;
#pragma unroll
    for (int i = 0; i < H; ++i) gw2[i] = 0.f;

    const int r0 = blockIdx.x * ROWS_PER_WG;
    const int r1 = min(n, r0 + ROWS_PER_WG);
    for (int r = r0 + wave; r < r1; r += GRAD_THREADS / 64) {
        float x[4], yt[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            x[c] = X[4 * r + c];
            yt[c] = Y[4 * r + c];
        }
        const Fwd f = forward(s, x, j);
        float dy[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const float d = f.y[o] - yt[o];
            sq = __builtin_fmaf(d, d, sq);
            dy[o] = scale * d;
            gw3[o] = __builtin_fmaf(dy[o], f.h2, gw3[o]);
            gb3[o] += dy[o];
        }
        float dh2 = 0.f;
#pragma unroll
        for (int o = 0; o < 4; ++o) dh2 = __builtin_fmaf(s.w3[o * H + j], dy[o], dh2);
        const float dz2 = f.z2 > 0.f ? dh2 : 0.f;
        gb2 += dz2;
#pragma unroll
        for (int i = 0; i < H; ++i) gw2[i] = __builtin_fmaf(dz2, bcast(f.h1, i), gw2[i]);
        // dh1 for unit j: sum over units jj of layer 2 of W2[jj][j] * dz2[jj]
        float dh1 = 0.f;
#pragma unroll 16
        for (int jj = 0; jj < H; ++jj) dh1 = __builtin_fmaf(s.w2[jj * H + j], bcast(dz2, jj), dh1);
        const float dz1 = f.z1 > 0.f ? dh1 : 0.f;
        gb1 += dz1;
#pragma unroll
        for (int c = 0; c < 4; ++c) gw1[c] = __builtin_fmaf(dz1, x[c], gw1[c]);
    }
    // fixed-order reduction over the waves of the workgroup
    for (int w = 0; w < GRAD_THREADS / 64; ++w) {
        if (wave == w) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[OFF_W1 + j * 4 + c] += gw1[c];
            acc[OFF_B1 + j] += gb1;
#pragma unroll
            for (int i = 0; i < H; ++i) acc[OFF_W2 + i * H + j] += gw2[i];  // transposed
            acc[OFF_B2 + j] += gb2;
#pragma unroll
            for (int o = 0; o < 4; ++o) acc[OFF_W3 + o * H + j] += gw3[o];
            if (j == 0) {
#pragma unroll
                for (int o = 0; o < 4; ++o) acc[OFF_B3 + o] += gb3[o];
                acc[NPAR] += sq;
            }
        }
        __syncthreads();
    }
    float* dst = part + (size_t)blockIdx.x * (NPAR + 1);
    for (int i = threadIdx.x; i < NPAR + 1; i += blockDim.x) {
        float val = acc[i];
        if (i >= OFF_W2 && i < OFF_B2) {
            const int q = i - OFF_W2;  // row-major index (unit q / H, input q % H)
            val = acc[OFF_W2 + (q % H) * H + q / H];
        }
        dst[i] = val;
    }
}

// Sum the workgroup partials (fixed order) and apply Adam step t (1-based), or
// only write the gradient when grad_out is set.
__global__ __launch_bounds__(1024) void mlp_adam_kernel(int nwg, int n, const float* __restrict__ part,
                                                        float* __restrict__ params,
                                                        float* __restrict__ m, float* __restrict__ v,
                                                        int t, float lr, float* __restrict__ loss_out,
                                                        float* __restrict__ grad_out) {
    const double bc1 = 1.0 - pow(0.9, (double)t), bc2 = 1.0 - pow(0.999, (double)t);
    for (int p = threadIdx.x; p < NPAR + 1; p += blockDim.x) {
        float g = 0.f;
        for (int w = 0; w < nwg; ++w) g += part[(size_t)w * (NPAR + 1) + p];
        if (p == NPAR) {
            if (loss_out) *loss_out = g / (4.f * (float)n);
            continue;
        }
        if (grad_out) {
            grad_out[p] = g;
            continue;
        }
        const float mm = 0.9f * m[p] + 0.1f * g;
        const float vv = 0.999f * v[p] + 0.001f * g * g;
        m[p] = mm;
        v[p] = vv;
        const float mh = (float)((double)mm / bc1);
        const float vh = (float)((double)vv / bc2);
        params[p] -= lr * mh / (sqrtf(vh) + 1e-8f);
    }
}

__global__ void fill_zero(float* __restrict__ p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0.f;
}

// Batched inference: one wave per sample, four samples per workgroup pass.
__global__ __launch_bounds__(256) void mlp_infer_kernel(int n, const float* __restrict__ X,
                                                        const float* __restrict__ params,
                                                        float* __restrict__ Y) {
    __shared__ SParams s;
    load_params(s, params);
    __syncthreads();
    const int j = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int r = blockIdx.x * 4 + wave; r < n; r += gridDim.x * 4) {
        float x[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = X[4 * r + c];
        const Fwd f = forward(s, x, j);
        if (j < 4) Y[4 * r + j] = j == 0 ? f.y[0] : j == 1 ? f.y[1] : j == 2 ? f.y[2] : f.y[3];
    }
}

}  // namespace

static_assert(MAX_WG * (NPAR + 1) <= kMlpPartFloats, "partial-gradient buffer");

hipError_t launch_mlp_train(int n, const float* X, const float* Y, float* params, float* m,
                            float* v, float* part, int steps, int t0, float lr, float* loss_trace,
                            float* grad_out, hipStream_t stream) {
    if (n < 1 || n > kMlpMaxRows) return hipErrorInvalidValue;
    const int nwg = (n + ROWS_PER_WG - 1) / ROWS_PER_WG;
    float* g_part = part;
    if (grad_out) {
        hipLaunchKernelGGL(mlp_grad_kernel, dim3(nwg), dim3(GRAD_THREADS), 0, stream, n, X, Y,
                           params, g_part);
        hipLaunchKernelGGL(mlp_adam_kernel, dim3(1), dim3(1024), 0, stream, nwg, n, g_part,
                           params, m, v, 1, 0.f, loss_trace, grad_out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(fill_zero, dim3(10), dim3(512), 0, stream, m, NPAR);
    hipLaunchKernelGGL(fill_zero, dim3(10), dim3(512), 0, stream, v, NPAR);
    for (int s = 0; s < steps; ++s) {
        hipLaunchKernelGGL(mlp_grad_kernel, dim3(nwg), dim3(GRAD_THREADS), 0, stream, n, X, Y,
                           params, g_part);
        hipLaunchKernelGGL(mlp_adam_kernel, dim3(1), dim3(1024), 0, stream, nwg, n, g_part,
                           params, m, v, t0 + s + 1, lr, loss_trace ? loss_trace + s : nullptr,
                           nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_infer(int n, const float* X, const float* params, float* Y,
                            hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    int b = (n + 3) / 4;
    if (b > 1024) b = 1024;
    hipLaunchKernelGGL(mlp_infer_kernel, dim3(b), dim3(256), 0, stream, n, X, params, Y);
    return hipGetLastError();
}

}  // namespace cmp
