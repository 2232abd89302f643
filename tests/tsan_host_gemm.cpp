// ThreadSanitizer driver for the host variant's FP32 GEMM (csrc/host_gemm.cpp), the part of the
// host runtime that runs on several std::threads: ragged shapes, 1 / 3 / 16 threads, beta = 0
// and beta != 0, and two callers at once on different outputs.  Small-integer operands make
// every result exact, so each one is compared with a plain binary64 loop.
#include <cstdint>
#include <cstdio>
#include <thread>
#include <vector>

namespace cmp {
void host_gemm_f32(int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                   const float* B, int64_t ldb, float beta, float* C, int64_t ldc, int max_threads);
}

static long check(int64_t M, int64_t N, int64_t K, float beta, int threads, int salt) {
    const int64_t lda = K + 3, ldb = N + 1, ldc = N + 2;
    std::vector<float> A(M * lda), B(K * ldb), C(M * ldc), C0;
    for (int64_t i = 0; i < M * lda; ++i) A[i] = (float)((i * 7 + salt) % 9) - 4.f;
    for (int64_t i = 0; i < K * ldb; ++i) B[i] = (float)((i * 5 + salt) % 9) - 4.f;
    for (int64_t i = 0; i < M * ldc; ++i) C[i] = (float)((i * 3 + salt) % 5) - 2.f;
    C0 = C;
    cmp::host_gemm_f32(M, N, K, 2.f, A.data(), lda, B.data(), ldb, beta, C.data(), ldc, threads);
    long bad = 0;
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double s = 0;
            for (int64_t k = 0; k < K; ++k) s += (double)A[i * lda + k] * B[k * ldb + j];
            const double want = 2.0 * s + (beta != 0.f ? (double)beta * C0[i * ldc + j] : 0.0);
            if (want != (double)C[i * ldc + j]) ++bad;
        }
    return bad;
}

int main() {
    long bad = 0;
    const int64_t shapes[][3] = {{1, 1, 1}, {33, 257, 65}, {300, 520, 200}, {129, 1031, 96}};
    for (const auto& s : shapes)
        for (int threads : {1, 3, 16})
            for (float beta : {0.f, -0.5f}) bad += check(s[0], s[1], s[2], beta, threads, (int)s[0] + threads);
    // two callers at once
    long b1 = 0, b2 = 0;
    std::thread t1([&] { b1 = check(300, 520, 200, 0.f, 16, 1); });
    std::thread t2([&] { b2 = check(257, 300, 129, 1.f, 16, 2); });
    t1.join();
    t2.join();
    bad += b1 + b2;
    std::printf("mismatches %ld\n", bad);
    return bad != 0;
}
