// Two-dimensional tensor-product plans: the transpose between the two
// passes (coefficients along x1 of every x2 node -> samples along x2 of
// every n1).
#include <hip/hip_runtime.h>

#include "lc_internal.h"

namespace lc {

// dst[c][r] = src[r][c] for an R x C row-major FP64 matrix: 32 x 32 tiles
// through LDS (padded against bank conflicts).
__global__ __launch_bounds__(256) void k_transpose64(const double *__restrict__ src, int64_t R, int64_t C,
                                                     double *__restrict__ dst) {
    __shared__ double tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int i = ty; i < 32; i += 8) {
        const int64_t r = r0 + i, c = c0 + tx;
        tile[i][tx] = (r < R && c < C) ? src[r * C + c] : 0.0;
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int64_t c = c0 + i, r = r0 + tx;
        if (c < C && r < R) dst[c * R + r] = tile[tx][i];
    }
}

hipError_t launch_transpose64(const double *src, int64_t R, int64_t C, double *dst, hipStream_t s) {
    const int64_t gy = (R + 31) / 32, gx = (C + 31) / 32;
    if (gy > 65535 || gx > 2147483647) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_transpose64, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, src, R, C, dst);
    return hipGetLastError();
}

// dst[r * n + i] = src[i] for r < reps (the row factors of every function)
__global__ __launch_bounds__(256) void k_repeat(const double *__restrict__ src, int64_t n, int64_t total,
                                                double *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i % n];
}

hipError_t launch_repeat(const double *src, int64_t n, int64_t reps, double *dst, hipStream_t s) {
    const int64_t total = n * reps;
    const int64_t grid = (total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536;
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(k_repeat, dim3((unsigned)grid), dim3(256), 0, s, src, n, total, dst);
    return hipGetLastError();
}

}  // namespace lc
