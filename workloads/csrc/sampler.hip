// Synthetic-input sampler (test and benchmark input generation only, not
// part of the Legendre-coefficient library): evaluates random finite
// Legendre series f_b(x) = sum_{n<N_b} c_{b,n} P_n(x) at device nodes with
// Clenshaw's backward recurrence
//   b_k = c_k + (2k+1)/(k+1) x b_{k+1} - (k+1)/(k+2) b_{k+2},  f = b_0,
// in FP64, so that batches too large to sample on the host can be built on
// the GPU.
#include <hip/hip_runtime.h>
#include <stdint.h>

__device__ __forceinline__ double clenshaw(const double *__restrict__ c, int64_t n, double x) {
    double b1 = 0.0, b2 = 0.0;
    for (int64_t k = n - 1; k >= 0; --k) {
        const double a = (double)(2 * k + 1) / (double)(k + 1);
        const double bb = (double)(k + 1) / (double)(k + 2);
        const double b0 = c[k] + a * x * b1 - bb * b2;
        b2 = b1;
        b1 = b0;
    }
    return b1;
}

// Ragged arena: function b owns nodes x[x_off[b] .. x_off[b+1]) and writes
// its samples at byte offset f_off[b] of f_arena, as FP64 or FP32.
__global__ void k_series_ragged(int32_t B, const double *__restrict__ coef, const int64_t *__restrict__ coef_off,
                                const double *__restrict__ x, const int64_t *__restrict__ x_off,
                                unsigned char *__restrict__ f_arena, const int64_t *__restrict__ f_off,
                                const int32_t *__restrict__ fp32) {
    const int64_t total = x_off[B];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = B - 1;  // last b with x_off[b] <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (x_off[mid] <= i) lo = mid; else hi = mid - 1;
        }
        const int b = lo;
        const int64_t e = i - x_off[b];
        const double v = clenshaw(coef + coef_off[b], coef_off[b + 1] - coef_off[b], x[i]);
        if (fp32[b]) reinterpret_cast<float *>(f_arena + f_off[b])[e] = (float)v;
        else reinterpret_cast<double *>(f_arena + f_off[b])[e] = v;
    }
}

// Fixed grid: F[p][b] = f_b(x_p), coefficients [B][deg+1] row-major.
__global__ void k_series_grid(int32_t B, int32_t ncoef, const double *__restrict__ coef, int32_t P,
                              const double *__restrict__ x, double *__restrict__ F) {
    const int64_t total = (int64_t)P * B;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = i / B, b = i - p * B;
        F[i] = clenshaw(coef + b * (int64_t)ncoef, ncoef, x[p]);
    }
}

extern "C" int synth_series_ragged(int32_t B, const double *coef, const int64_t *coef_off, const double *x,
                                   const int64_t *x_off, int64_t total, void *f_arena, const int64_t *f_off,
                                   const int32_t *fp32, hipStream_t s) {
    if (B < 1 || !coef || !coef_off || !x || !x_off || !f_arena || !f_off || !fp32) return 1;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 1 << 16) blocks = 1 << 16;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_series_ragged, dim3((unsigned)blocks), dim3(256), 0, s, B, coef, coef_off, x, x_off,
                       (unsigned char *)f_arena, f_off, fp32);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

extern "C" int synth_series_grid(int32_t B, int32_t ncoef, const double *coef, int32_t P, const double *x,
                                 double *F, hipStream_t s) {
    if (B < 1 || ncoef < 1 || P < 1 || !coef || !x || !F) return 1;
    const int64_t total = (int64_t)P * B;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 1 << 16) blocks = 1 << 16;
    hipLaunchKernelGGL(k_series_grid, dim3((unsigned)blocks), dim3(256), 0, s, B, ncoef, coef, P, x, F);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}
