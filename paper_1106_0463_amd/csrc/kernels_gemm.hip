// Abel-as-GEMM form (functions sampled on one fixed P-point Chebyshev-Gauss
// grid): phi = A F with the FP64 product-integration matrix
//   A[j][p] = integral_{cos y_j}^1 l_p(x) / sqrt(2 (x - cos y_j)) dx
//           = 2 s_j sum_q w_q l_p(x_{jq}),
// l_p the Lagrange cardinal polynomial of node p, evaluated with the
// barycentric formula for Chebyshev points of the first kind.
//
// Kernels:
//   k_amat        A in FP64, one workgroup per row j
//   k_split_rows  A -> 16-bit pieces (bf16, or fp16 with a power-of-two row
//                 scale), K-major [H][P]
//   k_colmax / k_split_cols  F [P][B] FP64 -> pieces [B][P] (transposed)
//   k_mgemm       Out[b][j] = sum_{(u,v)} sum_p X_u[b][p] Y_v[j][p] on MFMA
//                 (32x32x16, FP32 accumulation), fused over the piece
//                 products of the precision mode
//   k_gdst_lds    batched DST-III + rescale over the rows of Out
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "lc_internal.h"
#include "lc_gemm.h"

namespace lc {

// ------------------------------------------------------------ matrix A ---
// Block of 256 threads per row j = blockIdx.x + 1 (row 0, y = 0, is zero).
// Each thread owns columns p = tid + 256 i.  For every Abel node x_{jq}:
//   r_k = lam_k / (x - x_k),  D = sum_k r_k,  l_p(x) = r_p / D
// (an exact hit x == x_k gives l_p = delta_{pk}).
template <int PT>  // columns per thread (P <= 256 PT)
__global__ __launch_bounds__(256) void k_amat(int H, int P, int QA, const double *__restrict__ xc,
                                              const double *__restrict__ lam, const double2 *__restrict__ rowA,
                                              const double2 *__restrict__ omt2, const double *__restrict__ wq,
                                              const double *__restrict__ s2, double *__restrict__ A) {
#pragma clang fp contract(off)
    __shared__ double red[4];
    __shared__ int hitsh[4];
    const int r = blockIdx.x;  // row j = r + 1
    const int tid = threadIdx.x;
    double acc[PT];
    double xk[PT], lk[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int p = tid + 256 * i;
        acc[i] = 0.0;
        xk[i] = p < P ? xc[p] : 0.0;
        lk[i] = p < P ? lam[p] : 0.0;
    }
    const double2 a = rowA[r];
    const double sj2 = s2[r];
    for (int q = 0; q < QA; ++q) {
        // node x = 1 - A_j B_q in double-double (as for the sample nodes)
        const double2 b = omt2[q];
        const double pr = a.x * b.x;
        double e = fma(a.x, b.x, -pr);
        e = fma(a.x, b.y, fma(a.y, b.x, e));
        const double s = 1.0 - pr;
        const double bb = s - 1.0;
        const double err = (1.0 - (s - bb)) + (-pr - bb);
        const double x = s + (err - e);
        double rk[PT];
        double part = 0.0;
        int hit = -1;
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int p = tid + 256 * i;
            const double d = x - xk[i];
            rk[i] = 0.0;
            if (p < P) {
                if (d == 0.0) hit = p;
                else rk[i] = lk[i] / d;
            }
            part += rk[i];
        }
        // block sum of part, block max of hit
        for (int off = 32; off > 0; off >>= 1) {
            part += __shfl_xor(part, off, 64);
            hit = max(hit, __shfl_xor(hit, off, 64));
        }
        if ((tid & 63) == 0) {
            red[tid >> 6] = part;
            hitsh[tid >> 6] = hit;
        }
        __syncthreads();
        const double D = (red[0] + red[1]) + (red[2] + red[3]);
        const int h = max(max(hitsh[0], hitsh[1]), max(hitsh[2], hitsh[3]));
        __syncthreads();
        const double c = sj2 * wq[q];
        if (h < 0) {
            const double cd = c / D;
#pragma unroll
            for (int i = 0; i < PT; ++i) acc[i] = fma(cd, rk[i], acc[i]);
        } else {
#pragma unroll
            for (int i = 0; i < PT; ++i)
                if (tid + 256 * i == h) acc[i] += c;
        }
    }
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int p = tid + 256 * i;
        if (p < P) A[(int64_t)(r + 1) * P + p] = acc[i];
    }
}

hipError_t launch_amat(int H, int P, int QA, const double *xc, const double *lam, const double2 *rowA,
                       const double2 *omt2, const double *wq, const double *s2, double *A, hipStream_t s) {
    hipError_t e = hipMemsetAsync(A, 0, (size_t)P * sizeof(double), s);  // row 0
    if (e != hipSuccess) return e;
    const int pt = (P + 255) / 256;
#define LC_AMAT(PTV)                                                                                   \
    if (pt <= PTV) {                                                                                   \
        hipLaunchKernelGGL(k_amat<PTV>, dim3(H), dim3(256), 0, s, H, P, QA, xc, lam, rowA, omt2, wq, s2, A); \
        return hipGetLastError();                                                                      \
    }
    LC_AMAT(4)
    LC_AMAT(8)
    LC_AMAT(16)
    LC_AMAT(32)
    LC_AMAT(64)
#undef LC_AMAT
    return hipErrorInvalidValue;
}

// --------------------------------------------------------------- splits ---
// Piece extraction: v = sum of npc 16-bit pieces, each the nearest 16-bit
// value of the remainder.  FP16 uses a power-of-two scale 2^-e per row (A)
// or per function (F) so that |v 2^-e| < 1; BF16 has FP32's exponent range
// and needs none.
// Round-to-nearest-even FP32 -> 16-bit conversions written out on the bit
// pattern, so that the pieces do not depend on the default conversion mode.
template <typename H16> struct Round16;
template <> struct Round16<__bf16> {
    static __device__ __forceinline__ __bf16 from(float f) {
        unsigned u = __builtin_bit_cast(unsigned, f);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
    }
};
template <> struct Round16<_Float16> {
    static __device__ __forceinline__ _Float16 from(float f) { return (_Float16)f; }  // IEEE RNE
};

template <typename H16>
__device__ __forceinline__ void split_value(double v, int npc, H16 *out) {
    double r = v;
    for (int i = 0; i < npc; ++i) {
        // the remainder r - piece is exact in FP64, so a piece that is not the
        // nearest 16-bit value (double rounding through FP32) only shifts a
        // few bits to the next piece
        const H16 h = Round16<H16>::from((float)r);
        out[i] = h;
        r -= (double)(float)h;
    }
}

// A rows 1..H -> pieces Y_i[j-1][p]; fp16: scale row by 2^-e_j (e_j from the
// row's max |A|), exponent stored in rowexp[j-1].
template <typename H16>
__global__ __launch_bounds__(256) void k_split_rows(const double *__restrict__ A, int H, int P, int ldk, int npc,
                                                    H16 *__restrict__ Y, int64_t piece_stride,
                                                    int *__restrict__ rowexp, int scaled) {
    __shared__ double red[4];
    const int j = blockIdx.x;  // output row (A row j + 1)
    const double *a = A + (int64_t)(j + 1) * P;
    double m = 0.0;
    for (int p = threadIdx.x; p < P; p += 256) m = fmax(m, fabs(a[p]));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int ex = 0;
    if (scaled && m > 0.0) ex = ilogb(m) + 1;  // |a| 2^-ex < 1
    if (threadIdx.x == 0 && rowexp) rowexp[j] = ex;
    const double sc = ldexp(1.0, -ex);
    for (int p = threadIdx.x; p < P; p += 256) {
        H16 pcs[3];
        split_value<H16>(a[p] * sc, npc, pcs);
        for (int i = 0; i < npc; ++i) Y[i * piece_stride + (int64_t)j * ldk + p] = pcs[i];
    }
}

// per-function exponent colexp[b] = ilogb(max_p |F[p][b]|) + 1: a fill, then
// blocks of 256 functions x 64 rows fold their partial maxima in with an
// integer atomic max (the exponent is monotone in the magnitude).
__global__ __launch_bounds__(256) void k_colexp_init(int B, int *__restrict__ colexp) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b < B) colexp[b] = -2000;
}

__global__ __launch_bounds__(256) void k_colmax(const double *__restrict__ F, int P, int B,
                                                int *__restrict__ colexp) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    const int p0 = blockIdx.y * 64;
    if (b >= B) return;
    double m = 0.0;
    const int p1 = p0 + 64 < P ? p0 + 64 : P;
    for (int p = p0; p < p1; ++p) m = fmax(m, fabs(F[(int64_t)p * B + b]));
    if (m > 0.0) atomicMax(colexp + b, ilogb(m) + 1);
}

// F [P][B] -> pieces X_i[b][p] through a 64x64 LDS transpose tile.
template <typename H16>
__global__ __launch_bounds__(256) void k_split_cols(const double *__restrict__ F, int P, int B, int ldk, int npc,
                                                    H16 *__restrict__ X, int64_t piece_stride,
                                                    const int *__restrict__ colexp) {
    __shared__ double tile[64][65];
    const int p0 = blockIdx.y * 64, b0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int p = p0 + i, b = b0 + tx;
        tile[i][tx] = (p < P && b < B) ? F[(int64_t)p * B + b] : 0.0;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int b = b0 + i, p = p0 + tx;
        if (b < B && p < P) {
            const double sc = colexp ? ldexp(1.0, -max(colexp[b], -1000)) : 1.0;
            H16 pcs[3];
            split_value<H16>(tile[tx][i] * sc, npc, pcs);
            for (int k = 0; k < npc; ++k) X[k * piece_stride + (int64_t)b * ldk + p] = pcs[k];
        }
    }
}

hipError_t launch_split_rows(int h16, const double *A, int H, int P, int ldk, int npc, void *Y,
                             int64_t piece_stride, int *rowexp, int scaled, hipStream_t s) {
    if (h16 == kBF16)
        hipLaunchKernelGGL(k_split_rows<__bf16>, dim3(H), dim3(256), 0, s, A, H, P, ldk, npc, (__bf16 *)Y,
                           piece_stride, rowexp, scaled);
    else
        hipLaunchKernelGGL(k_split_rows<_Float16>, dim3(H), dim3(256), 0, s, A, H, P, ldk, npc, (_Float16 *)Y,
                           piece_stride, rowexp, scaled);
    return hipGetLastError();
}

hipError_t launch_split_cols(int h16, const double *F, int P, int B, int ldk, int npc, void *X,
                             int64_t piece_stride, int *colexp, int scaled, hipStream_t s) {
    if (scaled) {
        hipLaunchKernelGGL(k_colexp_init, dim3((B + 255) / 256), dim3(256), 0, s, B, colexp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_colmax, dim3((B + 255) / 256, (P + 63) / 64), dim3(256), 0, s, F, P, B, colexp);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    dim3 grid((B + 63) / 64, (P + 63) / 64);
    if (h16 == kBF16)
        hipLaunchKernelGGL(k_split_cols<__bf16>, grid, dim3(256), 0, s, F, P, B, ldk, npc, (__bf16 *)X,
                           piece_stride, scaled ? colexp : nullptr);
    else
        hipLaunchKernelGGL(k_split_cols<_Float16>, grid, dim3(256), 0, s, F, P, B, ldk, npc, (_Float16 *)X,
                           piece_stride, scaled ? colexp : nullptr);
    return hipGetLastError();
}

// ------------------------------------------------------------ MFMA GEMM ---
// Block tile 128 (b) x 128 (j), 4 waves in 2x2, each wave 64x64 = 2x2
// MFMA 32x32x16 tiles (16 FP32 accumulators each).  K advances 32 per LDS
// stage; all pieces of both operands for the stage are staged in LDS (rows
// padded to 40 halves = 80 B so that 16-byte fragment reads by 32
// consecutive rows spread over the banks); the next stage is prefetched
// into registers during the MFMAs.  Requires P % 32 == 0 (the host pads).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename H16> struct Mfma;
template <> struct Mfma<__bf16> {
    static __device__ __forceinline__ f32x16 run(u32x4 a, u32x4 b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
    }
};
template <> struct Mfma<_Float16> {
    static __device__ __forceinline__ f32x16 run(u32x4 a, u32x4 b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b),
                                                      c, 0, 0, 0);
    }
};

constexpr int GBM = 128, GBN = 128, GBK = 32, GLD = 40;  // LDS row: 40 halves

// Piece products of each mode (u indexes X pieces, v indexes Y pieces):
//   1: (0,0)                 one 16-bit product
//   3: (0,0) (1,0) (0,1)     hi*hi + lo*hi + hi*lo
//   6: the six products with u + v <= 2 of three pieces each
template <int MODE> struct Prods;
template <> struct Prods<1> { static constexpr int n = 1, nx = 1, ny = 1; static constexpr int u[1] = {0}, v[1] = {0}; };
template <> struct Prods<3> { static constexpr int n = 3, nx = 2, ny = 2; static constexpr int u[3] = {0, 1, 0}, v[3] = {0, 0, 1}; };
template <> struct Prods<6> {
    static constexpr int n = 6, nx = 3, ny = 3;
    static constexpr int u[6] = {0, 1, 0, 2, 1, 0}, v[6] = {0, 0, 1, 0, 1, 2};
};

template <typename H16, int MODE, int WM>
__global__ __launch_bounds__(128 * WM) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mgemm(
    const H16 *__restrict__ X, int64_t xps, const H16 *__restrict__ Y, int64_t yps, int Bn, int Hn, int P,
    float *__restrict__ Out, int ldo) {
    // block tile (64 WM) x 128: WM x 2 waves, each wave 64 x 64
    using PR = Prods<MODE>;
    constexpr int NX = PR::nx, NY = PR::ny;
    constexpr int BM = 64 * WM, NT = 128 * WM;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    H16 *sx = reinterpret_cast<H16 *>(smem);               // [NX][BM * GLD]
    H16 *sy = sx + NX * BM * GLD;                            // [NY][GBN * GLD]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    // tile coordinates, j fastest so that consecutive blocks share the X rows
    const int ntn = (Hn + GBN - 1) / GBN;
    const int bm0 = (blockIdx.x / ntn) * BM, bn0 = (blockIdx.x % ntn) * GBN;

    // global -> register staging: a tile row is 32 halves = 4 chunks of 16 B
    constexpr int CX = BM * 4 / NT, CY = GBN * 4 / NT;  // chunks per thread
    u32x4 rx[NX][CX], ry[NY][CY];
    auto gload = [&](int k0) {
#pragma unroll
        for (int c = 0; c < CX; ++c) {
            const int idx = tid + NT * c;
            const int row = idx >> 2, col = (idx & 3) * 8;
            const int gb = bm0 + row;
#pragma unroll
            for (int u = 0; u < NX; ++u)
                rx[u][c] = gb < Bn ? *reinterpret_cast<const u32x4 *>(X + u * xps + (int64_t)gb * P + k0 + col)
                                   : (u32x4)(0u);
        }
#pragma unroll
        for (int c = 0; c < CY; ++c) {
            const int idx = tid + NT * c;
            const int row = idx >> 2, col = (idx & 3) * 8;
            const int gj = bn0 + row;
#pragma unroll
            for (int v = 0; v < NY; ++v)
                ry[v][c] = gj < Hn ? *reinterpret_cast<const u32x4 *>(Y + v * yps + (int64_t)gj * P + k0 + col)
                                   : (u32x4)(0u);
        }
    };
    auto sstore = [&]() {
#pragma unroll
        for (int c = 0; c < CX; ++c) {
            const int idx = tid + NT * c;
            const int row = idx >> 2, col = (idx & 3) * 8;
#pragma unroll
            for (int u = 0; u < NX; ++u) *reinterpret_cast<u32x4 *>(&sx[u * BM * GLD + row * GLD + col]) = rx[u][c];
        }
#pragma unroll
        for (int c = 0; c < CY; ++c) {
            const int idx = tid + NT * c;
            const int row = idx >> 2, col = (idx & 3) * 8;
#pragma unroll
            for (int v = 0; v < NY; ++v) *reinterpret_cast<u32x4 *>(&sy[v * GBN * GLD + row * GLD + col]) = ry[v][c];
        }
    };

    // Two-level accumulation: the MFMA accumulator covers one K chunk of
    // KCH stages and is then added into a second FP32 total and cleared, so
    // that no FP32 chain runs over more than KCH*GBK/16 MFMA steps per
    // product (long chains of same-sign partial sums lose accuracy).
    constexpr int KCH = 4;
    f32x16 acc[2][2], tot[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acc[a][b][v] = 0.f;
                tot[a][b][v] = 0.f;
            }

    const int nk = P / GBK;
    gload(0);
    for (int kt = 0; kt < nk; ++kt) {
        if (kt % KCH == 0 && kt > 0) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    tot[a][b] += acc[a][b];
#pragma unroll
                    for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;
                }
        }
        __syncthreads();
        sstore();
        __syncthreads();
        if (kt + 1 < nk) gload((kt + 1) * GBK);
#pragma unroll
        for (int ks = 0; ks < GBK; ks += 16) {
            // fragments: lane holds row (lane % 32), k = ks + 8 (lane / 32) + 0..7
            const int fr = lane & 31, fk = ks + 8 * (lane >> 5);
            u32x4 fx[NX][2], fy[NY][2];
#pragma unroll
            for (int u = 0; u < NX; ++u)
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    fx[u][a] = *reinterpret_cast<const u32x4 *>(&sx[u * BM * GLD + (wm + 32 * a + fr) * GLD + fk]);
#pragma unroll
            for (int v = 0; v < NY; ++v)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    fy[v][b] = *reinterpret_cast<const u32x4 *>(&sy[v * GBN * GLD + (wn + 32 * b + fr) * GLD + fk]);
#pragma unroll
            for (int pi = 0; pi < PR::n; ++pi)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = Mfma<H16>::run(fx[PR::u[pi]][a], fy[PR::v[pi]][b], acc[a][b]);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) tot[a][b] += acc[a][b];
    // D layout: lane l, register v -> row 8 (v/4) + 4 (l/32) + (v%4), col l%32
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = bm0 + wm + 32 * a + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int col = bn0 + wn + 32 * b + (lane & 31);
                if (row < Bn && col < Hn) Out[(int64_t)row * ldo + col] = tot[a][b][v];
            }
}

int mgemm_wm = 2;  // waves along b per block (block tile 64*WM x 128); LC_MGEMM_WM overrides

hipError_t launch_mgemm(int h16, int mode, const void *X, int64_t xps, const void *Y, int64_t yps, int Bn, int Hn,
                        int P, float *Out, int ldo, hipStream_t s) {
    if (P % GBK) return hipErrorInvalidValue;
    const int WM = mgemm_wm == 2 ? 2 : 4;
    const int BM = 64 * WM;
    const int grid = ((Bn + BM - 1) / BM) * ((Hn + GBN - 1) / GBN);
    const int npx = mode == 1 ? 1 : (mode == 3 ? 2 : 3);
    const size_t lds = (size_t)npx * (BM + GBN) * GLD * 2;
#define LC_MG(T, MV, WMV)                                                                                      \
    if (mode == MV && WM == WMV) {                                                                             \
        if (lds > 65536) {                                                                                     \
            hipError_t e = hipFuncSetAttribute((const void *)k_mgemm<T, MV, WMV>,                              \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);          \
            if (e != hipSuccess) return e;                                                                     \
        }                                                                                                      \
        hipLaunchKernelGGL((k_mgemm<T, MV, WMV>), dim3(grid), dim3(128 * WMV), lds, s, (const T *)X, xps,    \
                           (const T *)Y, yps, Bn, Hn, P, Out, ldo);                                            \
        return hipGetLastError();                                                                              \
    }
    if (h16 == kBF16) {
        LC_MG(__bf16, 1, 2) LC_MG(__bf16, 3, 2) LC_MG(__bf16, 6, 2)
        LC_MG(__bf16, 1, 4) LC_MG(__bf16, 3, 4) LC_MG(__bf16, 6, 4)
    } else {
        LC_MG(_Float16, 1, 2) LC_MG(_Float16, 3, 2) LC_MG(_Float16, 6, 2)
        LC_MG(_Float16, 1, 4) LC_MG(_Float16, 3, 4) LC_MG(_Float16, 6, 4)
    }
#undef LC_MG
    return hipErrorInvalidValue;
}

// ------------------------------------------------- batched DST of rows ---
// Function b reads phi_j = Out[b][j-1] * 2^(rowexp[j-1] + colexp[b]) (no
// scaling when the exponent arrays are null).
template <int T, typename PhiT>
__global__ __launch_bounds__(T) void k_gdst_lds(const PhiT *__restrict__ Out, int ldo, const int *__restrict__ rowexp,
                                                const int *__restrict__ colexp, int64_t H, int L, int64_t N,
                                                const double2 *__restrict__ tw_pre,
                                                const double2 *__restrict__ tw_pack,
                                                const double2 *__restrict__ tw_fft, FftSched sch,
                                                double *__restrict__ C) {
    extern __shared__ double2 lds[];
    const int b = blockIdx.x;
    const PhiT *row = Out + (int64_t)b * ldo;
    const int ce = colexp ? max(colexp[b], -1000) : 0;
    struct Phi {
        const PhiT *p;
        const int *re;
        int ce;
        __device__ __forceinline__ double operator()(int64_t m) const {
            const double v = (double)p[m - 1];
            return re ? ldexp(v, re[m - 1] + ce) : v;
        }
    } ph{row, rowexp, ce};
    for (int k = threadIdx.x; k < L; k += T) lds[k] = dst_pack(k, ph, H, L, tw_pre, tw_pack);
    __syncthreads();
    fft_lds<T, 8>(lds, L, 1, sch, tw_fft, 1);
    double *c = C + (int64_t)b * N;
    for (int64_t n = threadIdx.x; n < N; n += T) c[n] = dst_post(n, lds, H);
}

hipError_t launch_gdst(int phi_is_fp32, const void *Out, int ldo, const int *rowexp, const int *colexp, int B,
                       int64_t H, int64_t L, int64_t N, const double2 *tw_pre, const double2 *tw_pack,
                       const double2 *tw_fft, const FftSched &sch, double *C, hipStream_t s) {
    const size_t lds = (size_t)L * sizeof(double2);
    int T = L <= 512 ? 64 : (L <= 2048 ? 256 : 1024);
    if (L > 8 * T) return hipErrorInvalidValue;
#define LC_GD(TV, PT)                                                                                  \
    if (T == TV) {                                                                                     \
        if (lds > 65536) {                                                                             \
            hipError_t e = hipFuncSetAttribute((const void *)k_gdst_lds<TV, PT>,                       \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);  \
            if (e != hipSuccess) return e;                                                             \
        }                                                                                              \
        hipLaunchKernelGGL((k_gdst_lds<TV, PT>), dim3(B), dim3(TV), lds, s, (const PT *)Out, ldo, rowexp, colexp, \
                           H, (int)L, N, tw_pre, tw_pack, tw_fft, sch, C);                             \
        return hipGetLastError();                                                                      \
    }
    if (phi_is_fp32) {
        LC_GD(64, float)
        LC_GD(256, float)
        LC_GD(1024, float)
    } else {
        LC_GD(64, double)
        LC_GD(256, double)
        LC_GD(1024, double)
    }
#undef LC_GD
    return hipErrorInvalidValue;
}

}  // namespace lc
