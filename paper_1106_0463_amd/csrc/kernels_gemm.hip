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
//                 scale, k_rowexp), in MFMA fragment order
//   k_split_cols  F [P][B] FP64 -> pieces of F^T, fragment order (FP16:
//                 one power-of-two scale per function and chunk of 256 p)
//   k_colscale    per-function exponent and chunk factors of the FP16 split
//   k_mgemm       Out[b][j] = sum_{(u,v)} sum_p X_u[b][p] Y_v[j][p] on MFMA
//                 (32x32x16, FP32 accumulation), fused over the piece
//                 products of the precision mode
//   k_gdst_lds    batched DST-III + rescale over the rows of Out
#include <hip/hip_runtime.h>

#include <type_traits>

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

// ---------------------------------------------------- fragment order ---
// Both 16-bit operands of the product are stored in the lane order of the
// MFMA 32x32x16 operand fragment: element (row r, k) of a piece lives at
//   ((r / 32) * K16 + k / 16) * 512 + ((r % 32) + 32 ((k / 8) % 2)) * 8 + k % 8
// (halves; K16 = Kp / 16 with Kp = P rounded up to 32).  One fragment is then
// 1 KiB in which lane l owns bytes [16 l, 16 l + 16): global loads, the
// global->LDS copies and the LDS reads of the product are all 16 contiguous
// bytes per lane, which no bank or channel pattern can split.  Rows are
// padded to the block tile and k to Kp with zeros.
constexpr int kSplitKW = 4;  // k fragments per wave in the column split
// K-steps of 16 per FP16 column-exponent chunk: one column-split block
static_assert(4 * kSplitKW == kExpChunk16, "a split block covers one exponent chunk");

__device__ __forceinline__ int64_t fo_offset(int64_t r, int k, int K16) {
    return ((r >> 5) * K16 + (k >> 4)) * 512 + (((r & 31) + ((k >> 3) & 1) * 32) << 3) + (k & 7);
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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Splits 8 consecutive-k values into npc pieces of 8 halves (16 bytes) each.
template <typename H16, int NPC>
__device__ __forceinline__ void split8(const double *v, u32x4 *out) {
    H16 h[NPC][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        double r = v[e];
#pragma unroll
        for (int i = 0; i < NPC; ++i) {
            // the remainder r - piece is exact in FP64, so a piece that is not
            // the nearest 16-bit value (double rounding through FP32) only
            // shifts a few bits to the next piece
            const H16 p = Round16<H16>::from((float)r);
            h[i][e] = p;
            r -= (double)(float)p;
        }
    }
#pragma unroll
    for (int i = 0; i < NPC; ++i) out[i] = __builtin_bit_cast(u32x4, h[i]);
}

// The Y operand is an FP64 matrix with rows r = 0..H-1 and columns k = 0..P-1
// read as S[(r + roff) rs + k cs]: the product-integration matrix A without
// its zero row (roff = 1, rs = P, cs = 1), or the direct Legendre matrix
// stored transposed (roff = 0, rs = 1, cs = N).
struct Strided {
    const double *p;
    int64_t roff, rs, cs;
    __device__ __forceinline__ double at(int64_t r, int64_t k) const { return p[(r + roff) * rs + k * cs]; }
};

// rowexp[r] = ilogb(max_k |S[r][k]|) + 1 (0 for a zero row): one block per row.
__global__ __launch_bounds__(256) void k_rowexp(Strided S, int P, int *__restrict__ rowexp) {
    __shared__ double red[4];
    const int r = blockIdx.x;
    double m = 0.0;
    for (int k = threadIdx.x; k < P; k += 256) m = fmax(m, fabs(S.at(r, k)));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (threadIdx.x == 0) rowexp[r] = m > 0.0 ? ilogb(m) + 1 : 0;
}

// S -> pieces Y_i in fragment order over Hpad rows; one thread per 8
// consecutive k of one row; rows >= H and k >= P are zero.
template <typename H16, int NPC>
__global__ __launch_bounds__(256) void k_split_rows(Strided S, int H, int P, int K16, int64_t nfrag,
                                                    H16 *__restrict__ Y, int64_t piece_stride,
                                                    const int *__restrict__ rowexp) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t frag = t >> 6;
    if (frag >= nfrag) return;
    const int lane = (int)(t & 63);
    const int64_t r = (frag / K16) * 32 + (lane & 31);
    const int k = (int)(frag % K16) * 16 + (lane >> 5) * 8;
    double v[8];
    const double sc = (rowexp && r < H) ? ldexp(1.0, -rowexp[r]) : 1.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (r < H && k + e < P) ? S.at(r, k + e) * sc : 0.0;
    u32x4 out[NPC];
    split8<H16, NPC>(v, out);
#pragma unroll
    for (int i = 0; i < NPC; ++i)
        *reinterpret_cast<u32x4 *>(Y + i * piece_stride + fo_offset(r, k, K16)) = out[i];
}

// AT[p][j] = A[j + 1][p] (the columns of A without its zero row, as rows):
// 32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose_a(const double *__restrict__ A, int H, int P,
                                                     double *__restrict__ AT) {
    __shared__ double tile[32][33];
    const int j0 = blockIdx.y * 32, p0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int i = ty; i < 32; i += 8) {
        const int j = j0 + i, p = p0 + tx;
        tile[i][tx] = (j < H && p < P) ? A[(int64_t)(j + 1) * P + p] : 0.0;
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int p = p0 + i, j = j0 + tx;
        if (p < P && j < H) AT[(int64_t)p * H + j] = tile[tx][i];
    }
}

hipError_t launch_transpose_a(const double *A, int H, int P, double *AT, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_a, dim3((P + 31) / 32, (H + 31) / 32), dim3(256), 0, s, A, H, P, AT);
    return hipGetLastError();
}

// Direct form (FP16): one exponent per function, colexp[b] = ilogb(max_p
// |F[p][b]|) + 1, before the split: a fill, then blocks of 256 functions x 64
// rows fold their partial maxima in with an integer atomic max (the exponent
// is monotone in the magnitude).  Its product folds FP64 totals every few
// K-steps, where a factor per chunk would double the fold's work.
__global__ __launch_bounds__(256) void k_colexp_init(int B, int *__restrict__ colexp) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b < B) colexp[b] = -2000;
}

__global__ __launch_bounds__(256) void k_colmax(const double *__restrict__ F, int P, int B,
                                                int *__restrict__ colexp) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    const int p0 = blockIdx.y * 64;
    if (b >= B) return;
    const int p1 = p0 + 64 < P ? p0 + 64 : P;
    double m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int p = p0;
    for (; p + 8 <= p1; p += 8) {
#pragma unroll
        for (int e = 0; e < 8; ++e) m[e] = fmax(m[e], fabs(__builtin_nontemporal_load(F + (int64_t)(p + e) * B + b)));
    }
    for (; p < p1; ++p) m[0] = fmax(m[0], fabs(F[(int64_t)p * B + b]));
    double mm = 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) mm = fmax(mm, m[e]);
    if (mm > 0.0) atomicMax(colexp + b, ilogb(mm) + 1);
}

// F [P][B] -> pieces X_i in fragment order over Bpad rows (function b is
// row b); one thread per (b, 8 consecutive p).  Fragments are numbered with
// the row block fastest, so that the waves resident together read long
// contiguous stretches of the same rows of F.
//
// FP16 (SCM 1): block (rb, kg) covers exactly the 256 samples p of exponent
// chunk kg for its 32 functions, so it scales them by 2^-e with its own
// chunk exponent e = ilogb(max |F|) + 1 (at least -1000) and stores e in
// cexp[kg][b]: one read of F instead of a maximum pass over all of it
// before the split.  The product rescales each chunk's FP32 sums by
// 2^(e - E_b) at the fold of its accumulators, E_b the function's largest
// chunk exponent (k_colscale).
// SCM 0: no scale (BF16); 1: chunk exponents (above); 2: the function's
// exponent colexp[b] from k_colmax (direct form).
template <typename H16, int NPC, int SCM>
__global__ __launch_bounds__(256) void k_split_cols(const double *__restrict__ F, int P, int B, int K16, int RB,
                                                    H16 *__restrict__ X, int64_t piece_stride,
                                                    int *__restrict__ cexp, int64_t Bpad) {
    // block (rb, kg): wave w writes the kSplitKW consecutive k fragments from
    // (4 kg + w) kSplitKW on, so a block's fragments of one piece are one
    // contiguous 4 kSplitKW KiB run; consecutive blocks take consecutive rb,
    // so the reads sweep rows of F in order
    const int rb = (int)(blockIdx.x % (unsigned)RB), kg = (int)(blockIdx.x / (unsigned)RB);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = rb * 32 + (lane & 31);
    // every load of the wave's kSplitKW fragments first, branch-free (indices
    // past F clamped, their values zeroed below), so that all are in flight
    // together; masked loads would each wait for the one before
    const int bc = b < B ? b : B - 1;
    double v[kSplitKW][8];
#pragma unroll
    for (int j = 0; j < kSplitKW; ++j) {
        const int k = ((kg * 4 + w) * kSplitKW + j) * 16 + (lane >> 5) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            v[j][e] = __builtin_nontemporal_load(F + (int64_t)(k + e < P ? k + e : P - 1) * B + bc);
    }
    // (the pieces of fragments past K16 are computed and dropped: only their
    // stores are conditional, so the loads above stay ahead of every use)
    double m = 0.0;
#pragma unroll
    for (int j = 0; j < kSplitKW; ++j) {
        const int k = ((kg * 4 + w) * kSplitKW + j) * 16 + (lane >> 5) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            v[j][e] = (b < B && k + e < P) ? v[j][e] : 0.0;
            m = fmax(m, fabs(v[j][e]));
        }
    }
    if constexpr (SCM == 2) {
        const double sc = b < B ? ldexp(1.0, -max(cexp[b], -1000)) : 1.0;
#pragma unroll
        for (int j = 0; j < kSplitKW; ++j)
#pragma unroll
            for (int e = 0; e < 8; ++e) v[j][e] *= sc;
    }
    if constexpr (SCM == 1) {
        __shared__ double red[4][32];
        m = fmax(m, __shfl_xor(m, 32, 64));  // lanes l and l + 32 hold the same function
        if (lane < 32) red[w][lane] = m;
        __syncthreads();
        const int l = lane & 31;
        m = fmax(fmax(red[0][l], red[1][l]), fmax(red[2][l], red[3][l]));
        const int ex = m > 0.0 ? max(ilogb(m) + 1, -1000) : -1000;
        if (w == 0 && lane < 32) cexp[(int64_t)kg * Bpad + b] = ex;
        const double sc = ldexp(1.0, -ex);
#pragma unroll
        for (int j = 0; j < kSplitKW; ++j)
#pragma unroll
            for (int e = 0; e < 8; ++e) v[j][e] *= sc;
    }
#pragma unroll
    for (int j = 0; j < kSplitKW; ++j) {
        const int k16 = (kg * 4 + w) * kSplitKW + j;
        const int k = k16 * 16 + (lane >> 5) * 8;
        u32x4 out[NPC];
        split8<H16, NPC>(v[j], out);
        if (k16 < K16) {
#pragma unroll
            for (int i = 0; i < NPC; ++i)
                *reinterpret_cast<u32x4 *>(X + i * piece_stride + fo_offset(b, k, K16)) = out[i];
        }
    }
}

// Per function b < Bt (the rows of the call's block tiles; cexp's row
// stride is Bpad): E_b = max over chunks of cexp[c][b] (the exponent
// of max_p |F[p][b]|, applied by the DST or the direct form's epilogue), and
// the chunk factors 2^(cexp[c][b] - E_b) as biased exponent bytes
// u = max(cexp - E_b + 127, 0) (the FP32 bit pattern u << 23; 0, a zero
// factor, for chunks 2^127 or more below the function's largest, whose share
// is far below FP32's rounding) in cs[b / 128][c][b % 128] for c < nchp (the
// product's block tile of 128 functions reads its nchp * 128 bytes as one
// run; chunks c >= nch are zero).
__global__ __launch_bounds__(256) void k_colscale(const int *__restrict__ cexp, int nch, int nchp, int64_t Bpad,
                                                  int64_t Bt, int B, int *__restrict__ colexp,
                                                  unsigned char *__restrict__ cs) {
    // thread (b, c): blockIdx.y = c < nchp; every thread takes E_b over all
    // chunks itself (nch independent, cached loads)
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (b >= Bt) return;
    int E = -1000;
    for (int i = 0; i < nch; ++i) E = max(E, cexp[i * Bpad + b]);
    if (c == 0 && b < B) colexp[b] = E;
    cs[(b >> 7) * nchp * 128 + c * 128 + (b & 127)] =
        c < nch ? (unsigned char)max(0, cexp[c * Bpad + b] - E + 127) : (unsigned char)0;
}

hipError_t launch_split_rows(int h16, const double *S, int64_t roff, int64_t rs, int64_t cs, int H, int P, int Kp,
                             int Hpad, int npc, void *Y, int64_t piece_stride, int *rowexp, int scaled,
                             hipStream_t s) {
    const Strided st{S, roff, rs, cs};
    if (scaled) {
        hipLaunchKernelGGL(k_rowexp, dim3(H), dim3(256), 0, s, st, P, rowexp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int K16 = Kp / 16;
    const int64_t nfrag = (int64_t)(Hpad / 32) * K16;
    const dim3 grid((unsigned)((nfrag * 64 + 255) / 256));
    const int *re = scaled ? rowexp : nullptr;
#define LC_SR(T, NP)                                                                                     \
    if (npc == NP) {                                                                                     \
        hipLaunchKernelGGL((k_split_rows<T, NP>), grid, dim3(256), 0, s, st, H, P, K16, nfrag, (T *)Y,  \
                           piece_stride, re);                                                            \
        return hipGetLastError();                                                                        \
    }
    if (h16 == kBF16) {
        LC_SR(__bf16, 1) LC_SR(__bf16, 2) LC_SR(__bf16, 3)
    } else {
        LC_SR(_Float16, 1) LC_SR(_Float16, 2) LC_SR(_Float16, 3)
    }
#undef LC_SR
    return hipErrorInvalidValue;
}

hipError_t launch_split_cols(int h16, const double *F, int P, int B, int Kp, int npc, void *X,
                             int64_t piece_stride, int64_t Bpad, int *cexp, int *colexp, unsigned char *cscale,
                             hipStream_t s, int bm) {
    const int K16 = Kp / 16;
    if (bm <= 0 || bm % kGemmBM) return hipErrorInvalidValue;
    const int64_t Bt = ((int64_t)B + bm - 1) / bm * bm;  // rows of the call's block tiles
    const int RB = (int)(Bt / 32);
    const int nch = (K16 + kExpChunk16 - 1) / kExpChunk16;
    const dim3 grid((unsigned)((int64_t)RB * nch));
    // FP16: chunk exponents when cscale is given (Abel form), else one
    // exponent per function (direct form)
    const int mode = h16 != kF16 ? 0 : (cscale ? 1 : 2);
    if (mode && !colexp) return hipErrorInvalidValue;
    if (mode == 1 && !cexp) return hipErrorInvalidValue;
    hipError_t e = hipSuccess;
    if (mode == 2) {
        hipLaunchKernelGGL(k_colexp_init, dim3((B + 255) / 256), dim3(256), 0, s, B, colexp);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_colmax, dim3((B + 255) / 256, (P + 63) / 64), dim3(256), 0, s, F, P, B, colexp);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    int *ce = mode == 1 ? cexp : colexp;
#define LC_SC(T, NP, SCV)                                                                                \
    if (npc == NP) {                                                                                     \
        hipLaunchKernelGGL((k_split_cols<T, NP, SCV>), grid, dim3(256), 0, s, F, P, B, K16, RB, (T *)X, \
                           piece_stride, ce, Bpad);                                                      \
        e = hipGetLastError();                                                                           \
    } else
    e = hipErrorInvalidValue;
    if (mode == 0) {
        LC_SC(__bf16, 1, 0) LC_SC(__bf16, 2, 0) LC_SC(__bf16, 3, 0) {}
        return e;
    }
    if (mode == 2) {
        LC_SC(_Float16, 1, 2) LC_SC(_Float16, 2, 2) LC_SC(_Float16, 3, 2) {}
        return e;
    }
    LC_SC(_Float16, 1, 1) LC_SC(_Float16, 2, 1) LC_SC(_Float16, 3, 1) {}
#undef LC_SC
    if (e != hipSuccess) return e;
    const int nchp = mgemm_scale_chunks(Kp);
    hipLaunchKernelGGL(k_colscale, dim3((unsigned)((Bt + 255) / 256), (unsigned)nchp), dim3(256), 0, s, cexp, nch,
                       nchp, Bpad, Bt, B, colexp, cscale);
    return hipGetLastError();
}

// ------------------------------------------------------------ MFMA GEMM ---
// Block tile 64 WR (b) x 128 (j), 2 WR waves in WR x 2 (WR = 2: 128 x 128,
// WR = 4: 256 x 128), each wave 64 x 64 = 2 x 2 MFMA 32x32x16 tiles; the
// 256-row block has twice the products per stage copy at the same two waves
// per SIMD.  K advances KS per stage through a ring of NS LDS
// stages filled by direct global->LDS copies (16 bytes per lane, one 1 KiB
// fragment per wave instruction): the copy of stage kt + NS - 1 is issued
// while stage kt is multiplied, and each wave waits only for the copies of
// the stage it is about to read.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

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

// s_waitcnt immediate that waits for at most n outstanding vector-memory
// operations and leaves the other counters alone.
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }
constexpr int kLgkmZero = 15 | (3 << 14) | (7 << 4);  // lgkmcnt(0) only

// Workgroup barrier that orders the LDS accesses around it (compiler fence
// plus s_barrier) without the full memory fence of __syncthreads, whose
// vmcnt(0) would drain the copies in flight for later stages.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_s_waitcnt(kLgkmZero);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Epilogue: D64 = false writes the FP32 sums to Out[b][j]; D64 = true writes
// FP64 C[b][j] = sum * 2^(rowexp[j] + colexp[b]) (exponent arrays may be
// null), the finished coefficients of the direct Legendre-matrix form.
template <typename H16, int MODE, int KS, int NS, bool D64, int KCH, int WR = 2, bool T64 = false>
__global__ __launch_bounds__(128 * WR) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mgemm(
    const H16 *__restrict__ X, int64_t xps, const H16 *__restrict__ Y, int64_t yps, int Bn, int Hn, int K16,
    float *__restrict__ Out, int ldo, double *__restrict__ C64, const int *__restrict__ rowexp,
    const int *__restrict__ colexp, const unsigned char *__restrict__ cscale, int nchp) {
    using PR = Prods<MODE>;
    // FP16 Abel form: per-chunk column factors (the direct form's FP16 pieces
    // carry one exponent per function, applied by the epilogue)
    constexpr bool CS = std::is_same<H16, _Float16>::value && !D64;
    constexpr int NX = PR::nx, NY = PR::ny;
    constexpr int KF = KS / 16;                         // fragments along k per stage
    constexpr int NW = 2 * WR, RX = 2 * WR;             // waves; row blocks of 32 of X per block
    constexpr int FX = NX * RX * KF, FY = NY * 4 * KF;  // fragments per stage
    constexpr int FST = FX + FY;
    static_assert(FST % NW == 0, "stage fragments must split over the waves");
    constexpr int DPW = FST / NW;  // copies per wave per stage
    static_assert(DPW * (NS - 2) < 64, "vmcnt range");
    extern __shared__ __attribute__((aligned(1024))) u32x4 ring[];  // [NS][FST][64]
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: the copies' LDS base
    const int wm = (wave >> 1) * 2, wn = (wave & 1) * 2;  // row blocks of 32 owned by the wave
    const int ntn = (Hn + 127) / 128;
    const int rbx = (blockIdx.x / ntn) * RX, rby = (blockIdx.x % ntn) * 4;  // first row blocks of X and Y

    // copy d of a stage (d = wave + 4 i): X fragments first (piece, row
    // block, k fragment), then Y fragments
    auto issue = [&](int kt) {
        u32x4 *st = ring + (kt % NS) * FST * 64;
#pragma unroll
        for (int i = 0; i < DPW; ++i) {
            const int d = wave + NW * i;
            const H16 *src;
            if (d < FX) {
                const int u = d / (RX * KF), r = (d / KF) % RX, kf = d % KF;
                src = X + u * xps + ((int64_t)(rbx + r) * K16 + kt * KF + kf) * 512;
            } else {
                const int e = d - FX;
                const int v = e / (4 * KF), r = (e / KF) % 4, kf = e % KF;
                src = Y + v * yps + ((int64_t)(rby + r) * K16 + kt * KF + kf) * 512;
            }
            __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(src + lane * 8),
                                             (__attribute__((address_space(3))) void *)(st + d * 64), 16, 0, 0);
        }
    };

    static_assert(kExpChunk16 % KCH == 0, "a fold must not span two exponent chunks");
    // Two-level accumulation: the MFMA accumulator covers KCH K-steps of 16
    // and is then added into a second total and cleared, so that no FP32
    // chain runs over more than KCH MFMA steps per product (each step
    // rounds relative to the running partial sum).  The total is FP32 for
    // the Abel product (whose output is FP32; the DST that follows averages
    // the errors of phi) and FP64 with shorter chunks for the direct form,
    // where nothing averages the accumulation error of a coefficient.
    using TotT = typename std::conditional<D64 || T64, double, float>::type;
    f32x16 acc[2][2];
    TotT tot[2][2][16];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acc[a][b][v] = 0.f;
                tot[a][b][v] = 0;
            }

    // FP16: the chunk factors of the block's 128 functions, [nchp][128] bytes
    // after the ring, copied before the first stage so that the first
    // stage's wait covers them
    const unsigned *scl = reinterpret_cast<const unsigned *>(ring + NS * FST * 64);
    if constexpr (CS) {  // RX/4 tiles of 128 functions, consecutive in cscale
        const unsigned char *src = cscale + (int64_t)(rbx / 4) * nchp * 128;
        for (int i = wave; i < (RX / 4) * nchp / 8; i += NW)
            __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(src + i * 1024 + lane * 16),
                                             (__attribute__((address_space(3))) void *)(ring + NS * FST * 64 + i * 64),
                                             16, 0, 0);
    }
    // fold of the accumulators into the totals; FP16 scales chunk c's sums of
    // row r by 2^(u - 127), u its factor byte (D rows of lane l, register v:
    // 8 (v/4) + 4 (l/32) + v%4, so four consecutive bytes per v/4)
    auto fold = [&](int c) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                unsigned wd = 0;
                if constexpr (CS)
                    wd = scl[(((wm + a) >> 2) * nchp * 128 + c * 128 + ((wm + a) & 3) * 32 + 8 * g + 4 * (lane >> 5)) >> 2];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float f = CS ? __builtin_bit_cast(float, ((wd >> (8 * i)) & 0xffu) << 23) : 1.f;
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int v = 4 * g + i;
                        tot[a][b][v] += CS ? (TotT)(acc[a][b][v] * f) : (TotT)acc[a][b][v];
                        acc[a][b][v] = 0.f;
                    }
                }
            }
    };

    const int nk = K16 / KF;  // stages
#pragma unroll
    for (int s = 0; s < NS - 1; ++s)
        if (s < nk) issue(s);
    int kstep = 0;
    for (int kt = 0; kt < nk; ++kt) {
        // the copies of stage kt are the oldest of this wave's outstanding ones
        if (kt + NS - 2 < nk) __builtin_amdgcn_s_waitcnt(vmcnt_imm(DPW * (NS - 2)));
        else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        lds_barrier();  // every wave's copies of stage kt have landed; stage kt - 1 is free
        if (kt + NS - 1 < nk) issue(kt + NS - 1);
        const u32x4 *st = ring + (kt % NS) * FST * 64;
#pragma unroll
        for (int kf = 0; kf < KF; ++kf) {
            u32x4 fx[NX][2], fy[NY][2];
#pragma unroll
            for (int u = 0; u < NX; ++u)
#pragma unroll
                for (int a = 0; a < 2; ++a) fx[u][a] = st[((u * RX + wm + a) * KF + kf) * 64 + lane];
#pragma unroll
            for (int v = 0; v < NY; ++v)
#pragma unroll
                for (int b = 0; b < 2; ++b) fy[v][b] = st[(FX + (v * 4 + wn + b) * KF + kf) * 64 + lane];
#pragma unroll
            for (int pi = 0; pi < PR::n; ++pi)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = Mfma<H16>::run(fx[PR::u[pi]][a], fy[PR::v[pi]][b], acc[a][b]);
            if (++kstep == KCH) {  // KCH divides kExpChunk16: a fold never spans two chunks
                kstep = 0;
                fold((kt * KF + kf) / kExpChunk16);
            }
        }
    }
    fold((K16 - 1) / kExpChunk16);
    // D layout: lane l, register v -> row 8 (v/4) + 4 (l/32) + (v%4), col l%32
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = (rbx + wm + a) * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int col = (rby + wn + b) * 32 + (lane & 31);
                if (row < Bn && col < Hn) {
                    if constexpr (D64) {
                        const int ex = (rowexp ? rowexp[col] : 0) + (colexp ? max(colexp[row], -1000) : 0);
                        C64[(int64_t)row * ldo + col] = ldexp(tot[a][b][v], ex);
                    } else {
                        Out[(int64_t)row * ldo + col] = (float)tot[a][b][v];
                    }
                }
            }
}

// stage depth (k per stage, ring length) of each mode: LDS per block is
// NS * (NX + NY) * 4 * KS/16 KiB (+ nchp / 8 KiB of FP16 chunk factors, at
// most 8 KiB for P <= 16384), at most 80 KiB so that two blocks share a CU
static void mgemm_defaults(int mode, int h16, bool d64, int &ks, int &ns, int &kch) {
    if (!ks) {
        ks = mode == 1 ? 32 : 16;
        ns = mode == 6 ? 3 : 4;
    }
    // FP64 chunk length of the direct form: 4 K-steps for fp16x3 and bf16x6
    // (at 8 their E_a reaches 1.0e-7 and 1.25e-7), 8 for bf16x3 and fp16x1,
    // whose 16-bit representation limits them above that anyway
    const bool long_chunks = mode == 1 || (mode == 3 && h16 == kBF16);
    // FP32 chunk length of the Abel form: 16 K-steps for the three-product
    // modes (their fold into the second total every 8 steps cost 5%; E_a at
    // full size 1.1e-8 either way), 8 for the six-product mode (no faster at
    // 16, E_a 1.8e-8 -> 2.9e-8) and for one product
    kch = d64 ? (kch ? kch : (long_chunks ? 8 : 4)) : (kch ? kch : (mode == 3 ? 16 : 8));
}

bool mgemm_shape_supported(int mode, int ks, int ns, int kch, bool direct) {
    if (direct ? (kch != 0 && kch != 2 && kch != 4 && kch != 8) : (kch != 0 && kch != 8 && kch != 16)) return false;
    if (ks == 0 && ns == 0) return true;
    static const int built[][3] = {{1, 32, 2}, {1, 32, 4}, {1, 16, 4}, {3, 32, 2}, {3, 16, 2},
                                   {3, 16, 3}, {3, 16, 4}, {6, 16, 2}, {6, 16, 3}};
    for (auto &b : built)
        if (b[0] == mode && b[1] == ks && b[2] == ns) return true;
    return false;
}

hipError_t launch_mgemm(int h16, int mode, const void *X, int64_t xps, const void *Y, int64_t yps, int Bn, int Hn,
                        int Kp, float *Out, int ldo, double *C64, const int *rowexp, const int *colexp,
                        const unsigned char *cscale, int ks, int ns, int kch, hipStream_t s, int wr, bool t64) {
    if (Kp % 32) return hipErrorInvalidValue;
    const bool d64 = C64 != nullptr;
    if (h16 == kF16 && !d64 && !cscale) return hipErrorInvalidValue;
    const int nchp = mgemm_scale_chunks(Kp);
    const int K16 = Kp / 16;
    int KS = ks, NS = ns;
    mgemm_defaults(mode, h16, d64, KS, NS, kch);
    if (wr != 2 && wr != 4) return hipErrorInvalidValue;
    const int grid = ((Bn + 64 * wr - 1) / (64 * wr)) * ((Hn + 127) / 128);
    const int npx = mode == 1 ? 1 : (mode == 3 ? 2 : 3);
    const size_t lds = (size_t)NS * npx * (2 * wr + 4) * (KS / 16) * 1024 +
                       (h16 == kF16 && !d64 ? (size_t)(wr / 2) * nchp * 128 : 0);
#define LC_MG3(T, MV, KSV, NSV, DV, KV, WV, TV)                                                                 \
    if (mode == MV && KS == KSV && NS == NSV && d64 == DV && kch == KV && wr == WV && t64 == TV) {              \
        if (lds > 65536) {                                                                                      \
            hipError_t e = hipFuncSetAttribute((const void *)k_mgemm<T, MV, KSV, NSV, DV, KV, WV, TV>,          \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);           \
            if (e != hipSuccess) return e;                                                                      \
        }                                                                                                       \
        hipLaunchKernelGGL((k_mgemm<T, MV, KSV, NSV, DV, KV, WV, TV>), dim3(grid), dim3(128 * WV), lds, s,      \
                           (const T *)X, xps, (const T *)Y, yps, Bn, Hn, K16, Out, ldo, C64, rowexp, colexp,    \
                           cscale, nchp);                                                                       \
        return hipGetLastError();                                                                               \
    }
#define LC_MG2(T, MV, KSV, NSV, DV, KV, WV) LC_MG3(T, MV, KSV, NSV, DV, KV, WV, false)
#define LC_MG1(T, MV, KSV, NSV, DV, KV) LC_MG2(T, MV, KSV, NSV, DV, KV, 2)
#define LC_MG(T, MV, KSV, NSV)                                                                                  \
    LC_MG1(T, MV, KSV, NSV, false, 8) LC_MG1(T, MV, KSV, NSV, false, 16)                                        \
    LC_MG1(T, MV, KSV, NSV, true, 2) LC_MG1(T, MV, KSV, NSV, true, 4)                                           \
    LC_MG1(T, MV, KSV, NSV, true, 8)
#define LC_MG_ALL(T)                                                                                            \
    LC_MG(T, 1, 32, 2) LC_MG(T, 1, 32, 4) LC_MG(T, 1, 16, 4)                                                    \
    LC_MG(T, 3, 32, 2) LC_MG(T, 3, 16, 2) LC_MG(T, 3, 16, 3) LC_MG(T, 3, 16, 4)                                 \
    LC_MG(T, 6, 16, 2) LC_MG(T, 6, 16, 3)
    if (h16 == kBF16) {
        LC_MG_ALL(__bf16)
        LC_MG2(__bf16, 3, 16, 4, false, 16, 4) LC_MG2(__bf16, 3, 16, 4, true, 8, 4)
        LC_MG3(__bf16, 6, 16, 3, false, 8, 2, true) LC_MG3(__bf16, 3, 16, 4, false, 16, 4, true)
        LC_MG3(__bf16, 3, 16, 4, false, 16, 2, true)
    } else {
        LC_MG_ALL(_Float16)
        LC_MG2(_Float16, 3, 16, 4, false, 16, 4) LC_MG2(_Float16, 3, 16, 4, true, 4, 4)
        LC_MG3(_Float16, 3, 16, 4, false, 16, 4, true) LC_MG3(_Float16, 3, 16, 4, false, 16, 2, true)
    }
#undef LC_MG3
#undef LC_MG2
#undef LC_MG_ALL
#undef LC_MG
#undef LC_MG1
    return hipErrorInvalidValue;
}

// ------------------------------------------------- batched DST of rows ---
// Function b reads phi_j = Out[b][j-1] * 2^(rowexp[j-1] + colexp[b]); SC
// (rowexp given) is a template argument, so that the reads of phi carry no
// branch and the pack can issue them together.
template <int T, typename PhiT, bool SC>
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
            if constexpr (SC) return ldexp(v, re[m - 1] + ce);
            return v;
        }
    } ph{row, rowexp, ce};
    const OctantRegs oc = octant_load<T>(tw_fft, L);
    dst_pack_lds<T, 8>(lds, ph, H, L, tw_pre, tw_pack);
    octant_store<T>(lds + L, oc, L);
    __syncthreads();
    fft_lds_one<T, 8>(lds, L, sch, tw_fft, lds + L);
    dst_post_block<T>(C + (int64_t)b * N, (int)N, lds, (int)H);
}

// ------------------------------------- twist folded into the Abel matrix ---
// The DST pack of eq. (2.4) (twist e^{i pi k/(2H)} and the half-length
// complex recombination of dst_pack) is linear in phi, so applied to the
// rows of A it gives the matrix whose product with F is the packed input Z
// of the FFT: rows 2k and 2k+1 of Ap are Re Z_k and Im Z_k (k < L = H/2) as
// combinations of the rows H-k, k, L-k, L+k of A (row 0, y = 0, is zero:
// that is phi_0 = 0 of V_0 = phi_H).  Block k, threads over the columns.
__global__ __launch_bounds__(256) void k_apack(const double *__restrict__ A, int P, int64_t H, int64_t L,
                                               const double2 *__restrict__ tw_pre,
                                               const double2 *__restrict__ tw_pack, double *__restrict__ Ap) {
    const int64_t k = blockIdx.x;
    const double2 t0 = tw_pre[k], t1 = tw_pre[k + L], tp = tw_pack[k];
    const double *rHk = A + (H - k) * P, *rk = A + k * P, *rLk = A + (L - k) * P, *rLpk = A + (L + k) * P;
    double *re = Ap + 2 * k * P, *im = re + P;
    for (int p = threadIdx.x; p < P; p += 256) {
        const double2 vk = cmul(t0, make_double2(rHk[p], -rk[p]));
        const double2 vkl = cmul(t1, make_double2(rLk[p], -rLpk[p]));
        const double2 sum = cadd(vk, vkl);
        const double2 r = cmul(tp, csub(vk, vkl));
        re[p] = sum.x - r.y;
        im[p] = sum.y + r.x;
    }
}

hipError_t launch_apack(const double *A, int P, int64_t H, int64_t L, const double2 *tw_pre, const double2 *tw_pack,
                        double *Ap, hipStream_t s) {
    hipLaunchKernelGGL(k_apack, dim3((unsigned)L), dim3(256), 0, s, A, P, H, L, tw_pre, tw_pack, Ap);
    return hipGetLastError();
}

// Batched FFT + unpack/rescale of rows that already hold the packed input:
// function b's Z_k is (Out[b][2k], Out[b][2k+1]) times 2^(rowexp[2k or
// 2k+1] + colexp[b]) when SC; every thread's loads (up to 8 values) are
// issued before the first is stored to LDS.
// FIX: L == 8T, the kernel holds only that length's compile-time passes.
template <int T, typename PhiT, bool SC, bool FIX>
__global__ __launch_bounds__(T) void k_gdst_z(const PhiT *__restrict__ Out, int ldo, const int *__restrict__ rowexp,
                                              const int *__restrict__ colexp, int64_t H, int Lr, int64_t N,
                                              const double2 *__restrict__ tw_fft, FftSched sch,
                                              double *__restrict__ C) {
    extern __shared__ double2 lds[];
    const int L = FIX ? 8 * T : Lr;
    using P2 = typename std::conditional<std::is_same<PhiT, float>::value, float2, double2>::type;
    const int b = blockIdx.x;
    const P2 *row = reinterpret_cast<const P2 *>(Out + (int64_t)b * ldo);
    const int ce = colexp ? max(colexp[b], -1000) : 0;
    const OctantRegs oc = octant_load<T>(tw_fft, L);
    P2 v[8];
    int2 ex[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = min((int)threadIdx.x + i * T, L - 1);
        v[i] = row[k];
        if constexpr (SC) ex[i] = reinterpret_cast<const int2 *>(rowexp)[k];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = (int)threadIdx.x + i * T;
        if (k < L) {
            if constexpr (SC) lds[k] = make_double2(ldexp((double)v[i].x, ex[i].x + ce), ldexp((double)v[i].y, ex[i].y + ce));
            else lds[k] = make_double2((double)v[i].x, (double)v[i].y);
        }
    }
    octant_store<T>(lds + L, oc, L);
    __syncthreads();
    if constexpr (FIX) fixed_passes<T, 8 * T, 1, true>(lds, tw_fft, lds + L);
    else fft_lds_one<T, 8>(lds, L, sch, tw_fft, lds + L);
    dst_post_block<T, true>(C + (int64_t)b * N, (int)N, lds, (int)H);
}

hipError_t launch_gdst_z(int phi_is_fp32, const void *Out, int ldo, const int *rowexp, const int *colexp, int B,
                         int64_t H, int64_t L, int64_t N, const double2 *tw_fft, const FftSched &sch, double *C,
                         hipStream_t s) {
    const size_t lds = fft_lds_bytes(L);
    // one radix-8 butterfly per thread and pass for power-of-two lengths
    // (compile-time passes); otherwise the length classes of launch_gdst
    int T = L <= 512 ? 64 : (L <= 2048 ? 256 : 1024);
    if ((L & (L - 1)) == 0 && L >= 512) T = (int)(L / 8);
    if (L > 8 * T || (ldo & 1)) return hipErrorInvalidValue;
    const bool fix = L == 8 * T;
#define LC_GZ1(TV, PT, SCV, FV)                                                                        \
    if (T == TV && (rowexp != nullptr) == SCV && fix == FV) {                                          \
        if (lds > 65536) {                                                                             \
            hipError_t e = hipFuncSetAttribute((const void *)k_gdst_z<TV, PT, SCV, FV>,                \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);  \
            if (e != hipSuccess) return e;                                                             \
        }                                                                                              \
        hipLaunchKernelGGL((k_gdst_z<TV, PT, SCV, FV>), dim3(B), dim3(TV), lds, s, (const PT *)Out, ldo, \
                           rowexp, colexp, H, (int)L, N, tw_fft, sch, C);                              \
        return hipGetLastError();                                                                      \
    }
#define LC_GZ(TV, PT) LC_GZ1(TV, PT, true, true) LC_GZ1(TV, PT, false, true) \
    LC_GZ1(TV, PT, true, false) LC_GZ1(TV, PT, false, false)
    if (phi_is_fp32) {
        LC_GZ(64, float)
        LC_GZ(128, float)
        LC_GZ(256, float)
        LC_GZ(512, float)
        LC_GZ(1024, float)
    } else {
        LC_GZ(64, double)
        LC_GZ(128, double)
        LC_GZ(256, double)
        LC_GZ(512, double)
        LC_GZ(1024, double)
    }
#undef LC_GZ
#undef LC_GZ1
    return hipErrorInvalidValue;
}

hipError_t launch_gdst(int phi_is_fp32, const void *Out, int ldo, const int *rowexp, const int *colexp, int B,
                       int64_t H, int64_t L, int64_t N, const double2 *tw_pre, const double2 *tw_pack,
                       const double2 *tw_fft, const FftSched &sch, double *C, hipStream_t s) {
    const size_t lds = fft_lds_bytes(L);
    int T = L <= 512 ? 64 : (L <= 2048 ? 256 : 1024);
    if (L > 8 * T) return hipErrorInvalidValue;
#define LC_GD1(TV, PT, SCV)                                                                            \
    if (T == TV && (rowexp != nullptr) == SCV) {                                                       \
        if (lds > 65536) {                                                                             \
            hipError_t e = hipFuncSetAttribute((const void *)k_gdst_lds<TV, PT, SCV>,                  \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);  \
            if (e != hipSuccess) return e;                                                             \
        }                                                                                              \
        hipLaunchKernelGGL((k_gdst_lds<TV, PT, SCV>), dim3(B), dim3(TV), lds, s, (const PT *)Out, ldo, rowexp, \
                           colexp, H, (int)L, N, tw_pre, tw_pack, tw_fft, sch, C);                     \
        return hipGetLastError();                                                                      \
    }
#define LC_GD(TV, PT) LC_GD1(TV, PT, true) LC_GD1(TV, PT, false)
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
#undef LC_GD1
    return hipErrorInvalidValue;
}

}  // namespace lc
