// Internal declarations of the Abel-as-GEMM kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lc_internal.h"

namespace lc {

constexpr int kBF16 = 0, kF16 = 1;

// rows of F^T per block tile of the MFMA product (also the padding unit of
// the fragment-order operands)
constexpr int kGemmBM = 128;

// FP16 column scaling: one power-of-two exponent per function and chunk of
// kExpChunk16 K-steps of 16 samples; the product's block tile keeps the
// chunk factors of its functions in LDS, nchp = chunks rounded up to 8
// (one 1 KiB copy per 8 chunks of 128 functions).
constexpr int kExpChunk16 = 16;
inline int mgemm_scale_chunks(int Kp) {
    const int nch = (Kp / 16 + kExpChunk16 - 1) / kExpChunk16;
    return (nch + 7) / 8 * 8;
}

// MFMA product shape of a plan: k per LDS stage and ring length (ks, ns;
// 0: the per-mode default), and K-steps of 16 per flush of the FP32 MFMA
// accumulators into the second total (kch: 2, 4 or 8 for the direct form's
// FP64 totals, 8 or 16 for the Abel form's FP32 totals; 0: per mode).  True
// when the library holds a kernel for it.
bool mgemm_shape_supported(int mode, int ks, int ns, int kch, bool direct);

hipError_t launch_amat(int H, int P, int QA, const double *xc, const double *lam, const double2 *rowA,
                       const double2 *omt2, const double *wq, const double *s2, double *A, hipStream_t s);
// Y operand rows r < H, columns k < P read as S[(r + roff) rs + k cs]
hipError_t launch_split_rows(int h16, const double *S, int64_t roff, int64_t rs, int64_t cs, int H, int P, int Kp,
                             int Hpad, int npc, void *Y, int64_t piece_stride, int *rowexp, int scaled,
                             hipStream_t s);
hipError_t launch_transpose_a(const double *A, int H, int P, double *AT, hipStream_t s);
// F [P][B] -> X pieces over Bpad rows.  FP16 with cscale (Abel form): the
// chunk exponents cexp [nch][Bpad], the function exponents colexp [B] and
// the chunk factors cscale [Bpad/128][nchp][128]; FP16 without cscale
// (direct form): one exponent per function in colexp (a maximum pass over F
// first); BF16: no scale
hipError_t launch_split_cols(int h16, const double *F, int P, int B, int Kp, int npc, void *X,
                             int64_t piece_stride, int64_t Bpad, int *cexp, int *colexp, unsigned char *cscale,
                             hipStream_t s, int bm = kGemmBM);
// C64 == nullptr: FP32 sums into Out[Bn][ldo]; otherwise finished FP64
// values into C64[Bn][ldo] scaled by 2^(rowexp[j] + colexp[b]); FP16 with
// FP32 output folds each chunk's sums in with the factors cscale of the
// column split (required there; unused with C64)
hipError_t launch_mgemm(int h16, int mode, const void *X, int64_t xps, const void *Y, int64_t yps, int Bn, int Hn,
                        int Kp, float *Out, int ldo, double *C64, const int *rowexp, const int *colexp,
                        const unsigned char *cscale, int ks, int ns, int kch, hipStream_t s, int wr = 2,
                        bool t64 = false);
hipError_t launch_gdst(int phi_is_fp32, const void *Out, int ldo, const int *rowexp, const int *colexp, int B,
                       int64_t H, int64_t L, int64_t N, const double2 *tw_pre, const double2 *tw_pack,
                       const double2 *tw_fft, const FftSched &sch, double *C, hipStream_t s);

// Ap [H][P]: rows 2k, 2k+1 = Re, Im of the DST pack Z_k applied to the rows
// of A ([H+1][P], row 0 zero), k < L = H/2
hipError_t launch_apack(const double *A, int P, int64_t H, int64_t L, const double2 *tw_pre, const double2 *tw_pack,
                        double *Ap, hipStream_t s);
// batched FFT + unpack/rescale of packed rows (Out[b][2k], Out[b][2k+1]) = Z_k
hipError_t launch_gdst_z(int phi_is_fp32, const void *Out, int ldo, const int *rowexp, const int *colexp, int B,
                         int64_t H, int64_t L, int64_t N, const double2 *tw_fft, const FftSched &sch, double *C,
                         hipStream_t s);

}  // namespace lc
