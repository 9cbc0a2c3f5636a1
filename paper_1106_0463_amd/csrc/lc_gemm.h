// Internal declarations of the Abel-as-GEMM kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lc_internal.h"

namespace lc {

constexpr int kBF16 = 0, kF16 = 1;

// waves along b per block of the MFMA product (2 or 4; block tile 64*WM x 128)
extern int mgemm_wm;

hipError_t launch_amat(int H, int P, int QA, const double *xc, const double *lam, const double2 *rowA,
                       const double2 *omt2, const double *wq, const double *s2, double *A, hipStream_t s);
hipError_t launch_split_rows(int h16, const double *A, int H, int P, int ldk, int npc, void *Y,
                             int64_t piece_stride, int *rowexp, int scaled, hipStream_t s);
hipError_t launch_split_cols(int h16, const double *F, int P, int B, int ldk, int npc, void *X,
                             int64_t piece_stride, int *colexp, int scaled, hipStream_t s);
hipError_t launch_mgemm(int h16, int mode, const void *X, int64_t xps, const void *Y, int64_t yps, int Bn, int Hn,
                        int P, float *Out, int ldo, hipStream_t s);
hipError_t launch_gdst(int phi_is_fp32, const void *Out, int ldo, const int *rowexp, const int *colexp, int B,
                       int64_t H, int64_t L, int64_t N, const double2 *tw_pre, const double2 *tw_pack,
                       const double2 *tw_fft, const FftSched &sch, double *C, hipStream_t s);

}  // namespace lc
