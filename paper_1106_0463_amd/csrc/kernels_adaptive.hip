// Composite Abel rule (breakpoints of f, geometric grading toward x = 1,
// per-row node counts): node construction and the segmented quadrature
// reduction.
//
// With x = 1 - 2 s_j^2 (1 - t^2) (s_j = sin(y_j / 2)), eq. (2.14) becomes
// phi_j = 2 s_j integral_0^1 f dt, and the rule cuts t in [0, 1] into
// panels.  Each panel is one segment of contiguous samples: its nodes are
// 1 - t = E + h d_i with d_i = 1 - tau_i from the panel's Gauss rule (the
// positive half of the 2q-point rule on the first panel, the q-point rule on
// the others), and its weights are scale * w_i.  Rows are stored in order,
// a row's panels in order of increasing t.
#include <hip/hip_runtime.h>

#include "dd_device.h"
#include "lc_internal.h"
#include "quad_device.h"

namespace lc {

// One block per segment: nodes in double-double, rounded once to FP64;
// padding slots repeat the last node.
__global__ __launch_bounds__(256) void k_anodes(const ASeg *__restrict__ segs, int64_t nseg,
                                                const double2 *__restrict__ dtab,
                                                const double2 *__restrict__ rowA, double *__restrict__ x) {
    const double2 two = make_double2(2.0, 0.0);
    for (int64_t k = blockIdx.x; k < nseg; k += gridDim.x) {
        const ASeg sg = segs[k];
        const double2 a = rowA[sg.row];
        for (int i = threadIdx.x; i < sg.qp; i += 256) {
            const int ii = i < sg.q ? i : sg.q - 1;
            const double2 e = dd_add(sg.E, dd_mul(sg.h, dtab[sg.woff + ii]));   // 1 - t
            const double2 omt2 = dd_mul(e, dd_add(two, make_double2(-e.x, -e.y)));  // 1 - t^2
            x[sg.off + i] = node_dd(a, omt2);
        }
    }
}

hipError_t launch_anodes(const ASeg *segs, int64_t nseg, const double2 *dtab, const double2 *rowA, double *x,
                         hipStream_t s) {
    const int64_t grid = nseg < 65536 ? nseg : 65536;
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(k_anodes, dim3((unsigned)grid), dim3(256), 0, s, segs, nseg, dtab, rowA, x);
    return hipGetLastError();
}

// G lanes per row: a group walks the segments of its row, each reduced with
// 16-byte loads of samples and of the (L2-resident) padded rule weights, and
// the lane partials are combined with the fixed-order butterfly.
//   phi[r] = s2[r] * sum_k scale_k sum_i w_i f_i
template <typename T, int G>
__global__ __launch_bounds__(256) void k_aquad(const T *__restrict__ f, const ASeg *__restrict__ segs,
                                               const int32_t *__restrict__ rseg, const int32_t *__restrict__ rows,
                                               int64_t nrows, const double *__restrict__ wtab,
                                               const double *__restrict__ s2, double *__restrict__ phi) {
    constexpr int VEC = 16 / sizeof(T);
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int64_t grp = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (64 / G) + lane / G;
    const int64_t ngrp = (int64_t)gridDim.x * (blockDim.x >> 6) * (64 / G);
    for (int64_t i = grp; i < nrows; i += ngrp) {
        const int r = rows[i];
        double acc = 0.0;
        for (int k = rseg[r]; k < rseg[r + 1]; ++k) {
            const ASeg sg = segs[k];
            // rule tables start at multiples of 4 doubles: 16-byte weight pairs
            const double part = row_partial<T, VEC, G, true>(f + sg.off, wtab + sg.woff, sg.qp / VEC, g);
            acc = fma(sg.scale, part, acc);
        }
        acc = group_sum<G>(acc);
        if (g == 0) phi[r] = s2[r] * acc;
    }
}

// Blocks of k_aquad<T, G> resident on one CU at once (occupancy API).
int aquad_blocks_per_cu(int prec, int G) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
#define LC_AO(T, GV)                                                                                   \
    if (G == GV) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)k_aquad<T, GV>, 256, 0);
    if (prec == LC_FP64) {
        LC_AO(double, 4) LC_AO(double, 8) LC_AO(double, 16) LC_AO(double, 32) LC_AO(double, 64)
    } else {
        LC_AO(float, 4) LC_AO(float, 8) LC_AO(float, 16) LC_AO(float, 32) LC_AO(float, 64)
    }
#undef LC_AO
    return (e == hipSuccess && n > 0) ? n : 4;
}

hipError_t launch_aquad(int prec, int G, int grid, const void *f, const ASeg *segs, const int32_t *rseg,
                        const int32_t *rows, int64_t nrows, const double *wtab, const double *s2, double *phi,
                        hipStream_t s) {
    if (nrows < 1) return hipSuccess;
#define LC_AQ(T, GV)                                                                                   \
    if (G == GV) {                                                                                     \
        hipLaunchKernelGGL((k_aquad<T, GV>), dim3(grid), dim3(256), 0, s, (const T *)f, segs, rseg, rows, \
                           nrows, wtab, s2, phi);                                                      \
        return hipGetLastError();                                                                      \
    }
    if (prec == LC_FP64) {
        LC_AQ(double, 4) LC_AQ(double, 8) LC_AQ(double, 16) LC_AQ(double, 32) LC_AQ(double, 64)
    } else {
        LC_AQ(float, 4) LC_AQ(float, 8) LC_AQ(float, 16) LC_AQ(float, 32) LC_AQ(float, 64)
    }
#undef LC_AQ
    return hipErrorInvalidValue;
}

}  // namespace lc
