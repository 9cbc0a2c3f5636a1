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

#include <climits>

#include "dd_device.h"
#include "lc_internal.h"
#include "quad_device.h"

namespace lc {

// One block per segment: nodes in double-double, rounded once to FP64;
// padding slots repeat the last node.
__global__ __launch_bounds__(256) void k_anodes(const ASeg *__restrict__ segs, int64_t nseg,
                                                const double2 *__restrict__ dtab,
                                                const double2 *__restrict__ rowA, double *__restrict__ x,
                                                bool comp) {
    const double2 two = make_double2(2.0, 0.0);
    for (int64_t k = blockIdx.x; k < nseg; k += gridDim.x) {
        const ASeg sg = segs[k];
        const double2 a = rowA[sg.row];
        for (int i = threadIdx.x; i < sg.qp; i += 256) {
            const int ii = i < sg.q ? i : sg.q - 1;
            const double2 e = dd_add(sg.E, dd_mul(sg.h, dtab[sg.woff + ii]));   // 1 - t
            const double2 omt2 = dd_mul(e, dd_add(two, make_double2(-e.x, -e.y)));  // 1 - t^2
            x[sg.off + i] = comp ? omx_dd(a, omt2) : node_dd(a, omt2);
        }
    }
}

hipError_t launch_anodes(const ASeg *segs, int64_t nseg, const double2 *dtab, const double2 *rowA, double *x,
                         hipStream_t s, bool comp) {
    const int64_t grid = nseg < 65536 ? nseg : 65536;
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(k_anodes, dim3((unsigned)grid), dim3(256), 0, s, segs, nseg, dtab, rowA, x, comp);
    return hipGetLastError();
}

// Orders the LDS accesses of one wave's lanes before and after it (a wave's
// LDS operations execute in order; this keeps the compiler from moving them
// across and waits for the writes).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Flattened reduction, G lanes per row: the panels of a row are contiguous
// in f, so the group reads the row as one run of chunks in windows of 4 G
// (one chunk per lane and step, four steps in flight), whatever the panel
// boundaries.  The row's panel table sits in the group's LDS slot.  A window
// inside one panel takes that panel's weights and scale; a window across
// boundaries looks the panel up per chunk.  All lanes of a wave reach the
// next row together (its groups reconverge after the window loop), so the
// table of the next row is written after every read of the current one.
//   phi[r] = s2[r] * sum_panels scale_k sum_i w_i f_i
// Blocks blk = 0 .. nblk - 1 of this lane count take rows blk * 256/G + group,
// striding by nblk * 256/G.
template <typename T, int G>
__device__ __forceinline__ void aflat_rows(const T *__restrict__ f, const ARow *__restrict__ rows, int64_t nrows,
                                           int blk, int nblk, const ATab *__restrict__ tab,
                                           const double *__restrict__ wtab, const double *__restrict__ s2,
                                           double *__restrict__ phi, ATab *lds) {
    constexpr int VEC = 16 / sizeof(T);
    constexpr int W = 4 * G;
    using V = typename VecOf<T, VEC>::type;
    const int g = threadIdx.x & (G - 1);
    const int gl = threadIdx.x / G;
    ATab *st = lds + gl * kAflatMaxSeg;
    const int64_t ngrp = (int64_t)nblk * (256 / G);
    for (int64_t i = (int64_t)blk * (256 / G) + gl; i < nrows; i += ngrp) {
        const ARow rd = rows[i];
        for (int j = g; j < rd.S; j += G) st[j] = tab[rd.k0 + j];
        wave_lds_sync();
        const V *p = reinterpret_cast<const V *>(f + rd.rbeg);
        const int nc = rd.nc, S = rd.S;
        int k = 0;
        int nxt = S > 1 ? st[1].cst : nc;
        int wb = st[0].wbase;
        double sc = st[0].scale;
        double acc = 0.0;
        for (int c0 = 0; c0 < nc; c0 += W) {
            const int c = c0 + g;
            V v[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) v[m] = (c + m * G < nc) ? ld_stream(p + c + m * G) : V{};
            if (c0 + W <= nxt) {
                double d[4][VEC], w[4][VEC];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    to_d(v[m], d[m]);
                    chunk_weights<VEC, true>(wtab, wb + c + m * G, w[m]);
                }
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    a0 = fma(w[0][e], d[0][e], a0);
                    a1 = fma(w[1][e], d[1][e], a1);
                    a0 = fma(w[2][e], d[2][e], a0);
                    a1 = fma(w[3][e], d[3][e], a1);
                }
                acc = fma(sc, a0 + a1, acc);
            } else {
                // a window across panel boundaries: the panel of each chunk
                // (and of the next window's first chunk) is the number of
                // panel starts at or below it.  Starts 1..k lie at or below
                // c0; the later ones are counted eight at a time with
                // independent LDS reads (no dependent walk), until a start
                // past the window ends the count.
                // Chunks past the row end (zero samples) take the last
                // chunk's panel and weights, so that all four weight loads
                // are unconditional and in flight together; their products
                // are dropped.
                int ce[4], kc[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    ce[m] = c + m * G < nc ? c + m * G : nc - 1;
                    kc[m] = k;
                }
                int kw = k;
                for (int j0 = k + 1; j0 < S; j0 += 8) {
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        const int j = j0 + jj;
                        const int cs = j < S ? st[j].cst : INT_MAX;
#pragma unroll
                        for (int m = 0; m < 4; ++m) kc[m] += cs <= ce[m] ? 1 : 0;
                        kw += cs <= c0 + W ? 1 : 0;
                    }
                    if (kw < j0 + 7) break;
                }
                double w[4][VEC];
#pragma unroll
                for (int m = 0; m < 4; ++m) chunk_weights<VEC, true>(wtab, st[kc[m]].wbase + ce[m], w[m]);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    double d[VEC];
                    to_d(v[m], d);
                    double part = 0.0;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) part = fma(w[m][e], d[e], part);
                    acc = fma(c + m * G < nc ? st[kc[m]].scale : 0.0, part, acc);  // + 0 past the end
                }
                k = kw;
                wb = st[k].wbase;
                sc = st[k].scale;
                nxt = k + 1 < S ? st[k + 1].cst : nc;
            }
        }
        acc = group_sum<G>(acc);
        if (g == 0) phi[rd.r] = s2[rd.r] * acc;
        wave_lds_sync();
    }
}

// One launch for every lane count: blocks [b0[j], b0[j+1]) take the rows of
// lane count 64 >> j (longest rows first in dispatch order); the LDS holds
// the table slots of the largest number of groups per block (G = 4).
template <typename T>
__global__ __launch_bounds__(256) void k_aflat(const T *__restrict__ f, AflatLaunch L, const ATab *__restrict__ tab,
                                               const double *__restrict__ wtab, const double *__restrict__ s2,
                                               double *__restrict__ phi) {
    __shared__ ATab lds[(256 / 4) * kAflatMaxSeg];
    const int b = blockIdx.x;
#define LC_AFR(J, GV)                                                                                  \
    if (b < L.b0[J + 1]) {                                                                             \
        aflat_rows<T, GV>(f, L.rows[J], L.nrows[J], b - L.b0[J], L.b0[J + 1] - L.b0[J], tab, wtab, s2, phi, lds); \
        return;                                                                                        \
    }
    LC_AFR(0, 64) LC_AFR(1, 32) LC_AFR(2, 16) LC_AFR(3, 8) LC_AFR(4, 4)
#undef LC_AFR
}

// Blocks of k_aflat<T> resident on one CU at once (occupancy API).
int aflat_blocks_per_cu(int prec) {
    int n = 0;
    const hipError_t e = prec == LC_FP64
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)k_aflat<double>, 256, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)k_aflat<float>, 256, 0);
    return (e == hipSuccess && n > 0) ? n : 4;
}

hipError_t launch_aflat(int prec, const AflatLaunch &L, const void *f, const ATab *tab, const double *wtab,
                        const double *s2, double *phi, hipStream_t s) {
    const int grid = L.b0[kAflatLanes];
    if (grid < 1) return hipSuccess;
    if (prec == LC_FP64)
        hipLaunchKernelGGL(k_aflat<double>, dim3(grid), dim3(256), 0, s, (const double *)f, L, tab, wtab, s2, phi);
    else
        hipLaunchKernelGGL(k_aflat<float>, dim3(grid), dim3(256), 0, s, (const float *)f, L, tab, wtab, s2, phi);
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
