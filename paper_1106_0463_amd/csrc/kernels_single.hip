// HIP kernels of the single-function path (gfx950, wave64):
//   * node construction  x_{jq} = 1 - 2 s_j^2 (1 - t_q^2)   (FP64, half-angle form)
//   * Abel quadrature reduction  phi_j = 2 s_j sum_q w_q f[j][q]   (HBM-bound)
//   * DST-III of eq. (2.4) through an LDS Stockham FFT of length H/2, fused
//     with the twist and the (2n+1) rescale; four-step form for long FFTs.
#include <hip/hip_runtime.h>

#include "dd_device.h"
#include "fft_lds.h"
#include "lc_internal.h"
#include "quad_device.h"

namespace lc {

// ---------------------------------------------------------------- nodes ---
// Row r (r = 0..H-1) is y_j = pi j / H with j = r + 1, column q the q-th
// largest positive Gauss node t_q.  x_{jq} = 1 - A_j B_q with
// A_j = 2 sin^2(y_j / 2) and B_q = 1 - t_q^2 (the half-angle form: no
// cancellation in cos y near y = 0), both given as double-double pairs
// (hi + lo, from long-double host values).  The product and the
// subtraction are carried out in double-double with FMA, so x is the FP64
// value nearest the exact node in all but rare half-way cases.
__global__ __launch_bounds__(256) void k_nodes(int64_t H, int Q, const double2 *__restrict__ A,
                                               const double2 *__restrict__ B, double *__restrict__ x, bool comp) {
    // the error-free transformations below must not be contracted into FMAs
#pragma clang fp contract(off)
    const int64_t total = H * (int64_t)Q;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx / Q;
        const int q = (int)(idx - r * Q);
        const double2 a = A[r], b = B[q];
        if (comp) {  // 1 - x = a b
            x[idx] = omx_dd(a, b);
            continue;
        }
        const double p = a.x * b.x;
        double e = fma(a.x, b.x, -p);                 // exact low part of a.x b.x
        e = fma(a.x, b.y, fma(a.y, b.x, e));          // + cross terms
        const double s = 1.0 - p;                     // two-sum(1, -p)
        const double bb = s - 1.0;
        const double err = (1.0 - (s - bb)) + (-p - bb);
        x[idx] = s + (err - e);
    }
}

// The same construction for many functions at once (batch plans): block t
// builds nodes [begin, end) of tiles[t].
// With comp set, the complements 1 - x go to comp + (t.x - x_base) + idx
// instead.
__global__ __launch_bounds__(256) void k_bnodes(const NodeTile *__restrict__ tiles, const double *x_base,
                                                double *comp) {
    const NodeTile t = tiles[blockIdx.x];
    for (int64_t idx = t.begin + threadIdx.x; idx < t.end; idx += 256) {
        const int64_t r = idx / t.Q;
        const int q = (int)(idx - r * t.Q);
        if (comp) comp[(t.x - x_base) + idx] = omx_dd(t.rowA[r], t.omt2[q]);
        else t.x[idx] = node_dd(t.rowA[r], t.omt2[q]);
    }
}

hipError_t launch_bnodes(const NodeTile *tiles, int64_t ntiles, hipStream_t s, const double *x_base,
                         double *comp) {
    for (int64_t a = 0; a < ntiles; a += 1 << 20) {
        const int64_t n = ntiles - a < (1 << 20) ? ntiles - a : (1 << 20);
        hipLaunchKernelGGL(k_bnodes, dim3((unsigned)n), dim3(256), 0, s, tiles + a, x_base, comp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_nodes(int64_t H, int Q, const double2 *A, const double2 *B, double *x, hipStream_t s,
                        bool comp) {
    const int64_t total = H * (int64_t)Q;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_nodes, dim3((unsigned)blocks), dim3(256), 0, s, H, Q, A, B, x, comp);
    return hipGetLastError();
}

// ---------------------------------------------------- quadrature reduction ---
// Exact-fit variant: a row of Q = G*CPL*VEC samples is read by G lanes, each
// lane always owning the same CPL chunks of VEC samples, so its weights stay
// in registers.  Each wave handles 64/G rows per step, U steps unrolled, so a
// lane keeps U*CPL 16-byte loads in flight.  Accumulation is FP64 with a
// fixed-order butterfly reduction over the G lanes (deterministic).
template <typename T, int VEC, int G, int CPL, int U>
__global__ __launch_bounds__(256) void k_quad_fit(const T *__restrict__ f, const double *__restrict__ w,
                                                  const double *__restrict__ s2, int64_t rows,
                                                  double *__restrict__ phi) {
    using V = typename VecOf<T, VEC>::type;
    constexpr int Q = G * CPL * VEC;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int rg = lane / G;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    double wr[CPL][VEC];
#pragma unroll
    for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) wr[c][e] = w[(g + c * G) * VEC + e];

    for (int64_t r0 = wave * (RPW * U); r0 < rows; r0 += nwaves * (RPW * U)) {
        V val[U][CPL];
        double s2v[U];  // read with the samples, not after the reduction
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = r0 + u * RPW + rg;
            if (row < rows) {
                const V *p = reinterpret_cast<const V *>(f + row * Q) + g;
#pragma unroll
                for (int c = 0; c < CPL; ++c) val[u][c] = ld_stream(p + c * G);
                s2v[u] = s2[row];
            } else {
#pragma unroll
                for (int c = 0; c < CPL; ++c) val[u][c] = (V)(T)0;
                s2v[u] = 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                double d[VEC];
                to_d(val[u][c], d);
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc = fma(wr[c][e], d[e], acc);
            }
            acc = group_sum<G>(acc);
            const int64_t row = r0 + u * RPW + rg;
            if (g == 0 && row < rows) st_stream(phi + row, s2v[u] * acc);
        }
    }
}

// Row-pair variant for short rows: a lane group reads rows 2p and 2p+1 (2Q
// contiguous samples) in the exact-fit pattern of one row of 2Q, each chunk
// inside one row (Q a multiple of VEC), and keeps one sum per row in chunk
// order; the per-row reduction and store are spread over twice the bytes.
template <typename T, int VEC, int G, int CPL, int U>
__global__ __launch_bounds__(256) void k_quad_pair(const T *__restrict__ f, const double *__restrict__ w,
                                                   const double *__restrict__ s2, int64_t rows,
                                                   double *__restrict__ phi) {
    using V = typename VecOf<T, VEC>::type;
    constexpr int HALF = G * CPL / 2;  // chunks per row
    static_assert((G * CPL) % 2 == 0, "a row pair splits into two rows of whole chunks");
    constexpr int Q = HALF * VEC;
    constexpr int RPW = 64 / G;  // row pairs per wave and unroll step
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int rg = lane / G;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t pairs = (rows + 1) / 2;
    double wr[CPL][VEC];
    bool second[CPL];  // chunk c of this lane lies in the pair's second row
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int ch = g + c * G;
        second[c] = ch >= HALF;
        const int q0 = (second[c] ? ch - HALF : ch) * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e) wr[c][e] = w[q0 + e];
    }

    for (int64_t p0 = wave * (RPW * U); p0 < pairs; p0 += nwaves * (RPW * U)) {
        V val[U][CPL];
        double s2a[U], s2b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t ra = 2 * (p0 + u * RPW + rg);
            const bool va = ra < rows, vb = ra + 1 < rows;
            const V *p = reinterpret_cast<const V *>(f + ra * Q) + g;
#pragma unroll
            for (int c = 0; c < CPL; ++c) val[u][c] = (second[c] ? vb : va) ? ld_stream(p + c * G) : (V)(T)0;
            s2a[u] = va ? s2[ra] : 0.0;
            s2b[u] = vb ? s2[ra + 1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                double d[VEC];
                to_d(val[u][c], d);
                double a = second[c] ? acc1 : acc0;
#pragma unroll
                for (int e = 0; e < VEC; ++e) a = fma(wr[c][e], d[e], a);
                if (second[c]) acc1 = a;
                else acc0 = a;
            }
            acc0 = group_sum<G>(acc0);
            acc1 = group_sum<G>(acc1);
            const int64_t ra = 2 * (p0 + u * RPW + rg);
            if (g == 0) {
                if (ra < rows) st_stream(phi + ra, s2a[u] * acc0);
                if (ra + 1 < rows) st_stream(phi + ra + 1, s2b[u] * acc1);
            }
        }
    }
}

// One-chunk variant for short rows of NCH = Q/VEC chunks, G/2 < NCH <= G:
// lane g < NCH reads chunk g, the other lanes idle.  The 64/G rows of one
// load instruction are adjacent in memory, so it reads whole cache lines
// even where a row is not a multiple of 128 bytes (FP32, Q = 48: four
// 192-byte rows per instruction, where the exact-fit shape has 4 lanes read
// 64-byte halves of lines).
template <typename T, int VEC, int G, int U>
__global__ __launch_bounds__(256) void k_quad_one(const T *__restrict__ f, const double *__restrict__ w,
                                                  const double *__restrict__ s2, int64_t rows, int Q,
                                                  double *__restrict__ phi) {
    using V = typename VecOf<T, VEC>::type;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int rg = lane / G;
    const bool act = g < Q / VEC;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    double wr[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) wr[e] = act ? w[g * VEC + e] : 0.0;

    for (int64_t r0 = wave * (RPW * U); r0 < rows; r0 += nwaves * (RPW * U)) {
        V val[U];
        double s2v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = r0 + u * RPW + rg;
            val[u] = (V)(T)0;
            s2v[u] = 0.0;
            if (row < rows) {
                if (act) val[u] = ld_stream(reinterpret_cast<const V *>(f + row * Q) + g);
                s2v[u] = s2[row];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double d[VEC];
            to_d(val[u], d);
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc = fma(wr[e], d[e], acc);
            acc = group_sum<G>(acc);
            const int64_t row = r0 + u * RPW + rg;
            if (g == 0 && row < rows) st_stream(phi + row, s2v[u] * acc);
        }
    }
}

// Generic variant for any Q (row_partial in quad_device.h).
template <typename T, int VEC, int G>
__global__ __launch_bounds__(256) void k_quad_gen(const T *__restrict__ f, const double *__restrict__ w,
                                                  const double *__restrict__ s2, int64_t rows, int Q,
                                                  double *__restrict__ phi) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int rg = lane / G;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int NC = Q / VEC;
    for (int64_t r0 = wave * RPW; r0 < rows; r0 += nwaves * RPW) {
        const int64_t row = r0 + rg;
        const double s2v = row < rows ? s2[row] : 0.0;  // read before the row, not after it
        double acc = 0.0;
        if (row < rows) acc = row_partial<T, VEC, G>(f + row * Q, w, NC, g);
        acc = group_sum<G>(acc);
        if (g == 0 && row < rows) st_stream(phi + row, s2v * acc);
    }
}

// When set, the dispatch below reports the resident blocks per CU of the
// selected variant (occupancy API) into *g_occ instead of launching it.
static thread_local int *g_occ = nullptr;

template <typename T, int VEC, int G, int CPL, int U>
static hipError_t go_fit(const QuadCfg &c, const void *f, const double *w, const double *s2, int64_t rows,
                         double *phi, hipStream_t s) {
    if (g_occ)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(g_occ, (const void *)k_quad_fit<T, VEC, G, CPL, U>,
                                                            c.block, 0);
    hipLaunchKernelGGL((k_quad_fit<T, VEC, G, CPL, U>), dim3(c.grid), dim3(c.block), 0, s,
                       (const T *)f, w, s2, rows, phi);
    return hipGetLastError();
}

template <typename T, int VEC, int G, int CPL, int U>
static hipError_t go_pair(const QuadCfg &c, const void *f, const double *w, const double *s2, int64_t rows,
                          double *phi, hipStream_t s) {
    if (g_occ)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(g_occ, (const void *)k_quad_pair<T, VEC, G, CPL, U>,
                                                            c.block, 0);
    hipLaunchKernelGGL((k_quad_pair<T, VEC, G, CPL, U>), dim3(c.grid), dim3(c.block), 0, s,
                       (const T *)f, w, s2, rows, phi);
    return hipGetLastError();
}

template <typename T, int VEC, int G, int U>
static hipError_t go_one(const QuadCfg &c, const void *f, const double *w, const double *s2, int64_t rows,
                         int Q, double *phi, hipStream_t s) {
    if (g_occ) return hipOccupancyMaxActiveBlocksPerMultiprocessor(g_occ, (const void *)k_quad_one<T, VEC, G, U>,
                                                                    c.block, 0);
    hipLaunchKernelGGL((k_quad_one<T, VEC, G, U>), dim3(c.grid), dim3(c.block), 0, s, (const T *)f, w, s2,
                       rows, Q, phi);
    return hipGetLastError();
}

template <typename T, int VEC, int G>
static hipError_t go_gen(const QuadCfg &c, const void *f, const double *w, const double *s2, int64_t rows,
                         int Q, double *phi, hipStream_t s) {
    if (g_occ) return hipOccupancyMaxActiveBlocksPerMultiprocessor(g_occ, (const void *)k_quad_gen<T, VEC, G>,
                                                                    c.block, 0);
    hipLaunchKernelGGL((k_quad_gen<T, VEC, G>), dim3(c.grid), dim3(c.block), 0, s, (const T *)f, w, s2,
                       rows, Q, phi);
    return hipGetLastError();
}

// Dispatch tables over the instantiated variants.
#define LC_FIT_CASES_K(K, TT, VV, GG)                                                                    \
    if (c.G == GG && c.vec == VV) {                                                              \
        switch (c.cpl * 16 + c.unroll) {                                                         \
            case 1 * 16 + 1: return K<TT, VV, GG, 1, 1>(c, f, w, s2, rows, phi, s);          \
            case 1 * 16 + 2: return K<TT, VV, GG, 1, 2>(c, f, w, s2, rows, phi, s);          \
            case 1 * 16 + 4: return K<TT, VV, GG, 1, 4>(c, f, w, s2, rows, phi, s);          \
            case 2 * 16 + 1: return K<TT, VV, GG, 2, 1>(c, f, w, s2, rows, phi, s);          \
            case 2 * 16 + 2: return K<TT, VV, GG, 2, 2>(c, f, w, s2, rows, phi, s);          \
            case 2 * 16 + 4: return K<TT, VV, GG, 2, 4>(c, f, w, s2, rows, phi, s);          \
            case 3 * 16 + 1: return K<TT, VV, GG, 3, 1>(c, f, w, s2, rows, phi, s);          \
            case 3 * 16 + 2: return K<TT, VV, GG, 3, 2>(c, f, w, s2, rows, phi, s);          \
            case 4 * 16 + 1: return K<TT, VV, GG, 4, 1>(c, f, w, s2, rows, phi, s);          \
            case 4 * 16 + 2: return K<TT, VV, GG, 4, 2>(c, f, w, s2, rows, phi, s);          \
            case 6 * 16 + 1: return K<TT, VV, GG, 6, 1>(c, f, w, s2, rows, phi, s);          \
            case 8 * 16 + 1: return K<TT, VV, GG, 8, 1>(c, f, w, s2, rows, phi, s);          \
            case 5 * 16 + 1: return K<TT, VV, GG, 5, 1>(c, f, w, s2, rows, phi, s);         \
            case 7 * 16 + 1: return K<TT, VV, GG, 7, 1>(c, f, w, s2, rows, phi, s);         \
            case 9 * 16 + 1: return K<TT, VV, GG, 9, 1>(c, f, w, s2, rows, phi, s);         \
            case 10 * 16 + 1: return K<TT, VV, GG, 10, 1>(c, f, w, s2, rows, phi, s);        \
            case 11 * 16 + 1: return K<TT, VV, GG, 11, 1>(c, f, w, s2, rows, phi, s);        \
            default: break;                                                                      \
        }                                                                                        \
    }
#define LC_FIT_CASES(TT, VV, GG) LC_FIT_CASES_K(go_fit, TT, VV, GG)

template <typename T>
static hipError_t dispatch_quad(const QuadCfg &c, const void *f, const double *w, const double *s2,
                                int64_t rows, int Q, double *phi, hipStream_t s) {
    if (c.rpg == 2) {
        if constexpr (sizeof(T) == 8) {
            LC_FIT_CASES_K(go_pair, T, 2, 4)
            LC_FIT_CASES_K(go_pair, T, 2, 8)
            LC_FIT_CASES_K(go_pair, T, 2, 16)
        } else {
            LC_FIT_CASES_K(go_pair, T, 4, 4)
            LC_FIT_CASES_K(go_pair, T, 4, 8)
            LC_FIT_CASES_K(go_pair, T, 4, 16)
        }
        return hipErrorInvalidValue;
    }
    if (c.rpg != 1) return hipErrorInvalidValue;
    if (c.cpl > 0) {
        if constexpr (sizeof(T) == 8) {
            LC_FIT_CASES(T, 2, 4)
            LC_FIT_CASES(T, 2, 8)
            LC_FIT_CASES(T, 2, 16)
        } else {
            LC_FIT_CASES(T, 4, 4)
            LC_FIT_CASES(T, 4, 8)
            LC_FIT_CASES(T, 4, 16)
        }
        return hipErrorInvalidValue;
    }
    if (c.cpl < 0) {
        constexpr int V = 16 / sizeof(T);
        switch (c.G * 16 + c.unroll) {
            case 8 * 16 + 1: return go_one<T, V, 8, 1>(c, f, w, s2, rows, Q, phi, s);
            case 8 * 16 + 2: return go_one<T, V, 8, 2>(c, f, w, s2, rows, Q, phi, s);
            case 8 * 16 + 4: return go_one<T, V, 8, 4>(c, f, w, s2, rows, Q, phi, s);
            case 8 * 16 + 8: return go_one<T, V, 8, 8>(c, f, w, s2, rows, Q, phi, s);
            case 16 * 16 + 1: return go_one<T, V, 16, 1>(c, f, w, s2, rows, Q, phi, s);
            case 16 * 16 + 2: return go_one<T, V, 16, 2>(c, f, w, s2, rows, Q, phi, s);
            case 16 * 16 + 4: return go_one<T, V, 16, 4>(c, f, w, s2, rows, Q, phi, s);
            case 16 * 16 + 8: return go_one<T, V, 16, 8>(c, f, w, s2, rows, Q, phi, s);
            case 32 * 16 + 1: return go_one<T, V, 32, 1>(c, f, w, s2, rows, Q, phi, s);
            case 32 * 16 + 2: return go_one<T, V, 32, 2>(c, f, w, s2, rows, Q, phi, s);
            case 32 * 16 + 4: return go_one<T, V, 32, 4>(c, f, w, s2, rows, Q, phi, s);
            case 32 * 16 + 8: return go_one<T, V, 32, 8>(c, f, w, s2, rows, Q, phi, s);
            case 64 * 16 + 1: return go_one<T, V, 64, 1>(c, f, w, s2, rows, Q, phi, s);
            case 64 * 16 + 2: return go_one<T, V, 64, 2>(c, f, w, s2, rows, Q, phi, s);
            case 64 * 16 + 4: return go_one<T, V, 64, 4>(c, f, w, s2, rows, Q, phi, s);
            case 64 * 16 + 8: return go_one<T, V, 64, 8>(c, f, w, s2, rows, Q, phi, s);
            default: break;
        }
        return hipErrorInvalidValue;
    }
    switch (c.vec * 1000 + c.G) {
        case 1004: return go_gen<T, 1, 4>(c, f, w, s2, rows, Q, phi, s);
        case 1008: return go_gen<T, 1, 8>(c, f, w, s2, rows, Q, phi, s);
        case 1016: return go_gen<T, 1, 16>(c, f, w, s2, rows, Q, phi, s);
        case 1032: return go_gen<T, 1, 32>(c, f, w, s2, rows, Q, phi, s);
        case 1064: return go_gen<T, 1, 64>(c, f, w, s2, rows, Q, phi, s);
        case 2016: return go_gen<T, 2, 16>(c, f, w, s2, rows, Q, phi, s);
        case 2032: return go_gen<T, 2, 32>(c, f, w, s2, rows, Q, phi, s);
        case 2064: return go_gen<T, 2, 64>(c, f, w, s2, rows, Q, phi, s);
        default: break;
    }
    return hipErrorInvalidValue;
}
#undef LC_FIT_CASES
#undef LC_FIT_CASES_K

int quad_blocks_per_cu(const QuadCfg &cfg, int prec) {
    int n = 0;
    g_occ = &n;
    QuadCfg c = cfg;
    c.grid = 1;
    const hipError_t e = prec == LC_FP64 ? dispatch_quad<double>(c, nullptr, nullptr, nullptr, 0, c.Qv, nullptr, 0)
                                         : dispatch_quad<float>(c, nullptr, nullptr, nullptr, 0, c.Qv, nullptr, 0);
    g_occ = nullptr;
    return (e == hipSuccess && n > 0) ? n : 0;
}

int quad_rows_per_block(const QuadCfg &c) {
    return (c.block / 64) * (64 / c.G) * (c.cpl != 0 ? c.unroll : 1) * (c.rpg == 2 ? 2 : 1);
}

bool quad_cfg_supported(const QuadCfg &c, int prec, int Q) {
    const int esz = prec == LC_FP64 ? 8 : 4;
    if (c.block != 256 || c.grid < 1) return false;
    if (Q % c.vec) return false;
    if (c.rpg != 1 && c.rpg != 2) return false;
    if (c.rpg == 2) {  // two rows of Q per lane group
        if (c.vec != 16 / esz || !(c.G == 4 || c.G == 8 || c.G == 16)) return false;
        if (c.G * c.cpl * c.vec != 2 * Q) return false;
        const int key = c.cpl * 16 + c.unroll;
        const int ok[] = {17, 18, 20, 33, 34, 36, 49, 50, 65, 66, 81, 97, 113, 129, 145, 161, 177};
        for (int k : ok)
            if (k == key) return true;
        return false;
    }
    if (c.cpl > 0) {
        const int vec_ok = esz == 8 ? 2 : 4;
        if (c.vec != vec_ok) return false;
        if (!(c.G == 4 || c.G == 8 || c.G == 16)) return false;
        if (c.G * c.cpl * c.vec != Q) return false;
        const int key = c.cpl * 16 + c.unroll;
        const int ok[] = {17, 18, 20, 33, 34, 36, 49, 50, 65, 66, 81, 97, 113, 129, 145, 161, 177};
        for (int k : ok)
            if (k == key) return true;
        return false;
    }
    if (c.cpl < 0) {  // one chunk per lane: G/2 < Q/vec <= G
        const int nch = Q / c.vec;
        if (c.cpl != -1 || c.vec != 16 / esz) return false;
        if (!(c.G == 8 || c.G == 16 || c.G == 32 || c.G == 64)) return false;
        if (!(c.unroll == 1 || c.unroll == 2 || c.unroll == 4 || c.unroll == 8)) return false;
        return 2 * nch > c.G && nch <= c.G;
    }
    if (c.vec == 1) return c.G == 4 || c.G == 8 || c.G == 16 || c.G == 32 || c.G == 64;
    if (c.vec == 2) return c.G == 16 || c.G == 32 || c.G == 64;
    return false;
}

hipError_t launch_quad(const QuadCfg &cfg, int prec, const void *f, const double *w, const double *s2,
                       int64_t rows, int Q, double *phi, hipStream_t s) {
    if (!quad_cfg_supported(cfg, prec, Q)) return hipErrorInvalidValue;
    if (prec == LC_FP64) return dispatch_quad<double>(cfg, f, w, s2, rows, Q, phi, s);
    return dispatch_quad<float>(cfg, f, w, s2, rows, Q, phi, s);
}

// ------------------------------------------------------------------ DST ---
struct GlobalPhi {
    const double *p;
    __device__ __forceinline__ double operator()(int64_t m) const { return p[m - 1]; }
};
struct LdsPhi {
    const double *p;
    __device__ __forceinline__ double operator()(int64_t m) const { return p[m - 1]; }
};

// Whole DST in one workgroup: pack phi into Z (LDS), Stockham FFT of length
// L = H/2, unpack + rescale into c.
template <int T>
__global__ __launch_bounds__(T) void k_dst_lds(const double *__restrict__ phi, int64_t H, int L, int64_t N,
                                               const double2 *__restrict__ tw_pre,
                                               const double2 *__restrict__ tw_pack,
                                               const double2 *__restrict__ tw_fft, FftSched sch,
                                               double *__restrict__ c) {
    extern __shared__ double2 lds[];
    GlobalPhi ph{phi};
    const OctantRegs oc = octant_load<T>(tw_fft, L);
    dst_pack_lds<T, 8>(lds, ph, H, L, tw_pre, tw_pack);
    octant_store<T>(lds + L, oc, L);
    __syncthreads();
    fft_lds_one<T, 8>(lds, L, sch, tw_fft, lds + L);
    dst_post_block<T, true>(c, (int)N, lds, (int)H);
}

// Four-step FFT of length L = L1 * L2 (k = L2 k1 + k2, p = p1 + L1 p2):
// columns:  A[p1][k2] = e^{2 pi i p1 k2 / L} sum_{k1} Z[L2 k1 + k2] e^{2 pi i p1 k1 / L1}
// rows:     z[p1 + L1 p2] = sum_{k2} A[p1][k2] e^{2 pi i p2 k2 / L2}
template <int T>
__global__ __launch_bounds__(T) void k_fft_cols(const double *__restrict__ phi, int64_t H, int L1, int L2,
                                                int CB, FftSched s1, const double2 *__restrict__ tw_pre,
                                                const double2 *__restrict__ tw_pack,
                                                const double2 *__restrict__ tw_fft, double2 *__restrict__ A) {
    extern __shared__ double2 lds[];
    const int64_t L = (int64_t)L1 * L2;
    const int k20 = blockIdx.x * CB;
    GlobalPhi ph{phi};
    // four values per thread at a time, every load issued before the first use
    for (int e0 = 0; e0 < CB * L1; e0 += 4 * T) {
        double2 z[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = min(e0 + (int)threadIdx.x + u * T, CB * L1 - 1);
            const int k1 = e / CB, cb = e - k1 * CB;
            z[u] = dst_pack((int64_t)L2 * k1 + k20 + cb, ph, H, L, tw_pre, tw_pack);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + (int)threadIdx.x + u * T;
            const int k1 = e / CB, cb = e - k1 * CB;
            if (e < CB * L1) lds[cb * L1 + k1] = z[u];
        }
    }
    __syncthreads();
    fft_lds<T, 8>(lds, L1, CB, s1, tw_fft, L2);
    for (int e = threadIdx.x; e < CB * L1; e += T) {
        const int p1 = e / CB, cb = e - p1 * CB;
        const int k2 = k20 + cb;
        A[(int64_t)p1 * L2 + k2] = cmul(lds[cb * L1 + p1], tw_fft[(int64_t)p1 * k2]);
    }
}

template <int T>
__global__ __launch_bounds__(T) void k_fft_rows(const double2 *__restrict__ A, int L1, int L2, int RB,
                                                FftSched s2, const double2 *__restrict__ tw_fft,
                                                double2 *__restrict__ z) {
    extern __shared__ double2 lds[];
    const int p10 = blockIdx.x * RB;
    for (int e0 = 0; e0 < RB * L2; e0 += 4 * T) {  // four loads in flight per thread
        double2 z[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) z[u] = A[(int64_t)p10 * L2 + min(e0 + (int)threadIdx.x + u * T, RB * L2 - 1)];
        // unconditional stores (past the end: the last element again, the
        // value loaded for it), so that no masked store pulls its load after
        // the previous one's wait
#pragma unroll
        for (int u = 0; u < 4; ++u) lds[min(e0 + (int)threadIdx.x + u * T, RB * L2 - 1)] = z[u];
    }
    __syncthreads();
    fft_lds<T, 8>(lds, L2, RB, s2, tw_fft, L1);
    for (int e = threadIdx.x; e < RB * L2; e += T) {
        const int p2 = e / RB, rb = e - p2 * RB;
        z[(int64_t)(p10 + rb) + (int64_t)L1 * p2] = lds[rb * L2 + p2];
    }
}

__global__ __launch_bounds__(256) void k_dst_post(const double2 *__restrict__ z, int64_t H, int64_t N,
                                                  double *__restrict__ c) {
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * blockDim.x)
        c[n] = dst_post(n, z, H);
}

template <typename K>
static hipError_t allow_lds(K kern, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_dst(const DstCfg &cfg, const double *phi, int64_t H, int64_t L, int64_t N,
                      const double2 *tw_pre, const double2 *tw_pack, const double2 *tw_fft, double2 *zA,
                      double2 *zB, double *c, hipStream_t s) {
    hipError_t e;
    if (L <= kLdsFftMax) {
        const size_t lds = fft_lds_bytes(L);
        if (L > 8 * cfg.threads) return hipErrorInvalidValue;
        switch (cfg.threads) {
            case 64:
                hipLaunchKernelGGL(k_dst_lds<64>, dim3(1), dim3(64), lds, s, phi, H, (int)L, N, tw_pre,
                                   tw_pack, tw_fft, cfg.sched, c);
                break;
            case 128:
                hipLaunchKernelGGL(k_dst_lds<128>, dim3(1), dim3(128), lds, s, phi, H, (int)L, N, tw_pre,
                                   tw_pack, tw_fft, cfg.sched, c);
                break;
            case 256:
                if ((e = allow_lds(k_dst_lds<256>, lds)) != hipSuccess) return e;
                hipLaunchKernelGGL(k_dst_lds<256>, dim3(1), dim3(256), lds, s, phi, H, (int)L, N, tw_pre,
                                   tw_pack, tw_fft, cfg.sched, c);
                break;
            case 512:
                if ((e = allow_lds(k_dst_lds<512>, lds)) != hipSuccess) return e;
                hipLaunchKernelGGL(k_dst_lds<512>, dim3(1), dim3(512), lds, s, phi, H, (int)L, N, tw_pre,
                                   tw_pack, tw_fft, cfg.sched, c);
                break;
            case 1024:
                if ((e = allow_lds(k_dst_lds<1024>, lds)) != hipSuccess) return e;
                hipLaunchKernelGGL(k_dst_lds<1024>, dim3(1), dim3(1024), lds, s, phi, H, (int)L, N, tw_pre,
                                   tw_pack, tw_fft, cfg.sched, c);
                break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    // four-step through global memory.  Sub-transforms of up to 512 points
    // run in one-wave blocks, as few per block as leave 256 blocks (one per
    // CU: at L1 = L2 = 256 a block per column), longer ones in 256-thread
    // blocks of up to 2048 elements
    const int L1 = cfg.L1, L2 = cfg.L2;
    if ((int64_t)L1 * L2 != L || L1 > 2048 || L2 > 2048) return hipErrorInvalidValue;
    // sub-transforms of length Lsub per block out of n: the largest divisor
    // of n with Lsub x <= cap and n / x >= min(n, 256)
    auto per_block = [](int Lsub, int n, int cap) {
        int x = cap / Lsub < n ? cap / Lsub : n;
        const int want = n < 256 ? n : 256;
        while (x > 1 && (n % x || n / x < want)) --x;
        return x;
    };
    const bool c64 = L1 <= 512, r64 = L2 <= 512;
    const int CB = c64 ? per_block(L1, L2, 512) : per_block(L1, L2, 2048);
    const int RB = r64 ? per_block(L2, L1, 512) : per_block(L2, L1, 2048);
    if (CB < 1 || RB < 1 || L2 % CB || L1 % RB || CB * L1 > (c64 ? 512 : 2048) || RB * L2 > (r64 ? 512 : 2048))
        return hipErrorInvalidValue;
    if (c64)
        hipLaunchKernelGGL(k_fft_cols<64>, dim3(L2 / CB), dim3(64), (size_t)CB * L1 * sizeof(double2), s, phi, H,
                           L1, L2, CB, cfg.s1, tw_pre, tw_pack, tw_fft, zA);
    else
        hipLaunchKernelGGL(k_fft_cols<256>, dim3(L2 / CB), dim3(256), (size_t)CB * L1 * sizeof(double2), s, phi,
                           H, L1, L2, CB, cfg.s1, tw_pre, tw_pack, tw_fft, zA);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (r64)
        hipLaunchKernelGGL(k_fft_rows<64>, dim3(L1 / RB), dim3(64), (size_t)RB * L2 * sizeof(double2), s, zA, L1,
                           L2, RB, cfg.s2, tw_fft, zB);
    else
        hipLaunchKernelGGL(k_fft_rows<256>, dim3(L1 / RB), dim3(256), (size_t)RB * L2 * sizeof(double2), s, zA,
                           L1, L2, RB, cfg.s2, tw_fft, zB);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int64_t blocks = (N + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_dst_post, dim3((unsigned)blocks), dim3(256), 0, s, zB, H, N, c);
    return hipGetLastError();
}

// ------------------------------------------------------ fused small path ---
// One workgroup does everything (quadrature into LDS, pack, FFT, unpack):
// one launch for problems whose samples are a few hundred KiB at most.
size_t fused_small_lds_bytes(int64_t H, int Q) {
    (void)Q;
    return (size_t)H * sizeof(double) + (size_t)(H / 2) * sizeof(double2);
}

template <typename T, int TH>
__global__ __launch_bounds__(TH) void k_fused_small(const T *__restrict__ f, const double *__restrict__ w,
                                                    const double *__restrict__ s2, int64_t H, int Q,
                                                    int64_t N, FftSched sch,
                                                    const double2 *__restrict__ tw_pre,
                                                    const double2 *__restrict__ tw_pack,
                                                    const double2 *__restrict__ tw_fft,
                                                    double *__restrict__ c) {
    extern __shared__ double2 lds[];
    const int L = (int)(H / 2);
    double *phs = reinterpret_cast<double *>(lds + L);
    constexpr int G = 16;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int rg = lane / G;
    const int wave = threadIdx.x >> 6;
    constexpr int NW = TH / 64;
    for (int64_t r0 = (int64_t)wave * RPW; r0 < H; r0 += NW * RPW) {
        const int64_t row = r0 + rg;
        double acc = 0.0;
        if (row < H) acc = row_partial<T, 1, G>(f + row * Q, w, Q, g);
        acc = group_sum<G>(acc);
        if (g == 0 && row < H) phs[row] = s2[row] * acc;
    }
    __syncthreads();
    LdsPhi ph{phs};
    for (int k = threadIdx.x; k < L; k += TH) lds[k] = dst_pack(k, ph, H, L, tw_pre, tw_pack);
    __syncthreads();
    fft_lds<TH, 8>(lds, L, 1, sch, tw_fft, 1);
    dst_post_block<TH>(c, (int)N, lds, (int)H);
}

hipError_t launch_fused_small(int threads, int prec, const void *f, const double *w, const double *s2,
                              int64_t H, int Q, int64_t N, const FftSched &sch, const double2 *tw_pre,
                              const double2 *tw_pack, const double2 *tw_fft, double *c, hipStream_t s) {
    const size_t lds = fused_small_lds_bytes(H, Q);
    if (H / 2 > 8 * threads || lds > 65536) return hipErrorInvalidValue;
    if (prec == LC_FP64) {
        if (threads == 256)
            hipLaunchKernelGGL((k_fused_small<double, 256>), dim3(1), dim3(256), lds, s, (const double *)f, w,
                               s2, H, Q, N, sch, tw_pre, tw_pack, tw_fft, c);
        else if (threads == 1024)
            hipLaunchKernelGGL((k_fused_small<double, 1024>), dim3(1), dim3(1024), lds, s, (const double *)f,
                               w, s2, H, Q, N, sch, tw_pre, tw_pack, tw_fft, c);
        else
            return hipErrorInvalidValue;
    } else {
        if (threads == 256)
            hipLaunchKernelGGL((k_fused_small<float, 256>), dim3(1), dim3(256), lds, s, (const float *)f, w,
                               s2, H, Q, N, sch, tw_pre, tw_pack, tw_fft, c);
        else if (threads == 1024)
            hipLaunchKernelGGL((k_fused_small<float, 1024>), dim3(1), dim3(1024), lds, s, (const float *)f, w,
                               s2, H, Q, N, sch, tw_pre, tw_pack, tw_fft, c);
        else
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lc
