// Batched kernels: many functions of uneven size in one execution.
//   * k_bquad_*: the Abel quadrature reduction over a table of row tiles
//     (each tile a run of rows of one function, its addresses resolved on
//     the host); one launch per class of functions sharing (Q, sample
//     precision), weights in registers.  A block reads the descriptor of its
//     next tile while the samples of the current one are in flight.
//   * k_bdst_lds: one workgroup per function, pack + LDS Stockham FFT +
//     unpack/rescale (the twist and the one FFT of eq. (2.4)), functions
//     listed longest first so the long ones start early.
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "lc_internal.h"
#include "quad_device.h"

namespace lc {

template <typename T, int VEC, int G, int CPL, int U>
__global__ __launch_bounds__(256) void k_bquad_fit(const unsigned char *__restrict__ f_arena,
                                                   const double *__restrict__ w,
                                                   const BatchTile *__restrict__ tiles, int ntiles,
                                                   double *__restrict__ phi_arena) {
    using V = typename VecOf<T, VEC>::type;
    constexpr int Q = G * CPL * VEC;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int rg = lane / G;
    const int wv = threadIdx.x >> 6;
    double wr[CPL][VEC];
#pragma unroll
    for (int c = 0; c < CPL; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) wr[c][e] = w[(g + c * G) * VEC + e];

    BatchTile nx{};
    if ((int)blockIdx.x < ntiles) nx = tiles[blockIdx.x];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BatchTile tl = nx;
        const T *f = reinterpret_cast<const T *>(f_arena + tl.f_off);
        double *phi = phi_arena + tl.phi_off;
        const int rend = tl.nrows;
        const int r0 = wv * (RPW * U);
        V val[U][CPL];
        double s2v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int row = r0 + u * RPW + rg;
            if (row < rend) {
                const V *p = reinterpret_cast<const V *>(f + (int64_t)row * Q) + g;
#pragma unroll
                for (int c = 0; c < CPL; ++c) val[u][c] = ld_stream(p + c * G);
                s2v[u] = ld_global(tl.s2 + row);
            } else {
#pragma unroll
                for (int c = 0; c < CPL; ++c) val[u][c] = (V)(T)0;
                s2v[u] = 0.0;
            }
        }
        // this tile's loads are in flight: read the next descriptor now (a
        // scalar load issued earlier would be waited for with this tile's)
        __builtin_amdgcn_sched_barrier(0);
        if (t + (int)gridDim.x < ntiles) nx = tiles[t + gridDim.x];
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
            const int row = r0 + u * RPW + rg;
            if (g == 0 && row < rend) st_stream(phi + row, s2v[u] * acc);
        }
    }
}

// Two rows per lane group for short rows: the G lanes of a group read the 2Q
// contiguous samples of rows 2p and 2p+1 in the exact-fit pattern of one row
// of 2Q (G * CPL chunks of VEC, lane g taking chunks g, g + G, ...), so that
// a row of 48 FP32 samples is read as a row of 48 FP64 samples is, and the
// per-row work (reduction, s2, phi store) is spread over twice the bytes.
// Q is a multiple of VEC, so each chunk lies in one row; each lane keeps
// one sum per row, in chunk order.
template <typename T, int VEC, int G, int CPL, int U>
__global__ __launch_bounds__(256) void k_bquad_pair(const unsigned char *__restrict__ f_arena,
                                                    const double *__restrict__ w,
                                                    const BatchTile *__restrict__ tiles, int ntiles,
                                                    double *__restrict__ phi_arena) {
    using V = typename VecOf<T, VEC>::type;
    constexpr int HALF = G * CPL / 2;  // chunks per row
    static_assert((G * CPL) % 2 == 0, "a row pair splits into two rows of whole chunks");
    constexpr int Q = HALF * VEC;
    constexpr int RPW = 64 / G;  // row pairs per wave and unroll step
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int rg = lane / G;
    const int wv = threadIdx.x >> 6;
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

    BatchTile nx{};
    if ((int)blockIdx.x < ntiles) nx = tiles[blockIdx.x];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BatchTile tl = nx;
        const T *f = reinterpret_cast<const T *>(f_arena + tl.f_off);
        double *phi = phi_arena + tl.phi_off;
        const int rend = tl.nrows;
        const int p0 = wv * (RPW * U);
        V val[U][CPL];
        double s2a[U], s2b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ra = 2 * (p0 + u * RPW + rg);
            const bool va = ra < rend, vb = ra + 1 < rend;
            const V *p = reinterpret_cast<const V *>(f + (int64_t)ra * Q) + g;
#pragma unroll
            for (int c = 0; c < CPL; ++c) val[u][c] = (second[c] ? vb : va) ? ld_stream(p + c * G) : (V)(T)0;
            s2a[u] = va ? ld_global(tl.s2 + ra) : 0.0;
            s2b[u] = vb ? ld_global(tl.s2 + ra + 1) : 0.0;
        }
        __builtin_amdgcn_sched_barrier(0);
        if (t + (int)gridDim.x < ntiles) nx = tiles[t + gridDim.x];
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
            const int ra = 2 * (p0 + u * RPW + rg);
            if (g == 0) {
                if (ra < rend) st_stream(phi + ra, s2a[u] * acc0);
                if (ra + 1 < rend) st_stream(phi + ra + 1, s2b[u] * acc1);
            }
        }
    }
}

// One 16-byte chunk per lane for short rows (G/2 < Q/VEC <= G, lanes past
// Q/VEC idle): the 64/G rows of a load instruction are adjacent, so it reads
// whole cache lines where the exact-fit shape would read halves of them.
template <typename T, int VEC, int G, int U>
__global__ __launch_bounds__(256) void k_bquad_one(const unsigned char *__restrict__ f_arena,
                                                   const double *__restrict__ w, int Q,
                                                   const BatchTile *__restrict__ tiles, int ntiles,
                                                   double *__restrict__ phi_arena) {
    using V = typename VecOf<T, VEC>::type;
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int rg = lane / G;
    const int wv = threadIdx.x >> 6;
    const bool act = g < Q / VEC;
    double wr[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) wr[e] = act ? w[g * VEC + e] : 0.0;

    BatchTile nx{};
    if ((int)blockIdx.x < ntiles) nx = tiles[blockIdx.x];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BatchTile tl = nx;
        const T *f = reinterpret_cast<const T *>(f_arena + tl.f_off);
        double *phi = phi_arena + tl.phi_off;
        const int rend = tl.nrows;
        const int r0 = wv * (RPW * U);
        V val[U];
        double s2v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int row = r0 + u * RPW + rg;
            val[u] = (V)(T)0;
            s2v[u] = 0.0;
            if (row < rend) {
                if (act) val[u] = ld_stream(reinterpret_cast<const V *>(f + (int64_t)row * Q) + g);
                s2v[u] = ld_global(tl.s2 + row);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        if (t + (int)gridDim.x < ntiles) nx = tiles[t + gridDim.x];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double d[VEC];
            to_d(val[u], d);
            double acc = 0.0;
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc = fma(wr[e], d[e], acc);
            acc = group_sum<G>(acc);
            const int row = r0 + u * RPW + rg;
            if (g == 0 && row < rend) st_stream(phi + row, s2v[u] * acc);
        }
    }
}

template <typename T, int VEC, int G>
__global__ __launch_bounds__(256) void k_bquad_gen(const unsigned char *__restrict__ f_arena,
                                                   const double *__restrict__ w, int Q,
                                                   const BatchTile *__restrict__ tiles, int ntiles,
                                                   double *__restrict__ phi_arena) {
    constexpr int RPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int g = lane & (G - 1);
    const int rg = lane / G;
    const int wv = threadIdx.x >> 6;
    const int NC = Q / VEC;
    BatchTile nx{};
    if ((int)blockIdx.x < ntiles) nx = tiles[blockIdx.x];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const BatchTile tl = nx;
        const T *f = reinterpret_cast<const T *>(f_arena + tl.f_off);
        const int row = wv * RPW + rg;
        const double s2v = row < tl.nrows ? ld_global(tl.s2 + row) : 0.0;
        __builtin_amdgcn_sched_barrier(0);
        if (t + (int)gridDim.x < ntiles) nx = tiles[t + gridDim.x];
        double acc = 0.0;
        if (row < tl.nrows) acc = row_partial<T, VEC, G>(f + (int64_t)row * Q, w, NC, g);
        acc = group_sum<G>(acc);
        if (g == 0 && row < tl.nrows) st_stream(phi_arena + tl.phi_off + row, s2v * acc);
    }
}

// When set, the dispatch below reports the resident blocks per CU of the
// selected variant (occupancy API) into *g_bocc instead of launching it.
static thread_local int *g_bocc = nullptr;

template <typename T, int VEC, int G, int CPL, int U>
static hipError_t bfit(const QuadCfg &c, const void *f, const double *w, const BatchTile *tiles, int ntiles,
                       double *phi, hipStream_t s) {
    if (g_bocc)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(g_bocc, (const void *)k_bquad_fit<T, VEC, G, CPL, U>,
                                                            c.block, 0);
    hipLaunchKernelGGL((k_bquad_fit<T, VEC, G, CPL, U>), dim3(c.grid), dim3(c.block), 0, s,
                       (const unsigned char *)f, w, tiles, ntiles, phi);
    return hipGetLastError();
}

template <typename T, int VEC, int G, int CPL, int U>
static hipError_t bpair(const QuadCfg &c, const void *f, const double *w, const BatchTile *tiles, int ntiles,
                        double *phi, hipStream_t s) {
    if (g_bocc)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(g_bocc, (const void *)k_bquad_pair<T, VEC, G, CPL, U>,
                                                            c.block, 0);
    hipLaunchKernelGGL((k_bquad_pair<T, VEC, G, CPL, U>), dim3(c.grid), dim3(c.block), 0, s,
                       (const unsigned char *)f, w, tiles, ntiles, phi);
    return hipGetLastError();
}

template <typename T, int VEC, int G, int U>
static hipError_t bone(const QuadCfg &c, const void *f, const double *w, int Q, const BatchTile *tiles,
                       int ntiles, double *phi, hipStream_t s) {
    if (g_bocc)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(g_bocc, (const void *)k_bquad_one<T, VEC, G, U>,
                                                            c.block, 0);
    hipLaunchKernelGGL((k_bquad_one<T, VEC, G, U>), dim3(c.grid), dim3(c.block), 0, s,
                       (const unsigned char *)f, w, Q, tiles, ntiles, phi);
    return hipGetLastError();
}

template <typename T, int VEC, int G>
static hipError_t bgen(const QuadCfg &c, const void *f, const double *w, int Q, const BatchTile *tiles,
                       int ntiles, double *phi, hipStream_t s) {
    if (g_bocc)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(g_bocc, (const void *)k_bquad_gen<T, VEC, G>, c.block, 0);
    hipLaunchKernelGGL((k_bquad_gen<T, VEC, G>), dim3(c.grid), dim3(c.block), 0, s,
                       (const unsigned char *)f, w, Q, tiles, ntiles, phi);
    return hipGetLastError();
}

#define LC_BFIT_CASES_K(K, TT, VV, GG)                                                             \
    if (c.G == GG && c.vec == VV) {                                                               \
        switch (c.cpl * 16 + c.unroll) {                                                          \
            case 1 * 16 + 1: return K<TT, VV, GG, 1, 1>(c, f, w, tiles, ntiles, phi, s);   \
            case 1 * 16 + 2: return K<TT, VV, GG, 1, 2>(c, f, w, tiles, ntiles, phi, s);   \
            case 1 * 16 + 4: return K<TT, VV, GG, 1, 4>(c, f, w, tiles, ntiles, phi, s);   \
            case 2 * 16 + 1: return K<TT, VV, GG, 2, 1>(c, f, w, tiles, ntiles, phi, s);   \
            case 2 * 16 + 2: return K<TT, VV, GG, 2, 2>(c, f, w, tiles, ntiles, phi, s);   \
            case 2 * 16 + 4: return K<TT, VV, GG, 2, 4>(c, f, w, tiles, ntiles, phi, s);   \
            case 3 * 16 + 1: return K<TT, VV, GG, 3, 1>(c, f, w, tiles, ntiles, phi, s);   \
            case 3 * 16 + 2: return K<TT, VV, GG, 3, 2>(c, f, w, tiles, ntiles, phi, s);   \
            case 4 * 16 + 1: return K<TT, VV, GG, 4, 1>(c, f, w, tiles, ntiles, phi, s);   \
            case 4 * 16 + 2: return K<TT, VV, GG, 4, 2>(c, f, w, tiles, ntiles, phi, s);   \
            case 6 * 16 + 1: return K<TT, VV, GG, 6, 1>(c, f, w, tiles, ntiles, phi, s);   \
            case 8 * 16 + 1: return K<TT, VV, GG, 8, 1>(c, f, w, tiles, ntiles, phi, s);   \
            case 5 * 16 + 1: return K<TT, VV, GG, 5, 1>(c, f, w, tiles, ntiles, phi, s);   \
            case 7 * 16 + 1: return K<TT, VV, GG, 7, 1>(c, f, w, tiles, ntiles, phi, s);   \
            case 9 * 16 + 1: return K<TT, VV, GG, 9, 1>(c, f, w, tiles, ntiles, phi, s);   \
            case 10 * 16 + 1: return K<TT, VV, GG, 10, 1>(c, f, w, tiles, ntiles, phi, s); \
            case 11 * 16 + 1: return K<TT, VV, GG, 11, 1>(c, f, w, tiles, ntiles, phi, s); \
            default: break;                                                                       \
        }                                                                                         \
    }
#define LC_BFIT_CASES(TT, VV, GG) LC_BFIT_CASES_K(bfit, TT, VV, GG)

template <typename T>
static hipError_t bdispatch(const QuadCfg &c, const void *f, const double *w, int Q, const BatchTile *tiles,
                            int ntiles, double *phi, hipStream_t s) {
    if (c.rpg == 2) {
        if constexpr (sizeof(T) == 8) {
            LC_BFIT_CASES_K(bpair, T, 2, 4)
            LC_BFIT_CASES_K(bpair, T, 2, 8)
            LC_BFIT_CASES_K(bpair, T, 2, 16)
        } else {
            LC_BFIT_CASES_K(bpair, T, 4, 4)
            LC_BFIT_CASES_K(bpair, T, 4, 8)
            LC_BFIT_CASES_K(bpair, T, 4, 16)
        }
        return hipErrorInvalidValue;
    }
    if (c.rpg != 1) return hipErrorInvalidValue;
    if (c.cpl > 0) {
        if constexpr (sizeof(T) == 8) {
            LC_BFIT_CASES(T, 2, 4)
            LC_BFIT_CASES(T, 2, 8)
            LC_BFIT_CASES(T, 2, 16)
        } else {
            LC_BFIT_CASES(T, 4, 4)
            LC_BFIT_CASES(T, 4, 8)
            LC_BFIT_CASES(T, 4, 16)
        }
        return hipErrorInvalidValue;
    }
    if (c.cpl < 0) {
        constexpr int V = 16 / sizeof(T);
        switch (c.G * 16 + c.unroll) {
            case 8 * 16 + 1: return bone<T, V, 8, 1>(c, f, w, Q, tiles, ntiles, phi, s);
            case 8 * 16 + 2: return bone<T, V, 8, 2>(c, f, w, Q, tiles, ntiles, phi, s);
            case 8 * 16 + 4: return bone<T, V, 8, 4>(c, f, w, Q, tiles, ntiles, phi, s);
            case 8 * 16 + 8: return bone<T, V, 8, 8>(c, f, w, Q, tiles, ntiles, phi, s);
            case 16 * 16 + 1: return bone<T, V, 16, 1>(c, f, w, Q, tiles, ntiles, phi, s);
            case 16 * 16 + 2: return bone<T, V, 16, 2>(c, f, w, Q, tiles, ntiles, phi, s);
            case 16 * 16 + 4: return bone<T, V, 16, 4>(c, f, w, Q, tiles, ntiles, phi, s);
            case 16 * 16 + 8: return bone<T, V, 16, 8>(c, f, w, Q, tiles, ntiles, phi, s);
            case 32 * 16 + 1: return bone<T, V, 32, 1>(c, f, w, Q, tiles, ntiles, phi, s);
            case 32 * 16 + 2: return bone<T, V, 32, 2>(c, f, w, Q, tiles, ntiles, phi, s);
            case 32 * 16 + 4: return bone<T, V, 32, 4>(c, f, w, Q, tiles, ntiles, phi, s);
            case 32 * 16 + 8: return bone<T, V, 32, 8>(c, f, w, Q, tiles, ntiles, phi, s);
            case 64 * 16 + 1: return bone<T, V, 64, 1>(c, f, w, Q, tiles, ntiles, phi, s);
            case 64 * 16 + 2: return bone<T, V, 64, 2>(c, f, w, Q, tiles, ntiles, phi, s);
            case 64 * 16 + 4: return bone<T, V, 64, 4>(c, f, w, Q, tiles, ntiles, phi, s);
            case 64 * 16 + 8: return bone<T, V, 64, 8>(c, f, w, Q, tiles, ntiles, phi, s);
            default: break;
        }
        return hipErrorInvalidValue;
    }
    switch (c.vec * 1000 + c.G) {
        case 1004: return bgen<T, 1, 4>(c, f, w, Q, tiles, ntiles, phi, s);
        case 1008: return bgen<T, 1, 8>(c, f, w, Q, tiles, ntiles, phi, s);
        case 1016: return bgen<T, 1, 16>(c, f, w, Q, tiles, ntiles, phi, s);
        case 1032: return bgen<T, 1, 32>(c, f, w, Q, tiles, ntiles, phi, s);
        case 1064: return bgen<T, 1, 64>(c, f, w, Q, tiles, ntiles, phi, s);
        case 2016: return bgen<T, 2, 16>(c, f, w, Q, tiles, ntiles, phi, s);
        case 2032: return bgen<T, 2, 32>(c, f, w, Q, tiles, ntiles, phi, s);
        case 2064: return bgen<T, 2, 64>(c, f, w, Q, tiles, ntiles, phi, s);
        default: break;
    }
    return hipErrorInvalidValue;
}
#undef LC_BFIT_CASES
#undef LC_BFIT_CASES_K

int bquad_blocks_per_cu(const QuadCfg &cfg, int prec) {
    int n = 0;
    g_bocc = &n;
    const hipError_t e = prec == LC_FP64 ? bdispatch<double>(cfg, nullptr, nullptr, cfg.Qv, nullptr, 1, nullptr, 0)
                                         : bdispatch<float>(cfg, nullptr, nullptr, cfg.Qv, nullptr, 1, nullptr, 0);
    g_bocc = nullptr;
    return (e == hipSuccess && n > 0) ? n : 0;
}

hipError_t launch_bquad(const QuadCfg &cfg, int prec, const void *f_arena, const double *w, const BatchTile *tiles,
                        int ntiles, double *phi_arena, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (prec == LC_FP64) return bdispatch<double>(cfg, f_arena, w, cfg.Qv, tiles, ntiles, phi_arena, s);
    return bdispatch<float>(cfg, f_arena, w, cfg.Qv, tiles, ntiles, phi_arena, s);
}

// One workgroup per listed function.
template <int T>
__global__ __launch_bounds__(T) void k_bdst_lds(const double *__restrict__ phi_arena,
                                                const BatchFn *__restrict__ fns,
                                                const int32_t *__restrict__ list,
                                                double *__restrict__ c_arena) {
    extern __shared__ double2 lds[];
    const BatchFn &fn = fns[list[blockIdx.x]];
    const int64_t H = fn.H;
    const int L = (int)fn.L;
    const FftSched &sch = fn.sched;  // uniform reads of the table, not a private copy
    struct Phi {
        const double *p;
        __device__ __forceinline__ double operator()(int64_t m) const { return p[m - 1]; }
    } ph{phi_arena + fn.phi_off};
    const OctantRegs oc = octant_load<T>(fn.tw_fft, L);
    dst_pack_lds<T, 8>(lds, ph, H, L, fn.tw_pre, fn.tw_pack);
    octant_store<T>(lds + L, oc, L);
    __syncthreads();
    fft_lds_one<T, 8>(lds, L, sch, fn.tw_fft, lds + L);
    double *c = c_arena + fn.c_off;
    dst_post_block<T, true>(c, (int)fn.N, lds, (int)H);
}

hipError_t prepare_bdst(int threads, int Lmax) {
    const size_t lds = fft_lds_bytes(Lmax);
    if (lds <= 65536) return hipSuccess;
    if (threads == 512)
        return hipFuncSetAttribute((const void *)k_bdst_lds<512>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (threads == 256)
        return hipFuncSetAttribute((const void *)k_bdst_lds<256>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (threads == 1024)
        return hipFuncSetAttribute((const void *)k_bdst_lds<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipSuccess;
}

hipError_t launch_bdst(int threads, int Lmax, const double *phi_arena, const BatchFn *fns, const int32_t *list,
                       int nlist, double *c_arena, hipStream_t s) {
    if (nlist <= 0) return hipSuccess;
    if (Lmax > 8 * threads) return hipErrorInvalidValue;
    const size_t lds = fft_lds_bytes(Lmax);
    switch (threads) {
        case 64:
            hipLaunchKernelGGL(k_bdst_lds<64>, dim3(nlist), dim3(64), lds, s, phi_arena, fns, list, c_arena);
            break;
        case 128:
            hipLaunchKernelGGL(k_bdst_lds<128>, dim3(nlist), dim3(128), lds, s, phi_arena, fns, list, c_arena);
            break;
        case 256:
            hipLaunchKernelGGL(k_bdst_lds<256>, dim3(nlist), dim3(256), lds, s, phi_arena, fns, list, c_arena);
            break;
        case 512:
            hipLaunchKernelGGL(k_bdst_lds<512>, dim3(nlist), dim3(512), lds, s, phi_arena, fns, list, c_arena);
            break;
        case 1024:
            hipLaunchKernelGGL(k_bdst_lds<1024>, dim3(nlist), dim3(1024), lds, s, phi_arena, fns, list, c_arena);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Short functions of one FFT length L, up to kMultiSlots per 64-thread
// workgroup (slot u of block b is list[b kMultiSlots + u], -1 when empty):
// they share H, twiddles and radix schedule, so their FFTs are nsub
// transforms of one LDS pass sequence.  The slots' phi offset, coefficient
// offset and N are staged in LDS first; an empty slot transforms the first
// slot's phi again and is not unpacked.
__global__ __launch_bounds__(64) void k_bdst_multi(const double *__restrict__ phi_arena,
                                                   const BatchFn *__restrict__ fns,
                                                   const int32_t *__restrict__ list,
                                                   double *__restrict__ c_arena) {
    constexpr int T = 64;
    extern __shared__ double2 lds[];
    __shared__ int64_t sphi[kMultiSlots], scoff[kMultiSlots];
    __shared__ int sn[kMultiSlots];
    const int32_t *mine = list + (int64_t)blockIdx.x * kMultiSlots;
    const BatchFn &f0 = fns[mine[0]];
    const int64_t H = f0.H;
    const int L = (int)f0.L;
    const int fpb = multi_slots(L);
    if ((int)threadIdx.x < fpb) {
        const int32_t fi = mine[threadIdx.x];
        const BatchFn &f = fns[fi < 0 ? mine[0] : fi];
        sphi[threadIdx.x] = f.phi_off;
        scoff[threadIdx.x] = f.c_off;
        sn[threadIdx.x] = fi < 0 ? 0 : (int)f.N;
    }
    __syncthreads();
    struct Phi {
        const double *p;
        __device__ __forceinline__ double operator()(int64_t m) const { return p[m - 1]; }
    };
    // Z_0 (and Z_{L/2} for even L) of slot threadIdx.x, then the mirror pairs
    // (Z_g, Z_{L-g}), g = 1 .. ceil(L/2) - 1, of every slot, each from one set
    // of four phi loads and three twiddle loads (the other three are exact
    // images in the tables), dst_pack's values bit for bit
    if ((int)threadIdx.x < fpb) {
        const Phi ph{phi_arena + sphi[threadIdx.x]};
        double2 *z = lds + threadIdx.x * L;
        z[0] = dst_pack(0, ph, H, L, f0.tw_pre, f0.tw_pack);
        if (!(L & 1) && L >= 2) z[L >> 1] = dst_pack(L >> 1, ph, H, L, f0.tw_pre, f0.tw_pack);
    }
    const int gp = ((L + 1) >> 1) - 1;  // pairs per slot
    const int tot = fpb * gp;
    const float rg = 1.0f / (float)(gp > 0 ? gp : 1);
#pragma unroll 1
    for (int e0 = 0; e0 < tot; e0 += 2 * T) {  // two pairs' reads in flight per thread
        double a[2], b[2], c[2], d[2];
        double2 t0[2], s0[2], tp[2];
        int slot[2], gg[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            int g;
            slot[u] = fdivmod(min(e0 + (int)threadIdx.x + u * T, tot - 1), gp, rg, g);
            g += 1;
            gg[u] = g;
            const Phi ph{phi_arena + sphi[slot[u]]};
            a[u] = ph(g);
            b[u] = ph(H - g);
            c[u] = ph(L - g);
            d[u] = ph(L + g);
            t0[u] = f0.tw_pre[g];
            s0[u] = f0.tw_pre[L - g];
            tp[u] = f0.tw_pack[g];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (e0 + (int)threadIdx.x + u * T < tot) {
                double2 *z = lds + slot[u] * L;
                const double2 t1 = make_double2(s0[u].y, s0[u].x), s1 = make_double2(t0[u].y, t0[u].x);
                const double2 sp = make_double2(-tp[u].x, tp[u].y);
                z[gg[u]] = dst_pack_from(b[u], a[u], c[u], d[u], t0[u], t1, tp[u]);
                z[L - gg[u]] = dst_pack_from(d[u], c[u], a[u], b[u], s0[u], s1, sp);
            }
    }
    __syncthreads();
    fft_passes<T, 8, false>(lds, L, fpb, f0.sched, f0.tw_fft, 1);  // fpb >= 2
    // unpack in quads: n = 4j .. 4j+3 of a slot read only z[j] and
    // z[H/2 - 1 - j] (H even), dst_post's values bit for bit, two 16-byte
    // non-temporal stores where the quad is whole and aligned (N <= H per slot)
    const int hq = (int)((H + 3) >> 2);
    const int tot4 = fpb * hq;
    const float rq = 1.0f / (float)hq;
    const double r = 1.0 / (double)(2 * H);
#pragma unroll 1
    for (int e = threadIdx.x; e < tot4; e += T) {
        int j;
        const int sl = fdivmod(e, hq, rq, j);
        const int nn = sn[sl], n0 = 4 * j;
        if (n0 >= nn) continue;
        const double2 *z = lds + sl * L;
        const double2 a = z[j], b = z[(H >> 1) - 1 - j];
        const double f = (double)(8 * j + 1);
        const double v[4] = {f * a.x * r, -(f + 2.0) * b.y * r, (f + 4.0) * a.y * r, -(f + 6.0) * b.x * r};
        double *c = c_arena + scoff[sl] + n0;
        if (n0 + 3 < nn && ((uintptr_t)c & 15) == 0) {
            __builtin_nontemporal_store(lc_f64x2{v[0], v[1]}, reinterpret_cast<lc_f64x2 *>(c));
            __builtin_nontemporal_store(lc_f64x2{v[2], v[3]}, reinterpret_cast<lc_f64x2 *>(c) + 1);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (n0 + i < nn) __builtin_nontemporal_store(v[i], c + i);
        }
    }
}

hipError_t launch_bdst_multi(const double *phi_arena, const BatchFn *fns, const int32_t *list, int nblocks,
                             double *c_arena, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bdst_multi, dim3(nblocks), dim3(64), (size_t)8 * 64 * sizeof(double2), s, phi_arena, fns,
                       list, c_arena);
    return hipGetLastError();
}

// --------------------------------------- fused small functions ---
// One workgroup per function small enough for its LDS (H <= kFuseHmax):
// every row's Abel sum goes to LDS (G lanes per row, U rows per group in
// flight, each lane's chunk weights in registers; chunk indices past the row
// are clamped and weighted 0 so that all loads issue together), then the
// twist, FFT and rescale of eq. (2.4) run from LDS and the coefficients go
// to the arena: phi never leaves the CU.  One launch covers every fused
// function of a sample precision, whatever its rule: block i takes
// list[i] = {function, Q, G, weights}, Q <= G * kFuseCpl * VEC.
constexpr int kFuseCpl = 4;
struct BLdsPhi {
    const double *p;
    __device__ __forceinline__ double operator()(int64_t m) const { return p[m - 1]; }
};
template <typename T, int G, int U>
__device__ __forceinline__ void fused_rows(const T *__restrict__ f, const double *__restrict__ w, int Q, int64_t H,
                                           const double *__restrict__ s2, double *__restrict__ phs) {
    constexpr int VEC = 16 / sizeof(T);
    constexpr int RPB = 256 / G;
    using V = typename VecOf<T, VEC>::type;
    const int NC = Q / VEC;
    const int g = threadIdx.x & (G - 1), rg = threadIdx.x / G;
    double wr[kFuseCpl][VEC];
    int cc[kFuseCpl];
#pragma unroll
    for (int j = 0; j < kFuseCpl; ++j) {
        const int c = g + j * G;
        cc[j] = c < NC ? c : NC - 1;
#pragma unroll
        for (int e = 0; e < VEC; ++e) wr[j][e] = c < NC ? w[c * VEC + e] : 0.0;
    }
    for (int64_t r0 = 0; r0 < H; r0 += RPB * U) {
        V v[U][kFuseCpl];
        double s2v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = r0 + rg + u * RPB;
            const int64_t rc = row < H ? row : H - 1;
            const V *p = reinterpret_cast<const V *>(f + rc * Q);
#pragma unroll
            for (int j = 0; j < kFuseCpl; ++j) v[u][j] = ld_stream(p + cc[j]);
            s2v[u] = ld_global(s2 + rc);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < kFuseCpl; ++j) {
                double d[VEC];
                to_d(v[u][j], d);
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc = fma(wr[j][e], d[e], acc);
            }
            acc = group_sum<G>(acc);
            const int64_t row = r0 + rg + u * RPB;
            if (g == 0 && row < H) phs[row] = s2v[u] * acc;
        }
    }
}

template <typename T, int U>
__global__ __launch_bounds__(256) void k_bfused(const unsigned char *__restrict__ f_arena,
                                                const BatchFn *__restrict__ fns,
                                                const FusedFn *__restrict__ list, double *__restrict__ c_arena) {
    extern __shared__ double2 lds[];
    const FusedFn fd = list[blockIdx.x];
    const BatchFn &fn = fns[fd.fn];
    const int64_t H = fn.H;
    const int L = (int)fn.L;
    double *phs = reinterpret_cast<double *>(lds + L);
    const T *f = reinterpret_cast<const T *>(f_arena + fn.f_off);
    switch (fd.G) {
        case 8: fused_rows<T, 8, U>(f, fd.w, fd.Q, H, fn.s2, phs); break;
        case 16: fused_rows<T, 16, U>(f, fd.w, fd.Q, H, fn.s2, phs); break;
        case 32: fused_rows<T, 32, U>(f, fd.w, fd.Q, H, fn.s2, phs); break;
        default: fused_rows<T, 64, U>(f, fd.w, fd.Q, H, fn.s2, phs); break;
    }
    __syncthreads();
    dst_pack_lds<256, 8>(lds, BLdsPhi{phs}, H, L, fn.tw_pre, fn.tw_pack);
    __syncthreads();
    fft_lds_one<256, 8>(lds, L, fn.sched, fn.tw_fft);
    double *c = c_arena + fn.c_off;
    dst_post_block<256>(c, (int)fn.N, lds, (int)H);
}

int fuse_lanes(int prec, int Q) {
    const int VEC = prec == LC_FP64 ? 2 : 4;
    if (Q % VEC) return 0;
    for (int G = 8; G <= 64; G *= 2)
        if (Q <= G * kFuseCpl * VEC) return G;
    return 0;
}

hipError_t launch_bfused(int prec, const void *f_arena, const BatchFn *fns, const FusedFn *list, int n, int64_t Hmax,
                         double *c_arena, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (Hmax > kFuseHmax) return hipErrorInvalidValue;
    const size_t lds = (size_t)Hmax * 16;  // L complex + H phi values
    if (prec == LC_FP64)
        hipLaunchKernelGGL((k_bfused<double, 4>), dim3(n), dim3(256), lds, s, (const unsigned char *)f_arena, fns,
                           list, c_arena);
    else
        hipLaunchKernelGGL((k_bfused<float, 4>), dim3(n), dim3(256), lds, s, (const unsigned char *)f_arena, fns,
                           list, c_arena);
    return hipGetLastError();
}

// ---------------------------------------------------- batched four-step ---
// The same three passes as the single-function four-step FFT, for every
// long function of a batch in one launch each: block t works on function
// tiles[t].fn starting at column (row, coefficient) tiles[t].first.
__global__ __launch_bounds__(256) void k_bbig_cols(const double *__restrict__ phi_arena,
                                                   const BigFn *__restrict__ fns,
                                                   const BigTile *__restrict__ tiles) {
    extern __shared__ double2 lds[];
    const BigTile tl = tiles[blockIdx.x];
    const BigFn &fn = fns[tl.fn];
    const int L1 = fn.L1, L2 = fn.L2, CB = fn.CB, k20 = tl.first;
    const FftSched s1 = fn.s1;
    struct Phi {
        const double *p;
        __device__ __forceinline__ double operator()(int64_t m) const { return p[m - 1]; }
    } ph{phi_arena + fn.phi_off};
    // four values per thread at a time, every load issued before the first use
    for (int e0 = 0; e0 < CB * L1; e0 += 4 * 256) {
        double2 z[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = min(e0 + (int)threadIdx.x + u * 256, CB * L1 - 1);
            const int k1 = e / CB, cb = e - k1 * CB;
            z[u] = dst_pack((int64_t)L2 * k1 + k20 + cb, ph, fn.H, fn.L, fn.tw_pre, fn.tw_pack);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + (int)threadIdx.x + u * 256;
            const int k1 = e / CB, cb = e - k1 * CB;
            if (e < CB * L1) lds[cb * L1 + k1] = z[u];
        }
    }
    __syncthreads();
    fft_lds<256, 8>(lds, L1, CB, s1, fn.tw_fft, L2);
    for (int e = threadIdx.x; e < CB * L1; e += 256) {
        const int p1 = e / CB, cb = e - p1 * CB;
        const int k2 = k20 + cb;
        fn.zA[(int64_t)p1 * L2 + k2] = cmul(lds[cb * L1 + p1], fn.tw_fft[(int64_t)p1 * k2]);
    }
}

__global__ __launch_bounds__(256) void k_bbig_rows(const BigFn *__restrict__ fns, const BigTile *__restrict__ tiles) {
    extern __shared__ double2 lds[];
    const BigTile tl = tiles[blockIdx.x];
    const BigFn &fn = fns[tl.fn];
    const int L1 = fn.L1, L2 = fn.L2, RB = fn.RB, p10 = tl.first;
    const FftSched s2 = fn.s2;
    for (int e0 = 0; e0 < RB * L2; e0 += 4 * 256) {  // four loads in flight per thread
        double2 z[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) z[u] = fn.zA[(int64_t)p10 * L2 + min(e0 + (int)threadIdx.x + u * 256, RB * L2 - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e0 + (int)threadIdx.x + u * 256 < RB * L2) lds[e0 + threadIdx.x + u * 256] = z[u];
    }
    __syncthreads();
    fft_lds<256, 8>(lds, L2, RB, s2, fn.tw_fft, L1);
    for (int e = threadIdx.x; e < RB * L2; e += 256) {
        const int p2 = e / RB, rb = e - p2 * RB;
        fn.zB[(int64_t)(p10 + rb) + (int64_t)L1 * p2] = lds[rb * L2 + p2];
    }
}

__global__ __launch_bounds__(256) void k_bbig_post(const BigFn *__restrict__ fns, const BigTile *__restrict__ tiles,
                                                   double *__restrict__ c_arena) {
    const BigTile tl = tiles[blockIdx.x];
    const BigFn &fn = fns[tl.fn];
    const int64_t n0 = tl.first, n1 = min((int64_t)tl.first + 1024, fn.N);
    double *c = c_arena + fn.c_off;
    for (int64_t n = n0 + threadIdx.x; n < n1; n += 256) c[n] = dst_post(n, fn.zB, fn.H);
}

int four_step_blocks(int L1, int L2, int *CB, int *RB) {
    int cb = 2048 / L1 < L2 ? 2048 / L1 : L2;
    while (cb > 1 && L2 % cb) --cb;
    int rb = 2048 / L2 < L1 ? 2048 / L2 : L1;
    while (rb > 1 && L1 % rb) --rb;
    *CB = cb;
    *RB = rb;
    return (cb >= 1 && rb >= 1 && cb * L1 <= 2048 && rb * L2 <= 2048) ? 0 : -1;
}

hipError_t launch_bbig(const double *phi_arena, const BigFn *fns, const BigTile *ctiles, int nct,
                       const BigTile *rtiles, int nrt, const BigTile *ptiles, int npt, double *c_arena,
                       hipStream_t s) {
    if (nct <= 0) return hipSuccess;
    const size_t lds = 2048 * sizeof(double2);
    hipLaunchKernelGGL(k_bbig_cols, dim3(nct), dim3(256), lds, s, phi_arena, fns, ctiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bbig_rows, dim3(nrt), dim3(256), lds, s, fns, rtiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bbig_post, dim3(npt), dim3(256), 0, s, fns, ptiles, c_arena);
    return hipGetLastError();
}

}  // namespace lc
