// Device helpers of the Abel quadrature reduction shared by the single and
// batched kernels: vector loads of FP64/FP32 samples, FP64 accumulation and
// fixed-order wave reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lc {

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));

template <typename T, int VEC> struct VecOf;
template <> struct VecOf<double, 1> { using type = double; };
template <> struct VecOf<double, 2> { using type = dv2; };
template <> struct VecOf<float, 1> { using type = float; };
template <> struct VecOf<float, 2> { using type = fv2; };
template <> struct VecOf<float, 4> { using type = fv4; };

__device__ __forceinline__ void to_d(double v, double *o) { o[0] = v; }
__device__ __forceinline__ void to_d(dv2 v, double *o) { o[0] = v.x; o[1] = v.y; }
__device__ __forceinline__ void to_d(float v, double *o) { o[0] = (double)v; }
__device__ __forceinline__ void to_d(fv2 v, double *o) { o[0] = (double)v.x; o[1] = (double)v.y; }
__device__ __forceinline__ void to_d(fv4 v, double *o) {
    o[0] = (double)v.x; o[1] = (double)v.y; o[2] = (double)v.z; o[3] = (double)v.w;
}

template <typename V>
__device__ __forceinline__ V ld_stream(const V *p) {
    return __builtin_nontemporal_load(p);
}

// Streaming store of one phi value.  The reductions write 8 bytes per row
// among many times that in sample reads; measured on 192- and 384-byte rows,
// these stores cost 12-22% of the kernel time as ordinary stores and 2.5-4%
// less as nontemporal ones.
__device__ __forceinline__ void st_stream(double *p, double v) { __builtin_nontemporal_store(v, p); }

// Load through a pointer known to address global memory (a pointer read out
// of a descriptor is otherwise a flat access, counted with the LDS ones).
__device__ __forceinline__ double ld_global(const double *p) {
    return *(const __attribute__((address_space(1))) double *)p;
}

// Lane i takes lane i + K of its 16-lane row (0 past the row's end): a DPP
// row shift, so a VALU move rather than a trip through the LDS crossbar.
template <int K>
__device__ __forceinline__ double row_shl(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x100 + K, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0x100 + K, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Total of each aligned group of G lanes, valid in the group's first lane
// (the others hold partial sums).  The offsets halve from G/2 down, so that
// lane sums the fixed pairwise tree of an xor butterfly; the steps inside a
// 16-lane row are DPP shifts, the steps across rows lane shuffles.  Every
// lane of a group must be active (groups never straddle divergent rows).
template <int G>
__device__ __forceinline__ double group_sum(double acc) {
    if constexpr (G >= 64) acc += __shfl_down(acc, 32, 64);
    if constexpr (G >= 32) acc += __shfl_down(acc, 16, 64);
    if constexpr (G >= 16) acc += row_shl<8>(acc);
    if constexpr (G >= 8) acc += row_shl<4>(acc);
    if constexpr (G >= 4) acc += row_shl<2>(acc);
    if constexpr (G >= 2) acc += row_shl<1>(acc);
    return acc;
}

// Generic variant for any Q: G lanes per row stride over the Q/VEC chunks
// with bounds checks, 4 chunks in flight per lane; weights from global
// memory (L1/L2 resident: every row reuses them).
// Weights of one chunk: VEC doubles at w + c VEC.  WV = true reads them as
// 16-byte pairs (w must then be 16-byte aligned).
template <int VEC, bool WV>
__device__ __forceinline__ void chunk_weights(const double *__restrict__ w, int c, double *o) {
    if constexpr (WV && VEC % 2 == 0) {
        const dv2 *q = reinterpret_cast<const dv2 *>(w + c * VEC);
#pragma unroll
        for (int e = 0; e < VEC / 2; ++e) {
            const dv2 v = q[e];
            o[2 * e] = v.x;
            o[2 * e + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) o[e] = w[c * VEC + e];
    }
}

template <typename T, int VEC, int G, bool WV = false>
__device__ __forceinline__ double row_partial(const T *__restrict__ frow, const double *__restrict__ w,
                                              int NC, int g) {
    using V = typename VecOf<T, VEC>::type;
    const V *p = reinterpret_cast<const V *>(frow);
    double acc0 = 0.0, acc1 = 0.0;
    int c = g;
    for (; c + 3 * G < NC; c += 4 * G) {
        V a = ld_stream(p + c), b = ld_stream(p + c + G), cc = ld_stream(p + c + 2 * G),
          dd = ld_stream(p + c + 3 * G);
        double da[VEC], db[VEC], dc[VEC], dd_[VEC];
        to_d(a, da); to_d(b, db); to_d(cc, dc); to_d(dd, dd_);
        double wa[VEC], wb[VEC], wc[VEC], wd[VEC];
        chunk_weights<VEC, WV>(w, c, wa);
        chunk_weights<VEC, WV>(w, c + G, wb);
        chunk_weights<VEC, WV>(w, c + 2 * G, wc);
        chunk_weights<VEC, WV>(w, c + 3 * G, wd);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            acc0 = fma(wa[e], da[e], acc0);
            acc1 = fma(wb[e], db[e], acc1);
            acc0 = fma(wc[e], dc[e], acc0);
            acc1 = fma(wd[e], dd_[e], acc1);
        }
    }
    // the lane's last (at most 3) chunks: all loads in flight before the
    // first use, rather than one dependent round trip per chunk
    if (c < NC) {
        const bool h1 = c + G < NC, h2 = c + 2 * G < NC;
        const V zero = V{};
        const V a = ld_stream(p + c);
        const V b = h1 ? ld_stream(p + c + G) : zero;
        const V cc = h2 ? ld_stream(p + c + 2 * G) : zero;
        double da[VEC], db[VEC], dc[VEC];
        to_d(a, da); to_d(b, db); to_d(cc, dc);
        double wa[VEC], wb[VEC], wc[VEC];
        chunk_weights<VEC, WV>(w, c, wa);
        if (h1) chunk_weights<VEC, WV>(w, c + G, wb);
        if (h2) chunk_weights<VEC, WV>(w, c + 2 * G, wc);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            acc0 = fma(wa[e], da[e], acc0);
            if (h1) acc1 = fma(wb[e], db[e], acc1);
            if (h2) acc0 = fma(wc[e], dc[e], acc0);
        }
    }
    return acc0 + acc1;
}

}  // namespace lc
