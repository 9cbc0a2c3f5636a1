// LDS-resident Stockham FFT building blocks (FP64 complex, wave64, gfx950)
// and the DST-III pack/unpack that turns the one FFT of eq. (2.4) into a
// complex FFT of half length.  Header-only: included by every kernel file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lc_internal.h"

namespace lc {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 mul_i(double2 a) { return make_double2(-a.y, a.x); }

// Small DFTs in the positive-exponent direction: X_s = sum_r v_r e^{+2 pi i r s / R}.
template <int R> struct Dft;

template <> struct Dft<2> {
    static __device__ __forceinline__ void run(double2 *v) {
        double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <> struct Dft<3> {
    static __device__ __forceinline__ void run(double2 *v) {
        const double h = 0.86602540378443864676;  // sqrt(3)/2
        double2 s = cadd(v[1], v[2]);
        double2 d = csub(v[1], v[2]);
        double2 m = make_double2(v[0].x - 0.5 * s.x, v[0].y - 0.5 * s.y);
        double2 t = make_double2(-h * d.y, h * d.x);  // i * (sqrt(3)/2) * d
        v[0] = cadd(v[0], s);
        v[1] = cadd(m, t);
        v[2] = csub(m, t);
    }
};

template <> struct Dft<4> {
    static __device__ __forceinline__ void run(double2 *v) {
        double2 t0 = cadd(v[0], v[2]);
        double2 t1 = csub(v[0], v[2]);
        double2 t2 = cadd(v[1], v[3]);
        double2 t3 = mul_i(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

// X_k = sum_j x_j w^{jk}, w = e^{+2 pi i/5}: with s1 = x1 + x4, d1 = x1 - x4,
// s2 = x2 + x3, d2 = x2 - x3, X_1,4 = x0 + c1 s1 + c2 s2 +- i (n1 d1 + n2 d2)
// and X_2,3 = x0 + c2 s1 + c1 s2 +- i (n2 d1 - n1 d2), with c1, c2 = cos(2 pi/5),
// cos(4 pi/5) = (sqrt 5 - 1)/4, -(sqrt 5 + 1)/4 and n1, n2 = sin(2 pi/5),
// sin(4 pi/5) = sqrt(10 + 2 sqrt 5)/4, sqrt(10 - 2 sqrt 5)/4.
template <> struct Dft<5> {
    static __device__ __forceinline__ void run(double2 *v) {
        const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
        const double n1 = 0.95105651629515357212, n2 = 0.58778525229247312917;
        const double2 s1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
        const double2 s2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
        const double2 a1 = make_double2(v[0].x + c1 * s1.x + c2 * s2.x, v[0].y + c1 * s1.y + c2 * s2.y);
        const double2 a2 = make_double2(v[0].x + c2 * s1.x + c1 * s2.x, v[0].y + c2 * s1.y + c1 * s2.y);
        // b1 = i (n1 d1 + n2 d2), b2 = i (n2 d1 - n1 d2)
        const double2 b1 = make_double2(-(n1 * d1.y + n2 * d2.y), n1 * d1.x + n2 * d2.x);
        const double2 b2 = make_double2(-(n2 * d1.y - n1 * d2.y), n2 * d1.x - n1 * d2.x);
        v[0] = cadd(v[0], cadd(s1, s2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    }
};

template <> struct Dft<8> {
    static __device__ __forceinline__ void run(double2 *v) {
        const double c = 0.70710678118654752440;  // sqrt(1/2)
        double2 e[4] = {v[0], v[2], v[4], v[6]};
        double2 o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4>::run(e);
        Dft<4>::run(o);
        // o_s *= e^{+2 pi i s / 8}
        o[1] = make_double2(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y));
        o[2] = mul_i(o[2]);
        o[3] = make_double2(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y));
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            v[s] = cadd(e[s], o[s]);
            v[s + 4] = csub(e[s], o[s]);
        }
    }
};

// q = a / d and rem = a % d for 0 <= a < 2^20, d >= 1, from an FP32
// reciprocal rd = 1/d: the estimate a rd is off by less than one, so one
// correction step makes both exact (a few instructions instead of a full
// integer division).
__device__ __forceinline__ int fdivmod(int a, int d, float rd, int &rem) {
    int q = (int)((float)a * rd);
    int r = a - q * d;
    if (r >= d) { ++q; r -= d; }
    if (r < 0) { --q; r += d; }
    rem = r;
    return q;
}

// One radix-R Stockham pass over nsub independent transforms of length Lsub
// stored back to back in LDS (in place: every thread first loads all of its
// butterflies, then the block synchronizes, then results are stored).
// Ns is the product of the radices of the previous passes.  Twiddles
// e^{2 pi i m / Lsub} are read from tw[m * tw_stride], requested with the
// LDS loads so that their latency passes while the block synchronizes.
// ONE: nsub == 1.  Requires nsub * Lsub <= EPT * T (checked by the host
// launchers) and Lsub * tw_stride < 2^31.
template <int R, int T, int EPT, bool ONE>
__device__ __forceinline__ void stockham_pass(double2 *__restrict__ lds, int Lsub, int nsub, int Ns,
                                              const double2 *__restrict__ tw, int tw_stride) {
    constexpr int MAXB = (EPT + R - 1) / R;
    const int nbs = Lsub / R;
    const int total = ONE ? nbs : nsub * nbs;
    const int tid = threadIdx.x;
    const int span = Ns * R;
    const int twstep = Lsub / span;
    const float rnbs = 1.0f / (float)nbs, rns = 1.0f / (float)Ns;
    double2 v[MAXB][R];
    double2 w[MAXB][R - 1];
    int base[MAXB];  // output index of the butterfly's first value
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * T;
        if (b < total) {
            int sub = 0, j = b;
            if constexpr (!ONE) sub = fdivmod(b, nbs, rnbs, j);
            const double2 *x = lds + sub * Lsub;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = x[j + r * nbs];
            int k;
            const int q = fdivmod(j, Ns, rns, k);
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) w[i][r - 1] = tw[k * r * twstep * tw_stride];
            }
            base[i] = sub * Lsub + q * span + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * T;
        if (b < total) {
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], w[i][r - 1]);
            }
            Dft<R>::run(v[i]);
#pragma unroll
            for (int s = 0; s < R; ++s) lds[base[i] + s * Ns] = v[i][s];
        }
    }
    __syncthreads();
}

template <int T, int EPT, bool ONE>
__device__ __forceinline__ void fft_passes(double2 *__restrict__ lds, int Lsub, int nsub, const FftSched &sch,
                                           const double2 *__restrict__ tw, int tw_stride) {
    int Ns = 1;
    for (int p = 0; p < sch.npass; ++p) {
        const int R = sch.radix[p];
        switch (R) {
            case 8: stockham_pass<8, T, EPT, ONE>(lds, Lsub, nsub, Ns, tw, tw_stride); break;
            case 4: stockham_pass<4, T, EPT, ONE>(lds, Lsub, nsub, Ns, tw, tw_stride); break;
            case 5: stockham_pass<5, T, EPT, ONE>(lds, Lsub, nsub, Ns, tw, tw_stride); break;
            case 3: stockham_pass<3, T, EPT, ONE>(lds, Lsub, nsub, Ns, tw, tw_stride); break;
            default: stockham_pass<2, T, EPT, ONE>(lds, Lsub, nsub, Ns, tw, tw_stride); break;
        }
        Ns *= R;
    }
}

// Unnormalized positive-exponent FFT of nsub transforms of length Lsub in LDS:
// z_p = sum_k Z_k e^{+2 pi i p k / Lsub}, natural order in and out.
template <int T, int EPT>
__device__ void fft_lds(double2 *__restrict__ lds, int Lsub, int nsub, const FftSched &sch,
                        const double2 *__restrict__ tw, int64_t tw_stride) {
    if (nsub == 1) fft_passes<T, EPT, true>(lds, Lsub, 1, sch, tw, (int)tw_stride);
    else fft_passes<T, EPT, false>(lds, Lsub, nsub, sch, tw, (int)tw_stride);
}

// ------------------------------------------------ octant twiddles ---
// The FFT twiddles tw[m] = e^{2 pi i m / L} (m < L, L divisible by 8) follow
// from the first octant tab[j] = tw[j], j <= L/8, by the exact quarter-turn
// and octant symmetries.  The host builds its table with the same reduction
// (quadrant, then the angle or its complement to a quarter turn, at most
// pi/4), so these are its values bit for bit.  The compile-time passes read
// an LDS copy of the octant (L/8 + 1 entries after the transform's L values)
// instead of the global table: global twiddle reads wait behind the
// streaming loads and stores of the kernels around the FFT.
template <int LS>
__device__ __forceinline__ double2 tw_octant(const double2 *__restrict__ tab, int m) {
    constexpr int Q = LS / 4, O = LS / 8;
    const int q = (m / Q) & 3, r = m % Q;
    const bool hi = r > O;  // angle past pi/4 in its quadrant: the complement's sine and cosine
    const double2 t = tab[hi ? Q - r : r];
    const double c = hi ? t.y : t.x, sn = hi ? t.x : t.y;
    return q == 0 ? make_double2(c, sn) : q == 1 ? make_double2(-sn, c) : q == 2 ? make_double2(-c, -sn)
                                                                             : make_double2(sn, -c);
}

// LDS bytes of a one-transform DST workgroup: L values and the octant.
__host__ __device__ constexpr size_t fft_lds_bytes(int64_t L) { return (size_t)(L + L / 8 + 1) * 16; }

// The octant of tw (L/8 + 1 <= 2T values: at most two per thread for
// L <= 8T), read at clamped indices so that both reads are issued at once
// with the caller's first loads; octant_store puts them in LDS, before the
// barrier that precedes the FFT.
struct OctantRegs {
    double2 a, b;
};
template <int T>
__device__ __forceinline__ OctantRegs octant_load(const double2 *__restrict__ tw, int L) {
    const int n = L / 8 + 1;
    return {tw[min((int)threadIdx.x, n - 1)], tw[min((int)threadIdx.x + T, n - 1)]};
}
template <int T>
__device__ __forceinline__ void octant_store(double2 *__restrict__ tab, const OctantRegs &o, int L) {
    const int n = L / 8 + 1;
    if ((int)threadIdx.x < n) tab[threadIdx.x] = o.a;
    if ((int)threadIdx.x + T < n) tab[threadIdx.x + T] = o.b;
}

// One transform of power-of-two length LS whose pass stride NS is a
// compile-time constant: the butterfly's quotient and remainder by NS and
// its twiddle offsets are shifts, masks and constants, where the run-time
// pass divides.  Each pass computes what stockham_pass computes for the same
// radix and stride.
template <int R, int T, int LS, int NS, bool OCT>
__device__ __forceinline__ void stockham_fixed(double2 *__restrict__ lds, const double2 *__restrict__ tw,
                                               const double2 *__restrict__ tab) {
    constexpr int nbs = LS / R, span = NS * R, twstep = LS / span;
    constexpr int MAXB = (nbs + T - 1) / T;
    const int tid = threadIdx.x;
    double2 v[MAXB][R];
    double2 w[MAXB][R > 1 ? R - 1 : 1];
    int base[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * T;
        if (nbs % T == 0 || b < nbs) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = lds[b + r * nbs];
            const int k = b % NS, q = b / NS;
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r)
                    w[i][r - 1] = OCT ? tw_octant<LS>(tab, k * r * twstep) : tw[k * r * twstep];
            }
            base[i] = q * span + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * T;
        if (nbs % T == 0 || b < nbs) {
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], w[i][r - 1]);
            }
            Dft<R>::run(v[i]);
#pragma unroll
            for (int s = 0; s < R; ++s) lds[base[i] + s * NS] = v[i][s];
        }
    }
    __syncthreads();
}

// Radix-8 passes, then one radix-4 or radix-2 pass for what is left;
// twiddles from the LDS octant tab when OCT.
template <int T, int LS, int NS, bool OCT>
__device__ __forceinline__ void fixed_passes(double2 *__restrict__ lds, const double2 *__restrict__ tw,
                                             const double2 *__restrict__ tab) {
    if constexpr (NS < LS) {
        constexpr int rest = LS / NS;
        constexpr int R = rest % 8 == 0 ? 8 : (rest % 4 == 0 ? 4 : 2);
        stockham_fixed<R, T, LS, NS, OCT>(lds, tw, tab);
        fixed_passes<T, LS, NS * R, OCT>(lds, tw, tab);
    }
}

// One transform of length L <= EPT T in LDS (as fft_lds with nsub = 1):
// the power-of-two lengths 2T, 4T and 8T take compile-time passes (radix 8
// first, whatever radix order the schedule names: the results differ from
// the schedule's by rounding only), every other length the run-time
// schedule.  tab: the LDS octant of tw, stored (octant_store) before a
// barrier that precedes this call, or null for global twiddle reads.
template <int T, int EPT>
__device__ __forceinline__ void fft_lds_one(double2 *__restrict__ lds, int L, const FftSched &sch, const double2 *__restrict__ tw,
                            const double2 *__restrict__ tab = nullptr) {
    static_assert(EPT == 8, "compile-time lengths assume 8 values per thread");
    if (tab) {
        if (L == 8 * T) return fixed_passes<T, 8 * T, 1, true>(lds, tw, tab);
        if (L == 4 * T) return fixed_passes<T, 4 * T, 1, true>(lds, tw, tab);
        if (L == 2 * T && T >= 4) return fixed_passes<T, 2 * T, 1, true>(lds, tw, tab);
    }
    if (L == 8 * T) fixed_passes<T, 8 * T, 1, false>(lds, tw, tab);
    else if (L == 4 * T) fixed_passes<T, 4 * T, 1, false>(lds, tw, tab);
    else if (L == 2 * T) fixed_passes<T, 2 * T, 1, false>(lds, tw, tab);
    else fft_passes<T, EPT, true>(lds, L, 1, sch, tw, 1);
}

// DST-III pack.  With phi_m = phi[m-1] for m = 1..H (H = 2L) and
//   V_k = e^{i pi k / (2H)} (phi_{H-k} - i phi_k)   (1 <= k < H),  V_0 = phi_H,
//   Z_k = (V_k + V_{k+L}) + i e^{2 pi i k / H} (V_k - V_{k+L}),  0 <= k < L,
// the length-L transform z = FFT(Z) carries the sums
//   v_q = sum_{k<H} V_k e^{2 pi i q k / H}  as  v_{2p} = Re z_p, v_{2p+1} = Im z_p,
// and the sine sums of eq. (2.4) follow in dst_post.  tw_pre[k] = e^{i pi k/(2H)}
// (k < H), tw_pack[k] = e^{2 pi i k / H} (k < L).
// Branch-free in k: V_0 = tw_pre[0] (phi_H - 0 i) with tw_pre[0] = 1 gives
// exactly (phi_H, +0), and phi_k is read at index max(k, 1) so that k = 0
// reads nothing outside phi.
template <typename PhiAt>
__device__ __forceinline__ double2 dst_pack(int64_t k, PhiAt phi, int64_t H, int64_t L,
                                            const double2 *__restrict__ tw_pre,
                                            const double2 *__restrict__ tw_pack) {
    const double pk = phi(k > 0 ? k : 1);
    const double2 vk = cmul(tw_pre[k], make_double2(phi(H - k), k > 0 ? -pk : 0.0));
    const double2 vkl = cmul(tw_pre[k + L], make_double2(phi(L - k), -phi(L + k)));
    const double2 sum = cadd(vk, vkl);
    const double2 r = cmul(tw_pack[k], csub(vk, vkl));
    return make_double2(sum.x - r.y, sum.y + r.x);
}

// Z_k from its four values of phi (k > 0): the arithmetic of dst_pack.
__device__ __forceinline__ double2 dst_pack_from(double phi_Hk, double phi_k, double phi_Lk, double phi_Lpk,
                                                 double2 t0, double2 t1, double2 tp) {
    const double2 vk = cmul(t0, make_double2(phi_Hk, -phi_k));
    const double2 vkl = cmul(t1, make_double2(phi_Lk, -phi_Lpk));
    const double2 sum = cadd(vk, vkl);
    const double2 r = cmul(tp, csub(vk, vkl));
    return make_double2(sum.x - r.y, sum.y + r.x);
}

// Z_k of every k < L into lds[k] (L <= EPT T), dst_pack's values bit for
// bit.  Z_g and Z_{L-g} read the same four values of phi (phi_g, phi_{H-g},
// phi_{L-g}, phi_{L+g}), so one thread forms both from one set of loads,
// and three of their six twiddles from the other three (the tables hold
// tw_pre[2L-g] = swap(tw_pre[g]), tw_pre[L+g] = swap(tw_pre[L-g]) and
// tw_pack[L-g] = (-tw_pack[g].x, tw_pack[g].y) exactly, by construction):
// pairs g = 1 .. ceil(L/2) - 1, two at a time with indices clamped so that
// every load is issued before the first use (only valid pairs are stored);
// thread T-1 adds Z_0 and, for even L, Z_{L/2}.
template <int T, int EPT, typename PhiAt>
__device__ __forceinline__ void dst_pack_lds(double2 *__restrict__ lds, PhiAt phi, int64_t H, int L,
                                             const double2 *__restrict__ tw_pre,
                                             const double2 *__restrict__ tw_pack) {
    const int G = (L + 1) >> 1;  // pairs g in [1, G)
    constexpr int NP = (EPT + 1) / 2;
    constexpr int U = NP < 2 ? NP : 2;
    if ((int)threadIdx.x == T - 1) {
        lds[0] = dst_pack(0, phi, H, L, tw_pre, tw_pack);
        if (!(L & 1) && L >= 2) lds[L >> 1] = dst_pack(L >> 1, phi, H, L, tw_pre, tw_pack);
    }
#pragma unroll
    for (int i0 = 0; i0 < NP; i0 += U) {
        if (1 + i0 * T >= G) break;
        double a[U], b[U], c[U], d[U];
        double2 t0[U], t1[U], tp[U], s0[U], s1[U], sp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int g0 = 1 + (int)threadIdx.x + (i0 + u) * T;
            const int g = g0 < G ? g0 : G - 1;
            a[u] = phi(g);
            b[u] = phi(H - g);
            c[u] = phi(L - g);
            d[u] = phi(L + g);
            t0[u] = tw_pre[g];
            s0[u] = tw_pre[L - g];
            tp[u] = tw_pack[g];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            t1[u] = make_double2(s0[u].y, s0[u].x);     // tw_pre[L + g]
            s1[u] = make_double2(t0[u].y, t0[u].x);     // tw_pre[2L - g]
            sp[u] = make_double2(-tp[u].x, tp[u].y);    // tw_pack[L - g]
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int g = 1 + (int)threadIdx.x + (i0 + u) * T;
            if (g < G) {
                lds[g] = dst_pack_from(b[u], a[u], c[u], d[u], t0[u], t1[u], tp[u]);
                lds[L - g] = dst_pack_from(d[u], c[u], a[u], b[u], s0[u], s1[u], sp[u]);
            }
        }
    }
}

// DST-III unpack and rescale: c_n = (2n+1) a_n with
//   a_n = (1/H) [ sum_{j<H} phi_j sin(pi (2n+1) j / (2H)) + (1/2)(-1)^n phi_H ]
//       = (-1)^n X_n / H,  X_{2m} = v_m / 2,  X_{2m+1} = v_{H-1-m} / 2,
// evaluated as ((2n+1) (-1)^n v) * r with r = 1/(2H) rounded (exact, so
// the same as dividing by 2H, when H is a power of two); r is loop-invariant
// in the callers' loops, so its division is done once.
__device__ __forceinline__ double dst_post(int64_t n, const double2 *z, int64_t H) {
    const int64_t q = (n & 1) ? (H - 1 - (n >> 1)) : (n >> 1);
    const double2 zz = z[q >> 1];
    const double v = (q & 1) ? zz.y : zz.x;
    const double sgn = (n & 1) ? -1.0 : 1.0;
    return (double)(2 * n + 1) * sgn * v * (1.0 / (double)(2 * H));
}

// dst_post for every n < N by the T threads of a block, four coefficients
// per thread and step: with H even, n = 4j .. 4j+3 read only z[j] and
// z[H/2 - 1 - j] (q = 2j, 2j+1 and H-1-2j, H-2-2j), so a step is two LDS
// reads, eight multiplications and, where c + 4j is 16-byte aligned, two
// 16-byte stores.  The values are dst_post's bit for bit.  N <= H.  NT:
// non-temporal stores, for coefficients that nothing in the library reads
// back (they leave the caches to the loads around them).
typedef double lc_f64x2 __attribute__((ext_vector_type(2)));
template <int T, bool NT = false>
__device__ __forceinline__ void dst_post_block(double *__restrict__ c, int N, const double2 *__restrict__ z, int H) {
    const double r = 1.0 / (double)(2 * H);
    const bool vec = ((uintptr_t)c & 15) == 0;
    const int nq = N >> 2;
#pragma unroll 2
    for (int j = threadIdx.x; j < nq; j += T) {
        const double2 a = z[j], b = z[(H >> 1) - 1 - j];
        const double f = (double)(8 * j + 1);
        const double c0 = f * a.x * r, c1 = -(f + 2.0) * b.y * r;
        const double c2 = (f + 4.0) * a.y * r, c3 = -(f + 6.0) * b.x * r;
        if (vec) {
            const lc_f64x2 u0 = {c0, c1}, u1 = {c2, c3};
            lc_f64x2 *p = reinterpret_cast<lc_f64x2 *>(c) + 2 * j;
            if constexpr (NT) {
                __builtin_nontemporal_store(u0, p);
                __builtin_nontemporal_store(u1, p + 1);
            } else {
                p[0] = u0;
                p[1] = u1;
            }
        } else if constexpr (NT) {
            __builtin_nontemporal_store(c0, c + 4 * j);
            __builtin_nontemporal_store(c1, c + 4 * j + 1);
            __builtin_nontemporal_store(c2, c + 4 * j + 2);
            __builtin_nontemporal_store(c3, c + 4 * j + 3);
        } else {
            c[4 * j] = c0;
            c[4 * j + 1] = c1;
            c[4 * j + 2] = c2;
            c[4 * j + 3] = c3;
        }
    }
    const int n = 4 * nq + (int)threadIdx.x;
    if (n < N) c[n] = dst_post(n, z, H);
}

}  // namespace lc
