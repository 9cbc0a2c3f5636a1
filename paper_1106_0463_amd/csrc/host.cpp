// Host runtime of the Legendre-coefficient library: argument validation,
// the Abel Gauss rule, twiddle tables, plan objects and the C ABI entry
// points for single-function plans (batch and GEMM plans live in their own
// files).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <sstream>
#include <thread>
#include <vector>

#include "lc_internal.h"

namespace lc {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

// Every device allocation of the library.  LC_ALLOC_LIMIT (bytes, read once)
// makes any single allocation larger than the limit fail as out of memory:
// a hook that lets a test drive the LC_ERR_NOMEM paths deterministically.
hipError_t device_alloc(void **p, size_t bytes) {
    static const long long limit = [] {
        const char *ev = getenv("LC_ALLOC_LIMIT");
        return ev ? atoll(ev) : -1LL;
    }();
    if (limit >= 0 && bytes > (size_t)limit) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

// LC_LOG=1 (read once): one stderr line per plan decision (grid size,
// launch shapes, radix schedules, batch classes and DST groups).
bool log_on() {
    static const bool on = [] {
        const char *ev = getenv("LC_LOG");
        return ev && atoi(ev) != 0;
    }();
    return on;
}

void log_line(const char *fmt, ...) {
    if (!log_on()) return;
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fprintf(stderr, "[lc] %s\n", buf);
}

std::string sched_str(const FftSched &s) {
    std::string r;
    for (int i = 0; i < s.npass; ++i) r += (i ? "x" : "") + std::to_string(s.radix[i]);
    return r.empty() ? "-" : r;
}

static lc_status fail(lc_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

static lc_status hip_fail(hipError_t e, const char *what) {
    return fail(LC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int device_cu_count() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

// ------------------------------------------------------------ sizes ---
// Smallest 2^a 3^b 5^c >= L with c <= 1: chains of radix-5 passes round
// more than the radix-8/4/3 passes they replace (e^{20x} at N = 20000: E_c
// 4.7e-13 to 9.3e-13 on L = 2^5 5^4 against 1.8e-13 on 2^12 5).
int64_t smooth_len_at_least(int64_t L) {
    if (L <= 1) return 1;
    int64_t best = INT64_MAX;
    for (int64_t p5 = 1; p5 <= 5; p5 *= 5) {
        for (int64_t p35 = p5;; p35 *= 3) {
            int64_t v = p35;
            while (v < L) v *= 2;
            best = std::min(best, v);
            if (p35 >= L) break;
        }
    }
    return best;
}

FftSched make_sched(int L, const int *order) {
    FftSched s{};
    s.n = L;
    int n = L, c8 = 0, c4 = 0, c2 = 0, c3 = 0, c5 = 0;
    while (n % 5 == 0) { n /= 5; ++c5; }
    while (n % 3 == 0) { n /= 3; ++c3; }
    while (n % 8 == 0) { n /= 8; ++c8; }
    if (n % 4 == 0) { n /= 4; ++c4; }
    if (n % 2 == 0) { n /= 2; ++c2; }
    // default order: largest radices first
    std::vector<int> r;
    if (order) {
        for (int i = 0; order[i]; ++i) r.push_back(order[i]);
    } else {
        for (int i = 0; i < c8; ++i) r.push_back(8);
        for (int i = 0; i < c5; ++i) r.push_back(5);
        for (int i = 0; i < c4; ++i) r.push_back(4);
        for (int i = 0; i < c3; ++i) r.push_back(3);
        for (int i = 0; i < c2; ++i) r.push_back(2);
    }
    s.npass = (int)r.size();
    for (int i = 0; i < s.npass && i < kMaxPasses; ++i) s.radix[i] = r[i];
    return s;
}

// ------------------------------------------------------- Gauss rule ---
// Positive half of the n = 2Q point Gauss-Legendre rule on [-1, 1]: the
// folded rule for integral_0^1 g(t) dt with g even, sum w_q = 1, exact for
// polynomials of degree <= 4Q-1 in t (degree <= 2Q-1 in x for the Abel map).
// Newton iteration on P_n in long double with Tricomi's initial guesses.
static void legendre_and_derivative(int n, long double x, long double &pn, long double &dpn) {
    long double pkm1 = 1.0L, pk = x;
    for (int k = 2; k <= n; ++k) {
        long double pk1 = ((long double)(2 * k - 1) * x * pk - (long double)(k - 1) * pkm1) / (long double)k;
        pkm1 = pk;
        pk = pk1;
    }
    pn = pk;
    dpn = (long double)n * (x * pk - pkm1) / (x * x - 1.0L);
}

double2 dd_split(long double v) {
    const double hi = (double)v;
    return make_double2(hi, (double)(v - (long double)hi));
}

// Positive half (n/2 nodes, decreasing, n even) of the n-point rule in long
// double: nodes x and weights w.
void gauss_positive_half_ld(int n, std::vector<long double> &x, std::vector<long double> &w) {
    const int h = n / 2;
    x.assign(h, 0.0L);
    w.assign(h, 0.0L);
    const long double PI = 3.141592653589793238462643383279502884L;
    auto work = [&](int i0, int i1) {
        for (int i = i0; i < i1; ++i) {
            const int k = i + 1;  // k-th largest root
            const long double nn = (long double)n;
            long double v = (1.0L - 1.0L / (8.0L * nn * nn) + 1.0L / (8.0L * nn * nn * nn)) *
                            cosl(PI * (4.0L * k - 1.0L) / (4.0L * nn + 2.0L));
            long double p, dp;
            for (int it = 0; it < 60; ++it) {
                legendre_and_derivative(n, v, p, dp);
                long double dx = p / dp;
                v -= dx;
                if (fabsl(dx) <= 4.0L * 1.0842e-19L * std::max(fabsl(v), 1e-3L)) break;
            }
            legendre_and_derivative(n, v, p, dp);
            x[i] = v;
            w[i] = 2.0L / ((1.0L - v * v) * dp * dp);
        }
    };
    const long long cost = (long long)h * n;
    int nth = 1;
    if (cost > 4000000LL) nth = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    if (nth == 1) {
        work(0, h);
    } else {
        std::vector<std::thread> th;
        const int chunk = (h + nth - 1) / nth;
        for (int a = 0; a < h; a += chunk) th.emplace_back(work, a, std::min(h, a + chunk));
        for (auto &t : th) t.join();
    }
}

void gauss_half_rule(int Q, std::vector<double> &t, std::vector<double> &w, std::vector<double2> &omt2) {
    std::vector<long double> x, wl;
    gauss_positive_half_ld(2 * Q, x, wl);
    t.resize(Q);
    w.resize(Q);
    omt2.resize(Q);
    for (int i = 0; i < Q; ++i) {
        t[i] = (double)x[i];
        w[i] = (double)wl[i];
        omt2[i] = dd_split((1.0L - x[i]) * (1.0L + x[i]));
    }
}

// --------------------------------------------------------- twiddles ---
// cos and sin of 2 pi num / den with exact integer reduction to an angle of
// at most pi/4 before calling the long-double routines.
static void sincos_turns(int64_t num, int64_t den, double *c, double *s) {
    const long double HALF_PI = 1.570796326794896619231321691639751442L;
    num %= den;
    if (num < 0) num += den;
    const int64_t q = (4 * num) / den;        // quadrant
    const int64_t r = 4 * num - q * den;      // angle = (pi/2) (q + r/den)
    long double cs, sn;
    if (2 * r > den) {
        const long double th = HALF_PI * (long double)(den - r) / (long double)den;
        cs = sinl(th);
        sn = cosl(th);
    } else {
        const long double th = HALF_PI * (long double)r / (long double)den;
        cs = cosl(th);
        sn = sinl(th);
    }
    long double rc, rs;
    switch (q & 3) {
        case 0: rc = cs; rs = sn; break;
        case 1: rc = -sn; rs = cs; break;
        case 2: rc = -cs; rs = -sn; break;
        default: rc = sn; rs = -cs; break;
    }
    *c = (double)rc;
    *s = (double)rs;
}

// The DST pack derives three of a mirror pair's six twiddles from the other
// three; the quadrant/octant reduction of sincos_turns already makes these
// entries exact images of their partners, and they are set from them so
// that this holds by construction (1 <= g < L/2, H = 2L):
//   pre[2L - g] = (pre[g].y, pre[g].x)          (angle pi/2 - theta)
//   pre[L + g]  = (pre[L - g].y, pre[L - g].x)  (reflection about pi/4)
//   pack[L - g] = (-pack[g].x, pack[g].y)        (angle pi - theta)
void twiddles(int64_t H, std::vector<double2> &pre, std::vector<double2> &pack, std::vector<double2> &fft) {
    const int64_t L = H / 2;
    pre.resize(H);
    pack.resize(L);
    fft.resize(L);
    for (int64_t k = 0; k < H; ++k) sincos_turns(k, 4 * H, &pre[k].x, &pre[k].y);
    for (int64_t k = 0; k < L; ++k) sincos_turns(k, H, &pack[k].x, &pack[k].y);
    for (int64_t k = 0; k < L; ++k) sincos_turns(k, L, &fft[k].x, &fft[k].y);
    for (int64_t g = 1; 2 * g < L; ++g) {
        pre[2 * L - g] = make_double2(pre[g].y, pre[g].x);
        pre[L + g] = make_double2(pre[L - g].y, pre[L - g].x);
        pack[L - g] = make_double2(-pack[g].x, pack[g].y);
    }
}

// Row factors of the node formula: A_j = 2 sin^2(pi j / (2H)) as a
// double-double pair, and 2 sin(pi j / (2H)) (the Abel Jacobian), j = 1..H.
long double row_half_sine(int64_t j, int64_t H) {
    const long double HALF_PI = 1.570796326794896619231321691639751442L;
    return (2 * j <= H) ? sinl(HALF_PI * (long double)j / (long double)H)
                        : cosl(HALF_PI * (long double)(H - j) / (long double)H);
}

void row_factors(int64_t H, std::vector<double2> &A, std::vector<double> &s2) {
    A.resize(H);
    s2.resize(H);
    for (int64_t r = 0; r < H; ++r) {
        const int64_t j = r + 1;                      // angle y/2 = (pi/2) j / H
        const long double sj = row_half_sine(j, H);
        A[r] = dd_split(2.0L * sj * sj);
        s2[r] = (double)(2.0L * sj);
    }
}

// -------------------------------------------------- launch configs ---
static bool fit_key_ok(int cpl, int u) {
    const int key = cpl * 16 + u;
    const int ok[] = {17, 18, 20, 33, 34, 36, 49, 50, 65, 66, 81, 97, 113, 129, 145, 161, 177};
    for (int k : ok)
        if (k == key) return true;
    return false;
}

QuadCfg default_quad_cfg(int prec, int Q, int64_t rows, int num_cu) {
    QuadCfg c{};
    c.block = 256;
    const int esz = prec == LC_FP64 ? 8 : 4;
    const int vfit = 16 / esz;
    bool fit = false;
    if (Q % vfit == 0) {
        const int nc = Q / vfit;
        for (int G : {8, 16, 4}) {
            if (nc % G) continue;
            const int cpl = nc / G;
            int u = cpl <= 2 ? 4 : (cpl <= 4 ? 2 : 1);
            while (u > 1 && !fit_key_ok(cpl, u)) u /= 2;
            if (!fit_key_ok(cpl, u)) continue;
            c.vec = vfit;
            c.G = G;
            c.cpl = cpl;
            c.unroll = u;
            fit = true;
            break;
        }
    }
    if (!fit) {
        c.cpl = 0;
        c.unroll = 1;
        if (esz == 8 && Q % 2 == 0 && Q >= 32) {
            c.vec = 2;
            const int nc = Q / 2;
            c.G = nc >= 64 ? 64 : (nc >= 32 ? 32 : 16);
        } else {
            c.vec = 1;
            c.G = Q >= 64 ? 64 : (Q >= 32 ? 32 : (Q >= 16 ? 16 : (Q >= 8 ? 8 : 4)));
        }
    }
    const int64_t rows_per_block = (int64_t)(c.block / 64) * (64 / c.G) * c.unroll;
    int64_t grid = (rows + rows_per_block - 1) / rows_per_block;
    // one round of resident blocks (occupancy of this variant)
    c.Qv = Q;
    c.grid = 1;
    int occ = quad_blocks_per_cu(c, prec);
    if (occ < 1) occ = 8;
    grid = std::min<int64_t>(grid, (int64_t)num_cu * occ);
    c.grid = (int)std::max<int64_t>(1, grid);
    return c;
}

bool pair_quad_cfg(int prec, int Q, QuadCfg &out) {
    const int vfit = prec == LC_FP64 ? 2 : 4;
    if (Q % vfit) return false;
    const int nc = 2 * Q / vfit;  // chunks of a row pair
    for (int G : {8, 16, 4}) {
        if (nc % G) continue;
        const int cpl = nc / G;
        int u = cpl <= 2 ? 4 : (cpl <= 4 ? 2 : 1);
        while (u > 1 && !fit_key_ok(cpl, u)) u /= 2;
        if (!fit_key_ok(cpl, u)) continue;
        QuadCfg c = out;
        c.vec = vfit;
        c.G = G;
        c.cpl = cpl;
        c.unroll = u;
        c.block = 256;
        c.grid = std::max(1, c.grid);
        c.Qv = Q;
        c.rpg = 2;
        out = c;
        return true;
    }
    return false;
}

// Workgroup size of an LDS FFT of length L: the smallest of 64 .. 1024
// threads with at most 8 values per thread (one radix-8 butterfly per thread
// and pass for L = 8T).
int dst_threads_for(int64_t L) {
    int T = 64;
    while (T < 1024 && L > 8 * T) T *= 2;
    return T;
}

bool dst_threads_ok(int T) { return T == 64 || T == 128 || T == 256 || T == 512 || T == 1024; }

DstCfg default_dst_cfg(int64_t L) {
    DstCfg d{};
    if (L <= kLdsFftMax) {
        d.threads = dst_threads_for(L);
        d.sched = make_sched((int)L);
        return d;
    }
    return four_step_cfg(L);
}

// Four-step split of an FFT of length L: L1 the largest divisor <= sqrt(L)
// with both factors <= 2048 (L1 = 0 if there is none).
DstCfg four_step_cfg(int64_t L) {
    DstCfg d{};
    int64_t best = 0;
    for (int64_t a = 2; a * a <= L; ++a)
        if (L % a == 0 && a <= 2048 && L / a <= 2048) best = a;
    d.threads = 256;
    if (best == 0) return d;  // unsupported (checked by the planner)
    d.L1 = (int)best;
    d.L2 = (int)(L / best);
    d.s1 = make_sched(d.L1);
    d.s2 = make_sched(d.L2);
    return d;
}

}  // namespace lc

using namespace lc;

// ================================================================ C ABI ===
extern "C" {

const char *lc_status_string(lc_status s) {
    switch (s) {
        case LC_OK: return "LC_OK";
        case LC_ERR_INVALID: return "LC_ERR_INVALID: invalid argument";
        case LC_ERR_NOMEM: return "LC_ERR_NOMEM: allocation failed";
        case LC_ERR_HIP: return "LC_ERR_HIP: HIP runtime error";
        case LC_ERR_UNSUPPORTED: return "LC_ERR_UNSUPPORTED: not supported by this library";
        case LC_ERR_INTERNAL: return "LC_ERR_INTERNAL: internal error";
    }
    return "unknown lc_status";
}

const char *lc_last_error(void) { return g_err.c_str(); }

lc_status lc_grid_size(int64_t M, int64_t *M_eff) {
    if (!M_eff) return fail(LC_ERR_INVALID, "lc_grid_size: M_eff is null");
    if (M < 2) return fail(LC_ERR_INVALID, "lc_grid_size: M=%lld < 2", (long long)M);
    if (M > ((int64_t)1 << 40)) return fail(LC_ERR_INVALID, "lc_grid_size: M=%lld too large", (long long)M);
    const int64_t L = smooth_len_at_least((std::max<int64_t>(M, 4) + 3) / 4);
    *M_eff = 4 * L;
    return LC_OK;
}

}  // extern "C"

namespace lc {

static void free_single(lc_plan_s *p) {
    hipFree(p->x);
    hipFree(p->w);
    hipFree(p->omt2);
    hipFree(p->rowA);
    hipFree(p->s2);
    hipFree(p->tw_pre);
    hipFree(p->tw_pack);
    hipFree(p->tw_fft);
    hipFree(p->phi);
    hipFree(p->zA);
    hipFree(p->zB);
    for (auto e : p->ev) hipEventDestroy(e);
    p->ev.clear();
}

template <typename T>
static hipError_t dalloc(T **ptr, size_t count, int64_t *acc) {
    *ptr = nullptr;
    if (count == 0) return hipSuccess;
    hipError_t e = device_alloc((void **)ptr, count * sizeof(T));
    if (e == hipSuccess && acc) *acc += (int64_t)(count * sizeof(T));
    return e;
}

lc_status validate_request(int64_t N, int64_t M, int32_t Q, int prec, const char *who) {
    if (N < 1) return fail(LC_ERR_INVALID, "%s: N=%lld must be >= 1", who, (long long)N);
    if (M < 2 || (M & 1)) return fail(LC_ERR_INVALID, "%s: M=%lld must be even and >= 2", who, (long long)M);
    if (N > M / 2) return fail(LC_ERR_INVALID, "%s: N=%lld exceeds M/2=%lld", who, (long long)N, (long long)(M / 2));
    if (Q < 1 || Q > 65536) return fail(LC_ERR_INVALID, "%s: Q=%d outside [1, 65536]", who, (int)Q);
    if (prec != LC_FP64 && prec != LC_FP32_QUAD) return fail(LC_ERR_INVALID, "%s: bad precision %d", who, prec);
    return LC_OK;
}

}  // namespace lc

extern "C" {

lc_status lc_plan(int64_t N, int64_t M, int32_t Q, lc_precision prec, lc_plan_t *out) {
    if (!out) return fail(LC_ERR_INVALID, "lc_plan: out is null");
    lc_status st = validate_request(N, M, Q, (int)prec, "lc_plan");
    if (st != LC_OK) return st;
    int64_t M_eff = 0;
    if ((st = lc_grid_size(M, &M_eff)) != LC_OK) return st;
    const int64_t H = M_eff / 2, L = H / 2;
    DstCfg dcfg = default_dst_cfg(L);
    if (L > kLdsFftMax && dcfg.L1 == 0)
        return fail(LC_ERR_UNSUPPORTED, "lc_plan: FFT length %lld has no supported four-step split",
                    (long long)L);
    if ((double)H * (double)Q > 4.0e10)
        return fail(LC_ERR_UNSUPPORTED, "lc_plan: H*Q=%.3g samples exceeds the library's limit",
                    (double)H * (double)Q);

    lc_plan_s *p = new (std::nothrow) lc_plan_s();
    if (!p) return fail(LC_ERR_NOMEM, "lc_plan: host allocation failed");
    p->kind = LC_PLAN_SINGLE;
    hipGetDevice(&p->device);
    p->fn.N = N;
    p->fn.M = M;
    p->fn.M_eff = M_eff;
    p->fn.H = H;
    p->fn.L = L;
    p->fn.Q = Q;
    p->fn.prec = (int)prec;

    std::vector<double> t, w, s2h;
    std::vector<double2> omt2, rowA;
    gauss_half_rule(Q, t, w, omt2);
    row_factors(H, rowA, s2h);
    std::vector<double2> pre, pack, fft;
    twiddles(H, pre, pack, fft);

    int64_t ws = 0;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    chk(dalloc(&p->x, (size_t)H * Q, &ws));
    chk(dalloc(&p->w, (size_t)Q, &ws));
    chk(dalloc(&p->omt2, (size_t)Q, &ws));
    chk(dalloc(&p->rowA, (size_t)H, &ws));
    chk(dalloc(&p->s2, (size_t)H, &ws));
    chk(dalloc(&p->tw_pre, (size_t)H, &ws));
    chk(dalloc(&p->tw_pack, (size_t)L, &ws));
    chk(dalloc(&p->tw_fft, (size_t)L, &ws));
    chk(dalloc(&p->phi, (size_t)H, &ws));
    if (L > kLdsFftMax) {
        chk(dalloc(&p->zA, (size_t)L, &ws));
        chk(dalloc(&p->zB, (size_t)L, &ws));
    }
    if (e != hipSuccess) {
        free_single(p);
        delete p;
        return e == hipErrorOutOfMemory ? fail(LC_ERR_NOMEM, "lc_plan: device allocation failed")
                                        : hip_fail(e, "lc_plan: hipMalloc");
    }
    p->workspace_bytes = ws;
    chk(hipMemcpy(p->w, w.data(), Q * sizeof(double), hipMemcpyHostToDevice));
    chk(hipMemcpy(p->omt2, omt2.data(), Q * sizeof(double2), hipMemcpyHostToDevice));
    chk(hipMemcpy(p->rowA, rowA.data(), H * sizeof(double2), hipMemcpyHostToDevice));
    chk(hipMemcpy(p->s2, s2h.data(), H * sizeof(double), hipMemcpyHostToDevice));
    chk(hipMemcpy(p->tw_pre, pre.data(), H * sizeof(double2), hipMemcpyHostToDevice));
    chk(hipMemcpy(p->tw_pack, pack.data(), L * sizeof(double2), hipMemcpyHostToDevice));
    chk(hipMemcpy(p->tw_fft, fft.data(), L * sizeof(double2), hipMemcpyHostToDevice));
    if (e == hipSuccess) chk(launch_nodes(H, Q, p->rowA, p->omt2, p->x, 0));
    if (e == hipSuccess) chk(hipDeviceSynchronize());
    if (e != hipSuccess) {
        free_single(p);
        delete p;
        return hip_fail(e, "lc_plan: building nodes");
    }
    p->quad = default_quad_cfg((int)prec, Q, H, device_cu_count());
    p->dst = dcfg;
    const int esz = prec == LC_FP64 ? 8 : 4;
    const double bytes = (double)H * Q * esz;
    p->fused_small = (bytes <= 256.0 * 1024 && H <= 4096 && fused_small_lds_bytes(H, Q) <= 65536);
    p->fused_threads = L <= 2048 ? 256 : 1024;
    log_line("lc_plan: N=%lld M=%lld M_eff=%lld H=%lld Q=%d %s; quad vec=%d G=%d cpl=%d unroll=%d grid=%d; %s",
             (long long)N, (long long)M, (long long)M_eff, (long long)H, Q, prec == LC_FP64 ? "fp64" : "fp32",
             p->quad.vec, p->quad.G, p->quad.cpl, p->quad.unroll, p->quad.grid,
             p->fused_small ? "one fused kernel" :
             (L > kLdsFftMax ? ("four-step " + std::to_string(dcfg.L1) + "x" + std::to_string(dcfg.L2) + " (" +
                                sched_str(dcfg.s1) + ", " + sched_str(dcfg.s2) + ")").c_str()
                             : ("LDS FFT L=" + std::to_string(L) + " T=" + std::to_string(dcfg.threads) + " radix " +
                                sched_str(dcfg.sched)).c_str()));
    *out = p;
    return LC_OK;
}

lc_status lc_plan_info(lc_plan_t p, lc_plan_desc *d);
lc_status lc_plan_nodes(lc_plan_t p, const double **x_dev, int64_t *rows, int32_t *Q);

}  // extern "C"

// Shared helpers for timing (used by all plan kinds).
namespace lc {
lc_status execute_adaptive(lc_plan_s *p, const void *f, double *c, hipStream_t s);
hipError_t timing_begin(lc_plan_s *p, hipStream_t s, int *slot) {
    *slot = -1;
    if (!p->timing) return hipSuccess;
    if (p->ev_used >= 4096) return hipSuccess;
    if ((int)p->ev.size() < 2 * (p->ev_used + 1)) {
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&b);
        if (e != hipSuccess) { hipEventDestroy(a); return e; }
        p->ev.push_back(a);
        p->ev.push_back(b);
    }
    *slot = p->ev_used++;
    return hipEventRecord(p->ev[2 * *slot], s);
}
hipError_t timing_end(lc_plan_s *p, hipStream_t s, int slot) {
    if (slot < 0) return hipSuccess;
    return hipEventRecord(p->ev[2 * slot + 1], s);
}
}  // namespace lc

extern "C" {

lc_status lc_execute(lc_plan_t p, const void *f_dev, double *c_dev, hipStream_t stream) {
    if (!p) return fail(LC_ERR_INVALID, "lc_execute: plan is null");
    if (p->kind != LC_PLAN_SINGLE && p->kind != LC_PLAN_ADAPTIVE)
        return fail(LC_ERR_INVALID, "lc_execute: not a single-function plan");
    if (!f_dev || !c_dev) return fail(LC_ERR_INVALID, "lc_execute: null f_dev or c_dev");
    if (((uintptr_t)f_dev) & 15) return fail(LC_ERR_INVALID, "lc_execute: f_dev must be 16-byte aligned");
    if (p->kind == LC_PLAN_ADAPTIVE) return execute_adaptive(p, f_dev, c_dev, stream);
    const FnDesc &d = p->fn;
    int slot = -1;
    hipError_t e = timing_begin(p, stream, &slot);
    if (e != hipSuccess) return hip_fail(e, "lc_execute: timing event");
    if (p->fused_small) {
        e = launch_fused_small(p->fused_threads, d.prec, f_dev, p->w, p->s2, d.H, d.Q, d.N, p->dst.sched,
                               p->tw_pre, p->tw_pack, p->tw_fft, c_dev, stream);
        if (e != hipSuccess) return hip_fail(e, "lc_execute: fused kernel launch");
        e = timing_end(p, stream, slot);
        if (e != hipSuccess) return hip_fail(e, "lc_execute: timing event");
        return LC_OK;
    }
    e = launch_quad(p->quad, d.prec, f_dev, p->w, p->s2, d.H, d.Q, p->phi, stream);
    if (e != hipSuccess) return hip_fail(e, "lc_execute: quadrature kernel launch");
    e = timing_end(p, stream, slot);
    if (e != hipSuccess) return hip_fail(e, "lc_execute: timing event");
    e = launch_dst(p->dst, p->phi, d.H, d.L, d.N, p->tw_pre, p->tw_pack, p->tw_fft, p->zA, p->zB, c_dev, stream);
    if (e != hipSuccess) return hip_fail(e, "lc_execute: FFT kernel launch");
    return LC_OK;
}

lc_status lc_plan_set_timing(lc_plan_t p, int32_t enable) {
    if (!p) return fail(LC_ERR_INVALID, "lc_plan_set_timing: plan is null");
    p->timing = enable != 0;
    p->ev_used = 0;
    return LC_OK;
}

lc_status lc_plan_kernel_ms(lc_plan_t p, double *avg_ms, int32_t *count) {
    if (!p || !avg_ms) return fail(LC_ERR_INVALID, "lc_plan_kernel_ms: null argument");
    if (!p->timing || p->ev_used == 0) return fail(LC_ERR_INVALID, "lc_plan_kernel_ms: nothing recorded");
    double sum = 0.0;
    for (int i = 0; i < p->ev_used; ++i) {
        hipError_t e = hipEventSynchronize(p->ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "lc_plan_kernel_ms: hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p->ev[2 * i], p->ev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(e, "lc_plan_kernel_ms: hipEventElapsedTime");
        sum += ms;
    }
    *avg_ms = sum / p->ev_used;
    if (count) *count = p->ev_used;
    return LC_OK;
}

}  // extern "C"

namespace lc {
// Implemented in host_batch.cpp / host_gemm.cpp.
void destroy_batch(lc_plan_s *p);
void destroy_gemm(lc_plan_s *p);
void destroy_adaptive(lc_plan_s *p);
void destroy_2d(lc_plan_s *p);
void info_batch(lc_plan_s *p, lc_plan_desc *d);
void info_gemm(lc_plan_s *p, lc_plan_desc *d);
void info_adaptive(lc_plan_s *p, lc_plan_desc *d);
void info_2d(lc_plan_s *p, lc_plan_desc *d);
lc_status nodes_batch(lc_plan_s *p, const double **x, int64_t *rows, int32_t *Q);
hipError_t adaptive_complement(const lc_plan_s *p, double *comp, hipStream_t s);
hipError_t batch_complement(const lc_plan_s *p, double *comp, hipStream_t s);
lc_status nodes_gemm(lc_plan_s *p, const double **x, int64_t *rows, int32_t *Q);
lc_status nodes_adaptive(lc_plan_s *p, const double **x, int64_t *rows, int32_t *Q);
lc_status nodes_2d(lc_plan_s *p, const double **x, int64_t *rows, int32_t *Q);
}  // namespace lc

extern "C" {

lc_status lc_plan_info(lc_plan_t p, lc_plan_desc *d) {
    if (!p || !d) return fail(LC_ERR_INVALID, "lc_plan_info: null argument");
    lc_plan_desc o{};
    o.kind = p->kind;
    if (p->kind == LC_PLAN_SINGLE) {
        o.precision = p->fn.prec;
        o.N = p->fn.N;
        o.M = p->fn.M;
        o.M_eff = p->fn.M_eff;
        o.H = p->fn.H;
        o.Q = p->fn.Q;
        o.samples = p->fn.H * (int64_t)p->fn.Q;
        o.sample_bytes = o.samples * (p->fn.prec == LC_FP64 ? 8 : 4);
        o.workspace_bytes = p->workspace_bytes;
    } else if (p->kind == LC_PLAN_BATCH) {
        info_batch(p, &o);
    } else if (p->kind == LC_PLAN_ADAPTIVE) {
        info_adaptive(p, &o);
    } else if (p->kind == LC_PLAN_2D) {
        info_2d(p, &o);
    } else {
        info_gemm(p, &o);
    }
    *d = o;
    return LC_OK;
}

lc_status lc_plan_nodes(lc_plan_t p, const double **x_dev, int64_t *rows, int32_t *Q) {
    if (!p || !x_dev) return fail(LC_ERR_INVALID, "lc_plan_nodes: null argument");
    if (p->kind == LC_PLAN_BATCH) return nodes_batch(p, x_dev, rows, Q);
    if (p->kind == LC_PLAN_GEMM) return nodes_gemm(p, x_dev, rows, Q);
    if (p->kind == LC_PLAN_ADAPTIVE) return nodes_adaptive(p, x_dev, rows, Q);
    if (p->kind == LC_PLAN_2D) return nodes_2d(p, x_dev, rows, Q);
    *x_dev = p->x;
    if (rows) *rows = p->fn.H;
    if (Q) *Q = p->fn.Q;
    return LC_OK;
}

lc_status lc_plan_nodes_complement(lc_plan_t p, double *omx_dev, hipStream_t stream) {
    if (!p || !omx_dev) return fail(LC_ERR_INVALID, "lc_plan_nodes_complement: null argument");
    hipError_t e;
    switch (p->kind) {
        case LC_PLAN_SINGLE:
            e = launch_nodes(p->fn.H, p->fn.Q, p->rowA, p->omt2, omx_dev, stream, true);
            break;
        case LC_PLAN_ADAPTIVE: e = adaptive_complement(p, omx_dev, stream); break;
        case LC_PLAN_BATCH: e = batch_complement(p, omx_dev, stream); break;
        default:
            return fail(LC_ERR_UNSUPPORTED, "lc_plan_nodes_complement: single, adaptive and batch plans only");
    }
    if (e != hipSuccess) return hip_fail(e, "lc_plan_nodes_complement: launch");
    return LC_OK;
}

lc_status lc_plan_destroy(lc_plan_t p) {
    if (!p) return LC_OK;
    hipDeviceSynchronize();
    if (p->kind == LC_PLAN_BATCH) destroy_batch(p);
    else if (p->kind == LC_PLAN_GEMM) destroy_gemm(p);
    else if (p->kind == LC_PLAN_ADAPTIVE) destroy_adaptive(p);
    else if (p->kind == LC_PLAN_2D) destroy_2d(p);
    free_single(p);
    delete p;
    return LC_OK;
}

}  // extern "C"

namespace lc {
lc_status fail_status(lc_status s, const std::string &msg) {
    g_err = msg;
    return s;
}
}  // namespace lc

// ------------------------------------------------------------ autotune ---
namespace lc {

static std::string sched_to_str(const FftSched &s) {
    std::string o = std::to_string(s.npass);
    for (int i = 0; i < s.npass; ++i) o += ' ' + std::to_string(s.radix[i]);
    return o;
}

static bool sched_from(std::istringstream &i, FftSched &s, int L) {
    FftSched t{};
    t.n = L;
    if (!(i >> t.npass) || t.npass < 0 || t.npass > kMaxPasses) return false;
    int64_t prod = 1;
    for (int k = 0; k < t.npass; ++k) {
        if (!(i >> t.radix[k])) return false;
        const int r = t.radix[k];
        if (r != 2 && r != 3 && r != 4 && r != 5 && r != 8) return false;  // the passes the kernels hold
        prod *= r;
    }
    if (prod != L) return false;
    s = t;
    return true;
}

lc_status tune_single(lc_plan_s *p, hipStream_t s) {
    const FnDesc &d = p->fn;
    const std::string key = arch_name() + "|single|" + std::to_string(d.H) + "|" + std::to_string(d.Q) + "|" +
                            std::to_string(d.prec) + "|" + std::to_string(d.N);
    std::string val;
    if (cache_get(key, val)) {
        std::istringstream in(val);
        std::string tag;
        QuadCfg q = p->quad;
        DstCfg dc = p->dst;
        int fused = 0, threads = 0;
        std::string qs;
        in >> tag;
        int v[7];
        bool ok = tag == "quad";
        for (int k = 0; ok && k < 7; ++k) ok = (bool)(in >> v[k]);
        if (ok) {
            q.vec = v[0]; q.G = v[1]; q.cpl = v[2]; q.unroll = v[3]; q.block = v[4]; q.grid = v[5]; q.rpg = v[6];
            ok = quad_cfg_supported(q, d.prec, d.Q) && (in >> tag) && tag == "dst" && (in >> threads);
        }
        if (ok && d.L <= kLdsFftMax) ok = sched_from(in, dc.sched, (int)d.L) && d.L <= 8 * threads && dst_threads_ok(threads);
        if (ok && d.L > kLdsFftMax) ok = sched_from(in, dc.s1, dc.L1) && sched_from(in, dc.s2, dc.L2);
        if (ok) ok = (in >> tag) && tag == "fused" && (in >> fused);
        if (ok) {
            p->quad = q;
            dc.threads = threads;
            p->dst = dc;
            p->fused_small = fused != 0 && p->fused_small;
            return LC_OK;
        }
    }
    hipError_t e = hipSuccess;
    double *cbuf = nullptr;
    if ((e = device_alloc((void **)&cbuf, (size_t)d.N * sizeof(double))) != hipSuccess)
        return fail_status(LC_ERR_NOMEM, "lc_autotune: workspace");
    const void *fsrc = p->x;  // same shape as the samples (FP64) or larger (FP32)
    double best = 1e30;
    QuadCfg bq = p->quad;
    for (const QuadCfg &c : quad_candidates(d.prec, d.Q, d.H, device_cu_count(), false)) {
        hipError_t er;
        const double t = time_launch([&](hipStream_t st) { return launch_quad(c, d.prec, fsrc, p->w, p->s2, d.H, d.Q, p->phi, st); }, s, 3, &er);
        if (er == hipSuccess && t < best) { best = t; bq = c; }
    }
    const double t_quad = best;
    DstCfg bd = p->dst;
    double bt = 1e30;
    if (d.L <= kLdsFftMax) {
        for (int T : {64, 128, 256, 512, 1024}) {
            if (d.L > 8 * T) continue;
            for (const FftSched &sc : sched_candidates((int)d.L)) {
                DstCfg c = p->dst;
                c.threads = T;
                c.sched = sc;
                hipError_t er;
                const double t = time_launch([&](hipStream_t st) { return launch_dst(c, p->phi, d.H, d.L, d.N, p->tw_pre, p->tw_pack, p->tw_fft, p->zA, p->zB, cbuf, st); }, s, 3, &er);
                if (er == hipSuccess && t < bt) { bt = t; bd = c; }
            }
        }
    } else {
        for (const FftSched &a : sched_candidates(p->dst.L1))
            for (const FftSched &b : sched_candidates(p->dst.L2)) {
                DstCfg c = p->dst;
                c.s1 = a;
                c.s2 = b;
                hipError_t er;
                const double t = time_launch([&](hipStream_t st) { return launch_dst(c, p->phi, d.H, d.L, d.N, p->tw_pre, p->tw_pack, p->tw_fft, p->zA, p->zB, cbuf, st); }, s, 3, &er);
                if (er == hipSuccess && t < bt) { bt = t; bd = c; }
            }
    }
    bool fused = false;
    if (p->fused_small) {
        hipError_t er;
        const double t = time_launch([&](hipStream_t st) { return launch_fused_small(p->fused_threads, d.prec, fsrc, p->w, p->s2, d.H, d.Q, d.N, bd.sched, p->tw_pre, p->tw_pack, p->tw_fft, cbuf, st); }, s, 3, &er);
        fused = er == hipSuccess && t < t_quad + bt;
    }
    hipFree(cbuf);
    p->quad = bq;
    p->dst = bd;
    p->fused_small = fused;
    std::string v = "quad " + quad_to_str(bq) + " dst " + std::to_string(bd.threads) + " ";
    v += d.L <= kLdsFftMax ? sched_to_str(bd.sched) : sched_to_str(bd.s1) + " " + sched_to_str(bd.s2);
    v += std::string(" fused ") + (fused ? "1" : "0");
    cache_put(key, v);
    return LC_OK;
}

}  // namespace lc
