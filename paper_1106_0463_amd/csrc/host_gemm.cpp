// Abel-as-GEMM plans: functions sampled on the fixed P-point Chebyshev-Gauss
// grid x_p = cos((2p+1) pi / (2P)).  The Abel step becomes phi = A F with the
// product-integration matrix A built in FP64 on the device (exact for f of
// degree < P: the Abel rule has Q_A = P/2 + 8 nodes); then the batched
// twist/FFT/rescale of eq. (2.4) over the functions.
//
// Precision modes: FP64 (rocBLAS DGEMM, the FP64 comparator) or split
// 16-bit pieces with FP32 accumulation on MFMA (hand-written kernel fusing
// the piece products); the DST and the (2n+1) rescale are FP64 in all modes.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cmath>
#include <cstdlib>
#include <type_traits>
#include <new>
#include <string>
#include <vector>

#include "lc_gemm.h"
#include "lc_internal.h"

namespace lc {

lc_status fail_status(lc_status s, const std::string &msg);
hipError_t timing_begin(lc_plan_s *p, hipStream_t s, int *slot);
hipError_t timing_end(lc_plan_s *p, hipStream_t s, int slot);

namespace {

struct GemmState {
    int P = 0, ldk = 0, QA = 0, mode = 0;
    int h16 = kBF16, npc = 1, kmode = 1, scaled = 0;
    int64_t N = 0, M = 0, M_eff = 0, H = 0, L = 0;
    double *xc = nullptr, *lam = nullptr, *A = nullptr;
    void *Y = nullptr;
    int *rowexp = nullptr;
    double2 *tw_pre = nullptr, *tw_pack = nullptr, *tw_fft = nullptr;
    FftSched sched{};
    int Bmax = 0;
    void *X = nullptr;
    int *colexp = nullptr;
    float *Out32 = nullptr;
    double *Out64 = nullptr;
    rocblas_handle rb = nullptr;
    int64_t ws_bytes = 0, b_bytes = 0;
    std::vector<void *> allocs;
    std::vector<void *> ballocs;  // per-B workspace
};

template <typename T>
hipError_t galloc(GemmState *g, T **p, size_t n, bool perB = false) {
    *p = nullptr;
    if (n == 0) return hipSuccess;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e == hipSuccess) {
        (perB ? g->ballocs : g->allocs).push_back(*p);
        (perB ? g->b_bytes : g->ws_bytes) += (int64_t)(n * sizeof(T));
    }
    return e;
}

void free_b(GemmState *g) {
    for (void *p : g->ballocs) hipFree(p);
    g->ballocs.clear();
    g->X = nullptr;
    g->colexp = nullptr;
    g->Out32 = nullptr;
    g->Out64 = nullptr;
    g->Bmax = 0;
}

void free_gemm(GemmState *g) {
    if (!g) return;
    free_b(g);
    for (void *p : g->allocs) hipFree(p);
    if (g->rb) rocblas_destroy_handle(g->rb);
    delete g;
}

hipError_t reserve(GemmState *g, int B) {
    free_b(g);
    g->b_bytes = 0;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    if (g->mode == LC_GEMM_FP64) {
        chk(galloc(g, &g->Out64, (size_t)B * g->H, true));
    } else {
        unsigned short *x = nullptr;
        chk(galloc(g, &x, (size_t)g->npc * B * g->ldk, true));
        g->X = x;
        if (e == hipSuccess && g->ldk != g->P) chk(hipMemset(x, 0, (size_t)g->npc * B * g->ldk * 2));
        chk(galloc(g, &g->colexp, (size_t)B, true));
        chk(galloc(g, &g->Out32, (size_t)B * g->H, true));
    }
    if (e == hipSuccess) g->Bmax = B;
    return e;
}

}  // namespace

void destroy_gemm(lc_plan_s *p) {
    free_gemm((GemmState *)p->ext);
    p->ext = nullptr;
}

void info_gemm(lc_plan_s *p, lc_plan_desc *d) {
    GemmState *g = (GemmState *)p->ext;
    d->precision = g->mode;
    d->N = g->N;
    d->M = g->M;
    d->M_eff = g->M_eff;
    d->H = g->H;
    d->Q = g->P;
    d->B = g->Bmax;
    d->samples = (int64_t)g->P * g->Bmax;
    d->sample_bytes = d->samples * 8;
    d->workspace_bytes = g->ws_bytes + g->b_bytes;
}

lc_status nodes_gemm(lc_plan_s *p, const double **x, int64_t *rows, int32_t *Q) {
    GemmState *g = (GemmState *)p->ext;
    *x = g->xc;
    if (rows) *rows = g->P;
    if (Q) *Q = 1;
    return LC_OK;
}

}  // namespace lc

using namespace lc;

extern "C" {

lc_status lc_plan_gemm(int32_t P, int64_t M, int64_t N, lc_gemm_mode mode, lc_plan_t *out) {
    if (!out) return fail_status(LC_ERR_INVALID, "lc_plan_gemm: out is null");
    if (P < 2 || P > 16384) return fail_status(LC_ERR_INVALID, "lc_plan_gemm: P must be in [2, 16384]");
    if (M < 2 || (M & 1)) return fail_status(LC_ERR_INVALID, "lc_plan_gemm: M must be even and >= 2");
    if (N < 1 || N > M / 2) return fail_status(LC_ERR_INVALID, "lc_plan_gemm: need 1 <= N <= M/2");
    if ((int)mode < LC_GEMM_FP64 || (int)mode > LC_GEMM_FP16X1)
        return fail_status(LC_ERR_INVALID, "lc_plan_gemm: bad mode");
    GemmState *g = new (std::nothrow) GemmState();
    if (!g) return fail_status(LC_ERR_NOMEM, "lc_plan_gemm: host allocation failed");
    if (const char *wm = getenv("LC_MGEMM_WM")) mgemm_wm = atoi(wm) == 2 ? 2 : 4;
    g->P = P;
    g->ldk = (P + 31) / 32 * 32;
    g->QA = P / 2 + 8;
    g->mode = (int)mode;
    switch (mode) {
        case LC_GEMM_BF16X3: g->h16 = kBF16; g->npc = 2; g->kmode = 3; g->scaled = 0; break;
        case LC_GEMM_BF16X6: g->h16 = kBF16; g->npc = 3; g->kmode = 6; g->scaled = 0; break;
        case LC_GEMM_FP16X3: g->h16 = kF16; g->npc = 2; g->kmode = 3; g->scaled = 1; break;
        case LC_GEMM_FP16X1: g->h16 = kF16; g->npc = 1; g->kmode = 1; g->scaled = 1; break;
        default: g->npc = 0; break;
    }
    g->N = N;
    g->M = M;
    lc_grid_size(M, &g->M_eff);
    g->H = g->M_eff / 2;
    g->L = g->H / 2;
    if (g->L > kLdsFftMax) {
        free_gemm(g);
        return fail_status(LC_ERR_UNSUPPORTED, "lc_plan_gemm: M/4 beyond the LDS FFT length (8192)");
    }
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    // Chebyshev-Gauss nodes and barycentric weights lam_p = (-1)^p sin((2p+1) pi / (2P))
    std::vector<double> xc(P), lam(P);
    const long double PI = 3.141592653589793238462643383279502884L;
    for (int p = 0; p < P; ++p) {
        const long double th = PI * (2.0L * p + 1.0L) / (2.0L * P);
        xc[p] = (double)cosl(th);
        lam[p] = (double)((p % 2 ? -1.0L : 1.0L) * sinl(th));
    }
    std::vector<double> t, w, s2;
    std::vector<double2> omt2, rowA, pre, pack, fft;
    gauss_half_rule(g->QA, t, w, omt2);
    row_factors(g->H, rowA, s2);
    twiddles(g->H, pre, pack, fft);
    g->sched = make_sched((int)g->L);
    double *d_w = nullptr, *d_s2 = nullptr;
    double2 *d_omt2 = nullptr, *d_rowA = nullptr;
    auto up = [&](auto **dst, const auto &v) {
        using T = typename std::decay<decltype(v[0])>::type;
        chk(galloc(g, (T **)dst, v.size()));
        if (e == hipSuccess) chk(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    };
    up(&g->xc, xc);
    up(&g->lam, lam);
    up(&d_w, w);
    up(&d_s2, s2);
    up(&d_omt2, omt2);
    up(&d_rowA, rowA);
    up(&g->tw_pre, pre);
    up(&g->tw_pack, pack);
    up(&g->tw_fft, fft);
    chk(galloc(g, &g->A, (size_t)(g->H + 1) * P));
    if (e == hipSuccess) chk(launch_amat((int)g->H, P, g->QA, g->xc, g->lam, d_rowA, d_omt2, d_w, d_s2, g->A, 0));
    if (e == hipSuccess && g->mode != LC_GEMM_FP64) {
        unsigned short *y = nullptr;
        chk(galloc(g, &y, (size_t)g->npc * g->H * g->ldk));
        g->Y = y;
        if (e == hipSuccess) chk(hipMemset(y, 0, (size_t)g->npc * g->H * g->ldk * 2));
        chk(galloc(g, &g->rowexp, (size_t)g->H));
        if (e == hipSuccess)
            chk(launch_split_rows(g->h16, g->A, (int)g->H, P, g->ldk, g->npc, g->Y, (int64_t)g->H * g->ldk,
                                  g->rowexp, g->scaled, 0));
    }
    if (e == hipSuccess && g->mode == LC_GEMM_FP64) {
        if (rocblas_create_handle(&g->rb) != rocblas_status_success) e = hipErrorUnknown;
    }
    if (e == hipSuccess) chk(hipDeviceSynchronize());
    if (e == hipSuccess) chk(reserve(g, 16384));
    if (e != hipSuccess) {
        free_gemm(g);
        return fail_status(e == hipErrorOutOfMemory ? LC_ERR_NOMEM : LC_ERR_HIP,
                           std::string("lc_plan_gemm: ") + hipGetErrorString(e));
    }
    lc_plan_s *p = new (std::nothrow) lc_plan_s();
    if (!p) {
        free_gemm(g);
        return fail_status(LC_ERR_NOMEM, "lc_plan_gemm: host allocation failed");
    }
    p->kind = LC_PLAN_GEMM;
    hipGetDevice(&p->device);
    p->ext = g;
    *out = p;
    return LC_OK;
}

lc_status lc_plan_gemm_reserve(lc_plan_t p, int32_t B_max) {
    if (!p || p->kind != LC_PLAN_GEMM) return fail_status(LC_ERR_INVALID, "lc_plan_gemm_reserve: not a GEMM plan");
    if (B_max < 1) return fail_status(LC_ERR_INVALID, "lc_plan_gemm_reserve: B_max must be >= 1");
    GemmState *g = (GemmState *)p->ext;
    hipDeviceSynchronize();
    hipError_t e = reserve(g, B_max);
    if (e != hipSuccess)
        return fail_status(e == hipErrorOutOfMemory ? LC_ERR_NOMEM : LC_ERR_HIP,
                           std::string("lc_plan_gemm_reserve: ") + hipGetErrorString(e));
    return LC_OK;
}

lc_status lc_plan_gemm_matrix(lc_plan_t p, const double **A_dev) {
    if (!p || p->kind != LC_PLAN_GEMM || !A_dev) return fail_status(LC_ERR_INVALID, "lc_plan_gemm_matrix: bad argument");
    *A_dev = ((GemmState *)p->ext)->A;
    return LC_OK;
}

lc_status lc_execute_gemm(lc_plan_t p, const double *F_dev, int32_t B, double *C_dev, hipStream_t stream) {
    if (!p || p->kind != LC_PLAN_GEMM) return fail_status(LC_ERR_INVALID, "lc_execute_gemm: not a GEMM plan");
    if (!F_dev || !C_dev) return fail_status(LC_ERR_INVALID, "lc_execute_gemm: null pointer");
    GemmState *g = (GemmState *)p->ext;
    if (B < 1 || B > g->Bmax) return fail_status(LC_ERR_INVALID, "lc_execute_gemm: B outside [1, reserved]");
    hipError_t e;
    int slot = -1;
    if (g->mode == LC_GEMM_FP64) {
        rocblas_set_stream(g->rb, stream);
        const double one = 1.0, zero = 0.0;
        if ((e = timing_begin(p, stream, &slot)) != hipSuccess) return fail_status(LC_ERR_HIP, "lc_execute_gemm: timing");
        // column-major: Out^T (H x B) = A[1:] (H x P) * F (P x B)
        rocblas_status rs = rocblas_dgemm(g->rb, rocblas_operation_transpose, rocblas_operation_transpose, (int)g->H, B,
                                          g->P, &one, g->A + g->P, g->P, F_dev, B, &zero, g->Out64, (int)g->H);
        if (rs != rocblas_status_success) return fail_status(LC_ERR_HIP, "lc_execute_gemm: rocblas_dgemm failed");
        if ((e = timing_end(p, stream, slot)) != hipSuccess) return fail_status(LC_ERR_HIP, "lc_execute_gemm: timing");
        e = launch_gdst(0, g->Out64, (int)g->H, nullptr, nullptr, B, g->H, g->L, g->N, g->tw_pre, g->tw_pack,
                        g->tw_fft, g->sched, C_dev, stream);
        if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_gemm: dst: ") + hipGetErrorString(e));
        return LC_OK;
    }
    const int64_t xps = (int64_t)g->Bmax * g->ldk;
    e = launch_split_cols(g->h16, F_dev, g->P, B, g->ldk, g->npc, g->X, xps, g->colexp, g->scaled, stream);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_gemm: split: ") + hipGetErrorString(e));
    if ((e = timing_begin(p, stream, &slot)) != hipSuccess) return fail_status(LC_ERR_HIP, "lc_execute_gemm: timing");
    e = launch_mgemm(g->h16, g->kmode, g->X, xps, g->Y, (int64_t)g->H * g->ldk, B, (int)g->H, g->ldk, g->Out32,
                     (int)g->H, stream);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_gemm: mfma: ") + hipGetErrorString(e));
    if ((e = timing_end(p, stream, slot)) != hipSuccess) return fail_status(LC_ERR_HIP, "lc_execute_gemm: timing");
    e = launch_gdst(1, g->Out32, (int)g->H, g->scaled ? g->rowexp : nullptr, g->scaled ? g->colexp : nullptr, B, g->H,
                    g->L, g->N, g->tw_pre, g->tw_pack, g->tw_fft, g->sched, C_dev, stream);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_gemm: dst: ") + hipGetErrorString(e));
    return LC_OK;
}

}  // extern "C"
