// Abel-as-GEMM plans: functions sampled on the fixed P-point Chebyshev-Gauss
// grid x_p = cos((2p+1) pi / (2P)).  The Abel step becomes phi = A F with the
// product-integration matrix A built in FP64 on the device (exact for f of
// degree < P: the Abel rule has Q_A = P/2 + 8 nodes); then the batched
// twist/FFT/rescale of eq. (2.4) over the functions.
//
// Precision modes: FP64 (rocBLAS DGEMM, the FP64 comparator) or split
// 16-bit pieces with FP32 accumulation on MFMA (hand-written kernel fusing
// the piece products); the DST and the (2n+1) rescale are FP64 in all modes.
//
// Direct Legendre-matrix plans fold the twist/DST/rescale into the matrix:
// Lmat = D A (N x P), D the map phi -> c of eq. (2.4) on the M-grid, built
// once in FP64 by running the batched FP64 DST over the columns of A.  An
// execute is then the single product C = F^T Lmat^T with finished FP64
// coefficients written by the product's epilogue.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cmath>
#include <cstdio>
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
    int P = 0, Kp = 0, QA = 0, mode = 0;
    int direct = 0;  // direct Legendre-matrix form
    int64_t R = 0;   // rows of the Y operand: H (Abel form) or N (direct)
    double *LT = nullptr;  // direct form: Lmat^T [P][N] FP64
    int64_t Hpad = 0, Bpad = 0;  // operand rows padded to the MFMA block tile
    int h16 = kBF16, npc = 1, kmode = 1, scaled = 0;
    int ks = 0, ns = 0, kch = 0;  // MFMA product shape (0: per-mode defaults)
    int wr = 2;                   // rows of waves per product block (2: 128 functions, 4: 256)
    bool t64 = false;             // Abel form: FP64 second-level totals (grids above 4096)
    int64_t N = 0, M = 0, M_eff = 0, H = 0, L = 0;
    double *xc = nullptr, *lam = nullptr, *A = nullptr;
    double *Ap = nullptr;  // Abel form: A with the DST pack applied to its rows ([H][P])
    void *Y = nullptr;
    int *rowexp = nullptr;
    double2 *tw_pre = nullptr, *tw_pack = nullptr, *tw_fft = nullptr;
    FftSched sched{};
    int Bmax = 0;
    void *X = nullptr;
    int *colexp = nullptr;
    int *cexp = nullptr;              // FP16: chunk exponents [nch][Bpad]
    unsigned char *cscale = nullptr;  // FP16: chunk factors [Bpad/128][nchp][128]
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
    hipError_t e = device_alloc((void **)p, n * sizeof(T));
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
    g->cexp = nullptr;
    g->cscale = nullptr;
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
        if (!g->direct) chk(galloc(g, &g->Out64, (size_t)B * g->H, true));
    } else {
        // the split writes every padded row and k of the pieces it uses
        unsigned short *x = nullptr;
        const int bm = 64 * g->wr;  // rows of the product's block tile
        g->Bpad = ((int64_t)B + bm - 1) / bm * bm;
        chk(galloc(g, &x, (size_t)g->npc * g->Bpad * g->Kp, true));
        g->X = x;
        chk(galloc(g, &g->colexp, (size_t)B, true));
        if (g->scaled && !g->direct) {  // the Abel form's chunk exponents
            const int nchp = mgemm_scale_chunks(g->Kp);
            chk(galloc(g, &g->cexp, (size_t)(g->Kp / 16 + kExpChunk16 - 1) / kExpChunk16 * g->Bpad, true));
            chk(galloc(g, &g->cscale, (size_t)nchp * g->Bpad, true));
        }
        if (!g->direct) chk(galloc(g, &g->Out32, (size_t)B * g->H, true));
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
    if (g->direct) d->kind = LC_PLAN_LEGENDRE_MATRIX;
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

namespace {

lc_status plan_gemm_common(int32_t P, int64_t M, int64_t N, lc_gemm_mode mode, int direct, lc_plan_t *out,
                           const char *fn) {
    const std::string who = std::string(fn) + ": ";
    if (!out) return fail_status(LC_ERR_INVALID, who + "out is null");
    if (P < 2 || P > 16384) return fail_status(LC_ERR_INVALID, who + "P must be in [2, 16384]");
    if (M < 2 || (M & 1)) return fail_status(LC_ERR_INVALID, who + "M must be even and >= 2");
    if (N < 1 || N > M / 2) return fail_status(LC_ERR_INVALID, who + "need 1 <= N <= M/2");
    if ((int)mode < LC_GEMM_FP64 || (int)mode > LC_GEMM_FP16X1) return fail_status(LC_ERR_INVALID, who + "bad mode");
    GemmState *g = new (std::nothrow) GemmState();
    if (!g) return fail_status(LC_ERR_NOMEM, who + "host allocation failed");
    g->direct = direct;
    // tuning overrides, fixed for the plan's lifetime
    if (const char *kc = getenv("LC_MGEMM_KCH")) g->kch = atoi(kc);
    int rows = 256;
    if (const char *br = getenv("LC_MGEMM_BLOCK_ROWS")) rows = atoi(br);
    if (rows != 128 && rows != 256) {
        free_gemm(g);
        return fail_status(LC_ERR_INVALID, who + "LC_MGEMM_BLOCK_ROWS must be 128 or 256");
    }
    if (const char *st = getenv("LC_MGEMM_STAGES")) {
        if (sscanf(st, "%d,%d", &g->ks, &g->ns) != 2) g->ks = g->ns = -1;
    }
    g->P = P;
    g->Kp = (P + 31) / 32 * 32;
    g->QA = P / 2 + 8;
    g->mode = (int)mode;
    switch (mode) {
        case LC_GEMM_BF16X3: g->h16 = kBF16; g->npc = 2; g->kmode = 3; g->scaled = 0; break;
        case LC_GEMM_BF16X6: g->h16 = kBF16; g->npc = 3; g->kmode = 6; g->scaled = 0; break;
        case LC_GEMM_FP16X3: g->h16 = kF16; g->npc = 2; g->kmode = 3; g->scaled = 1; break;
        case LC_GEMM_FP16X1: g->h16 = kF16; g->npc = 1; g->kmode = 1; g->scaled = 1; break;
        default: g->npc = 0; break;
    }
    // product block of 256 functions (8 waves) for the three-product modes
    // at the default stage shape, 2-3% faster there than 128 (one ring stage
    // feeds twice the products); 128 (4 waves) for the others
    g->wr = rows == 256 && g->kmode == 3 && g->ks <= 0 && !g->kch ? 4 : 2;
    // FP64 second-level totals for the Abel form's three- and six-product
    // modes where K exceeds 4096: the FP32 totals round once per fold, and
    // at P = 16384 that took bf16x6 to E_a 1.16e-7 and fp16x3 to 6.4e-8
    // (8.4e-9 and 9.2e-9 with FP64 totals); at P = 4096 they cost 0-3% and
    // E_a is 0.9-1.8e-8 either way.  LC_MGEMM_T64=0/1 overrides the choice.
    {
        bool t64 = g->Kp > 4096;
        if (const char *t = getenv("LC_MGEMM_T64")) t64 = atoi(t) != 0;
        g->t64 = t64 && !direct && (g->kmode == 3 || g->kmode == 6) && g->ks <= 0 && !g->kch;
    }
    if (g->kmode && g->npc && !mgemm_shape_supported(g->kmode, g->ks, g->ns, g->kch, direct != 0)) {
        free_gemm(g);
        return fail_status(LC_ERR_INVALID, who + "LC_MGEMM_STAGES / LC_MGEMM_KCH name no built product kernel");
    }
    g->N = N;
    g->M = M;
    lc_grid_size(M, &g->M_eff);
    g->H = g->M_eff / 2;
    g->L = g->H / 2;
    if (g->L > kLdsFftMax) {
        free_gemm(g);
        return fail_status(LC_ERR_UNSUPPORTED, who + "M/4 beyond the LDS FFT length (8192)");
    }
    g->R = direct ? N : g->H;
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
    if (e == hipSuccess && !direct) {
        chk(galloc(g, &g->Ap, (size_t)g->H * P));
        if (e == hipSuccess) chk(launch_apack(g->A, P, g->H, g->L, g->tw_pre, g->tw_pack, g->Ap, 0));
    }
    if (e == hipSuccess && direct) {
        // Lmat^T [P][N]: the FP64 twist/DST/rescale of every column of A
        double *AT = nullptr;
        chk(device_alloc((void **)&AT, (size_t)P * g->H * sizeof(double)));
        chk(galloc(g, &g->LT, (size_t)P * N));
        if (e == hipSuccess) chk(launch_transpose_a(g->A, (int)g->H, P, AT, 0));
        if (e == hipSuccess)
            chk(launch_gdst(0, AT, (int)g->H, nullptr, nullptr, P, g->H, g->L, N, g->tw_pre, g->tw_pack, g->tw_fft,
                            g->sched, g->LT, 0));
        if (AT) {
            hipError_t s2e = hipDeviceSynchronize();
            if (e == hipSuccess) e = s2e;
            hipFree(AT);
        }
    }
    if (e == hipSuccess && g->mode != LC_GEMM_FP64) {
        unsigned short *y = nullptr;
        g->Hpad = (g->R + 127) / 128 * 128;
        chk(galloc(g, &y, (size_t)g->npc * g->Hpad * g->Kp));
        g->Y = y;
        chk(galloc(g, &g->rowexp, (size_t)g->R));
        if (e == hipSuccess) {
            if (direct)  // rows n of Lmat = columns of Lmat^T
                chk(launch_split_rows(g->h16, g->LT, 0, 1, N, (int)N, P, g->Kp, (int)g->Hpad, g->npc, g->Y,
                                      g->Hpad * g->Kp, g->rowexp, g->scaled, 0));
            else  // rows of Ap (A with the DST pack applied)
                chk(launch_split_rows(g->h16, g->Ap, 0, P, 1, (int)g->H, P, g->Kp, (int)g->Hpad, g->npc, g->Y,
                                      g->Hpad * g->Kp, g->rowexp, g->scaled, 0));
        }
    }
    if (e == hipSuccess && g->mode == LC_GEMM_FP64) {
        if (rocblas_create_handle(&g->rb) != rocblas_status_success) e = hipErrorUnknown;
    }
    if (e == hipSuccess) chk(hipDeviceSynchronize());
    if (e == hipSuccess) chk(reserve(g, 16384));
    if (e != hipSuccess) {
        free_gemm(g);
        return fail_status(e == hipErrorOutOfMemory ? LC_ERR_NOMEM : LC_ERR_HIP, who + hipGetErrorString(e));
    }
    lc_plan_s *p = new (std::nothrow) lc_plan_s();
    if (!p) {
        free_gemm(g);
        return fail_status(LC_ERR_NOMEM, who + "host allocation failed");
    }
    p->kind = LC_PLAN_GEMM;
    hipGetDevice(&p->device);
    p->ext = g;
    log_line("%sP=%d M_eff=%lld H=%lld N=%lld mode=%d (%d pieces, %d products) rows=%lld padded=%lld "
             "stages=%s chunk=%s block=%d totals=%s", who.c_str(), P, (long long)g->M_eff, (long long)g->H,
             (long long)N, g->mode, g->npc, g->kmode, (long long)g->R, (long long)g->Hpad,
             g->ks ? (std::to_string(g->ks) + "," + std::to_string(g->ns)).c_str() : "default",
             g->kch ? std::to_string(g->kch).c_str() : "default", 64 * g->wr,
             g->direct || g->t64 ? "fp64" : "fp32");
    *out = p;
    return LC_OK;
}

}  // namespace

extern "C" {

lc_status lc_plan_gemm(int32_t P, int64_t M, int64_t N, lc_gemm_mode mode, lc_plan_t *out) {
    return plan_gemm_common(P, M, N, mode, 0, out, "lc_plan_gemm");
}

lc_status lc_plan_legendre_matrix(int32_t P, int64_t M, int64_t N, lc_gemm_mode mode, lc_plan_t *out) {
    return plan_gemm_common(P, M, N, mode, 1, out, "lc_plan_legendre_matrix");
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
    const GemmState *g = (const GemmState *)p->ext;
    *A_dev = g->direct ? g->LT : g->A;
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
        rocblas_status rs;
        if (g->direct)  // column-major: C^T (N x B) = Lmat (N x P, stored as Lmat^T [P][N]) * F (P x B)
            rs = rocblas_dgemm(g->rb, rocblas_operation_none, rocblas_operation_transpose, (int)g->N, B, g->P, &one,
                               g->LT, (int)g->N, F_dev, B, &zero, C_dev, (int)g->N);
        else  // column-major: Out^T (H x B) = Ap (H x P) * F (P x B)
            rs = rocblas_dgemm(g->rb, rocblas_operation_transpose, rocblas_operation_transpose, (int)g->H, B, g->P,
                               &one, g->Ap, g->P, F_dev, B, &zero, g->Out64, (int)g->H);
        if (rs != rocblas_status_success) return fail_status(LC_ERR_HIP, "lc_execute_gemm: rocblas_dgemm failed");
        if ((e = timing_end(p, stream, slot)) != hipSuccess) return fail_status(LC_ERR_HIP, "lc_execute_gemm: timing");
        if (g->direct) return LC_OK;
        e = launch_gdst_z(0, g->Out64, (int)g->H, nullptr, nullptr, B, g->H, g->L, g->N, g->tw_fft, g->sched, C_dev,
                          stream);
        if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_gemm: dst: ") + hipGetErrorString(e));
        return LC_OK;
    }
    const int64_t xps = g->Bpad * g->Kp;
    // the Abel form's FP16 split takes chunk exponents (cscale), the direct
    // form's one exponent per function (cscale null)
    e = launch_split_cols(g->h16, F_dev, g->P, B, g->Kp, g->npc, g->X, xps, g->Bpad, g->cexp, g->colexp,
                          g->direct ? nullptr : g->cscale, stream, 64 * g->wr);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_gemm: split: ") + hipGetErrorString(e));
    if ((e = timing_begin(p, stream, &slot)) != hipSuccess) return fail_status(LC_ERR_HIP, "lc_execute_gemm: timing");
    if (g->direct)
        e = launch_mgemm(g->h16, g->kmode, g->X, xps, g->Y, g->Hpad * g->Kp, B, (int)g->N, g->Kp, nullptr, (int)g->N,
                         C_dev, g->scaled ? g->rowexp : nullptr, g->scaled ? g->colexp : nullptr, nullptr, g->ks,
                         g->ns, g->kch, stream, g->wr);
    else
        e = launch_mgemm(g->h16, g->kmode, g->X, xps, g->Y, g->Hpad * g->Kp, B, (int)g->H, g->Kp, g->Out32,
                         (int)g->H, nullptr, nullptr, nullptr, g->cscale, g->ks, g->ns, g->kch, stream, g->wr,
                         g->t64);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_gemm: mfma: ") + hipGetErrorString(e));
    if ((e = timing_end(p, stream, slot)) != hipSuccess) return fail_status(LC_ERR_HIP, "lc_execute_gemm: timing");
    if (g->direct) return LC_OK;
    e = launch_gdst_z(1, g->Out32, (int)g->H, g->scaled ? g->rowexp : nullptr, g->scaled ? g->colexp : nullptr, B,
                      g->H, g->L, g->N, g->tw_fft, g->sched, C_dev, stream);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_gemm: dst: ") + hipGetErrorString(e));
    return LC_OK;
}

}  // extern "C"
