// Two-dimensional tensor-product plans:
//   c_{n1 n2} = (n1 + 1/2)(n2 + 1/2) integral integral f(x1, x2) P_n1(x1) P_n2(x2)
// by the method along x1 for every node of x2, then along x2 for every n1.
// Both axes use the S = H Q Abel nodes of one single plan (N, M, Q), whose
// weights, row factors, twiddles and FFT schedule it reuses:
//   pass 1: Abel sums over the S*H rows of F (S functions of [H][Q] samples),
//           batched DST -> c1[b][n1]               (S x N)
//   transpose -> c1T[n1][b]                        (N x S: N functions)
//   pass 2: Abel sums over the N*H rows of c1T, batched DST -> C[n1][n2].
#include <hip/hip_runtime.h>

#include <new>
#include <string>
#include <vector>

#include "lc_gemm.h"
#include "lc_internal.h"

namespace lc {

lc_status fail_status(lc_status s, const std::string &msg);
hipError_t timing_begin(lc_plan_s *p, hipStream_t s, int *slot);
hipError_t timing_end(lc_plan_s *p, hipStream_t s, int slot);
QuadCfg default_quad_cfg(int prec, int Q, int64_t rows, int num_cu);

namespace {

struct Plan2D {
    lc_plan_t p1 = nullptr;     // single plan of the 1-D node set
    int64_t S = 0;              // nodes per axis, H * Q
    double *s2rep = nullptr;    // [S * H] row factors, repeated per function
    double *phi1 = nullptr;     // [S * H]
    double *c1 = nullptr;       // [S][N]
    double *c1T = nullptr;      // [N][S]
    double *phi2 = nullptr;     // [N * H]
    QuadCfg q1{}, q2{};
    int64_t ws = 0;
    std::vector<void *> allocs;
};

void free_2d(Plan2D *t) {
    if (!t) return;
    for (void *p : t->allocs) hipFree(p);
    if (t->p1) lc_plan_destroy(t->p1);
    delete t;
}

template <typename T>
hipError_t talloc(Plan2D *t, T **p, size_t n) {
    *p = nullptr;
    hipError_t e = device_alloc((void **)p, n * sizeof(T));
    if (e == hipSuccess) {
        t->allocs.push_back(*p);
        t->ws += (int64_t)(n * sizeof(T));
    }
    return e;
}

}  // namespace

void destroy_2d(lc_plan_s *p) {
    free_2d((Plan2D *)p->ext);
    p->ext = nullptr;
}

void info_2d(lc_plan_s *p, lc_plan_desc *d) {
    const Plan2D *t = (const Plan2D *)p->ext;
    lc_plan_info(t->p1, d);
    d->kind = LC_PLAN_2D;
    d->samples = t->S * t->S;
    d->sample_bytes = d->samples * (p->fn.prec == LC_FP64 ? 8 : 4);
    d->workspace_bytes += t->ws;
}

lc_status nodes_2d(lc_plan_s *p, const double **x, int64_t *rows, int32_t *Q) {
    return lc_plan_nodes(((Plan2D *)p->ext)->p1, x, rows, Q);
}

}  // namespace lc

using namespace lc;

extern "C" {

lc_status lc_plan_2d(int64_t N, int64_t M, int32_t Q, lc_precision prec, lc_plan_t *out) {
    if (!out) return fail_status(LC_ERR_INVALID, "lc_plan_2d: out is null");
    Plan2D *t = new (std::nothrow) Plan2D();
    if (!t) return fail_status(LC_ERR_NOMEM, "lc_plan_2d: host allocation failed");
    lc_status st = lc_plan(N, M, Q, prec, &t->p1);
    if (st != LC_OK) {
        delete t;
        return st;  // the error string is lc_plan's
    }
    const FnDesc d = t->p1->fn;
    if (d.L > kLdsFftMax) {
        free_2d(t);
        return fail_status(LC_ERR_UNSUPPORTED, "lc_plan_2d: M/4 beyond the LDS FFT length (8192)");
    }
    t->S = d.H * (int64_t)Q;
    if ((double)t->S * (double)t->S > 4.0e10 || t->S > 2000000) {
        free_2d(t);
        return fail_status(LC_ERR_UNSUPPORTED, "lc_plan_2d: (H Q)^2 samples exceed the library's limit");
    }
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    const int64_t SH = t->S * d.H;
    chk(talloc(t, &t->s2rep, (size_t)SH));
    chk(talloc(t, &t->phi1, (size_t)SH));
    chk(talloc(t, &t->c1, (size_t)t->S * N));
    chk(talloc(t, &t->c1T, (size_t)t->S * N));
    chk(talloc(t, &t->phi2, (size_t)N * d.H));
    if (e == hipSuccess) chk(launch_repeat(t->p1->s2, d.H, t->S, t->s2rep, 0));
    if (e == hipSuccess) chk(hipDeviceSynchronize());
    if (e != hipSuccess) {
        free_2d(t);
        return fail_status(e == hipErrorOutOfMemory ? LC_ERR_NOMEM : LC_ERR_HIP,
                           std::string("lc_plan_2d: ") + hipGetErrorString(e));
    }
    t->q1 = default_quad_cfg((int)prec, Q, SH, device_cu_count());
    t->q2 = default_quad_cfg(LC_FP64, Q, N * d.H, device_cu_count());
    if (const char *ev = getenv("LC_2D_ROW_PAIRS"))
        if (atoi(ev)) {
            pair_quad_cfg((int)prec, Q, t->q1);
            pair_quad_cfg(LC_FP64, Q, t->q2);
        }
    lc_plan_s *p = new (std::nothrow) lc_plan_s();
    if (!p) {
        free_2d(t);
        return fail_status(LC_ERR_NOMEM, "lc_plan_2d: host allocation failed");
    }
    p->kind = LC_PLAN_2D;
    p->device = t->p1->device;
    p->fn = d;
    p->ext = t;
    *out = p;
    return LC_OK;
}

lc_status lc_execute_2d(lc_plan_t p, const void *F_dev, double *C_dev, hipStream_t s) {
    if (!p || p->kind != LC_PLAN_2D) return fail_status(LC_ERR_INVALID, "lc_execute_2d: not a 2-D plan");
    if (!F_dev || !C_dev) return fail_status(LC_ERR_INVALID, "lc_execute_2d: null pointer");
    if (((uintptr_t)F_dev) & 15) return fail_status(LC_ERR_INVALID, "lc_execute_2d: F_dev must be 16-byte aligned");
    Plan2D *t = (Plan2D *)p->ext;
    const lc_plan_s *p1 = t->p1;
    const FnDesc &d = p->fn;
    int slot = -1;
    hipError_t e = timing_begin(p, s, &slot);
    if (e == hipSuccess) e = launch_quad(t->q1, d.prec, F_dev, p1->w, t->s2rep, t->S * d.H, d.Q, t->phi1, s);
    if (e == hipSuccess) e = timing_end(p, s, slot);
    if (e == hipSuccess)
        e = launch_gdst(0, t->phi1, (int)d.H, nullptr, nullptr, (int)t->S, d.H, d.L, d.N, p1->tw_pre, p1->tw_pack,
                        p1->tw_fft, p1->dst.sched, t->c1, s);
    if (e == hipSuccess) e = launch_transpose64(t->c1, t->S, d.N, t->c1T, s);
    if (e == hipSuccess) e = launch_quad(t->q2, LC_FP64, t->c1T, p1->w, t->s2rep, d.N * d.H, d.Q, t->phi2, s);
    if (e == hipSuccess)
        e = launch_gdst(0, t->phi2, (int)d.H, nullptr, nullptr, (int)d.N, d.H, d.L, d.N, p1->tw_pre, p1->tw_pack,
                        p1->tw_fft, p1->dst.sched, C_dev, s);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_2d: ") + hipGetErrorString(e));
    return LC_OK;
}

}  // extern "C"
