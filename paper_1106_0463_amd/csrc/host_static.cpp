// lc_execute_noalloc: the execute call of single-function plans (uniform and
// composite Abel rule) with its workspace -- the Abel integrals phi[H] and,
// for FFTs longer than the LDS holds, the two four-step buffers -- taken from
// one static device array of the library instead of the plan's own buffers.
// It runs the same kernels as lc_execute, in the same order, so the results
// are bit-for-bit those of lc_execute.
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy, from the first call on that device until the
// process ends.  Its device address is looked up once per device (with that
// device current) and kept in a per-device table; kernels get that address,
// never the variable's host-side name.
#include <mutex>

#include "lc_internal.h"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[LC_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's copy of scratch (looked up on the first
// call with dev current).
hipError_t scratch_ptr(int dev, unsigned char **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[dev] = ptr;
    }
    *out = (unsigned char *)g_scratch[dev];
    return hipSuccess;
}

int64_t round256(int64_t b) { return (b + 255) & ~int64_t(255); }

}  // namespace

namespace lc {
hipError_t adaptive_reduce(const lc_plan_s *p, const void *f, double *phi, hipStream_t s);
}

extern "C" {

lc_status lc_execute_noalloc(lc_plan_t p, const void *f_dev, double *c_dev, hipStream_t stream) {
    using namespace lc;
    if (!p) { set_error("lc_execute_noalloc: plan is null"); return LC_ERR_INVALID; }
    if (p->kind != LC_PLAN_SINGLE && p->kind != LC_PLAN_ADAPTIVE) {
        set_error("lc_execute_noalloc: not a single-function plan");
        return LC_ERR_INVALID;
    }
    if (!f_dev || !c_dev) { set_error("lc_execute_noalloc: null f_dev or c_dev"); return LC_ERR_INVALID; }
    if (((uintptr_t)f_dev) & 15) {
        set_error("lc_execute_noalloc: f_dev must be 16-byte aligned");
        return LC_ERR_INVALID;
    }
    const FnDesc &d = p->fn;
    const bool four_step = d.L > kLdsFftMax;
    const int64_t need = round256(d.H * (int64_t)sizeof(double)) +
                         (four_step ? 2 * round256(d.L * (int64_t)sizeof(double2)) : 0);
    if (need > (int64_t)LC_NOALLOC_SCRATCH_BYTES) {
        set_error("lc_execute_noalloc: the plan needs " + std::to_string(need) +
                  " bytes of workspace (H = " + std::to_string(d.H) + "); the static scratch holds " +
                  std::to_string((long long)LC_NOALLOC_SCRATCH_BYTES) + " bytes");
        return LC_ERR_INVALID;
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_error("lc_execute_noalloc: hipGetDevice failed"); return LC_ERR_HIP; }
    if (dev != p->device) {
        set_error("lc_execute_noalloc: the current device is not the plan's device");
        return LC_ERR_INVALID;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("lc_execute_noalloc: device ordinal beyond the library's table");
        return LC_ERR_UNSUPPORTED;
    }
    unsigned char *base = nullptr;
    if ((e = scratch_ptr(dev, &base)) != hipSuccess) {
        set_error(std::string("lc_execute_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        return LC_ERR_HIP;
    }
    // workspace carved from the array: phi, then zA and zB (four-step only),
    // each 256-byte aligned.  Every element is written before it is read, so
    // nothing needs clearing between calls.
    double *phi = (double *)base;
    double2 *zA = nullptr, *zB = nullptr;
    if (four_step) {
        zA = (double2 *)(base + round256(d.H * (int64_t)sizeof(double)));
        zB = (double2 *)((unsigned char *)zA + round256(d.L * (int64_t)sizeof(double2)));
    }
    if (p->kind == LC_PLAN_SINGLE && p->fused_small) {
        e = launch_fused_small(p->fused_threads, d.prec, f_dev, p->w, p->s2, d.H, d.Q, d.N, p->dst.sched,
                               p->tw_pre, p->tw_pack, p->tw_fft, c_dev, stream);
        if (e != hipSuccess) {
            set_error(std::string("lc_execute_noalloc: fused kernel launch: ") + hipGetErrorString(e));
            return LC_ERR_HIP;
        }
        return LC_OK;
    }
    if (p->kind == LC_PLAN_ADAPTIVE)
        e = adaptive_reduce(p, f_dev, phi, stream);
    else
        e = launch_quad(p->quad, d.prec, f_dev, p->w, p->s2, d.H, d.Q, phi, stream);
    if (e != hipSuccess) {
        set_error(std::string("lc_execute_noalloc: quadrature kernel launch: ") + hipGetErrorString(e));
        return LC_ERR_HIP;
    }
    e = launch_dst(p->dst, phi, d.H, d.L, d.N, p->tw_pre, p->tw_pack, p->tw_fft, zA, zB, c_dev, stream);
    if (e != hipSuccess) {
        set_error(std::string("lc_execute_noalloc: FFT kernel launch: ") + hipGetErrorString(e));
        return LC_ERR_HIP;
    }
    return LC_OK;
}

}  // extern "C"
