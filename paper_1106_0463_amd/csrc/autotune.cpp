// Autotuner: times the launch variants of a plan's kernels on the plan's own
// buffers (the node arrays stand in for samples of the same size) and keeps
// the fastest; choices persist in a text cache (one "key<TAB>value" line per
// entry) named by the environment variable LC_AUTOTUNE_CACHE, keyed by the
// device architecture and the problem shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "lc_internal.h"

namespace lc {

lc_status fail_status(lc_status s, const std::string &msg);
lc_status tune_single(lc_plan_s *p, hipStream_t s);
lc_status tune_batch(lc_plan_s *p, hipStream_t s);
lc_status tune_adaptive(lc_plan_s *p, hipStream_t s);

static std::mutex g_cache_mu;

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

bool cache_get(const std::string &key, std::string &val) {
    const char *path = getenv("LC_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        const size_t t = line.find('\t');
        if (t != std::string::npos && line.compare(0, t, key) == 0 && t == key.size()) {
            val = line.substr(t + 1);  // the last entry wins
            found = true;
        }
    }
    return found;
}

void cache_put(const std::string &key, const std::string &val) {
    const char *path = getenv("LC_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::ofstream out(path, std::ios::app);
    out << key << '\t' << val << '\n';
}

std::string quad_to_str(const QuadCfg &c) {
    std::ostringstream o;
    o << c.vec << ' ' << c.G << ' ' << c.cpl << ' ' << c.unroll << ' ' << c.block << ' ' << c.grid << ' ' << c.rpg;
    return o.str();
}

bool quad_from_str(const std::string &s, QuadCfg &c) {
    std::istringstream i(s);
    QuadCfg t = c;
    if (!(i >> t.vec >> t.G >> t.cpl >> t.unroll >> t.block >> t.grid >> t.rpg)) return false;
    c = t;
    return true;
}

// Every supported quadrature launch shape for (precision, Q), each with
// grids of one half, one and two rounds of the blocks the device holds at
// once for that variant (occupancy API; a grid-stride launch whose grid is
// not a whole number of rounds ends on a partial round), capped by the
// useful number of blocks, and with the useful number itself (one pass per
// block: the blocks are handed out as CUs free up).
std::vector<QuadCfg> quad_candidates(int prec, int Q, int64_t rows, int cu, bool batch) {
    std::vector<QuadCfg> out;
    auto add = [&](QuadCfg c) {
        if (!quad_cfg_supported(c, prec, Q)) return;
        const int64_t rpb = quad_rows_per_block(c);
        const int64_t useful = (rows + rpb - 1) / rpb;
        int occ = batch ? bquad_blocks_per_cu(c, prec) : quad_blocks_per_cu(c, prec);
        if (occ < 1) occ = 8;
        for (int half_rounds : {1, 2, 4, 0}) {
            QuadCfg g = c;
            const int64_t want = half_rounds ? (int64_t)cu * occ * half_rounds / 2 : useful;
            g.grid = (int)std::max<int64_t>(1, std::min<int64_t>({useful, want, (int64_t)INT32_MAX}));
            bool dup = false;
            for (auto &o : out) dup |= quad_to_str(o) == quad_to_str(g);
            if (!dup) out.push_back(g);
        }
    };
    const int vfit = prec == LC_FP64 ? 2 : 4;
    for (int G : {4, 8, 16})
        for (int cpl : {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11})
            for (int u : {1, 2, 4}) {
                QuadCfg c{};
                c.vec = vfit;
                c.G = G;
                c.cpl = cpl;
                c.unroll = u;
                c.block = 256;
                c.grid = 1;
                c.Qv = Q;
                add(c);
            }
    // two rows per lane group (short rows: halves the per-row work per byte)
    for (int G : {4, 8, 16})
        for (int cpl : {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11})
            for (int u : {1, 2, 4}) {
                QuadCfg c{};
                c.vec = vfit;
                c.G = G;
                c.cpl = cpl;
                c.unroll = u;
                c.block = 256;
                c.grid = 1;
                c.Qv = Q;
                c.rpg = 2;
                add(c);
            }
    for (int G : {8, 16, 32, 64})
        for (int u : {1, 2, 4, 8}) {
            QuadCfg c{};
            c.vec = vfit;
            c.G = G;
            c.cpl = -1;
            c.unroll = u;
            c.block = 256;
            c.grid = 1;
            c.Qv = Q;
            add(c);
        }
    for (int vec : {1, 2})
        for (int G : {4, 8, 16, 32, 64}) {
            QuadCfg c{};
            c.vec = vec;
            c.G = G;
            c.cpl = 0;
            c.unroll = 1;
            c.block = 256;
            c.grid = 1;
            c.Qv = Q;
            add(c);
        }
    return out;
}

// Mean time (ms) of `reps` launches after one warm-up, with HIP events on s.
double time_launch(const std::function<hipError_t(hipStream_t)> &f, hipStream_t s, int reps, hipError_t *err) {
    hipEvent_t a, b;
    *err = hipEventCreate(&a);
    if (*err != hipSuccess) return 1e30;
    *err = hipEventCreate(&b);
    if (*err != hipSuccess) {
        hipEventDestroy(a);
        return 1e30;
    }
    double ms = 1e30;
    if ((*err = f(s)) == hipSuccess && (*err = hipEventRecord(a, s)) == hipSuccess) {
        for (int r = 0; r < reps && *err == hipSuccess; ++r) *err = f(s);
        if (*err == hipSuccess) *err = hipEventRecord(b, s);
        if (*err == hipSuccess) *err = hipEventSynchronize(b);
        float t = 0.f;
        if (*err == hipSuccess && (*err = hipEventElapsedTime(&t, a, b)) == hipSuccess) ms = t / reps;
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    return ms;
}

// Radix orders tried for an FFT of length L: largest radices first, the
// reverse, and radix-4 passes in place of radix-8 ones.
std::vector<FftSched> sched_candidates(int L) {
    std::vector<FftSched> out;
    FftSched d = make_sched(L);
    out.push_back(d);
    FftSched r = d;
    for (int i = 0; i < d.npass; ++i) r.radix[i] = d.radix[d.npass - 1 - i];
    out.push_back(r);
    int n = L, c2 = 0, c3 = 0, c5 = 0;
    while (n % 5 == 0) { n /= 5; ++c5; }
    while (n % 3 == 0) { n /= 3; ++c3; }
    while (n % 2 == 0) { n /= 2; ++c2; }
    std::vector<int> v;
    for (int i = 0; i + 1 < c2; i += 2) v.push_back(4);
    if (c2 % 2) v.push_back(2);
    for (int i = 0; i < c5; ++i) v.push_back(5);
    for (int i = 0; i < c3; ++i) v.push_back(3);
    v.push_back(0);
    out.push_back(make_sched(L, v.data()));
    return out;
}

}  // namespace lc

extern "C" lc_status lc_autotune(lc_plan_t p, hipStream_t stream) {
    if (!p) return lc::fail_status(LC_ERR_INVALID, "lc_autotune: plan is null");
    if (p->kind == LC_PLAN_SINGLE) return lc::tune_single(p, stream);
    if (p->kind == LC_PLAN_BATCH) return lc::tune_batch(p, stream);
    if (p->kind == LC_PLAN_ADAPTIVE) return lc::tune_adaptive(p, stream);
    return LC_OK;  // GEMM plans have a single launch shape
}
