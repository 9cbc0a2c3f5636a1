// Adaptive single-function plans: the composite Abel rule of lc_abel_rule
// (breakpoints, grading toward x = 1, per-row node counts) on the M-point
// grid, then the twist / FFT / rescale of eq. (2.4) as in a single plan.
//
// Host planning follows the rule's specification in long double: per row
// the cut distances e = 1 - t (breakpoint b: r / (1 + sqrt(1 - r)) with
// r = (1 - b) / (2 s^2); grading: sigma^k), the panels between them, and for
// every panel a segment {offset, node count, rule, scale, E, h} with
// 1 - t_i = E + h d_i.  Distinct (q, kind) Gauss rules are built once
// (long double Newton) into a padded weight table and a double-double node
// table.  Rows are grouped by the lanes per row G that their length fills,
// one reduction launch per group, longest rows first.  Rows of at most
// kAflatMaxSeg panels take the flattened reduction (one run of chunks per
// row), rows with more panels the panel-by-panel one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "lc_internal.h"

namespace lc {

lc_status fail_status(lc_status s, const std::string &msg);
std::string arch_name();
bool cache_get(const std::string &key, std::string &val);
void cache_put(const std::string &key, const std::string &val);
double time_launch(const std::function<hipError_t(hipStream_t)> &f, hipStream_t s, int reps, hipError_t *err);
hipError_t timing_begin(lc_plan_s *p, hipStream_t s, int *slot);
hipError_t timing_end(lc_plan_s *p, hipStream_t s, int slot);

namespace {

constexpr int kNG = 5;  // lane groups G = 4, 8, 16, 32, 64

struct AdaptiveState {
    int64_t nnz = 0, nseg = 0;
    int qmax = 0;
    int gcap = 3;                // largest lane group used (G = 4 << gcap)
    int prec = LC_FP64;
    int gmul = 0;                // grid = resident blocks * gmul / 2 (0: one row per group)
    std::vector<int64_t> rlen;   // chunks per row (host), for regrouping
    std::vector<ARow> rdesc;     // flattened-row descriptors by row (host)
    ASeg *segs = nullptr;
    ATab *tab = nullptr;
    int32_t *rseg = nullptr;
    double *wtab = nullptr;
    double2 *dtab = nullptr;
    // rows of more than kAflatMaxSeg panels: panel-by-panel reduction
    int32_t *rows[kNG] = {};
    int64_t nrows[kNG] = {};
    int grid[kNG] = {};
    // the other rows: flattened reduction
    ARow *frows[kNG] = {};
    int64_t nfrows[kNG] = {};
    int fgrid[kNG] = {};
    AflatLaunch fl = {};
    std::vector<void *> allocs;
};

void free_adaptive(AdaptiveState *a) {
    if (!a) return;
    for (void *p : a->allocs) hipFree(p);
    delete a;
}

template <typename T>
hipError_t aalloc(AdaptiveState *a, T **p, size_t n, int64_t *ws) {
    *p = nullptr;
    if (n == 0) return hipSuccess;
    hipError_t e = device_alloc((void **)p, n * sizeof(T));
    if (e == hipSuccess) {
        a->allocs.push_back(*p);
        *ws += (int64_t)(n * sizeof(T));
    }
    return e;
}

int ladder(long long n) {
    if (n <= 128) return (int)(8 * ((n + 7) / 8));
    int bl = 0;
    for (long long v = n; v; v >>= 1) ++bl;
    const long long step = 1LL << (bl - 1 - 4);
    return (int)(step * ((n + step - 1) / step));
}

// node count of the panel [t_lo, t_hi] of a row with s = sin(y/2): the band
// count D s^2 / 2 of a whole row, shared in proportion to t^2 (the phase of
// cos(D (1 - 2 s^2 (1 - t^2))) over the panel), plus the pad
int panel_q(long double s, long double t_lo, long double t_hi, const lc_abel_rule &r) {
    if (!(r.band > 0)) return r.q;
    long double g = (long double)r.band * s * s / 2 * (t_hi * t_hi - t_lo * t_lo);
    g += 6.5L * cbrtl(g);
    const long long n = (long long)r.q + (long long)ceill(g);
    return (int)std::min<long long>(r.q_max, ladder(n));
}

// cut distances e = 1 - t in (0, 1), decreasing
void row_cuts(long double s, const lc_abel_rule &r, std::vector<long double> &out) {
    std::vector<long double> es;
    const long double c = 1 - 2 * s * s;
    for (int i = 0; i < r.nbreak; ++i) {
        const long double b = r.breaks[i];
        if (c < b && b < 1) {
            const long double rr = (1 - b) / (2 * s * s);
            es.push_back(rr / (1 + sqrtl(1 - rr)));
        }
    }
    if (r.grade_ratio > 0)
        for (int k = 1; k <= r.grade_levels; ++k) es.push_back(powl((long double)r.grade_ratio, (long double)k));
    std::sort(es.begin(), es.end(), [](long double a, long double b) { return a > b; });
    out.clear();
    for (long double e : es) {
        if (!(e > 1e-15L && e < 1 - 1e-7L)) continue;  // t <= 1e-7: a breakpoint at the row's end point
        if (!out.empty() && out.back() - e < 1e-12L * out.front()) continue;
        out.push_back(e);
    }
}

// Lane groups: G = the largest power of two <= a quarter of the row's chunks
// (4 .. 4 << gcap; lanes past a short panel's end idle through it); within a
// group the longest rows go first, so that a launch does not end on a few
// long rows.
void group_rows(const std::vector<int64_t> &rlen, int gcap, std::vector<int32_t> *grows) {
    for (int gi = 0; gi < kNG; ++gi) grows[gi].clear();
    for (size_t rr = 0; rr < rlen.size(); ++rr) {
        int gi = 0;
        while (gi + 1 <= gcap && (int64_t)(4 << (gi + 1)) * 4 <= rlen[rr]) ++gi;
        grows[gi].push_back((int32_t)rr);
    }
    for (int gi = 0; gi < kNG; ++gi)
        std::stable_sort(grows[gi].begin(), grows[gi].end(),
                         [&](int32_t a, int32_t b) { return rlen[a] > rlen[b]; });
}

// uploads the row lists of grows into a's (preallocated, H entries in all)
// group arrays, rows of up to kAflatMaxSeg panels as flattened-row
// descriptors and the others as row indices, and sets the launch grids: the
// blocks one round of the device holds (occupancy) times gmul / 2, so that a
// grid-stride launch ends without a partial round of blocks, or (gmul = 0)
// one row per group, the blocks then taken longest rows first as CUs free
// up.  A grid-stride launch gives group g the rows at positions g + k ngrp;
// the longest-first list is laid out in serpentine order (every other round
// reversed), so that no group collects the longest row of every round.
template <typename T>
void serpentine(std::vector<T> &v, int64_t ngrp) {
    const int64_t n = (int64_t)v.size();
    for (int64_t k0 = ngrp; k0 < n; k0 += 2 * ngrp) std::reverse(v.begin() + k0, v.begin() + std::min(n, k0 + ngrp));
}

hipError_t set_groups(AdaptiveState *a, const std::vector<int32_t> *grows) {
    int64_t off = 0, foff = 0;
    auto grid_of = [&](int64_t n, int gi, int per_cu) {
        const int64_t per_block = 256 / (4 << gi);
        const int64_t need = std::max<int64_t>(1, (n + per_block - 1) / per_block);
        if (a->gmul == 0) return (int)std::min<int64_t>(need, INT32_MAX);
        const int64_t resident = (int64_t)device_cu_count() * per_cu;
        return (int)std::min<int64_t>(need, std::max<int64_t>(1, resident * a->gmul / 2));
    };
    for (int gi = 0; gi < kNG; ++gi) {
        std::vector<int32_t> slow;
        std::vector<ARow> fast;
        for (int32_t r : grows[gi]) {
            if (a->rdesc[r].S <= kAflatMaxSeg) fast.push_back(a->rdesc[r]);
            else slow.push_back(r);
        }
        a->rows[gi] = a->rows[0] + off;
        a->nrows[gi] = (int64_t)slow.size();
        a->frows[gi] = a->frows[0] + foff;
        a->nfrows[gi] = (int64_t)fast.size();
        a->grid[gi] = grid_of(a->nrows[gi], gi, aquad_blocks_per_cu(a->prec, 4 << gi));
        a->fgrid[gi] = a->nfrows[gi] ? grid_of(a->nfrows[gi], gi, aflat_blocks_per_cu(a->prec)) : 0;
        serpentine(slow, (int64_t)a->grid[gi] * (256 / (4 << gi)));
        serpentine(fast, (int64_t)a->fgrid[gi] * (256 / (4 << gi)));
        if (!slow.empty()) {
            hipError_t e = hipMemcpy(a->rows[gi], slow.data(), slow.size() * sizeof(int32_t), hipMemcpyHostToDevice);
            if (e != hipSuccess) return e;
        }
        if (!fast.empty()) {
            hipError_t e = hipMemcpy(a->frows[gi], fast.data(), fast.size() * sizeof(ARow), hipMemcpyHostToDevice);
            if (e != hipSuccess) return e;
        }
        off += a->nrows[gi];
        foff += a->nfrows[gi];
    }
    // one flattened launch, the longest rows' blocks first
    int b = 0;
    for (int j = 0; j < kAflatLanes; ++j) {
        const int gi = kNG - 1 - j;  // G = 64 >> j
        a->fl.rows[j] = a->frows[gi];
        a->fl.nrows[j] = a->nfrows[gi];
        a->fl.b0[j] = b;
        b += a->fgrid[gi];
    }
    a->fl.b0[kAflatLanes] = b;
    return hipSuccess;
}

// every reduction launch of the plan: flattened rows, then the others
hipError_t launch_reductions(const AdaptiveState *a, int prec, const void *f, const double *s2, double *phi,
                             hipStream_t s) {
    hipError_t e = launch_aflat(prec, a->fl, f, a->tab, a->wtab, s2, phi, s);
    for (int gi = 0; gi < kNG && e == hipSuccess; ++gi)
        e = launch_aquad(prec, 4 << gi, a->grid[gi], f, a->segs, a->rseg, a->rows[gi], a->nrows[gi], a->wtab, s2,
                         phi, s);
    return e;
}

lc_status check_rule(const lc_abel_rule *r) {
    if (!r) return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: rule is null");
    if (r->q < 1 || r->q > 65536) return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: q must be in [1, 65536]");
    if (!(r->band >= 0) || !std::isfinite(r->band))
        return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: band must be finite and >= 0");
    if (r->band > 0 && (r->q_max < r->q || r->q_max > 65536))
        return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: need q <= q_max <= 65536 when band > 0");
    if (r->nbreak < 0 || r->nbreak > 64 || (r->nbreak > 0 && !r->breaks))
        return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: nbreak must be in [0, 64] with a breaks array");
    for (int i = 0; i < r->nbreak; ++i)
        if (!(r->breaks[i] > -1.0 && r->breaks[i] < 1.0))
            return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: breakpoints must lie in (-1, 1)");
    if (!(r->grade_ratio >= 0 && r->grade_ratio < 1) || r->grade_levels < 0 || r->grade_levels > 64)
        return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: grade_ratio in [0, 1), grade_levels in [0, 64]");
    const bool cuts = r->nbreak > 0 || (r->grade_ratio > 0 && r->grade_levels > 0);
    const int qcap = r->band > 0 ? r->q_max : r->q;
    if (cuts && (qcap % 2))
        return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: q (or q_max) must be even when the rule has cuts");
    return LC_OK;
}

}  // namespace

// The adaptive state owns every device buffer of the plan, including those
// kept in the shared plan fields: detach them so the single-plan free skips
// them.
void detach_shared(lc_plan_s *p) {
    p->x = nullptr;
    p->rowA = nullptr;
    p->s2 = nullptr;
    p->tw_pre = nullptr;
    p->tw_pack = nullptr;
    p->tw_fft = nullptr;
    p->phi = nullptr;
    p->zA = nullptr;
    p->zB = nullptr;
}

void destroy_adaptive(lc_plan_s *p) {
    free_adaptive((AdaptiveState *)p->ext);
    p->ext = nullptr;
    detach_shared(p);
}

void info_adaptive(lc_plan_s *p, lc_plan_desc *d) {
    const AdaptiveState *a = (const AdaptiveState *)p->ext;
    d->precision = p->fn.prec;
    d->N = p->fn.N;
    d->M = p->fn.M;
    d->M_eff = p->fn.M_eff;
    d->H = p->fn.H;
    d->Q = a->qmax;
    d->samples = a->nnz;
    d->sample_bytes = a->nnz * (p->fn.prec == LC_FP64 ? 8 : 4);
    d->workspace_bytes = p->workspace_bytes;
}

lc_status nodes_adaptive(lc_plan_s *p, const double **x, int64_t *rows, int32_t *Q) {
    *x = p->x;
    if (rows) *rows = ((AdaptiveState *)p->ext)->nnz;
    if (Q) *Q = 1;
    return LC_OK;
}

// 1 - x of every node of the plan into comp (the node array's layout).
hipError_t adaptive_complement(const lc_plan_s *p, double *comp, hipStream_t s) {
    const AdaptiveState *a = (const AdaptiveState *)p->ext;
    return launch_anodes(a->segs, a->nseg, a->dtab, p->rowA, comp, s, true);
}

// The plan's reduction launches writing phi[H] to the given buffer.
hipError_t adaptive_reduce(const lc_plan_s *p, const void *f, double *phi, hipStream_t s) {
    return launch_reductions((const AdaptiveState *)p->ext, p->fn.prec, f, p->s2, phi, s);
}

lc_status execute_adaptive(lc_plan_s *p, const void *f, double *c, hipStream_t s) {
    const AdaptiveState *a = (const AdaptiveState *)p->ext;
    const FnDesc &d = p->fn;
    int slot = -1;
    hipError_t e = timing_begin(p, s, &slot);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, "lc_execute: timing event");
    e = launch_reductions(a, d.prec, f, p->s2, p->phi, s);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute: quadrature: ") + hipGetErrorString(e));
    e = timing_end(p, s, slot);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, "lc_execute: timing event");
    e = launch_dst(p->dst, p->phi, d.H, d.L, d.N, p->tw_pre, p->tw_pack, p->tw_fft, p->zA, p->zB, c, s);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute: FFT: ") + hipGetErrorString(e));
    return LC_OK;
}

// Autotuning: the largest lane group (G = 8 .. 64 lanes per row for the
// long rows) and the grid (gmul 1, 2, 4 or one row per group), timed on the
// plan's own node array standing in for samples.
lc_status tune_adaptive(lc_plan_s *p, hipStream_t s) {
    AdaptiveState *a = (AdaptiveState *)p->ext;
    const std::string key = arch_name() + "|adaptive|" + std::to_string(p->fn.H) + "|" +
                            std::to_string(a->nnz) + "|" + std::to_string(a->nseg) + "|" + std::to_string(p->fn.prec);
    std::string cached;
    std::vector<int32_t> grows[kNG];
    int best = a->gcap;
    if (cache_get(key, cached)) {
        int gc = best, mul = a->gmul;
        if (sscanf(cached.c_str(), "%d %d", &gc, &mul) >= 1) best = std::max(0, std::min(kNG - 1, gc));
        a->gmul = std::max(0, std::min(4, mul));
    } else {
        double best_ms = 1e30;
        int best_mul = a->gmul;
        for (int cand = 0; cand < 4 * (kNG - 1); ++cand) {
            // grid: 1/2, 1, 2 rounds of resident blocks, or one row per group
            const int gc = 1 + cand / 4, mul = cand % 4 == 3 ? 0 : 1 << (cand % 4);
            a->gmul = mul;
            group_rows(a->rlen, gc, grows);
            hipError_t e = set_groups(a, grows);
            if (e != hipSuccess) return fail_status(LC_ERR_HIP, "lc_autotune: row groups");
            auto run = [&](hipStream_t st) { return launch_reductions(a, p->fn.prec, p->x, p->s2, p->phi, st); };
            const double ms = time_launch(run, s, 5, &e);
            if (e != hipSuccess) return fail_status(LC_ERR_HIP, "lc_autotune: timing");
            if (ms < best_ms) {
                best_ms = ms;
                best = gc;
                best_mul = mul;
            }
        }
        a->gmul = best_mul;
        cache_put(key, std::to_string(best) + " " + std::to_string(best_mul));
    }
    group_rows(a->rlen, best, grows);
    if (set_groups(a, grows) != hipSuccess) return fail_status(LC_ERR_HIP, "lc_autotune: row groups");
    a->gcap = best;
    return LC_OK;
}

}  // namespace lc

using namespace lc;

extern "C" lc_status lc_plan_adaptive(int64_t N, int64_t M, const lc_abel_rule *rule, lc_precision prec,
                                      lc_plan_t *out) {
    if (!out) return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: out is null");
    lc_status st = check_rule(rule);
    if (st != LC_OK) return st;
    if (N < 1 || M < 2 || (M & 1) || N > M / 2)
        return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: need N >= 1, M even >= 2, N <= M/2");
    if (prec != LC_FP64 && prec != LC_FP32_QUAD) return fail_status(LC_ERR_INVALID, "lc_plan_adaptive: bad precision");
    int64_t M_eff = 0;
    if ((st = lc_grid_size(M, &M_eff)) != LC_OK) return st;
    const int64_t H = M_eff / 2, L = H / 2;
    DstCfg dcfg = default_dst_cfg(L);
    if (L > kLdsFftMax && dcfg.L1 == 0)
        return fail_status(LC_ERR_UNSUPPORTED, "lc_plan_adaptive: FFT length has no supported four-step split");
    const lc_abel_rule r = *rule;
    const int vec = prec == LC_FP64 ? 2 : 4;

    // ---- rows -> panels -> segments (long double, the rule's specification)
    std::map<std::pair<int, int>, int> rule_id;  // (q, full) -> index
    std::vector<std::pair<int, int>> rules;
    struct HSeg {
        int32_t row, q, rid;
        long double E, h, scale;
    };
    std::vector<HSeg> hs;
    std::vector<int32_t> rseg(H + 1, 0);
    std::vector<long double> cuts;
    auto rid_of = [&](int q, int full) {
        auto key = std::make_pair(q, full);
        auto it = rule_id.find(key);
        if (it != rule_id.end()) return it->second;
        const int id = (int)rules.size();
        rule_id[key] = id;
        rules.push_back(key);
        return id;
    };
    int qmax = 0;
    for (int64_t rr = 0; rr < H; ++rr) {
        rseg[rr] = (int32_t)hs.size();
        const long double sj = row_half_sine(rr + 1, H);
        row_cuts(sj, r, cuts);
        const long double e1 = cuts.empty() ? 0.0L : cuts[0];
        const int q1 = panel_q(sj, 0.0L, 1 - e1, r);
        qmax = std::max(qmax, q1);
        hs.push_back({(int32_t)rr, q1, rid_of(q1, 0), e1, 1 - e1, 1 - e1});  // first panel [0, t_1]
        for (size_t k = 0; k < cuts.size(); ++k) {
            // panel [1 - hi, 1 - lo] in t
            const long double hi = cuts[k], lo = k + 1 < cuts.size() ? cuts[k + 1] : 0.0L;
            const long double h = (hi - lo) / 2;
            const int q = panel_q(sj, 1 - hi, 1 - lo, r);
            qmax = std::max(qmax, q);
            hs.push_back({(int32_t)rr, q, rid_of(q, 1), lo, h, h});
        }
        if (hs.size() > (size_t)INT32_MAX / 2)
            return fail_status(LC_ERR_UNSUPPORTED, "lc_plan_adaptive: too many panels");
    }
    rseg[H] = (int32_t)hs.size();

    // ---- Gauss tables: weights padded with zeros, node offsets d = 1 - tau
    std::vector<int64_t> woff(rules.size());
    int64_t wlen = 0;
    for (size_t i = 0; i < rules.size(); ++i) {
        woff[i] = wlen;
        wlen += (rules[i].first + 3) / 4 * 4;
    }
    std::vector<double> wt(wlen, 0.0);
    std::vector<double2> dt(wlen, make_double2(0.0, 0.0));
    for (size_t i = 0; i < rules.size(); ++i) {
        const int q = rules[i].first;
        std::vector<long double> x, w;
        if (rules[i].second == 0) {  // positive half of the 2q-point rule, nodes decreasing
            gauss_positive_half_ld(2 * q, x, w);
            for (int k = 0; k < q; ++k) {
                wt[woff[i] + k] = (double)w[k];
                dt[woff[i] + k] = dd_split(1.0L - x[k]);
            }
        } else {  // the q-point rule (q even), nodes increasing
            gauss_positive_half_ld(q, x, w);
            const int h = q / 2;
            for (int k = 0; k < h; ++k) {
                wt[woff[i] + k] = (double)w[k];
                dt[woff[i] + k] = dd_split(1.0L + x[k]);              // tau = -x_k
                wt[woff[i] + q - 1 - k] = (double)w[k];
                dt[woff[i] + q - 1 - k] = dd_split(1.0L - x[k]);      // tau = +x_k
            }
        }
    }

    // ---- device segments (sample offsets padded to 4)
    std::vector<ASeg> segs(hs.size());
    int64_t off = 0;
    for (size_t k = 0; k < hs.size(); ++k) {
        const HSeg &h = hs[k];
        ASeg &a = segs[k];
        a.off = off;
        a.q = h.q;
        a.qp = (h.q + 3) / 4 * 4;
        a.woff = (int32_t)woff[h.rid];
        a.scale = (double)h.scale;
        a.row = h.row;
        a.E = dd_split(h.E);
        a.h = dd_split(h.h);
        off += a.qp;
    }
    const int64_t nnz = off;
    if ((double)nnz > 4.0e10) return fail_status(LC_ERR_UNSUPPORTED, "lc_plan_adaptive: too many samples");

    std::vector<int64_t> rlen(H, 0);
    std::vector<ATab> tab(segs.size());
    std::vector<ARow> rdesc(H);
    for (int64_t rr = 0; rr < H; ++rr) {
        const int k0 = rseg[rr];
        for (int k = k0; k < rseg[rr + 1]; ++k) {
            const int64_t cst = (segs[k].off - segs[k0].off) / vec;
            tab[k].cst = (int32_t)cst;
            tab[k].wbase = (int32_t)(segs[k].woff / vec - cst);
            tab[k].scale = segs[k].scale;
            rlen[rr] += segs[k].qp / vec;
        }
        rdesc[rr] = ARow{segs[k0].off, (int32_t)rr, (int32_t)rlen[rr], k0, rseg[rr + 1] - k0, {0, 0}};
    }
    std::vector<int32_t> grows[kNG];
    int gcap = 3;  // G <= 32 lanes per row, one row per group: measured best on the large band-limited rule
    if (const char *ev = getenv("LC_AQUAD_GMAX")) gcap = std::max(0, std::min(kNG - 1, atoi(ev)));
    int gmul = 0;  // one row per group: measured best
    if (const char *ev = getenv("LC_AQUAD_GMUL")) gmul = std::max(0, std::min(4, atoi(ev)));
    group_rows(rlen, gcap, grows);

    std::vector<double2> rowA, pre, pack, fft;
    std::vector<double> s2h;
    row_factors(H, rowA, s2h);
    twiddles(H, pre, pack, fft);

    lc_plan_s *p = new (std::nothrow) lc_plan_s();
    AdaptiveState *a = new (std::nothrow) AdaptiveState();
    if (!p || !a) {
        delete p;
        delete a;
        return fail_status(LC_ERR_NOMEM, "lc_plan_adaptive: host allocation failed");
    }
    p->kind = LC_PLAN_ADAPTIVE;
    hipGetDevice(&p->device);
    p->ext = a;
    p->fn.N = N;
    p->fn.M = M;
    p->fn.M_eff = M_eff;
    p->fn.H = H;
    p->fn.L = L;
    p->fn.Q = 1;
    p->fn.prec = (int)prec;
    p->dst = dcfg;
    a->nnz = nnz;
    a->nseg = (int64_t)segs.size();
    a->qmax = qmax;

    int64_t ws = 0;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    auto up = [&](auto *dst, const auto &v) {
        if (e == hipSuccess && !v.empty())
            chk(hipMemcpy(dst, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice));
    };
    chk(aalloc(a, &p->x, (size_t)nnz, &ws));
    chk(aalloc(a, &a->segs, segs.size(), &ws));
    chk(aalloc(a, &a->tab, tab.size(), &ws));
    chk(aalloc(a, &a->rseg, rseg.size(), &ws));
    chk(aalloc(a, &a->wtab, wt.size(), &ws));
    chk(aalloc(a, &a->dtab, dt.size(), &ws));
    chk(aalloc(a, &p->rowA, (size_t)H, &ws));
    chk(aalloc(a, &p->s2, (size_t)H, &ws));
    chk(aalloc(a, &p->tw_pre, (size_t)H, &ws));
    chk(aalloc(a, &p->tw_pack, (size_t)L, &ws));
    chk(aalloc(a, &p->tw_fft, (size_t)L, &ws));
    chk(aalloc(a, &p->phi, (size_t)H, &ws));
    if (L > kLdsFftMax) {
        chk(aalloc(a, &p->zA, (size_t)L, &ws));
        chk(aalloc(a, &p->zB, (size_t)L, &ws));
    }
    a->prec = (int)prec;
    a->gmul = gmul;
    chk(aalloc(a, &a->rows[0], (size_t)H, &ws));   // all groups' row lists, back to back
    chk(aalloc(a, &a->frows[0], (size_t)H, &ws));  // the same for flattened rows
    a->rdesc = std::move(rdesc);
    if (e == hipSuccess) chk(set_groups(a, grows));
    a->gcap = gcap;
    a->rlen = std::move(rlen);
    up(a->segs, segs);
    up(a->tab, tab);
    up(a->rseg, rseg);
    up(a->wtab, wt);
    up(a->dtab, dt);
    up(p->rowA, rowA);
    up(p->s2, s2h);
    up(p->tw_pre, pre);
    up(p->tw_pack, pack);
    up(p->tw_fft, fft);
    if (e == hipSuccess) chk(launch_anodes(a->segs, a->nseg, a->dtab, p->rowA, p->x, 0));
    if (e == hipSuccess) chk(hipDeviceSynchronize());
    if (e != hipSuccess) {
        detach_shared(p);
        free_adaptive(a);
        delete p;
        return fail_status(e == hipErrorOutOfMemory ? LC_ERR_NOMEM : LC_ERR_HIP,
                           std::string("lc_plan_adaptive: ") + hipGetErrorString(e));
    }
    p->workspace_bytes = ws;
    log_line("lc_plan_adaptive: N=%lld M_eff=%lld H=%lld samples=%lld panels=%lld (%.2f per row) max q=%d "
             "rules=%zu lane cap G=%d %s", (long long)N, (long long)M_eff, (long long)H, (long long)nnz,
             (long long)a->nseg, (double)a->nseg / (double)H, qmax, rules.size(), 4 << gcap,
             L > kLdsFftMax ? "four-step FFT" : "LDS FFT");
    *out = p;
    return LC_OK;
}
