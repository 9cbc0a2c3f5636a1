// Batched plans: B independent functions of uneven N/M/Q/precision.
//
// Layout: one sample arena (per function [H_b][R_b] FP64 or FP32 at a
// 256-byte aligned byte offset), one node arena (per function [H_b][R_b]
// FP64), one coefficient arena (N_b doubles each, packed) and a phi
// workspace arena (H_b doubles each).  R_b is the number of Abel nodes per
// row: Q_b for the uniform rule, or the padded panel counts of a composite
// rule whose panels are the same in every row (grading toward x = 1, no
// breakpoints, no band).  Either way a row is phi_j = 2 s_j sum_i W_i f_ji
// with weights W and nodes 1 - 2 s_j^2 (1 - t_i^2) shared by the row, so
// both run on the same kernels.  Rules are shared by all functions with the
// same rule, twiddles and row factors by all functions with the same H.
//
// Execution: the Abel quadrature reduction of every function runs as one
// launch per (Q, precision) class over a table of row tiles (each tile a run
// of rows of one function), then one LDS DST launch per FFT-length class
// (one workgroup per function, longest first), then the four-step DST for
// the few functions whose FFT exceeds the LDS.  The sequence is captured
// once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <sstream>
#include <new>
#include <string>
#include <vector>

#include "lc_internal.h"

namespace lc {

lc_status fail_status(lc_status s, const std::string &msg);
lc_status validate_request(int64_t N, int64_t M, int32_t Q, int prec, const char *who);
hipError_t timing_begin(lc_plan_s *p, hipStream_t s, int *slot);
hipError_t timing_end(lc_plan_s *p, hipStream_t s, int slot);

namespace {

struct HSet {
    int64_t H = 0, L = 0;
    double *s2 = nullptr;
    double2 *rowA = nullptr, *tw_pre = nullptr, *tw_pack = nullptr, *tw_fft = nullptr;
    DstCfg dcfg{};
};
// A quadrature rule of a batch: the uniform rule (kind 0: the positive half
// of the 2q-point Gauss-Legendre rule) or a composite rule with the grading
// cuts 1 - t = ratio^k, k = 1..levels (kind 1), R nodes per row.
struct RuleKey {
    int kind = 0, q = 0;
    double ratio = 0.0;
    int levels = 0;
    bool operator<(const RuleKey &o) const {
        if (kind != o.kind) return kind < o.kind;
        if (q != o.q) return q < o.q;
        if (ratio != o.ratio) return ratio < o.ratio;
        return levels < o.levels;
    }
};
struct QSet {
    RuleKey key;
    int Q = 0;                 // R: nodes per row
    double *w = nullptr;       // [R] weights W_i (0 on padding)
    double2 *omt2 = nullptr;   // [R] 1 - t_i^2, double-double
};

// Weights and 1 - t^2 of a composite rule whose panels are the same in every
// row: the specification of lc_abel_rule without breakpoints or band, in
// long double.  Cuts e = 1 - t = ratio^k (decreasing; cuts outside
// (1e-15, 1 - 1e-7) are dropped and cuts closer than 1e-12 of the first
// merge); the first panel [0, 1 - e_1] takes the positive half of the
// 2q-point rule (nodes in decreasing t), every later panel [1 - e_k,
// 1 - e_{k+1}] the q-point rule (nodes in increasing t); every panel is
// padded to a multiple of 4 nodes (the last node repeated, weight 0).  This
// is the row layout of an adaptive plan with the same rule.
std::vector<long double> grade_cuts(double ratio, int levels) {
    std::vector<long double> cuts;
    for (int i = 1; i <= levels && ratio > 0; ++i) {
        const long double e = powl((long double)ratio, (long double)i);
        if (!(e > 1e-15L && e < 1 - 1e-7L)) continue;
        if (!cuts.empty() && cuts.back() - e < 1e-12L * cuts.front()) continue;
        cuts.push_back(e);
    }
    return cuts;
}

void composite_rule(const RuleKey &k, std::vector<double> &w, std::vector<double2> &omt2) {
    const std::vector<long double> cuts = grade_cuts(k.ratio, k.levels);
    w.clear();
    omt2.clear();
    std::vector<long double> x, wq, d, ww;
    auto panel = [&](bool first, long double E, long double h, long double scale) {
        const int q = k.q;
        d.assign(q, 0.0L);
        ww.assign(q, 0.0L);
        if (first) {
            gauss_positive_half_ld(2 * q, x, wq);
            for (int i = 0; i < q; ++i) {
                d[i] = 1 - x[i];
                ww[i] = wq[i];
            }
        } else {
            gauss_positive_half_ld(q, x, wq);
            for (int i = 0; i < q / 2; ++i) {
                d[i] = 1 + x[i];
                ww[i] = wq[i];
                d[q - 1 - i] = 1 - x[i];
                ww[q - 1 - i] = wq[i];
            }
        }
        const int qp = (q + 3) / 4 * 4;
        for (int i = 0; i < qp; ++i) {
            const int ii = i < q ? i : q - 1;
            const long double e = E + h * d[ii];  // 1 - t
            w.push_back(i < q ? (double)(scale * ww[i]) : 0.0);
            omt2.push_back(dd_split(e * (2 - e)));
        }
    };
    const long double e1 = cuts.empty() ? 0.0L : cuts[0];
    panel(true, e1, 1 - e1, 1 - e1);
    for (size_t i = 0; i < cuts.size(); ++i) {
        const long double hi = cuts[i], lo = i + 1 < cuts.size() ? cuts[i + 1] : 0.0L;
        const long double h = (hi - lo) / 2;
        panel(false, lo, h, h);
    }
}
constexpr int kParts = 4;  // pipeline parts of a captured batch execution

struct QuadClass {
    int Q = 0, prec = 0;
    QuadCfg cfg{};
    double *w = nullptr;
    BatchTile *tiles = nullptr;
    int ntiles = 0;
    int64_t rows = 0;
    std::vector<int> fns;
    int tstart[kParts + 1] = {};  // tiles of part k: [tstart[k], tstart[k+1])
};
struct DstGroup {
    int threads = 0, Lmax = 0, n = 0;
    int32_t *list = nullptr;
    int lstart[kParts + 1] = {};  // list entries of part k (list sorted by part, then length)
    // short functions packed kMultiSlots list entries per 64-thread block
    // (blocks of one FFT length each; n and lstart count blocks)
    bool multi = false;
};

// tiles are in function order and parts are contiguous function ranges, so
// the tiles of part k are one contiguous range
void part_starts(const std::vector<BatchTile> &tiles, const std::vector<int> &part_of, int nparts, int *start) {
    int k = 0;
    start[0] = 0;
    for (int t = 0; t < (int)tiles.size(); ++t)
        while (k < nparts - 1 && part_of[tiles[t].fn] > k) start[++k] = t;
    while (k < nparts) start[++k] = (int)tiles.size();
}

// rpt rows per tile, addresses resolved: samples at f_off + r Q s bytes,
// phi and s2 from row r of the function
std::vector<BatchTile> make_tiles(const std::vector<FnDesc> &fn, const std::map<int64_t, HSet> &hs,
                                  const std::vector<int> &fns, int rpt) {
    std::vector<BatchTile> tiles;
    for (int b : fns) {
        const FnDesc &d = fn[b];
        const int64_t esz = d.prec == LC_FP64 ? 8 : 4;
        const double *s2 = hs.at(d.H).s2;
        for (int64_t r = 0; r < d.H; r += rpt)
            tiles.push_back({d.f_off + r * d.Q * esz, d.phi_off + r, s2 + r, (int32_t)std::min<int64_t>(rpt, d.H - r), b});
    }
    return tiles;
}

struct BatchState {
    int B = 0;
    std::vector<FnDesc> fn;
    BatchFn *dfn = nullptr;
    std::map<int64_t, HSet> hs;
    std::vector<QSet> qs;              // rules, indexed by FnDesc::w_id
    std::vector<QuadClass> classes;
    std::vector<DstGroup> groups;
    std::vector<int> large;
    BigFn *dbig = nullptr;
    BigTile *ctiles = nullptr, *rtiles = nullptr, *ptiles = nullptr;
    int nct = 0, nrt = 0, npt = 0;
    int cst[kParts + 1] = {}, rst[kParts + 1] = {}, pst[kParts + 1] = {};  // big tiles per part
    std::vector<int> part_of;          // part of each function
    std::vector<char> fused;           // functions run whole by the fused kernel
    FusedFn *flist[2] = {};            // their descriptors per sample precision, largest first
    int nfused[2] = {};
    int64_t fHmax[2] = {};
    int nparts = 1;
    hipStream_t side = nullptr;        // second stream of the captured pipeline
    hipEvent_t evq[kParts] = {}, evj = nullptr;
    double *x_arena = nullptr, *phi_arena = nullptr;
    NodeTile *node_tiles = nullptr;    // node construction blocks (kept for the complements)
    int64_t n_node_tiles = 0;
    double2 *zA = nullptr, *zB = nullptr;
    int64_t f_bytes = 0, x_elems = 0, c_elems = 0, phi_elems = 0, ws_bytes = 0;
    std::vector<void *> allocs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void *gf = nullptr;
    double *gc = nullptr;
    hipStream_t gs = nullptr;
};

template <typename T>
hipError_t balloc(BatchState *st, T **p, size_t n) {
    *p = nullptr;
    if (n == 0) return hipSuccess;
    hipError_t e = device_alloc((void **)p, n * sizeof(T));
    if (e == hipSuccess) {
        st->allocs.push_back(*p);
        st->ws_bytes += (int64_t)(n * sizeof(T));
    }
    return e;
}

template <typename T>
hipError_t upload(BatchState *st, T **p, const std::vector<T> &v) {
    hipError_t e = balloc(st, p, v.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

void free_state(BatchState *st) {
    if (!st) return;
    for (auto &e : st->evq)
        if (e) hipEventDestroy(e);
    if (st->evj) hipEventDestroy(st->evj);
    if (st->side) hipStreamDestroy(st->side);
    if (st->gexec) hipGraphExecDestroy(st->gexec);
    if (st->graph) hipGraphDestroy(st->graph);
    for (void *p : st->allocs) hipFree(p);
    delete st;
}

// DST work of part k.  With a second stream s2 the DST groups (independent
// functions) are spread over s and s2, largest estimated work first onto
// the less loaded stream, so that one group's last round of workgroups
// overlaps the others; the batched four-step passes stay on s.
hipError_t launch_part_dst(BatchState *st, int k, double *c_arena, hipStream_t s, hipStream_t s2 = nullptr) {
    hipError_t e;
    std::vector<int> order(st->groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    auto cost = [&](int i) {
        const DstGroup &g = st->groups[i];
        return (double)(g.lstart[k + 1] - g.lstart[k]) * g.Lmax;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    double load[2] = {0.0, 0.0};
    for (int i : order) {
        const DstGroup &g = st->groups[i];
        const int n = g.lstart[k + 1] - g.lstart[k];
        const int w = (s2 && load[1] < load[0]) ? 1 : 0;
        load[w] += cost(i);
        e = g.multi ? launch_bdst_multi(st->phi_arena, st->dfn, g.list + (int64_t)g.lstart[k] * kMultiSlots, n,
                                        c_arena, w ? s2 : s)
                    : launch_bdst(g.threads, g.Lmax, st->phi_arena, st->dfn, g.list + g.lstart[k], n, c_arena,
                                  w ? s2 : s);
        if (e != hipSuccess) return e;
    }
    return launch_bbig(st->phi_arena, st->dbig, st->ctiles + st->cst[k], st->cst[k + 1] - st->cst[k],
                       st->rtiles + st->rst[k], st->rst[k + 1] - st->rst[k], st->ptiles + st->pst[k],
                       st->pst[k + 1] - st->pst[k], c_arena, s);
}

hipError_t launch_part_quad(BatchState *st, int k, const void *f_arena, double *c_arena, hipStream_t s) {
    for (int pr = 0; pr < 2; ++pr) {  // the fused functions (one part only), first
        if (k > 0 || st->nfused[pr] == 0) continue;
        hipError_t e = launch_bfused(pr == 0 ? LC_FP64 : LC_FP32_QUAD, f_arena, st->dfn, st->flist[pr],
                                     st->nfused[pr], st->fHmax[pr], c_arena, s);
        if (e != hipSuccess) return e;
    }
    for (auto &qc : st->classes) {
        const int n = qc.tstart[k + 1] - qc.tstart[k];
        if (n <= 0) continue;
        QuadCfg c = qc.cfg;
        c.grid = std::max(1, std::min(c.grid, n));
        hipError_t e = launch_bquad(c, qc.prec, f_arena, qc.w, qc.tiles + qc.tstart[k], n, st->phi_arena, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Eager order: all quadrature (timed as one region), then all DST work.
hipError_t launch_all(lc_plan_s *p, BatchState *st, const void *f_arena, double *c_arena, hipStream_t s,
                      bool timed) {
    hipError_t e;
    int slot = -1;
    if (timed && (e = timing_begin(p, s, &slot)) != hipSuccess) return e;
    for (int k = 0; k < st->nparts; ++k)
        if ((e = launch_part_quad(st, k, f_arena, c_arena, s)) != hipSuccess) return e;
    if (timed && (e = timing_end(p, s, slot)) != hipSuccess) return e;
    for (int k = 0; k < st->nparts; ++k)
        if ((e = launch_part_dst(st, k, c_arena, s)) != hipSuccess) return e;
    return hipSuccess;
}

// Captured order: a two-stream pipeline.  The quadrature of part k runs on
// the caller's stream; the DST of part k runs on the side stream once part
// k's quadrature is done, so it overlaps the (HBM-bound) quadrature of part
// k+1.  The last part's DST groups use both streams (the caller's has no
// quadrature left).  The side stream joins back before the graph ends.
hipError_t launch_pipeline(BatchState *st, const void *f_arena, double *c_arena, hipStream_t s) {
    hipError_t e;
    for (int k = 0; k < st->nparts; ++k) {
        if ((e = launch_part_quad(st, k, f_arena, c_arena, s)) != hipSuccess) return e;
        if ((e = hipEventRecord(st->evq[k], s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(st->side, st->evq[k], 0)) != hipSuccess) return e;
        const bool last = k + 1 == st->nparts;
        if ((e = launch_part_dst(st, k, c_arena, st->side, last ? s : nullptr)) != hipSuccess) return e;
    }
    if ((e = hipEventRecord(st->evj, st->side)) != hipSuccess) return e;
    return hipStreamWaitEvent(s, st->evj, 0);
}

lc_status build_batch(int32_t B, const int64_t *N, const int64_t *M, const std::vector<RuleKey> &keys,
                      const lc_precision *prec, const char *who, lc_plan_t *out);

}  // namespace

void destroy_batch(lc_plan_s *p) {
    free_state((BatchState *)p->ext);
    p->ext = nullptr;
}

void info_batch(lc_plan_s *p, lc_plan_desc *d) {
    BatchState *st = (BatchState *)p->ext;
    d->B = st->B;
    int64_t samples = 0, N = 0;
    for (auto &f : st->fn) {
        samples += f.H * f.Q;
        N += f.N;
    }
    d->N = N;
    d->samples = samples;
    d->sample_bytes = st->f_bytes;
    d->workspace_bytes = st->ws_bytes;
}

hipError_t batch_complement(const lc_plan_s *p, double *comp, hipStream_t s) {
    const BatchState *st = (const BatchState *)p->ext;
    return launch_bnodes(st->node_tiles, st->n_node_tiles, s, st->x_arena, comp);
}

lc_status nodes_batch(lc_plan_s *p, const double **x, int64_t *rows, int32_t *Q) {
    BatchState *st = (BatchState *)p->ext;
    *x = st->x_arena;
    if (rows) *rows = st->x_elems;
    if (Q) *Q = 0;
    return LC_OK;
}

// Autotuning of a batch plan: the launch shape of every quadrature class
// (tiles rebuilt for each candidate) and the threads of every DST group.
lc_status tune_batch(lc_plan_s *p, hipStream_t s) {
    BatchState *st = (BatchState *)p->ext;
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the batch shape
    auto mix = [&](int64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (uint64_t)((v >> (8 * k)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (auto &d : st->fn) {
        mix(d.N);
        mix(d.M_eff);
        mix(d.Q);
        mix(d.prec);
        const RuleKey &k = st->qs[d.w_id].key;
        mix(k.kind);
        mix(k.q);
        int64_t rb = 0;
        memcpy(&rb, &k.ratio, sizeof rb);
        mix(rb);
        mix(k.levels);
    }
    const std::string key = arch_name() + "|batch2|" + std::to_string(st->B) + "|" + std::to_string(h);
    std::string val;
    std::vector<QuadCfg> qcfg;
    std::vector<int> gthreads;
    bool cached = false;
    if (cache_get(key, val)) {
        std::istringstream in(val);
        size_t nc = 0, ng = 0;
        cached = (bool)(in >> nc) && nc == st->classes.size();
        for (size_t i = 0; cached && i < nc; ++i) {
            QuadCfg c = st->classes[i].cfg;
            cached = (bool)(in >> c.vec >> c.G >> c.cpl >> c.unroll >> c.block >> c.grid >> c.rpg) &&
                     quad_cfg_supported(c, st->classes[i].prec, st->classes[i].Q);
            qcfg.push_back(c);
        }
        cached = cached && (in >> ng) && ng == st->groups.size();
        for (size_t i = 0; cached && i < ng; ++i) {
            int t = 0;
            cached = (bool)(in >> t) && st->groups[i].Lmax <= 8 * t && dst_threads_ok(t);
            gthreads.push_back(t);
        }
    }
    hipError_t e = hipSuccess;
    if (!cached) {
        qcfg.clear();
        gthreads.clear();
        const int cu = device_cu_count();
        for (auto &qc : st->classes) {
            double best = 1e30;
            QuadCfg bc = qc.cfg;
            if (qc.fns.empty()) {  // every function of the class runs in the fused kernel
                qcfg.push_back(bc);
                continue;
            }
            for (QuadCfg c : quad_candidates(qc.prec, qc.Q, qc.rows, cu, true)) {
                c.Qv = qc.Q;
                std::vector<BatchTile> tl = make_tiles(st->fn, st->hs, qc.fns, quad_rows_per_block(c));
                BatchTile *dt = nullptr;
                if ((e = device_alloc((void **)&dt, tl.size() * sizeof(BatchTile))) != hipSuccess) break;
                e = hipMemcpy(dt, tl.data(), tl.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
                c.grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)tl.size(), c.grid * 1));
                if (e == hipSuccess) {
                    hipError_t er;
                    const int nt = (int)tl.size();
                    const double t = time_launch([&](hipStream_t ss) { return launch_bquad(c, qc.prec, st->x_arena, qc.w, dt, nt, st->phi_arena, ss); }, s, 3, &er);
                    if (er == hipSuccess && t < best) { best = t; bc = c; }
                }
                hipFree(dt);
            }
            qcfg.push_back(bc);
        }
        double *cbuf = nullptr;
        if (e == hipSuccess) e = device_alloc((void **)&cbuf, (size_t)std::max<int64_t>(1, st->c_elems) * sizeof(double));
        for (auto &g : st->groups) {
            double best = 1e30;
            int bt = g.threads;
            if (g.multi) {
                gthreads.push_back(bt);
                continue;
            }
            for (int T : {64, 128, 256, 512, 1024}) {
                if (e != hipSuccess || g.Lmax > 8 * T || prepare_bdst(T, g.Lmax) != hipSuccess) continue;
                hipError_t er;
                const double t = time_launch([&](hipStream_t ss) { return launch_bdst(T, g.Lmax, st->phi_arena, st->dfn, g.list, g.n, cbuf, ss); }, s, 3, &er);
                if (er == hipSuccess && t < best) { best = t; bt = T; }
            }
            gthreads.push_back(bt);
        }
        hipFree(cbuf);
        if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_autotune: ") + hipGetErrorString(e));
        std::string v = std::to_string(qcfg.size());
        for (auto &c : qcfg) v += " " + quad_to_str(c);
        v += " " + std::to_string(gthreads.size());
        for (int t : gthreads) v += " " + std::to_string(t);
        cache_put(key, v);
    }
    // apply: new tiles per class, thread counts per group, fresh graph
    for (size_t i = 0; i < st->classes.size(); ++i) {
        QuadClass &qc = st->classes[i];
        QuadCfg c = qcfg[i];
        c.Qv = qc.Q;
        std::vector<BatchTile> tl = make_tiles(st->fn, st->hs, qc.fns, quad_rows_per_block(c));
        BatchTile *dt = nullptr;
        if ((e = upload(st, &dt, tl)) != hipSuccess) return fail_status(LC_ERR_HIP, "lc_autotune: tiles");
        qc.tiles = dt;
        qc.ntiles = (int)tl.size();
        part_starts(tl, st->part_of, st->nparts, qc.tstart);
        qc.cfg = c;
        qc.cfg.grid = (int)std::max<int64_t>(1, std::min<int64_t>(qc.ntiles, c.grid));
        log_line("lc_autotune: class R=%d %s: vec=%d G=%d cpl=%d unroll=%d grid=%d%s%s", qc.Q,
                 qc.prec == LC_FP64 ? "fp64" : "fp32", qc.cfg.vec, qc.cfg.G, qc.cfg.cpl, qc.cfg.unroll, qc.cfg.grid,
                 qc.cfg.rpg == 2 ? " (row pairs)" : "", cached ? " (cached)" : "");
    }
    for (size_t i = 0; i < st->groups.size(); ++i) {
        if (st->groups[i].multi) continue;  // 64 threads by construction
        if (prepare_bdst(gthreads[i], st->groups[i].Lmax) == hipSuccess) st->groups[i].threads = gthreads[i];
    }
    if (st->gexec) {
        hipGraphExecDestroy(st->gexec);
        st->gexec = nullptr;
    }
    if (st->graph) {
        hipGraphDestroy(st->graph);
        st->graph = nullptr;
    }
    return LC_OK;
}

}  // namespace lc

using namespace lc;

extern "C" {

lc_status lc_plan_batch(int32_t B, const int64_t *N, const int64_t *M, const int32_t *Q, const lc_precision *prec,
                        lc_plan_t *out) {
    if (!out || !N || !M || !Q || !prec) return fail_status(LC_ERR_INVALID, "lc_plan_batch: null argument");
    if (B < 1) return fail_status(LC_ERR_INVALID, "lc_plan_batch: B must be >= 1");
    for (int b = 0; b < B; ++b) {
        char who[64];
        snprintf(who, sizeof who, "lc_plan_batch[%d]", b);
        lc_status s = validate_request(N[b], M[b], Q[b], (int)prec[b], who);
        if (s != LC_OK) return s;
    }
    std::vector<RuleKey> keys(B);
    for (int b = 0; b < B; ++b) {
        keys[b].kind = 0;
        keys[b].q = Q[b];
    }
    return build_batch(B, N, M, keys, prec, "lc_plan_batch", out);
}

lc_status lc_plan_batch_rules(int32_t B, const int64_t *N, const int64_t *M, const lc_abel_rule *rules,
                              const lc_precision *prec, lc_plan_t *out) {
    if (!out || !N || !M || !rules || !prec) return fail_status(LC_ERR_INVALID, "lc_plan_batch_rules: null argument");
    if (B < 1) return fail_status(LC_ERR_INVALID, "lc_plan_batch_rules: B must be >= 1");
    std::vector<RuleKey> keys(B);
    for (int b = 0; b < B; ++b) {
        char who[80];
        snprintf(who, sizeof who, "lc_plan_batch_rules[%d]", b);
        const lc_abel_rule &r = rules[b];
        if (r.band != 0.0 || r.nbreak != 0)
            return fail_status(LC_ERR_UNSUPPORTED, std::string(who) +
                               ": batch rules take no band or breakpoints (every row must have the same panels)");
        if (r.q < 1 || r.q > 65536) return fail_status(LC_ERR_INVALID, std::string(who) + ": q must be in [1, 65536]");
        if (!(r.grade_ratio >= 0 && r.grade_ratio < 1) || r.grade_levels < 0 || r.grade_levels > 64)
            return fail_status(LC_ERR_INVALID, std::string(who) + ": grade_ratio in [0, 1), grade_levels in [0, 64]");
        const bool cuts = r.grade_ratio > 0 && r.grade_levels > 0;
        if (cuts && (r.q % 2))
            return fail_status(LC_ERR_INVALID, std::string(who) + ": q must be even when the rule has cuts");
        keys[b].kind = 1;
        keys[b].q = r.q;
        keys[b].ratio = cuts ? r.grade_ratio : 0.0;
        keys[b].levels = cuts ? r.grade_levels : 0;
        if ((int)grade_cuts(keys[b].ratio, keys[b].levels).size() != keys[b].levels)
            return fail_status(LC_ERR_INVALID, std::string(who) +
                               ": grading cuts ratio^k must lie in (1e-15, 1 - 1e-7) and not merge");
        const int64_t R = (int64_t)(keys[b].levels + 1) * ((r.q + 3) / 4 * 4);
        if (R > 65536)
            return fail_status(LC_ERR_UNSUPPORTED, std::string(who) + ": more than 65536 nodes per row");
        lc_status s = validate_request(N[b], M[b], (int32_t)R, (int)prec[b], who);
        if (s != LC_OK) return s;
    }
    return build_batch(B, N, M, keys, prec, "lc_plan_batch_rules", out);
}

}  // extern "C"

namespace lc {
namespace {

lc_status build_batch(int32_t B, const int64_t *N, const int64_t *M, const std::vector<RuleKey> &keys,
                      const lc_precision *prec, const char *who, lc_plan_t *out) {
    const std::string whos(who);
    BatchState *st = new (std::nothrow) BatchState();
    if (!st) return fail_status(LC_ERR_NOMEM, whos + ": host allocation failed");
    st->B = B;
    st->fn.resize(B);
    const int cu = device_cu_count();
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };

    // ---- rules (host tables; uploaded with the other shared tables)
    std::map<RuleKey, int> rule_id;
    std::vector<std::vector<double>> rw;
    std::vector<std::vector<double2>> ro;
    std::vector<int> wid(B);
    for (int b = 0; b < B; ++b) {
        auto it = rule_id.find(keys[b]);
        if (it != rule_id.end()) {
            wid[b] = it->second;
            continue;
        }
        const int id = (int)st->qs.size();
        rule_id[keys[b]] = id;
        wid[b] = id;
        std::vector<double> w, t;
        std::vector<double2> o;
        if (keys[b].kind == 0) gauss_half_rule(keys[b].q, t, w, o);
        else composite_rule(keys[b], w, o);
        QSet q;
        q.key = keys[b];
        q.Q = (int)w.size();
        st->qs.push_back(q);
        rw.push_back(std::move(w));
        ro.push_back(std::move(o));
    }

    // ---- sizes and offsets
    int64_t foff = 0, xoff = 0, coff = 0, poff = 0;
    for (int b = 0; b < B; ++b) {
        FnDesc &d = st->fn[b];
        int64_t Me = 0;
        lc_grid_size(M[b], &Me);
        d.N = N[b];
        d.M = M[b];
        d.M_eff = Me;
        d.H = Me / 2;
        d.L = d.H / 2;
        d.Q = st->qs[wid[b]].Q;
        d.w_id = wid[b];
        d.prec = (int)prec[b];
        const int esz = d.prec == LC_FP64 ? 8 : 4;
        d.f_off = foff;
        foff += (d.H * d.Q * esz + 255) / 256 * 256;
        d.x_off = xoff;
        xoff += (d.H * d.Q + 31) / 32 * 32;
        d.c_off = coff;
        coff += d.N;
        d.phi_off = poff;
        poff += d.H;
        if (d.L > kLdsFftMax && four_step_cfg(d.L).L1 == 0) {
            free_state(st);
            return fail_status(LC_ERR_UNSUPPORTED, whos + ": an FFT length has no four-step split");
        }
    }
    st->f_bytes = foff;
    st->x_elems = xoff;
    st->c_elems = coff;
    st->phi_elems = poff;
    // pipeline parts: contiguous function ranges of about equal sample bytes
    // (LC_BATCH_PARTS = 1..4; one part by default: measured fastest on the
    // uneven-batch and mixed-stream workloads)
    {
        int want = 1;
        if (const char *ev = getenv("LC_BATCH_PARTS")) want = std::max(1, std::min(kParts, atoi(ev)));
        st->nparts = B >= 4 * want ? want : 1;
    }
    st->part_of.assign(B, 0);
    if (st->nparts > 1) {
        int64_t acc = 0;
        for (int b = 0; b < B; ++b) {
            const int64_t sz = st->fn[b].H * st->fn[b].Q * (st->fn[b].prec == LC_FP64 ? 8 : 4);
            st->part_of[b] = (int)std::min<int64_t>(st->nparts - 1, (acc + sz / 2) * st->nparts / std::max<int64_t>(1, foff));
            acc += sz;
        }
    }

    // functions small enough for one workgroup can run quadrature, twist, FFT
    // and rescale in the fused kernel (LC_BATCH_FUSE=1; off by default: it
    // measured within 1% of the two-phase execution on the uneven batch and
    // the mixed stream, one way or the other)
    {
        bool fuse = false;
        if (const char *ev = getenv("LC_BATCH_FUSE")) fuse = atoi(ev) != 0;
        int64_t hmin = 512;  // below: tiled reduction and packed DSTs (one workgroup would idle)
        if (const char *ev = getenv("LC_BATCH_FUSE_HMIN")) hmin = std::max<int64_t>(2, atoll(ev));
        st->fused.assign(B, 0);
        for (int b = 0; b < B; ++b) {
            const FnDesc &d = st->fn[b];
            st->fused[b] = fuse && st->nparts == 1 && d.H >= hmin && d.H <= kFuseHmax && fuse_lanes(d.prec, d.Q) > 0;
        }
    }
    // ---- shared tables
    for (auto &d : st->fn) {
        if (!st->hs.count(d.H)) {
            HSet h;
            h.H = d.H;
            h.L = d.L;
            std::vector<double2> pre, pack, fft, rowA;
            std::vector<double> s2;
            twiddles(d.H, pre, pack, fft);
            row_factors(d.H, rowA, s2);
            chk(upload(st, &h.tw_pre, pre));
            chk(upload(st, &h.tw_pack, pack));
            chk(upload(st, &h.tw_fft, fft));
            chk(upload(st, &h.rowA, rowA));
            chk(upload(st, &h.s2, s2));
            h.dcfg = four_step_cfg(d.L);
            st->hs[d.H] = h;
        }
    }
    for (size_t i = 0; i < st->qs.size(); ++i) {
        chk(upload(st, &st->qs[i].w, rw[i]));
        chk(upload(st, &st->qs[i].omt2, ro[i]));
    }
    chk(balloc(st, &st->x_arena, (size_t)st->x_elems));
    chk(balloc(st, &st->phi_arena, (size_t)st->phi_elems));
    // functions whose FFT runs as the batched four-step (several workgroups
    // per function) rather than in one workgroup's LDS: L > big_L
    // (LC_BATCH_BIG_L overrides; a length without a split stays in LDS;
    // moving lengths 1024..8192 to the four-step measured slower)
    int64_t big_L = kLdsFftMax;
    if (const char *ev = getenv("LC_BATCH_BIG_L")) big_L = std::max<int64_t>(64, atoll(ev));
    auto is_big = [&](int64_t L) { return L > kLdsFftMax || (L > big_L && four_step_cfg(L).L1 != 0); };
    int64_t Lsum = 0;
    for (int b = 0; b < B; ++b)
        if (is_big(st->fn[b].L)) Lsum += st->fn[b].L;
    if (Lsum) {
        chk(balloc(st, &st->zA, (size_t)Lsum));
        chk(balloc(st, &st->zB, (size_t)Lsum));
    }
    if (e != hipSuccess) {
        free_state(st);
        return fail_status(e == hipErrorOutOfMemory ? LC_ERR_NOMEM : LC_ERR_HIP,
                           whos + ": allocation/upload failed: " + hipGetErrorString(e));
    }
    // ---- nodes: one launch over blocks of 4096 nodes of one function each
    if (e == hipSuccess) {
        std::vector<NodeTile> nt;
        for (auto &d : st->fn) {
            const int64_t n = d.H * d.Q;
            for (int64_t a = 0; a < n; a += 4096)
                nt.push_back({st->x_arena + d.x_off, st->hs[d.H].rowA, st->qs[d.w_id].omt2, a,
                              std::min<int64_t>(n, a + 4096), d.Q});
        }
        NodeTile *dnt = nullptr;
        chk(upload(st, &dnt, nt));
        if (e == hipSuccess) chk(launch_bnodes(dnt, (int64_t)nt.size(), 0));
        st->node_tiles = dnt;
        st->n_node_tiles = (int64_t)nt.size();
    }
    chk(hipDeviceSynchronize());
    // ---- device descriptors
    std::vector<BatchFn> hfn(B);
    for (int b = 0; b < B; ++b) {
        const FnDesc &d = st->fn[b];
        const HSet &h = st->hs[d.H];
        BatchFn &f = hfn[b];
        f.f_off = d.f_off;
        f.phi_off = d.phi_off;
        f.c_off = d.c_off;
        f.N = d.N;
        f.H = d.H;
        f.L = d.L;
        f.s2 = h.s2;
        f.tw_pre = h.tw_pre;
        f.tw_pack = h.tw_pack;
        f.tw_fft = h.tw_fft;
        if (d.L <= kLdsFftMax) f.sched = make_sched((int)d.L);
    }
    chk(upload(st, &st->dfn, hfn));
    // ---- quadrature classes and their tiles
    // two rows per lane group wherever 2Q fits: by default for FP32 samples
    // (the uneven batch's 192-byte rows: 0.98 against 1.08 ms per step),
    // not for FP64 (1.64 against 1.63 ms); LC_BATCH_ROW_PAIRS=0 or 1 sets
    // it for both.  The autotuner weighs both shapes either way.
    int row_pairs = -1;
    if (const char *ev = getenv("LC_BATCH_ROW_PAIRS")) row_pairs = atoi(ev) != 0;
    std::map<std::pair<int, int>, std::vector<int>> cls;
    for (int b = 0; b < B; ++b) cls[{st->fn[b].w_id, st->fn[b].prec}].push_back(b);
    for (auto &kv : cls) {
        QuadClass qc;
        qc.Q = st->qs[kv.first.first].Q;
        qc.prec = kv.first.second;
        {   // the functions that run whole in the fused kernel leave the tiles
            std::vector<int> rest;
            for (int b : kv.second)
                if (!st->fused[b]) rest.push_back(b);
            kv.second = rest;
        }
        for (int b : kv.second) qc.rows += st->fn[b].H;
        qc.cfg = default_quad_cfg(qc.prec, qc.Q, qc.rows, cu);
        if (row_pairs == 1 || (row_pairs < 0 && qc.prec != LC_FP64))
            pair_quad_cfg(qc.prec, qc.Q, qc.cfg);  // keeps the default where it does not fit
        qc.cfg.Qv = qc.Q;
        qc.w = st->qs[kv.first.first].w;
        qc.fns = kv.second;
        std::vector<BatchTile> tiles = make_tiles(st->fn, st->hs, qc.fns, quad_rows_per_block(qc.cfg));
        qc.ntiles = (int)tiles.size();
        part_starts(tiles, st->part_of, st->nparts, qc.tstart);
        {   // one round of resident blocks of this variant
            int occ = bquad_blocks_per_cu(qc.cfg, qc.prec);
            if (occ < 1) occ = 8;
            qc.cfg.grid = (int)std::max<int64_t>(1, std::min<int64_t>(qc.ntiles, (int64_t)cu * occ));
        }
        chk(upload(st, &qc.tiles, tiles));
        st->classes.push_back(qc);
    }
    // ---- fused functions: one list per sample precision, largest first
    for (int pr = 0; pr < 2; ++pr) {
        std::vector<int> fz;
        for (int b = 0; b < B; ++b)
            if (st->fused[b] && (st->fn[b].prec == LC_FP64) == (pr == 0)) fz.push_back(b);
        std::stable_sort(fz.begin(), fz.end(), [&](int a, int c) { return st->fn[a].H > st->fn[c].H; });
        std::vector<FusedFn> fl;
        for (int b : fz) {
            const FnDesc &d = st->fn[b];
            fl.push_back({b, d.Q, fuse_lanes(d.prec, d.Q), 0, st->qs[d.w_id].w});
            st->fHmax[pr] = std::max(st->fHmax[pr], d.H);
        }
        st->nfused[pr] = (int)fl.size();
        if (!fl.empty()) chk(upload(st, &st->flist[pr], fl));
    }
    // ---- DST groups (one workgroup per function, longest first; short
    // functions of equal FFT length packed several per workgroup)
    std::map<int, std::vector<int>> grp;
    std::map<std::pair<int, int64_t>, std::vector<int>> packed;  // (part, L) -> functions
    bool pack = true;
    if (const char *ev = getenv("LC_BATCH_MULTI")) pack = atoi(ev) != 0;
    for (int b = 0; b < B; ++b) {
        const int64_t L = st->fn[b].L;
        if (st->fused[b]) continue;  // its DST runs in the fused kernel
        if (is_big(L)) {
            st->large.push_back(b);
            continue;
        }
        if (pack && L <= kMultiMaxL) {
            packed[{st->part_of[b], L}].push_back(b);
            continue;
        }
        // group by power-of-two length class so that the LDS reserved per
        // workgroup (the group's longest FFT) stays close to what it needs
        int cls = 512;
        while (cls < L) cls *= 2;
        grp[cls].push_back(b);
    }
    // long functions: batched four-step descriptors and block tables
    if (!st->large.empty()) {
        std::vector<BigFn> big;
        std::vector<BigTile> ct, rt, pt;
        int64_t zoff = 0;
        for (int b : st->large) {
            const FnDesc &d = st->fn[b];
            const HSet &h = st->hs[d.H];
            BigFn f{};
            f.H = d.H;
            f.L = d.L;
            f.N = d.N;
            f.L1 = h.dcfg.L1;
            f.L2 = h.dcfg.L2;
            four_step_blocks(f.L1, f.L2, &f.CB, &f.RB);
            f.phi_off = d.phi_off;
            f.c_off = d.c_off;
            f.tw_pre = h.tw_pre;
            f.tw_pack = h.tw_pack;
            f.tw_fft = h.tw_fft;
            f.zA = st->zA + zoff;
            f.zB = st->zB + zoff;
            zoff += d.L;
            f.s1 = h.dcfg.s1;
            f.s2 = h.dcfg.s2;
            const int id = (int)big.size();
            for (int k = 0; k < f.L2; k += f.CB) ct.push_back({id, k});
            for (int k = 0; k < f.L1; k += f.RB) rt.push_back({id, k});
            for (int64_t n = 0; n < f.N; n += 1024) pt.push_back({id, (int32_t)n});
            big.push_back(f);
        }
        auto starts = [&](const std::vector<BigTile> &v, int *out) {
            int k = 0;
            out[0] = 0;
            for (int t = 0; t < (int)v.size(); ++t)
                while (k < st->nparts - 1 && st->part_of[st->large[v[t].fn]] > k) out[++k] = t;
            while (k < st->nparts) out[++k] = (int)v.size();
        };
        starts(ct, st->cst);
        starts(rt, st->rst);
        starts(pt, st->pst);
        chk(upload(st, &st->dbig, big));
        chk(upload(st, &st->ctiles, ct));
        chk(upload(st, &st->rtiles, rt));
        chk(upload(st, &st->ptiles, pt));
        st->nct = (int)ct.size();
        st->nrt = (int)rt.size();
        st->npt = (int)pt.size();
    }
    for (auto &kv : grp) {
        DstGroup g;
        g.threads = dst_threads_for(kv.first);
        auto v = kv.second;
        std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
            if (st->part_of[a] != st->part_of[b]) return st->part_of[a] < st->part_of[b];
            return st->fn[a].L > st->fn[b].L;
        });
        g.Lmax = 0;
        for (int b : v) g.Lmax = std::max<int>(g.Lmax, (int)st->fn[b].L);
        g.n = (int)v.size();
        {
            int k = 0;
            g.lstart[0] = 0;
            for (int i = 0; i < g.n; ++i)
                while (k < st->nparts - 1 && st->part_of[v[i]] > k) g.lstart[++k] = i;
            while (k < st->nparts) g.lstart[++k] = g.n;
        }
        std::vector<int32_t> list(v.begin(), v.end());
        chk(upload(st, &g.list, list));
        chk(prepare_bdst(g.threads, g.Lmax));
        st->groups.push_back(g);
    }
    if (!packed.empty()) {
        // blocks of multi_slots(L) functions of one length, by part, longest
        // lengths first within a part
        DstGroup g;
        g.multi = true;
        g.threads = 64;
        g.Lmax = kMultiMaxL;
        std::vector<int32_t> list;
        int k = 0;
        g.lstart[0] = 0;
        for (auto it = packed.begin(); it != packed.end();) {
            const int part = it->first.first;
            while (k < part) g.lstart[++k] = (int)(list.size() / kMultiSlots);
            auto end = it;
            while (end != packed.end() && end->first.first == part) ++end;
            std::vector<std::pair<int64_t, const std::vector<int> *>> byL;
            for (auto jt = it; jt != end; ++jt) byL.push_back({jt->first.second, &jt->second});
            std::sort(byL.begin(), byL.end(), [](auto &a, auto &b) { return a.first > b.first; });
            for (auto &pl : byL) {
                const int slots = multi_slots((int)pl.first);
                const std::vector<int> &fs = *pl.second;
                for (size_t i = 0; i < fs.size(); i += slots)
                    for (int u = 0; u < kMultiSlots; ++u)
                        list.push_back(u < slots && i + u < fs.size() ? fs[i + u] : -1);
            }
            it = end;
        }
        while (k < st->nparts) g.lstart[++k] = (int)(list.size() / kMultiSlots);
        g.n = (int)(list.size() / kMultiSlots);
        chk(upload(st, &g.list, list));
        st->groups.push_back(g);
    }
    if (e != hipSuccess) {
        free_state(st);
        return fail_status(LC_ERR_HIP, whos + ": setup failed: " + hipGetErrorString(e));
    }
    chk(hipStreamCreateWithFlags(&st->side, hipStreamNonBlocking));
    for (int k = 0; k < kParts; ++k) chk(hipEventCreateWithFlags(&st->evq[k], hipEventDisableTiming));
    chk(hipEventCreateWithFlags(&st->evj, hipEventDisableTiming));
    if (e != hipSuccess) {
        free_state(st);
        return fail_status(LC_ERR_HIP, whos + ": stream/event setup: " + hipGetErrorString(e));
    }
    lc_plan_s *p = new (std::nothrow) lc_plan_s();
    if (!p) {
        free_state(st);
        return fail_status(LC_ERR_NOMEM, whos + ": host allocation failed");
    }
    p->kind = LC_PLAN_BATCH;
    hipGetDevice(&p->device);
    p->ext = st;
    p->workspace_bytes = st->ws_bytes;
    if (log_on()) {
        log_line("%s: B=%d sample bytes=%lld rules=%zu classes=%zu fused=%d+%d four-step=%zu parts=%d", who, B,
                 (long long)st->f_bytes, st->qs.size(), st->classes.size(), st->nfused[0], st->nfused[1],
                 st->large.size(), st->nparts);
        for (auto &qc : st->classes)
            log_line("  class R=%d %s: %zu functions, %lld rows, %d tiles; vec=%d G=%d cpl=%d unroll=%d grid=%d%s", qc.Q,
                     qc.prec == LC_FP64 ? "fp64" : "fp32", qc.fns.size(), (long long)qc.rows, qc.ntiles, qc.cfg.vec,
                     qc.cfg.G, qc.cfg.cpl, qc.cfg.unroll, qc.cfg.grid, qc.cfg.rpg == 2 ? " (row pairs)" : "");
        for (auto &g : st->groups)
            log_line("  DST group: %s T=%d Lmax=%d, %d %s", g.multi ? "packed" : "LDS", g.threads, g.Lmax, g.n,
                     g.multi ? "workgroups" : "functions");
    }
    *out = p;
    return LC_OK;
}

}  // namespace
}  // namespace lc

extern "C" {

lc_status lc_plan_batch_offsets(lc_plan_t p, int64_t *f_off, int64_t *x_off, int64_t *c_off) {
    if (!p || p->kind != LC_PLAN_BATCH) return fail_status(LC_ERR_INVALID, "lc_plan_batch_offsets: not a batch plan");
    BatchState *st = (BatchState *)p->ext;
    for (int b = 0; b < st->B; ++b) {
        if (f_off) f_off[b] = st->fn[b].f_off;
        if (x_off) x_off[b] = st->fn[b].x_off;
        if (c_off) c_off[b] = st->fn[b].c_off;
    }
    if (f_off) f_off[st->B] = st->f_bytes;
    if (x_off) x_off[st->B] = st->x_elems;
    if (c_off) c_off[st->B] = st->c_elems;
    return LC_OK;
}

lc_status lc_execute_batch(lc_plan_t p, const void *f_arena, double *c_arena, hipStream_t stream) {
    if (!p || p->kind != LC_PLAN_BATCH) return fail_status(LC_ERR_INVALID, "lc_execute_batch: not a batch plan");
    if (!f_arena || !c_arena) return fail_status(LC_ERR_INVALID, "lc_execute_batch: null arena");
    if (((uintptr_t)f_arena) & 255) return fail_status(LC_ERR_INVALID, "lc_execute_batch: f_arena must be 256-byte aligned");
    BatchState *st = (BatchState *)p->ext;
    hipError_t e;
    // Timed executions and executions on the null stream run eagerly; every
    // other execution replays the captured graph.
    if (p->timing || stream == nullptr) {
        e = launch_all(p, st, f_arena, c_arena, stream, p->timing);
        if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_batch: ") + hipGetErrorString(e));
        return LC_OK;
    }
    if (!st->gexec || st->gf != f_arena || st->gc != c_arena || st->gs != stream) {
        if (st->gexec) {
            hipGraphExecDestroy(st->gexec);
            st->gexec = nullptr;
        }
        if (st->graph) {
            hipGraphDestroy(st->graph);
            st->graph = nullptr;
        }
        e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_batch: begin capture: ") + hipGetErrorString(e));
        hipError_t el = launch_pipeline(st, f_arena, c_arena, stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(stream, &g);
        if (el != hipSuccess || e != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return fail_status(LC_ERR_HIP, std::string("lc_execute_batch: capture: ") +
                                               hipGetErrorString(el != hipSuccess ? el : e));
        }
        st->graph = g;
        e = hipGraphInstantiate(&st->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            st->gexec = nullptr;
            return fail_status(LC_ERR_HIP, std::string("lc_execute_batch: instantiate: ") + hipGetErrorString(e));
        }
        st->gf = f_arena;
        st->gc = c_arena;
        st->gs = stream;
    }
    e = hipGraphLaunch(st->gexec, stream);
    if (e != hipSuccess) return fail_status(LC_ERR_HIP, std::string("lc_execute_batch: graph launch: ") + hipGetErrorString(e));
    return LC_OK;
}

}  // extern "C"
