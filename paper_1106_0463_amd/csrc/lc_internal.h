// Internal declarations shared by the host runtime and the HIP kernels of
// the Legendre-coefficient library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/lc.h"

namespace lc {

// Longest complex FFT that one workgroup keeps resident in LDS
// (8192 complex doubles = 128 KiB of the 160 KiB per CU).
constexpr int kLdsFftMax = 8192;
constexpr int kMaxPasses = 24;

// Radix schedule of a Stockham FFT, passed to kernels by value.
struct FftSched {
    int n;                   // transform length
    int npass;
    int radix[kMaxPasses];
};

// Quadrature-reduction launch configuration.
struct QuadCfg {
    int vec;        // elements per lane load (16 B loads where the row allows)
    int G;          // lanes per row (power of two, <= 64)
    int cpl;        // chunks per lane (0: generic loop with bounds checks; -1: one
                    // 16-byte chunk per lane, lanes past Q/vec idle)
    int unroll;     // rows per row-group per iteration
    int block;      // threads per block
    int grid;       // blocks
    int Qv;         // Q (used by the batched generic kernel)
    int rpg = 1;    // rows per lane group: 1, or 2 (exact fit over row pairs,
                    // G * cpl * vec = 2 Q)
};

struct DstCfg {
    int threads;    // threads per workgroup of the LDS FFT kernels
    FftSched sched; // schedule for the whole length (single pass)
    int L1, L2;     // four-step split (L1 * L2 = L) when L > kLdsFftMax
    FftSched s1, s2;
};

// One function's worth of plan data (single plans use one; batch plans many).
struct FnDesc {
    int64_t N, M, M_eff, H, L;
    int32_t Q;
    int32_t prec;        // lc_precision
    int64_t f_off;       // byte offset in the sample arena (batch)
    int64_t x_off;       // element offset in the node arena (batch)
    int64_t c_off;       // element offset in the coefficient arena (batch)
    int64_t phi_off;     // element offset in the phi arena (batch)
    int32_t tw_id;       // index of its twiddle set (batch)
    int32_t w_id;        // index of its Gauss rule (batch)
};

// Device-side descriptor of a batch function (plain data for kernels).
struct BatchFn {
    int64_t f_off;     // bytes into the sample arena
    int64_t phi_off;   // elements into the phi arena
    int64_t c_off;     // elements into the coefficient arena
    int64_t N, H, L;
    const double *s2;  // 2 sin(y_j / 2), j = 1..H
    const double2 *tw_pre, *tw_pack, *tw_fft;
    FftSched sched;    // LDS schedule for L (when L <= kLdsFftMax)
};

// A function whose FFT exceeds the LDS: four-step form L = L1 * L2 with its
// own schedules and workspace (zA, zB: L complex each).
struct BigFn {
    int64_t H, L, N;
    int32_t L1, L2, CB, RB;
    int64_t phi_off, c_off;
    const double2 *tw_pre, *tw_pack, *tw_fft;
    double2 *zA, *zB;
    FftSched s1, s2;
};
// One block of a batched four-step pass: function index and first column
// (row) of the block.
struct BigTile {
    int32_t fn;
    int32_t first;
};

// Nodes [begin, end) (flat index r*Q + q) of one function of a batch.
struct NodeTile {
    double *x;
    const double2 *rowA, *omt2;
    int64_t begin, end;
    int32_t Q, pad;
};

// A run of rows of one function handled by one block of the batched
// quadrature kernel, resolved on the host: byte offset of its first row's
// samples in the sample arena, element offset of its first phi, the s2 of
// its first row, its row count, and the function (host bookkeeping).
struct BatchTile {
    int64_t f_off;
    int64_t phi_off;
    const double *s2;
    int32_t nrows;
    int32_t fn;
};

}  // namespace lc

struct lc_plan_s {
    int kind = LC_PLAN_SINGLE;
    int device = 0;
    lc::FnDesc fn{};
    // device buffers (single plans)
    double *x = nullptr;      // [H][Q] nodes
    double *w = nullptr;      // [Q] folded Gauss weights
    double2 *omt2 = nullptr;  // [Q] 1 - t_q^2 (double-double)
    double2 *rowA = nullptr;  // [H] 2 sin^2(y_j/2) (double-double)
    double *s2 = nullptr;     // [H] 2 sin(y_j / 2)
    double2 *tw_pre = nullptr, *tw_pack = nullptr, *tw_fft = nullptr;
    double *phi = nullptr;    // [H] workspace
    double2 *zA = nullptr, *zB = nullptr;  // [L] four-step workspace
    lc::QuadCfg quad{};
    lc::DstCfg dst{};
    bool fused_small = false;
    int fused_threads = 256;
    int64_t workspace_bytes = 0;
    // timing of the dominant kernel
    bool timing = false;
    std::vector<hipEvent_t> ev;  // pairs
    int ev_used = 0;
    // batch and GEMM plans keep their own state here
    void *ext = nullptr;
};

namespace lc {

// --- launchers (kernels_single.hip) ---------------------------------------
// One panel of one row of a composite Abel rule: q nodes (padded to qp, a
// multiple of 4) at element offset off of the sample array, with
// 1 - t = E + h d_i (d_i from the rule's node table at woff) and weights
// scale * w_i (the rule's padded weight table at woff).
struct ASeg {
    int64_t off;
    int32_t qp;
    int32_t woff;
    double scale;
    int32_t q;
    int32_t row;
    double2 E;
    double2 h;
};

// The same panel for the flattened row reduction: its first chunk (VEC
// samples) counted from the row's start, the weight-table chunk that row
// chunk 0 would map to (row chunk c of the panel takes weight chunk
// wbase + c) and the scale.
struct ATab {
    int32_t cst;
    int32_t wbase;
    double scale;
};
// A row of the flattened reduction, in launch order: samples from element
// rbeg, nc chunks, panels k0 .. k0 + S - 1 (S <= kAflatMaxSeg).
struct ARow {
    int64_t rbeg;
    int32_t r;
    int32_t nc;
    int32_t k0;
    int32_t S;
    int32_t pad[2];
};
constexpr int kAflatMaxSeg = 16;
// One launch of the flattened reduction over every lane count: entry j holds
// the rows of G = 64 >> j lanes per row, taken by blocks [b0[j], b0[j + 1]).
constexpr int kAflatLanes = 5;
struct AflatLaunch {
    const ARow *rows[kAflatLanes];
    int64_t nrows[kAflatLanes];
    int b0[kAflatLanes + 1];
};

// comp: write the complements 1 - x instead of the nodes
hipError_t launch_anodes(const ASeg *segs, int64_t nseg, const double2 *dtab, const double2 *rowA, double *x,
                         hipStream_t s, bool comp = false);
int aflat_blocks_per_cu(int prec);
hipError_t launch_aflat(int prec, const AflatLaunch &L, const void *f, const ATab *tab, const double *wtab,
                        const double *s2, double *phi, hipStream_t s);
int aquad_blocks_per_cu(int prec, int G);
hipError_t launch_aquad(int prec, int G, int grid, const void *f, const ASeg *segs, const int32_t *rseg,
                        const int32_t *rows, int64_t nrows, const double *wtab, const double *s2, double *phi,
                        hipStream_t s);
// dst[c][r] = src[r][c], R x C row-major FP64
hipError_t launch_transpose64(const double *src, int64_t R, int64_t C, double *dst, hipStream_t s);
// dst[r * n + i] = src[i], r < reps
hipError_t launch_repeat(const double *src, int64_t n, int64_t reps, double *dst, hipStream_t s);
hipError_t launch_nodes(int64_t H, int Q, const double2 *A, const double2 *B, double *x,
                        hipStream_t s, bool comp = false);
// comp: write 1 - x to comp at each node's offset from x_base instead
hipError_t launch_bnodes(const NodeTile *tiles, int64_t ntiles, hipStream_t s, const double *x_base = nullptr,
                         double *comp = nullptr);
hipError_t launch_quad(const QuadCfg &cfg, int prec, const void *f, const double *w,
                       const double *s2, int64_t rows, int Q, double *phi, hipStream_t s);
hipError_t launch_dst(const DstCfg &cfg, const double *phi, int64_t H, int64_t L, int64_t N,
                      const double2 *tw_pre, const double2 *tw_pack, const double2 *tw_fft,
                      double2 *zA, double2 *zB, double *c, hipStream_t s);
hipError_t launch_fused_small(int threads, int prec, const void *f, const double *w,
                              const double *s2, int64_t H, int Q, int64_t N, const FftSched &sch,
                              const double2 *tw_pre, const double2 *tw_pack,
                              const double2 *tw_fft, double *c, hipStream_t s);
bool quad_cfg_supported(const QuadCfg &cfg, int prec, int Q);
int quad_rows_per_block(const QuadCfg &cfg);

// --- batched launchers (kernels_batch.hip) ---------------------------------
hipError_t launch_bquad(const QuadCfg &cfg, int prec, const void *f_arena, const double *w,
                        const BatchTile *tiles, int ntiles, double *phi_arena,
                        hipStream_t s);
hipError_t launch_bdst(int threads, int Lmax, const double *phi_arena, const BatchFn *fns,
                       const int32_t *list, int nlist, double *c_arena, hipStream_t s);
hipError_t prepare_bdst(int threads, int Lmax);
// Short functions packed per 64-thread workgroup: kMultiSlots list entries
// per block (-1 = empty), all of one FFT length L <= kMultiMaxL, of which the
// first multi_slots(L) are used.
constexpr int kMultiSlots = 32;
constexpr int kMultiMaxL = 256;  // at least 2 functions per workgroup
__host__ __device__ inline int multi_slots(int L) {
    const int n = 512 / L;
    return n < kMultiSlots ? n : kMultiSlots;
}
hipError_t launch_bdst_multi(const double *phi_arena, const BatchFn *fns, const int32_t *list, int nblocks,
                             double *c_arena, hipStream_t s);
// Functions of at most kFuseHmax rows whose Q suits the fused kernel run
// quadrature, twist, FFT and rescale in one workgroup; one launch per
// sample precision (list: n entries, Hmax their largest H).
constexpr int64_t kFuseHmax = 2048;
struct FusedFn {
    int32_t fn;        // function (index into the BatchFn table)
    int32_t Q;         // samples per row
    int32_t G;         // lanes per row (fuse_lanes)
    int32_t pad;
    const double *w;   // the rule's weights [Q]
};
int fuse_lanes(int prec, int Q);  // lanes per row of the fused kernel, 0 if Q does not suit it
hipError_t launch_bfused(int prec, const void *f_arena, const BatchFn *fns, const FusedFn *list, int n, int64_t Hmax,
                         double *c_arena, hipStream_t s);
hipError_t launch_bbig(const double *phi_arena, const BigFn *fns, const BigTile *ctiles, int nct,
                       const BigTile *rtiles, int nrt, const BigTile *ptiles, int npt, double *c_arena,
                       hipStream_t s);
int four_step_blocks(int L1, int L2, int *CB, int *RB);
size_t fused_small_lds_bytes(int64_t H, int Q);

// --- host helpers (host.cpp) ---------------------------------------------
void set_error(const std::string &msg);
hipError_t device_alloc(void **p, size_t bytes);  // hipMalloc behind the LC_ALLOC_LIMIT test hook
bool log_on();                                   // LC_LOG=1
void log_line(const char *fmt, ...);             // one "[lc] ..." line on stderr when LC_LOG=1
std::string sched_str(const FftSched &s);        // "8x8x4" 
int64_t smooth_len_at_least(int64_t L);           // smallest 2^a 3^b 5^c >= L, c <= 1
FftSched make_sched(int L, const int *order = nullptr);
void gauss_half_rule(int Q, std::vector<double> &t, std::vector<double> &w,
                     std::vector<double2> &omt2);
void row_factors(int64_t H, std::vector<double2> &A, std::vector<double> &s2);
void gauss_positive_half_ld(int n, std::vector<long double> &x, std::vector<long double> &w);
long double row_half_sine(int64_t j, int64_t H);  // sin(pi j / (2H))
double2 dd_split(long double v);
void twiddles(int64_t H, std::vector<double2> &pre, std::vector<double2> &pack,
              std::vector<double2> &fft);
QuadCfg default_quad_cfg(int prec, int Q, int64_t rows, int num_cu);
// the batch's exact fit over row pairs for (prec, Q) into out (grid kept);
// false when 2Q does not split into whole 16-byte chunks of a built shape
bool pair_quad_cfg(int prec, int Q, QuadCfg &out);
// resident blocks per CU of the quadrature variant cfg selects (single
// plans / batch plans; cfg.Qv must hold Q); 0 if unknown
int quad_blocks_per_cu(const QuadCfg &cfg, int prec);
int bquad_blocks_per_cu(const QuadCfg &cfg, int prec);
DstCfg default_dst_cfg(int64_t L);
int dst_threads_for(int64_t L);   // smallest of 64 .. 1024 with L <= 8 T
bool dst_threads_ok(int T);       // a built LDS FFT workgroup size
DstCfg four_step_cfg(int64_t L);
int device_cu_count();

// --- autotuner helpers (autotune.cpp) --------------------------------------
std::string arch_name();
bool cache_get(const std::string &key, std::string &val);
void cache_put(const std::string &key, const std::string &val);
std::string quad_to_str(const QuadCfg &c);
bool quad_from_str(const std::string &s, QuadCfg &c);
std::vector<QuadCfg> quad_candidates(int prec, int Q, int64_t rows, int cu, bool batch);
std::vector<FftSched> sched_candidates(int L);
double time_launch(const std::function<hipError_t(hipStream_t)> &f, hipStream_t s, int reps, hipError_t *err);

}  // namespace lc
