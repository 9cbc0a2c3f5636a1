/*
 * lc.h -- C ABI of the MI355X (gfx950) implementation of the Legendre-
 * coefficient method of E. De Micheli and G. A. Viano, "A new and efficient
 * method for the computation of Legendre coefficients", arXiv 1106.0463.
 *
 * Problem (Section 2, eqs. (2.1) and (2.3)): given f summable on [-1, 1],
 * compute
 *     c_n = (n + 1/2) * integral_{-1}^{1} f(x) P_n(x) dx,   n = 0 .. N-1.
 *
 * Method (Theorem 1, eqs. (2.4), (2.5), (2.12)-(2.14)): a_n = c_n / (2n+1)
 * are the Fourier coefficients (n >= 0) of the Abel-type transform
 *     fhat(y) = (1/(2 pi i)) eps(y) e^{i y/2} phi(|y|),
 *     phi(y)  = integral_{cos y}^{1} f(x) / sqrt(2 (x - cos y)) dx.
 * The library evaluates phi on the grid y_j = pi j / H (j = 1..H, H = M/2)
 * after the change of variable x = cos y + 2 sin^2(y/2) t^2, which turns the
 * end-point singularity into a smooth integrand, with the positive half of
 * the 2Q-point Gauss-Legendre rule in t:
 *     phi_j = 2 s_j * sum_{q<Q} w_q f(x_{jq}),
 *     x_{jq} = 1 - 2 s_j^2 (1 - t_q^2) = cos y_j + 2 sin^2(y_j/2) t_q^2,
 *     s_j = sin(y_j / 2),
 * (exact for polynomial f of degree <= 2Q-1), then applies the twist and the
 * one FFT of eq. (2.4) (as a DST-III of length H computed with a complex FFT
 * of length H/2) and the rescale c_n = (2n+1) a_n.  For real f only
 * y in (0, pi] needs Abel integrals: fhat(-y) follows from eq. (2.12).
 *
 * Conventions for every entry point:
 *  - Return value is an lc_status; LC_OK (0) on success.  On error nothing
 *    is written to out-parameters and lc_last_error() (thread-local) holds a
 *    message.  No C++ exception crosses this interface.
 *  - "device pointer": memory on the current HIP device (hipMalloc or a
 *    torch CUDA/HIP tensor).  "host pointer": ordinary process memory.
 *  - Execute calls are asynchronous on the given stream: they enqueue work
 *    and return without synchronizing; faults inside kernels surface at the
 *    caller's next synchronization.  They allocate nothing.
 *  - A plan is bound to the device that was current when it was created and
 *    owns all of its device buffers (nodes, weights, twiddles, workspace).
 *    One plan must not be executed concurrently from two streams (the
 *    workspace is per plan); distinct plans are independent.
 */
#ifndef LC_H
#define LC_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LC_OK = 0,
    LC_ERR_INVALID = 1,      /* bad argument (sizes, null pointer, wrong plan kind) */
    LC_ERR_NOMEM = 2,        /* device or host allocation failed                   */
    LC_ERR_HIP = 3,          /* a HIP runtime call or kernel launch failed          */
    LC_ERR_UNSUPPORTED = 4,  /* valid request outside what this library implements */
    LC_ERR_INTERNAL = 5
} lc_status;

/* Sample / accumulation precision of a request. */
typedef enum {
    LC_FP64 = 0,       /* f samples FP64; Abel sums, twist, FFT, rescale FP64   */
    LC_FP32_QUAD = 1   /* f samples FP32 (half the bytes); everything after the
                          load (Abel sums, FFT, rescale) in FP64                */
} lc_precision;

/* Arithmetic of the Abel-as-GEMM form (product-integration matrix times
 * samples).  Split modes write each FP64 operand as a sum of 16-bit pieces
 * and accumulate the piece products on MFMA in FP32.  Accuracy on
 * a_n = c_n / (2n+1), E_a = max|da| / max|a|: FP16X3 and BF16X6 hold
 * E_a <= 1e-7; BF16X3 (~1.2e-7 at P = 4096) and FP16X1 (~1e-5) do not, the
 * limit of their two and one 16-bit pieces. */
typedef enum {
    LC_GEMM_FP64 = 0,    /* FP64 product (reference arithmetic)                   */
    LC_GEMM_BF16X3 = 1,  /* A=Ah+Al, F=Fh+Fl (bf16): Ah Fh + Ah Fl + Al Fh        */
    LC_GEMM_BF16X6 = 2,  /* three bf16 pieces each: the six products of order <=2 */
    LC_GEMM_FP16X3 = 3,  /* power-of-two-scaled fp16 pieces: three products       */
    LC_GEMM_FP16X1 = 4   /* one scaled fp16 piece each: one product                */
} lc_gemm_mode;

typedef enum {
    LC_PLAN_SINGLE = 0,
    LC_PLAN_BATCH = 1,
    LC_PLAN_GEMM = 2,            /* Abel product + batched twist/FFT/rescale     */
    LC_PLAN_LEGENDRE_MATRIX = 3, /* one product with the full N x P matrix       */
    LC_PLAN_ADAPTIVE = 4,        /* single function, composite Abel rule         */
    LC_PLAN_2D = 5               /* two-dimensional tensor-product transform     */
} lc_plan_kind;

/* Composite Abel rule of an adaptive plan (lc_plan_adaptive).  With
 * x = 1 - 2 s^2 (1 - t^2), s = sin(y/2), eq. (2.14) reads
 * phi(y) = 2 s integral_0^1 f dt; the rule cuts t in [0, 1] into panels:
 *   - each breakpoint b with cos y < b < 1 (a point where f or a derivative
 *     of f jumps, e.g. x = 0 for |x|^{3/2}) becomes the cut whose node is
 *     x = b;
 *   - grade_levels > 0 with 0 < grade_ratio < 1 adds the cuts
 *     1 - t = grade_ratio^k, k = 1..grade_levels (panels shrinking toward
 *     x = 1, for f singular just beyond x = 1);
 * cuts closer than 1e-12 (relative, in 1 - t) merge, and cuts at t <= 1e-7
 * (a breakpoint within ~1e-14 of cos y) are dropped.  The first panel uses
 * the positive half of the 2q-point Gauss-Legendre rule (the integrand is
 * even in t there), the others the q-point rule.  Node count of a panel
 * [t_lo, t_hi]:
 *   band == 0: q;
 *   band  > 0: min(q_max, ladder(q + ceil(g))), g = G + 6.5 G^{1/3},
 *              G = (band s^2 / 2) (t_hi^2 - t_lo^2),
 *              for f band-limited to degree ~band: about band s^2 / 2 nodes
 *              per row (instead of a uniform band / 2), shared among the
 *              panels in proportion to the phase of cos(band x) they cover;
 *              ladder() rounds up to a multiple of 8 up to 128 and to 16
 *              steps per octave above.
 * Limits: 1 <= q <= 65536; q (band = 0) or q_max (band > 0, q_max >= q)
 * even whenever cuts are requested; nbreak <= 64, breaks in (-1, 1);
 * grade_levels <= 64. */
typedef struct {
    int32_t q;             /* nodes per panel, or the base count when band > 0 */
    int32_t q_max;         /* cap of the per-row count (band > 0)              */
    double band;           /* 0, or the degree f is band-limited to            */
    int32_t nbreak;        /* number of breakpoints                            */
    const double *breaks;  /* host array of nbreak values (may be null if 0)   */
    double grade_ratio;    /* 0, or the grading ratio in (0, 1)                */
    int32_t grade_levels;  /* number of graded cuts                            */
} lc_abel_rule;

typedef struct lc_plan_s *lc_plan_t;

typedef struct {
    int32_t kind;        /* lc_plan_kind                                         */
    int32_t precision;   /* lc_precision (single plans) / lc_gemm_mode (GEMM)    */
    int64_t N;           /* coefficients returned (single / GEMM plans)          */
    int64_t M;           /* y-grid size requested                                */
    int64_t M_eff;       /* y-grid size used (see lc_grid_size)                  */
    int64_t H;           /* M_eff / 2: rows of the node array                    */
    int32_t Q;           /* Abel nodes per row (single); P sample nodes (GEMM)   */
    int32_t B;           /* functions (batch plans), 0 otherwise                 */
    int64_t samples;     /* f samples the caller provides per execute           */
    int64_t sample_bytes;/* bytes of those samples                               */
    int64_t workspace_bytes; /* device bytes owned by the plan                   */
} lc_plan_desc;

/* Size rule for the y-grid (host only, no device work).  The FFT of eq. (2.4)
 * is computed as a complex FFT of length H/2; this library supports lengths
 * 2^a 3^b 5^c.  M_eff is the smallest M' >= max(M, 4) with M' = 4 * 2^a 3^b 5^c
 * and c <= 1 (at most one radix-5 pass, whose rounding exceeds the others').
 * Using M_eff >= M only refines the trapezoid grid of eq. (2.4).
 * Errors: LC_ERR_INVALID if M < 2 or M_eff is null or the size overflows. */
lc_status lc_grid_size(int64_t M, int64_t *M_eff);

/* Single-function plan (eq. (2.4) on the M-point grid, Q Abel nodes).
 * N >= 1, M even >= 2, N <= M/2, 1 <= Q <= 65536, prec in lc_precision.
 * Builds on the current device: the Gauss rule (host, long double), the
 * nodes x_{jq} (device, FP64, half-angle form), FFT twiddles (host, long
 * double with exact integer argument reduction, stored FP64) and a
 * workspace.  *out is written only on success.
 * Errors: LC_ERR_INVALID, LC_ERR_NOMEM, LC_ERR_HIP. */
lc_status lc_plan(int64_t N, int64_t M, int32_t Q, lc_precision prec, lc_plan_t *out);

/* Single-function plan with the composite Abel rule *rule (see
 * lc_abel_rule) in place of the uniform Q-point rule; N, M and prec as in
 * lc_plan.  The nodes are one flat FP64 array (lc_plan_nodes: rows = the
 * number of samples, Q = 1): rows j = 1..M_eff/2 in order, a row's panels in
 * order of increasing t, every panel padded to a multiple of 4 samples
 * (padding repeats the panel's last node and has weight 0); nodes are the
 * correctly rounded values of 1 - 2 s_j^2 (1 - t^2).  Executed with
 * lc_execute on samples in that layout.
 * Errors: LC_ERR_INVALID (bad rule or sizes), LC_ERR_NOMEM, LC_ERR_HIP,
 * LC_ERR_UNSUPPORTED (too many samples). */
lc_status lc_plan_adaptive(int64_t N, int64_t M, const lc_abel_rule *rule, lc_precision prec, lc_plan_t *out);

/* Two-dimensional tensor-product plan, the extension of the method to
 * functions on the square:
 *   c[n1][n2] = (n1 + 1/2)(n2 + 1/2) integral integral f(x1, x2) P_n1(x1) P_n2(x2),
 * n1, n2 < N, by the one-dimensional method (eq. (2.4) with the Abel rule of
 * a single plan (N, M, Q)) along x1 for every sample point of x2, then along
 * x2 for every n1.  Both axes use the S = H Q nodes X of that single plan
 * (lc_plan_nodes: x[H][Q], flattened as X_a, a = 0..S-1).  The caller
 * samples F[b][a] = f(X_a, X_b) (S x S row-major, FP64 or FP32 per prec).
 * Limits: those of lc_plan, M/4 <= 8192, S <= 2e6 and S^2 <= 4e10.
 * Errors: as lc_plan; LC_ERR_UNSUPPORTED beyond the limits. */
lc_status lc_plan_2d(int64_t N, int64_t M, int32_t Q, lc_precision prec, lc_plan_t *out);

/* Executes a 2-D plan: F_dev the S x S samples (16-byte aligned), C_dev an
 * N x N FP64 array (row n1, column n2).  Asynchronous on stream.
 * Errors: LC_ERR_INVALID, LC_ERR_HIP. */
lc_status lc_execute_2d(lc_plan_t plan, const void *F_dev, double *C_dev, hipStream_t stream);

/* Describes any plan.  Errors: LC_ERR_INVALID on null arguments. */
lc_status lc_plan_info(lc_plan_t plan, lc_plan_desc *desc);

/* Device pointer to the sample nodes, owned by the plan and valid until
 * lc_plan_destroy.  Single plans: x[H][Q] row-major FP64, row r holds
 * y_{r+1} = pi (r+1)/H; the caller writes f(x[r][q]) into f[r][q].
 * Batch plans: the node arena, function b at element offset x_off[b] (see
 * lc_plan_batch_offsets), laid out like a single plan.  GEMM and
 * Legendre-matrix plans: the P Chebyshev-Gauss nodes x_p = cos((2p+1) pi / (2P)).
 * rows / Q may be null.  Errors: LC_ERR_INVALID. */
lc_status lc_plan_nodes(lc_plan_t plan, const double **x_dev, int64_t *rows, int32_t *Q);

/* Complements of the nodes: writes 1 - x for every node of a single,
 * adaptive or batch plan into omx_dev (device FP64, the node array's layout
 * and length: H*Q, the sample count, or the node arena), each the FP64 value
 * nearest 2 s_j^2 (1 - t^2) (computed in double-double).  Near x = 1 the
 * FP64 node x carries an absolute rounding error of up to 2^-53 that is
 * large relative to 1 - x; a caller sampling f with a singularity just
 * beyond x = 1 (e.g. (1 - 2xt + t^2)^{-1/2} = ((1-t)^2 + 2t(1-x))^{-1/2} with
 * t near 1) evaluates f from 1 - x instead, at the same node.  Asynchronous
 * on stream.  Errors: LC_ERR_INVALID (null argument), LC_ERR_UNSUPPORTED
 * (other plan kinds), LC_ERR_HIP. */
lc_status lc_plan_nodes_complement(lc_plan_t plan, double *omx_dev, hipStream_t stream);

/* Executes a single plan: f_dev is the device array of samples f[H][Q]
 * (FP64, or FP32 for LC_FP32_QUAD), c_dev a device array of N doubles that
 * receives c_0..c_{N-1}.  Asynchronous on stream (0 = null stream); no
 * allocation, no host synchronization.  f_dev must be 16-byte aligned.
 * Errors: LC_ERR_INVALID (null pointer, wrong plan kind, misaligned f_dev),
 * LC_ERR_HIP (launch failure). */
lc_status lc_execute(lc_plan_t plan, const void *f_dev, double *c_dev, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * execute call of a single plan (lc_plan or lc_plan_adaptive) whose
 * workspace -- phi[H] and, when H/2 > 8192, two four-step buffers of H/2
 * complex values -- lives in one static device array of the library
 * (LC_NOALLOC_SCRATCH_BYTES per device, held from the first call on that
 * device until the process ends) instead of the plan's workspace.  Same
 * arguments, kernels and results (bit for bit) as lc_execute; it calls no
 * allocation routine and records no timing events.  The plan needs
 * 8 H bytes (H/2 <= 8192) or 8 H + 32 (H/2) bytes, each part rounded up to
 * 256 bytes; larger plans are rejected.  The current device must be the
 * plan's.  Every call on one device shares that device's array: calls that
 * overlap in time on one device (two streams, or two threads) race and give
 * wrong results; calls ordered on one stream are safe.  Nothing in the
 * array needs clearing between calls (every value is written before it is
 * read).
 * Errors: LC_ERR_INVALID (as lc_execute; a plan larger than the array; the
 * current device is not the plan's), LC_ERR_HIP (symbol lookup or launch
 * failure), LC_ERR_UNSUPPORTED (device ordinal >= 64). */
#define LC_NOALLOC_SCRATCH_BYTES (8u << 20)
lc_status lc_execute_noalloc(lc_plan_t plan, const void *f_dev, double *c_dev, hipStream_t stream);

/* Batched plan for B independent functions of uneven sizes (N[b], M[b],
 * Q[b], prec[b], host arrays of length B, each entry validated as in
 * lc_plan).  Samples live in one device arena (byte offsets f_off, every
 * function 256-byte aligned, FP64 or FP32 per prec[b]); coefficients in one
 * FP64 arena (element offsets c_off).  Execution is a fixed sequence of
 * kernels captured once into a HIP graph on the first lc_execute_batch and
 * replayed afterwards.  Errors: LC_ERR_INVALID, LC_ERR_NOMEM, LC_ERR_HIP. */
lc_status lc_plan_batch(int32_t B, const int64_t *N, const int64_t *M, const int32_t *Q,
                        const lc_precision *prec, lc_plan_t *out);

/* Batched plan with a composite Abel rule per function (the remarks after
 * eq. (2.14): a change of variable and Gauss-Legendre panels), for batches
 * that mix smooth functions with functions singular just beyond x = 1
 * (e.g. the generating function eq. (2.2) with t near 1).  rules[b] follows
 * lc_abel_rule with the batch's restriction that every row has the same
 * panels: band = 0 and nbreak = 0 (LC_ERR_UNSUPPORTED otherwise); grading
 * (grade_ratio, grade_levels) and the node count q are free per function,
 * except that every cut grade_ratio^k must be kept by the cut rule of
 * lc_abel_rule (none at or below 1e-15, none merged: LC_ERR_INVALID
 * otherwise).  Function b has R_b = (grade_levels + 1) * (q rounded up to a
 * multiple of 4) samples per row (grade_levels = 0 when grade_ratio = 0), in the
 * row layout of lc_plan_adaptive with the same rule (panels by increasing t,
 * each padded to a multiple of 4 with the last node repeated at weight 0),
 * rows j = 1..M_eff/2 in order: [H_b][R_b].  Everything else -- arenas,
 * offsets (lc_plan_batch_offsets), nodes (lc_plan_nodes), execution
 * (lc_execute_batch), autotuning, timing -- is that of lc_plan_batch.
 * Limits: those of lc_plan_batch with Q = R_b <= 65536.
 * Errors: LC_ERR_INVALID, LC_ERR_UNSUPPORTED, LC_ERR_NOMEM, LC_ERR_HIP. */
lc_status lc_plan_batch_rules(int32_t B, const int64_t *N, const int64_t *M, const lc_abel_rule *rules,
                              const lc_precision *prec, lc_plan_t *out);

/* Host copies of the batch layout, each array of length B+1 (may be null):
 * f_off  byte offset of function b's samples in the f arena (f_off[B] =
 *        arena bytes);
 * x_off  element offset (doubles) of its nodes in the node arena;
 * c_off  element offset (doubles) of its coefficients in the c arena.
 * Errors: LC_ERR_INVALID (not a batch plan). */
lc_status lc_plan_batch_offsets(lc_plan_t plan, int64_t *f_off, int64_t *x_off, int64_t *c_off);

/* Executes a batch plan (graph replay on stream).  f_arena: device arena of
 * samples (layout of lc_plan_batch_offsets), c_arena: device FP64 arena.
 * Pointers must be 256-byte aligned.  The first call on a given
 * (f_arena, c_arena, stream) triple captures the graph; a call with other
 * pointers re-captures it.  Errors: LC_ERR_INVALID, LC_ERR_HIP. */
lc_status lc_execute_batch(lc_plan_t plan, const void *f_arena, double *c_arena, hipStream_t stream);

/* Abel-as-GEMM plan: functions sampled on the fixed P-point Chebyshev-Gauss
 * grid.  The Abel step becomes phi = A F with the product-integration matrix
 * A[j][p] = integral_{cos y_j}^{1} l_p(x) / sqrt(2 (x - cos y_j)) dx
 * (l_p the Lagrange cardinal polynomial of node p; exact for f of degree
 * < P), built in FP64 on the device.  Then the twist/FFT/rescale of a
 * single plan, batched over the functions.  2 <= P <= 16384, M even with
 * M/2 >= N, N >= 1.  Errors: LC_ERR_INVALID, LC_ERR_NOMEM, LC_ERR_HIP. */
lc_status lc_plan_gemm(int32_t P, int64_t M, int64_t N, lc_gemm_mode mode, lc_plan_t *out);

/* Direct Legendre-matrix plan on the same fixed grid.  For a fixed grid the
 * whole map from samples to coefficients (Abel step, twist, the FFT of
 * eq. (2.4) and the (2n+1) rescale) is linear, i.e. one N x P matrix
 *   Lmat = D A,
 * with A the product-integration matrix above and D the map phi -> c of
 * eq. (2.4) on the M-point grid.  Lmat is built once in FP64 on the device
 * by applying the plan's FP64 twist/DST/rescale to the columns of A, so
 * that it equals the Legendre coefficients of the Lagrange cardinal
 * polynomials of the grid whenever the method is exact for them
 * (M >= N + P).  Each execute is then a single product C = F^T Lmat^T,
 * with no FFT; the split modes accumulate the piece products in FP32 on
 * MFMA and write finished FP64 coefficients.  The plan is executed, sized
 * and destroyed with the GEMM calls (lc_execute_gemm, lc_plan_gemm_reserve,
 * lc_plan_destroy); lc_plan_info reports kind LC_PLAN_LEGENDRE_MATRIX.
 * Arguments and errors as lc_plan_gemm. */
lc_status lc_plan_legendre_matrix(int32_t P, int64_t M, int64_t N, lc_gemm_mode mode, lc_plan_t *out);

/* Executes a GEMM plan on B functions: F_dev device FP64 [P][B] (row p holds
 * f_b(x_p) for every b), C_dev device FP64 [B][N].  B <= the plan's
 * capacity (lc_plan_gemm_reserve, default 16384).  Asynchronous on stream.
 * Errors: LC_ERR_INVALID, LC_ERR_HIP. */
lc_status lc_execute_gemm(lc_plan_t plan, const double *F_dev, int32_t B, double *C_dev,
                          hipStream_t stream);

/* Sets the largest B a GEMM plan accepts (allocates its workspace).
 * Errors: LC_ERR_INVALID, LC_ERR_NOMEM. */
lc_status lc_plan_gemm_reserve(lc_plan_t plan, int32_t B_max);

/* Device pointer to the GEMM plan's FP64 matrix, valid until destroy:
 * the product-integration matrix A, [H+1][P] row-major (row 0, y = 0, is
 * zero), for lc_plan_gemm plans; the transposed Legendre matrix Lmat^T,
 * [P][N] row-major, for lc_plan_legendre_matrix plans.
 * Errors: LC_ERR_INVALID. */
lc_status lc_plan_gemm_matrix(lc_plan_t plan, const double **A_dev);

/* Times the plan's kernel variants (quadrature lanes per row and rows per
 * block, FFT radix schedule and threads; for adaptive plans the largest
 * lane group of the segmented reduction) on the plan's own buffers and
 * keeps the fastest; results persist in the file named by LC_AUTOTUNE_CACHE
 * (if set), keyed by device architecture and the plan's shape.  GEMM plans
 * have one launch shape: LC_OK.  Synchronizes stream.
 * Errors: LC_ERR_INVALID, LC_ERR_HIP, LC_ERR_NOMEM. */
lc_status lc_autotune(lc_plan_t plan, hipStream_t stream);

/* Frees the plan and all of its device memory (synchronizes the device
 * first).  A null plan is accepted.  Returns LC_OK. */
lc_status lc_plan_destroy(lc_plan_t plan);

/* Static string for a status code. */
const char *lc_status_string(lc_status s);

/* Message of the last error on the calling thread ("" if none). */
const char *lc_last_error(void);

/* Kernel timing of the plan's dominant kernel (the Abel quadrature
 * reduction for single and batch plans, the MFMA product for GEMM plans).
 * lc_plan_set_timing(plan, 1) starts recording a pair of HIP events around
 * that kernel, on the execute stream, at every execute (up to 4096 executes;
 * later ones are not recorded); enable = 0 stops and discards the record.
 * lc_plan_kernel_ms synchronizes the recorded events and returns the mean
 * kernel duration in milliseconds over the recorded executes and their
 * number.  Errors: LC_ERR_INVALID (null arguments, timing disabled or
 * nothing recorded), LC_ERR_HIP. */
lc_status lc_plan_set_timing(lc_plan_t plan, int32_t enable);
lc_status lc_plan_kernel_ms(lc_plan_t plan, double *avg_ms, int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* LC_H */
