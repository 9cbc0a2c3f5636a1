/*
 * CPU oracle for the Legendre-coefficient method of De Micheli & Viano,
 * "A new and efficient method for the computation of Legendre coefficients"
 * (arXiv 1106.0463).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * Everything is plain long double (x87 80-bit) with straightforward loops:
 *
 *   oracle_gauss_legendre   the K-point Gauss-Legendre rule on [-1,1], by
 *                           Newton iteration on P_K (textbook construction).
 *   oracle_legendre_coeffs  the definition, eq. (2.3):
 *                           c_n = (n+1/2) * integral_{-1}^{1} f(x) P_n(x) dx,
 *                           evaluated as (n+1/2) * sum_k w_k f(x_k) P_n(x_k)
 *                           with the three-term recurrence for P_n
 *                           (the O(N^2) "standard quadrature" the paper's
 *                           introduction names as the slow baseline).
 *   oracle_fourier_coeffs   the Fourier coefficient of eq. (2.4),
 *                           a_n = integral_{-pi}^{pi} fhat(y) e^{i n y} dy,
 *                           as a plain M-point trapezoid sum over a uniform
 *                           periodic grid y_j = -pi + 2*pi*j/M (no FFT).
 *
 * Parallel loops use OpenMP with a static schedule and a fixed-order final
 * reduction, so a given thread count gives bit-identical results.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef long double ld;

static const ld PI_L = 3.141592653589793238462643383279502884L;

/* P_K(x) and P_{K-1}(x) by the three-term recurrence
 * (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1},  P_0 = 1, P_1 = x. */
static void legendre_pair(long K, ld x, ld *pk, ld *pkm1)
{
    ld p0 = 1.0L, p1 = x;
    if (K == 0) { *pk = 1.0L; *pkm1 = 0.0L; return; }
    for (long n = 1; n < K; ++n) {
        ld p2 = ((ld)(2 * n + 1) * x * p1 - (ld)n * p0) / (ld)(n + 1);
        p0 = p1;
        p1 = p2;
    }
    *pk = p1;
    *pkm1 = p0;
}

/* K-point Gauss-Legendre rule: nodes are the zeros of P_K, weights
 * w_k = 2 / ((1 - x_k^2) P_K'(x_k)^2), with
 * P_K'(x) = K (x P_K(x) - P_{K-1}(x)) / (x^2 - 1) (Newton steps).
 * Nodes are returned in decreasing order; the rule is made exactly
 * symmetric by computing the upper half and mirroring it.
 * Returns 0 on success, -1 on bad K, -2 if Newton failed to converge. */
int oracle_gauss_legendre(long K, ld *x, ld *w)
{
    if (K < 1 || !x || !w) return -1;
    long half = (K + 1) / 2;
    int failed = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : failed)
    for (long k = 0; k < half; ++k) {
        /* initial guess for the (k+1)-th largest zero */
        ld xi = cosl(PI_L * ((ld)k + 0.75L) / ((ld)K + 0.5L));
        ld pk, pkm1, dp, prev = 1.0L;
        int it, ok = 0;
        for (it = 0; it < 100; ++it) {
            legendre_pair(K, xi, &pk, &pkm1);
            dp = (ld)K * (xi * pk - pkm1) / (xi * xi - 1.0L);
            ld dx = pk / dp;
            xi -= dx;
            /* relative test, with an absolute floor for the node at x = 0 of
             * odd K (nodes are ~pi/K apart, so 1e-3 is far below spacing) */
            if (fabsl(dx) <= 4.0L * LDBL_EPSILON * fmaxl(fabsl(xi), 1e-3L)) { ok = 1; break; }
            /* quadratic convergence has stopped: the step is at the rounding
             * level of P_K (grows like K eps near the ends) */
            if (it >= 3 && fabsl(dx) > 0.25L * prev && fabsl(dx) < 1e-15L) { ok = 1; break; }
            prev = fabsl(dx);
        }
        /* weight at the converged node, with P_K' from the same recurrence
         * (the rounding errors of P_K and P_{K-1} are correlated and cancel
         * in x P_K - P_{K-1}; the shortcut P_K' = K P_{K-1}/(1-x^2) that
         * assumes P_K(x_k) = 0 loses ~1e-12 at the outermost nodes) */
        legendre_pair(K, xi, &pk, &pkm1);
        dp = (ld)K * (xi * pk - pkm1) / (xi * xi - 1.0L);
        if (!ok) failed |= 1;
        ld wk = 2.0L / ((1.0L - xi * xi) * dp * dp);
        x[k] = xi;
        w[k] = wk;
        x[K - 1 - k] = -xi;
        w[K - 1 - k] = wk;
    }
    if (K % 2 == 1) x[K / 2] = 0.0L; /* exact zero of odd-degree P_K */
    return failed ? -2 : 0;
}

/* Definition (2.3): c_n = (n + 1/2) sum_k w_k f_k P_n(x_k), n = 0..N-1.
 * f holds f(x_k) at the caller's nodes.  Returns 0, or -1 on bad args,
 * -3 on allocation failure. */
int oracle_legendre_coeffs(long K, const ld *x, const ld *w, const ld *f,
                           long N, ld *c)
{
    if (K < 1 || N < 1 || !x || !w || !f || !c) return -1;
    int nt = omp_get_max_threads();
    ld *part = (ld *)calloc((size_t)nt * (size_t)N, sizeof(ld));
    if (!part) return -3;
#pragma omp parallel num_threads(nt)
    {
        ld *acc = part + (size_t)omp_get_thread_num() * (size_t)N;
#pragma omp for schedule(static)
        for (long k = 0; k < K; ++k) {
            ld wf = w[k] * f[k];
            ld xk = x[k];
            ld p0 = 1.0L, p1 = xk;
            acc[0] += wf * p0;
            if (N > 1) acc[1] += wf * p1;
            for (long n = 1; n + 1 < N; ++n) {
                ld p2 = ((ld)(2 * n + 1) * xk * p1 - (ld)n * p0) / (ld)(n + 1);
                acc[n + 1] += wf * p2;
                p0 = p1;
                p1 = p2;
            }
        }
    }
    for (long n = 0; n < N; ++n) {
        ld s = 0.0L;
        for (int t = 0; t < nt; ++t) s += part[(size_t)t * (size_t)N + (size_t)n];
        c[n] = ((ld)n + 0.5L) * s;
    }
    free(part);
    return 0;
}

/* Trapezoid form of (2.4) on the periodic grid y_j = -pi + 2 pi j / M,
 * j = 0..M-1:   a_n = (2 pi / M) sum_j fhat_j e^{i n y_j},  n = 0..N-1.
 * Angles are reduced exactly in integers:
 *   n y_j = -n pi + 2 pi (n j mod M) / M,   e^{-i n pi} = (-1)^n.
 * Returns 0, -1 on bad args, -3 on allocation failure. */
int oracle_fourier_coeffs(long M, const ld *fhat_re, const ld *fhat_im,
                          long N, ld *a_re, ld *a_im)
{
    if (M < 1 || N < 1 || !fhat_re || !fhat_im || !a_re || !a_im) return -1;
    ld *cs = (ld *)malloc((size_t)M * sizeof(ld));
    ld *sn = (ld *)malloc((size_t)M * sizeof(ld));
    if (!cs || !sn) { free(cs); free(sn); return -3; }
    for (long m = 0; m < M; ++m) {
        ld ang = 2.0L * PI_L * (ld)m / (ld)M;
        cs[m] = cosl(ang);
        sn[m] = sinl(ang);
    }
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        ld sr = 0.0L, si = 0.0L;
        long nm = n % M;
        long idx = 0; /* (n * j) mod M, advanced incrementally */
        for (long j = 0; j < M; ++j) {
            ld er = cs[idx], ei = sn[idx];
            sr += fhat_re[j] * er - fhat_im[j] * ei;
            si += fhat_re[j] * ei + fhat_im[j] * er;
            idx += nm;
            if (idx >= M) idx -= M;
        }
        ld sign = (n % 2 == 0) ? 1.0L : -1.0L;
        a_re[n] = sign * (2.0L * PI_L / (ld)M) * sr;
        a_im[n] = sign * (2.0L * PI_L / (ld)M) * si;
    }
    free(cs);
    free(sn);
    return 0;
}

/* The same sum for a list of indices n = idx[i] (sampled outputs). */
int oracle_fourier_coeffs_idx(long M, const ld *fhat_re, const ld *fhat_im,
                              long nidx, const long *idx, ld *a_re, ld *a_im)
{
    if (M < 1 || nidx < 0 || !fhat_re || !fhat_im || !idx || !a_re || !a_im) return -1;
    ld *cs = (ld *)malloc((size_t)M * sizeof(ld));
    ld *sn = (ld *)malloc((size_t)M * sizeof(ld));
    if (!cs || !sn) { free(cs); free(sn); return -3; }
    for (long m = 0; m < M; ++m) {
        ld ang = 2.0L * PI_L * (ld)m / (ld)M;
        cs[m] = cosl(ang);
        sn[m] = sinl(ang);
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nidx; ++i) {
        long n = idx[i];
        ld sr = 0.0L, si = 0.0L;
        long nm = n % M;
        long id = 0;
        for (long j = 0; j < M; ++j) {
            ld er = cs[id], ei = sn[id];
            sr += fhat_re[j] * er - fhat_im[j] * ei;
            si += fhat_re[j] * ei + fhat_im[j] * er;
            id += nm;
            if (id >= M) id -= M;
        }
        ld sign = (n % 2 == 0) ? 1.0L : -1.0L;
        a_re[i] = sign * (2.0L * PI_L / (ld)M) * sr;
        a_im[i] = sign * (2.0L * PI_L / (ld)M) * si;
    }
    free(cs);
    free(sn);
    return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
