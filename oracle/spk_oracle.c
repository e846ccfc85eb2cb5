/*
 * spk_oracle.c -- reference results for the autotuned kernels.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU implementation that every GPU variant is checked against.  It plays
 * the part of the unannotated program in the paper's method (Section 2,
 * "Approach": the original code is kept as the reference implementation
 * whose outputs every tuned variant must reproduce).  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * HIP library never links, loads or calls it, and the two share no code.
 *
 * Conventions
 *   - FP64 arithmetic throughout; FP32 inputs are promoted exactly (a
 *     product of two floats is exact in double).
 *   - Built with -O2 -ffp-contract=off; every fused multiply-add is an
 *     explicit fma(), so results do not depend on compiler contraction.
 *   - OpenMP only splits independent rows or elements, so the output is
 *     bit-identical for any thread count.  dot() combines fixed 4096-element
 *     chunks in index order for the same reason.
 *
 * Operations (the abstract does not print the kernels' formulas; the
 * vector update of Figure 1 is read as WAXPY, w = alpha*x + y, and the
 * sparse kernels of the prior GPU work in Section 3 as CSR y = A*x):
 *   waxpy   w_i = alpha*x_i + y_i          (one fused rounding)
 *   axpy    y_i <- alpha*x_i + y_i         (waxpy with w == y)
 *   dot     sum_i x_i*y_i                  (compensated, index order)
 *   spmv    y_i = sum_k val_k * x[col_k]   over row i's entries in storage order
 *   spmv_waxpy  y = A*x, then w = alpha*y + x  (one Krylov-style step)
 * plus the acceptance checks used by the tests (ulp distance, per-row
 * tolerance test).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_API __attribute__((visibility("default")))

ORC_API int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

ORC_API void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ---------------------------------------------------------------- WAXPY -- */

/* w_i = alpha*x_i + y_i, rounded once (fma). */
ORC_API void orc_waxpy_f64(int64_t n, double alpha, const double *x, const double *y, double *w)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        w[i] = fma(alpha, x[i], y[i]);
}

/* FP32 data: alpha is first rounded to float (the operation acts on float
 * operands), the fused result is formed in double and rounded to float. */
ORC_API void orc_waxpy_f32(int64_t n, double alpha, const float *x, const float *y, float *w)
{
    const double a = (double)(float)alpha;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        w[i] = (float)fma(a, (double)x[i], (double)y[i]);
}

/* y_i <- alpha*x_i + y_i (in place). */
ORC_API void orc_axpy_f64(int64_t n, double alpha, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        y[i] = fma(alpha, x[i], y[i]);
}

ORC_API void orc_axpy_f32(int64_t n, double alpha, const float *x, float *y)
{
    const double a = (double)(float)alpha;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        y[i] = (float)fma(a, (double)x[i], (double)y[i]);
}

/* ------------------------------------------------------------------ dot -- */

/* Neumaier's improvement of Kahan summation: (s, c) with s + c the running
 * sum.  Terms are added strictly in index order. */
typedef struct { double s, c; } orc_cs;

static inline void orc_cs_add(orc_cs *acc, double t)
{
    double s = acc->s + t;
    if (fabs(acc->s) >= fabs(t))
        acc->c += (acc->s - s) + t;
    else
        acc->c += (t - s) + acc->s;
    acc->s = s;
}

#define ORC_DOT_CHUNK 4096

/* sum_i x_i*y_i.  Each product is formed in double; sums are compensated.
 * Fixed 4096-element chunks are summed independently and then combined in
 * chunk order, so the value does not depend on the thread count. */
static double orc_dot_impl(int64_t n, const double *xd, const double *yd,
                           const float *xf, const float *yf)
{
    if (n <= 0) return 0.0;
    const int64_t nchunk = (n + ORC_DOT_CHUNK - 1) / ORC_DOT_CHUNK;
    orc_cs total = {0.0, 0.0};
    double tail = 0.0;
    /* chunks are processed in parallel blocks of a fixed size and
     * merged in order */
    enum { BLOCK = 1024 };
    orc_cs part[BLOCK];
    for (int64_t c0 = 0; c0 < nchunk; c0 += BLOCK) {
        const int64_t cn = (nchunk - c0 < BLOCK) ? nchunk - c0 : BLOCK;
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < cn; ++c) {
            const int64_t lo = (c0 + c) * ORC_DOT_CHUNK;
            const int64_t hi = (lo + ORC_DOT_CHUNK < n) ? lo + ORC_DOT_CHUNK : n;
            orc_cs a = {0.0, 0.0};
            for (int64_t i = lo; i < hi; ++i) {
                double p = xd ? xd[i] * yd[i] : (double)xf[i] * (double)yf[i];
                orc_cs_add(&a, p);
            }
            part[c] = a;
        }
        for (int64_t c = 0; c < cn; ++c) {
            orc_cs_add(&total, part[c].s);
            tail += part[c].c;
        }
    }
    return total.s + (total.c + tail);
}

ORC_API double orc_dot_f64(int64_t n, const double *x, const double *y)
{
    return orc_dot_impl(n, x, y, NULL, NULL);
}

ORC_API double orc_dot_f32(int64_t n, const float *x, const float *y)
{
    return orc_dot_impl(n, NULL, NULL, x, y);
}

/* sum_i |x_i*y_i| (scale of the dot tolerance), plain summation. */
ORC_API double orc_dot_absum_f64(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i)
        s += fabs(x[i] * y[i]);
    return s;
}

ORC_API double orc_dot_absum_f32(int64_t n, const float *x, const float *y)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i)
        s += fabs((double)x[i] * (double)y[i]);
    return s;
}

/* ----------------------------------------------------------------- SpMV -- */

/* y_i = sum over row i's stored entries, in storage order, of val_k*x[col_k];
 * duplicates and explicit zeros all contribute; an empty row gives +0.
 * absum (nullable) receives sum_k |val_k*x[col_k]|, the scale of the
 * per-row tolerance. */
ORC_API void orc_spmv_csr_f64(int64_t m, const int32_t *row_ptr, const int32_t *col_idx,
                              const double *val, const double *x, double *y, double *absum)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double acc = 0.0, mag = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const double a = val[k], xv = x[col_idx[k]];
            acc = fma(a, xv, acc);
            mag += fabs(a * xv);
        }
        y[i] = acc;
        if (absum) absum[i] = mag;
    }
}

/* FP32 operands promoted to double: every product is exact, the sum is
 * formed in double, and y is returned in double. */
ORC_API void orc_spmv_csr_f32(int64_t m, const int32_t *row_ptr, const int32_t *col_idx,
                              const float *val, const float *x, double *y, double *absum)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double acc = 0.0, mag = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const double a = (double)val[k], xv = (double)x[col_idx[k]];
            acc = fma(a, xv, acc);
            mag += fabs(a * xv);
        }
        y[i] = acc;
        if (absum) absum[i] = mag;
    }
}

/* One Krylov-style step on a square matrix: y = A*x, then w = alpha*y + x. */
ORC_API void orc_spmv_waxpy_f64(int64_t m, const int32_t *row_ptr, const int32_t *col_idx,
                                const double *val, const double *x, double alpha,
                                double *y, double *w, double *absum)
{
    orc_spmv_csr_f64(m, row_ptr, col_idx, val, x, y, absum);
    orc_waxpy_f64(m, alpha, y, x, w);
}

/* Batched form: ``count`` independent square instances laid out back to back
 * (instance i: row_ptr at rp_off[i] with local values, entries at nz_off[i],
 * vectors at vec_off[i]).  Each instance is exactly orc_spmv_waxpy_f64. */
ORC_API void orc_batch_spmv_waxpy_f64(int64_t count, const int64_t *m, const int64_t *rp_off,
                                      const int64_t *nz_off, const int64_t *vec_off,
                                      const int32_t *row_ptr, const int32_t *col_idx,
                                      const double *val, const double *x, double alpha,
                                      double *y, double *w, double *absum)
{
    for (int64_t b = 0; b < count; ++b) {
        const int64_t vo = vec_off[b];
        orc_spmv_waxpy_f64(m[b], row_ptr + rp_off[b], col_idx + nz_off[b], val + nz_off[b],
                           x + vo, alpha, y + vo, w + vo, absum ? absum + vo : NULL);
    }
}

/* ---------------------------------------------------- acceptance checks -- */

/* Monotone integer image of an IEEE double: ord(a) < ord(b) iff a < b for
 * non-NaN values, +0 and -0 map to 0, adjacent doubles differ by 1. */
static inline int64_t orc_ord_f64(double a)
{
    int64_t b;
    memcpy(&b, &a, sizeof b);
    return b < 0 ? -(b & INT64_MAX) : b;
}

static inline int64_t orc_ord_f32(float a)
{
    int32_t b;
    memcpy(&b, &a, sizeof b);
    return b < 0 ? -(int64_t)(b & INT32_MAX) : (int64_t)b;
}

/* Largest ulp distance between a and b.  A NaN in exactly one of a pair
 * counts as INT64_MAX; two NaNs count as 0. */
ORC_API int64_t orc_max_ulp_f64(int64_t n, const double *a, const double *b, int64_t *where)
{
    int64_t worst = 0, at = -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t d;
        const int na = isnan(a[i]), nb = isnan(b[i]);
        if (na || nb)
            d = (na && nb) ? 0 : INT64_MAX;
        else {
            const int64_t oa = orc_ord_f64(a[i]), ob = orc_ord_f64(b[i]);
            d = oa > ob ? oa - ob : ob - oa;
        }
        if (d > worst) { worst = d; at = i; }
    }
    if (where) *where = at;
    return worst;
}

ORC_API int64_t orc_max_ulp_f32(int64_t n, const float *a, const float *b, int64_t *where)
{
    int64_t worst = 0, at = -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t d;
        const int na = isnan(a[i]), nb = isnan(b[i]);
        if (na || nb)
            d = (na && nb) ? 0 : INT64_MAX;
        else {
            const int64_t oa = orc_ord_f32(a[i]), ob = orc_ord_f32(b[i]);
            d = oa > ob ? oa - ob : ob - oa;
        }
        if (d > worst) { worst = d; at = i; }
    }
    if (where) *where = at;
    return worst;
}

/* Per-row acceptance of a computed y (promoted to double) against the
 * reference: |y_i - ref_i| <= tau * absum_i for finite references (so an
 * empty row must be exactly zero); a NaN reference needs a NaN, an infinite
 * one the same infinity.  Returns the number of failing rows; *worst gets
 * the largest |y_i - ref_i| / absum_i seen on finite rows (or +inf when a
 * row with absum 0 differs) and *where its index. */
ORC_API int64_t orc_check_rows(int64_t m, const double *y, const double *ref, const double *absum,
                               double tau, double *worst, int64_t *where)
{
    int64_t bad = 0, at = -1;
    double wr = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        int ok;
        double ratio = 0.0;
        if (isnan(ref[i]))
            ok = isnan(y[i]);
        else if (isinf(ref[i]))
            ok = (y[i] == ref[i]);
        else {
            const double err = fabs(y[i] - ref[i]);
            ok = err <= tau * absum[i];
            if (err > 0.0) ratio = absum[i] > 0.0 ? err / absum[i] : INFINITY;
            if (isnan(y[i])) { ok = 0; ratio = INFINITY; }
        }
        if (!ok) ++bad;
        if (ratio > wr || (!ok && at < 0)) { wr = ratio > wr ? ratio : wr; at = i; }
    }
    if (worst) *worst = wr;
    if (where) *where = at;
    return bad;
}

/* ------------------------------------------------------------------- CG -- */

/* Conjugate gradients on a square symmetric positive definite CSR matrix
 * (FP64), the textbook recurrence in its usual order: r = b - A x, p = r,
 * rr = r.r; then per iteration q = A p, alpha = rr / (p.q), x += alpha p,
 * r -= alpha q, rr' = r.r, beta = rr' / rr, p = r + beta p.  x holds the
 * initial guess on entry and the iterate on return; rr_hist[k] = r_k.r_k for
 * k = 0..iters.  Every update is one fused multiply-add per element.  Once
 * the residual is exactly zero the step sizes are taken as zero (instead of
 * 0/0), so the iterate stays put. */
ORC_API void orc_cg_f64(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                        const double *b, double *x, int64_t iters, double *rr_hist,
                        double *r, double *p, double *q)
{
    orc_spmv_csr_f64(n, row_ptr, col_idx, val, x, q, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        r[i] = fma(-1.0, q[i], b[i]);
        p[i] = r[i];
    }
    double rr = orc_dot_f64(n, r, r);
    rr_hist[0] = rr;
    for (int64_t k = 0; k < iters; ++k) {
        orc_spmv_csr_f64(n, row_ptr, col_idx, val, p, q, NULL);
        const double pq = orc_dot_f64(n, p, q);
        const double alpha = pq != 0.0 ? rr / pq : 0.0;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            x[i] = fma(alpha, p[i], x[i]);
            r[i] = fma(-alpha, q[i], r[i]);
        }
        const double rr_new = orc_dot_f64(n, r, r);
        const double beta = rr != 0.0 ? rr_new / rr : 0.0;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            p[i] = fma(beta, p[i], r[i]);
        rr = rr_new;
        rr_hist[k + 1] = rr;
    }
}
