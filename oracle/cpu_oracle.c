/*
 * FP64 CPU oracle: plain COO loops for SpMTTKRP (Eq. 6), SpTTM (Eq. 3) and
 * the CP model at the nonzeros.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into its own shared
 * library (liborc.so) that only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load.  It includes nothing from the
 * product package and the product package includes nothing from here.
 *
 * Parallelism is the plainest that keeps the loops exact and repeatable:
 * every thread owns a contiguous, equal share of the nonzeros and a private
 * float64 copy of the output; the copies are added in thread order.  The
 * result is therefore deterministic for a given thread count, and equal (up
 * to float64 rounding order) to the serial loop.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

int orc_max_threads(void) { return omp_get_max_threads(); }

static int clamp_threads(int nthreads, int64_t private_bytes, int64_t cap_bytes)
{
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    while (nthreads > 1 && private_bytes * (int64_t)nthreads > cap_bytes) nthreads--;
    return nthreads;
}

/*
 * SpMTTKRP on `mode` (Eq. 6, generalised to N modes):
 *   out[i_mode(e), r] += vals[e] * prod_{m != mode} factors[m][i_m(e) * R + r]
 * out is dims[mode] x R, row-major, overwritten.  factors[mode] is not read.
 * Returns the number of threads used (>= 1), or -1 on allocation failure.
 */
int orc_mttkrp(int order, const int64_t *dims, int64_t nnz, const int32_t *const *idx,
               const double *vals, const double *const *factors, int R, int mode,
               double *out, int nthreads)
{
    const int64_t rows = dims[mode];
    const int64_t obytes = rows * (int64_t)R * (int64_t)sizeof(double);
    nthreads = clamp_threads(nthreads, obytes, (int64_t)24 << 30);
    double *priv = (double *)calloc((size_t)nthreads * (size_t)rows * (size_t)R, sizeof(double));
    if (!priv && rows * R > 0) return -1;

    #pragma omp parallel num_threads(nthreads)
    {
        const int t = omp_get_thread_num();
        const int nt = omp_get_num_threads();
        const int64_t e0 = nnz * t / nt, e1 = nnz * (t + 1) / nt;
        double *acc = priv + (size_t)t * (size_t)rows * (size_t)R;
        double *h = (double *)malloc(sizeof(double) * (size_t)(R > 0 ? R : 1));
        for (int64_t e = e0; e < e1; ++e) {
            for (int r = 0; r < R; ++r) h[r] = vals[e];
            for (int m = 0; m < order; ++m) {
                if (m == mode) continue;
                const double *row = factors[m] + (int64_t)idx[m][e] * R;
                for (int r = 0; r < R; ++r) h[r] *= row[r];
            }
            double *o = acc + (int64_t)idx[mode][e] * R;
            for (int r = 0; r < R; ++r) o[r] += h[r];
        }
        free(h);
    }
    #pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t i = 0; i < rows * R; ++i) {
        double s = 0.0;
        for (int t = 0; t < nthreads; ++t) s += priv[(size_t)t * (size_t)rows * (size_t)R + i];
        out[i] = s;
    }
    free(priv);
    return nthreads;
}

/* ---- SpTTM: grouping pass (fibres of the index modes) ------------------- */

typedef struct { int order; int mode; const int32_t *const *idx; } grp_ctx;

static int cmp_fibre(const void *pa, const void *pb, void *pc)
{
    const grp_ctx *c = (const grp_ctx *)pc;
    const int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    for (int m = 0; m < c->order; ++m) {
        if (m == c->mode) continue;
        const int32_t x = c->idx[m][a], y = c->idx[m][b];
        if (x != y) return x < y ? -1 : 1;
    }
    return a < b ? -1 : (a > b);
}

/*
 * Groups the nonzeros by their index-mode tuple (every mode but `mode`), in
 * lexicographic order.  order_out[nnz] receives nonzero ids grouped by
 * fibre, fib_ptr[nfib + 1] the start of each group (caller sizes it nnz + 1).
 * Returns nfib.
 */
int64_t orc_ttm_group(int order, int64_t nnz, const int32_t *const *idx, int mode,
                      int64_t *order_out, int64_t *fib_ptr)
{
    grp_ctx c = { order, mode, idx };
    for (int64_t e = 0; e < nnz; ++e) order_out[e] = e;
    qsort_r(order_out, (size_t)nnz, sizeof(int64_t), cmp_fibre, &c);
    int64_t nf = 0;
    for (int64_t s = 0; s < nnz; ++s) {
        int newf = (s == 0);
        if (!newf) {
            for (int m = 0; m < order; ++m) {
                if (m == mode) continue;
                if (idx[m][order_out[s]] != idx[m][order_out[s - 1]]) { newf = 1; break; }
            }
        }
        if (newf) fib_ptr[nf++] = s;
    }
    fib_ptr[nf] = nnz;
    return nf;
}

/*
 * SpTTM on `mode` (Eq. 3): Y[f, :] = sum over the nonzeros e of fibre f of
 * vals[e] * U[i_mode(e), :], U being dims[mode] x R row-major.  Fibres come
 * from orc_ttm_group.  Fibres are disjoint, so threads split them freely.
 */
int orc_ttm(int64_t nfib, const int64_t *order_in, const int64_t *fib_ptr,
            const int32_t *idx_mode, const double *vals, const double *U, int R,
            double *Y, int nthreads)
{
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    #pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1024)
    for (int64_t f = 0; f < nfib; ++f) {
        double *y = Y + f * R;
        for (int r = 0; r < R; ++r) y[r] = 0.0;
        for (int64_t s = fib_ptr[f]; s < fib_ptr[f + 1]; ++s) {
            const int64_t e = order_in[s];
            const double *u = U + (int64_t)idx_mode[e] * R;
            for (int r = 0; r < R; ++r) y[r] += vals[e] * u[r];
        }
    }
    return nthreads;
}

/*
 * CP model at the nonzeros: xhat[e] = sum_r prod_m factors[m][i_m(e) * R + r].
 */
int orc_model(int order, int64_t nnz, const int32_t *const *idx,
              const double *const *factors, int R, double *xhat, int nthreads)
{
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    #pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t e = 0; e < nnz; ++e) {
        double s = 0.0;
        for (int r = 0; r < R; ++r) {
            double p = 1.0;
            for (int m = 0; m < order; ++m) p *= factors[m][(int64_t)idx[m][e] * R + r];
            s += p;
        }
        xhat[e] = s;
    }
    return nthreads;
}
