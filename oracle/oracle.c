/*
 * CPU oracle for the sparse CP-ALS hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain FP64 loops written to be checked by eye against the paper, not for
 * speed.  Nothing in the HIP library includes, links or calls this file; only
 * the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * Notation (Section III, Algorithm 1): a sparse tensor X with N modes of
 * lengths I_0..I_{N-1}, factor matrices A_m (I_m x R, row-major), and the
 * MTTKRP of mode n, Y_n = X_(n) (Khatri-Rao product of the other factors).
 * Written element-wise, which is independent of the Khatri-Rao column order:
 *
 *     Y_n(i, r) = sum over nonzeros (i_0..i_{N-1}; x) with i_n = i of
 *                 x * prod_{m != n} A_m(i_m, r).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* MTTKRP by a direct loop over the COO nonzeros in storage order.
 * inds: N x nnz int64 (mode-major), vals: nnz doubles, factors: N pointers
 * (the entry for `mode` is not read), Y: I_mode x R, overwritten.
 * Returns 0, or -1 when the row scratch cannot be allocated. */
int oracle_mttkrp_coo(int nmodes, const int64_t *dims, int64_t nnz, const int64_t *inds,
                      const double *vals, const double *const *factors, int rank, int mode,
                      double *Y)
{
    double *row = (double *)malloc(sizeof(double) * (size_t)rank);
    if (!row) return -1;
    memset(Y, 0, sizeof(double) * (size_t)dims[mode] * (size_t)rank);
    for (int64_t k = 0; k < nnz; ++k) {
        for (int r = 0; r < rank; ++r) row[r] = vals[k];
        for (int m = 0; m < nmodes; ++m) {
            if (m == mode) continue;
            const double *a = factors[m] + inds[(int64_t)m * nnz + k] * rank;
            for (int r = 0; r < rank; ++r) row[r] *= a[r];
        }
        double *y = Y + inds[(int64_t)mode * nnz + k] * rank;
        for (int r = 0; r < rank; ++r) y[r] += row[r];
    }
    free(row);
    return 0;
}

/* The same MTTKRP with the nonzeros split into `nthreads` contiguous ranges,
 * thread t summing range t into a private copy of Y; the copies are then
 * added into Y in range order (the privatised parallel MTTKRP the paper
 * times, Section IV-B, with OpenMP threads in place of Chapel tasks).  It
 * differs from the sequential loop only in the order of the FP64 additions;
 * it serves to time the oracle on all host cores.  Returns 0, or -1 when the
 * copies cannot be allocated. */
int oracle_mttkrp_coo_par(int nmodes, const int64_t *dims, int64_t nnz, const int64_t *inds,
                          const double *vals, const double *const *factors, int rank, int mode,
                          int nthreads, double *Y)
{
    if (nthreads < 1) nthreads = 1;
    const size_t ylen = (size_t)dims[mode] * (size_t)rank;
    double *copies = (double *)calloc((size_t)nthreads * ylen, sizeof(double));
    if (!copies) return -1;
    int failed = 0;
#pragma omp parallel num_threads(nthreads) reduction(|| : failed)
    {
#ifdef _OPENMP
        const int t = omp_get_thread_num(), nt = omp_get_num_threads();
#else
        const int t = 0, nt = 1;
#endif
        const int64_t k0 = nnz * t / nt, k1 = nnz * (t + 1) / nt;
        double *Yt = copies + (size_t)t * ylen;
        double *row = (double *)malloc(sizeof(double) * (size_t)rank);
        if (!row) {
            failed = 1;
        } else {
            for (int64_t k = k0; k < k1; ++k) {
                for (int r = 0; r < rank; ++r) row[r] = vals[k];
                for (int m = 0; m < nmodes; ++m) {
                    if (m == mode) continue;
                    const double *a = factors[m] + inds[(int64_t)m * nnz + k] * rank;
                    for (int r = 0; r < rank; ++r) row[r] *= a[r];
                }
                double *y = Yt + inds[(int64_t)mode * nnz + k] * rank;
                for (int r = 0; r < rank; ++r) y[r] += row[r];
            }
            free(row);
        }
    }
    if (failed) {
        free(copies);
        return -1;
    }
    memset(Y, 0, sizeof(double) * ylen);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t j = 0; j < (int64_t)ylen; ++j) {
        double s = 0.0;
        for (int t = 0; t < nthreads; ++t) s += copies[(size_t)t * ylen + (size_t)j];
        Y[j] = s;
    }
    free(copies);
    return 0;
}

/* The same MTTKRP, restricted to the output rows listed in `rows` (nrows
 * distinct row indices); Yrows is nrows x R, overwritten.  Used to check
 * single rows of very large outputs.  Returns 0, -1 on allocation failure,
 * -2 on an out-of-range or repeated row. */
int oracle_mttkrp_coo_rows(int nmodes, const int64_t *dims, int64_t nnz, const int64_t *inds,
                           const double *vals, const double *const *factors, int rank,
                           int mode, int64_t nrows, const int64_t *rows, double *Yrows)
{
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)dims[mode]);
    double *row = (double *)malloc(sizeof(double) * (size_t)rank);
    if (!slot || !row) { free(slot); free(row); return -1; }
    for (int64_t i = 0; i < dims[mode]; ++i) slot[i] = -1;
    for (int64_t s = 0; s < nrows; ++s) {
        if (rows[s] < 0 || rows[s] >= dims[mode] || slot[rows[s]] >= 0) {
            free(slot); free(row); return -2;
        }
        slot[rows[s]] = s;
    }
    memset(Yrows, 0, sizeof(double) * (size_t)nrows * (size_t)rank);
    for (int64_t k = 0; k < nnz; ++k) {
        int64_t s = slot[inds[(int64_t)mode * nnz + k]];
        if (s < 0) continue;
        for (int r = 0; r < rank; ++r) row[r] = vals[k];
        for (int m = 0; m < nmodes; ++m) {
            if (m == mode) continue;
            const double *a = factors[m] + inds[(int64_t)m * nnz + k] * rank;
            for (int r = 0; r < rank; ++r) row[r] *= a[r];
        }
        double *y = Yrows + s * rank;
        for (int r = 0; r < rank; ++r) y[r] += row[r];
    }
    free(slot);
    free(row);
    return 0;
}

/* Sum of squares of the values, the ||X||^2 term of the fit. */
double oracle_sumsq(int64_t nnz, const double *vals)
{
    double s = 0.0;
    for (int64_t k = 0; k < nnz; ++k) s += vals[k] * vals[k];
    return s;
}
