/*
 * TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously correct FP64 CPU
 * implementation of sparse MTTKRP used to check the GPU library.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the library never does.  It shares no code with the GPU path.
 *
 * Definition (Sec. II-A, Eq. (1) in its elementwise form, "Elementwise
 * computation"): for output mode n of an N-mode sparse tensor with
 * nonzeros (p_k, val_k), p_k = (c_0 .. c_{N-1}), and dense factors A_m
 * (I_m x R, row-major),
 *
 *     M_n[i, r] = sum over k with c_n(k) == i of  val_k * prod_{m != n} A_m[c_m(k), r]
 *
 * for 0 <= i < I_n, 0 <= r < R.  Rows that no nonzero touches are zero.
 * Duplicate coordinates are simply two terms of the sum.
 *
 * Everything is accumulated in double precision.  With threads > 1 every
 * thread owns a contiguous slice of the nonzeros and a private output; the
 * private outputs are added in thread order, so a fixed thread count gives a
 * fixed result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Returns 0 on success, -1 on an index out of range, -2 on bad arguments,
 * -3 when memory runs out. */
static int check_args(const uint32_t* idx, uint64_t nnz, int N, const uint32_t* dims, int mode, int R)
{
    if (N < 2 || mode < 0 || mode >= N || R < 1) return -2;
    for (uint64_t k = 0; k < nnz; ++k)
        for (int m = 0; m < N; ++m)
            if (idx[k * (uint64_t)N + m] >= dims[m]) return -1;
    return 0;
}

/* One nonzero's contribution, added into row `dst` (R doubles). */
static void add_term(const uint32_t* p, double v, int N, const double* const* factors, int mode, int R,
                     double* dst)
{
    for (int r = 0; r < R; ++r) {
        double t = v;
        for (int m = 0; m < N; ++m) {
            if (m == mode) continue;
            t *= factors[m][(uint64_t)p[m] * R + r];
        }
        dst[r] += t;
    }
}

int oracle_mttkrp(const uint32_t* idx, const double* val, uint64_t nnz, int N, const uint32_t* dims,
                  const double* const* factors, int mode, int R, double* out, int threads)
{
    int rc = check_args(idx, nnz, N, dims, mode, R);
    if (rc) return rc;
    const uint64_t I = dims[mode];
    const uint64_t osz = I * (uint64_t)R;
    memset(out, 0, osz * sizeof(double));
    if (threads < 1) threads = 1;
    if (threads == 1 || nnz < 4096) {
        for (uint64_t k = 0; k < nnz; ++k) {
            const uint32_t* p = idx + k * (uint64_t)N;
            add_term(p, val[k], N, factors, mode, R, out + (uint64_t)p[mode] * R);
        }
        return 0;
    }
    double* priv = (double*)calloc((size_t)threads * osz, sizeof(double));
    if (!priv) return -3;
#pragma omp parallel num_threads(threads)
    {
#ifdef _OPENMP
        const int t = omp_get_thread_num();
        const int T = omp_get_num_threads();
#else
        const int t = 0, T = 1;
#endif
        const uint64_t lo = nnz * (uint64_t)t / (uint64_t)T;
        const uint64_t hi = nnz * (uint64_t)(t + 1) / (uint64_t)T;
        double* mine = priv + (uint64_t)t * osz;
        for (uint64_t k = lo; k < hi; ++k) {
            const uint32_t* p = idx + k * (uint64_t)N;
            add_term(p, val[k], N, factors, mode, R, mine + (uint64_t)p[mode] * R);
        }
    }
    for (int t = 0; t < threads; ++t) {
        const double* mine = priv + (uint64_t)t * osz;
        for (uint64_t e = 0; e < osz; ++e) out[e] += mine[e];
    }
    free(priv);
    return 0;
}

/* The same sum for a subset of output rows only: out is (nrows x R), row j of
 * out holds M_n[rows[j], :].  Used to check single outputs of tensors too
 * large for a full oracle pass in a test. */
int oracle_mttkrp_rows(const uint32_t* idx, const double* val, uint64_t nnz, int N, const uint32_t* dims,
                       const double* const* factors, int mode, int R, const uint32_t* rows,
                       uint64_t nrows, double* out)
{
    int rc = check_args(idx, nnz, N, dims, mode, R);
    if (rc) return rc;
    int64_t* slot = (int64_t*)malloc((size_t)dims[mode] * sizeof(int64_t));
    if (!slot) return -3;
    for (uint64_t i = 0; i < dims[mode]; ++i) slot[i] = -1;
    for (uint64_t j = 0; j < nrows; ++j) {
        if (rows[j] >= dims[mode]) { free(slot); return -1; }
        slot[rows[j]] = (int64_t)j;
    }
    memset(out, 0, nrows * (uint64_t)R * sizeof(double));
    for (uint64_t k = 0; k < nnz; ++k) {
        const uint32_t* p = idx + k * (uint64_t)N;
        int64_t j = slot[p[mode]];
        if (j < 0) continue;
        add_term(p, val[k], N, factors, mode, R, out + (uint64_t)j * R);
    }
    /* rows listed twice: copy the accumulated row into every listed slot */
    for (uint64_t j = 0; j < nrows; ++j) {
        int64_t s = slot[rows[j]];
        if ((uint64_t)s != j) memcpy(out + j * (uint64_t)R, out + (uint64_t)s * R, (size_t)R * sizeof(double));
    }
    free(slot);
    return 0;
}
