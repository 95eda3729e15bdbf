/*
 * Test infrastructure only: the plain, slow FP64 CPU oracle for the GLS grid.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use it;
 * the GPU library neither links nor calls it, and it shares no code with it.
 *
 * For every requested (SNP i, trait j) problem it computes the generalized
 * least-squares estimate of Section 2, Eq. (1),
 *
 *     b_ij = (X_i^T M_j^{-1} X_i)^{-1} X_i^T M_j^{-1} y_j,   X_i = [X_L | x_i],
 *
 * with the covariance of Eq. (2),  M_j = sigma2_j (h2_j Phi + (1 - h2_j) I),
 * by the single-instance method the paper names as the fastest for one
 * problem (Section 3.1, the "LAPACK" row of Table 1): a Cholesky factorisation
 * M_j = L L^T (n^3/3 flops), then triangular solves A = L^{-1} X_i and
 * c = L^{-1} y_j, so that X_i^T M_j^{-1} X_i = A^T A and X_i^T M_j^{-1} y_j = A^T c,
 * and finally the p x p system (A^T A) b = A^T c by a second Cholesky.
 *
 * No BLAS, no LAPACK, no eigendecomposition. The factor of M_j is computed
 * once per distinct trait of a call and reused for that trait's SNPs; the
 * arithmetic per problem is otherwise exactly the definition above.
 *
 * Conventions
 *   - every matrix is row-major; Phi is n x n; X_L is given column by column
 *     ((p-1) rows of n values), SNP columns and traits likewise (n values each);
 *   - a non-positive or non-finite pivot of M_j is an error (M_j must be SPD);
 *   - a pivot of A^T A at or below 1e-10 of its diagonal entry, or not
 *     finite (X_i numerically not of full rank), gives b_ij = NaN and is
 *     counted.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* In-place lower Cholesky of the row-major n x n matrix a (only the lower
 * triangle is read and written). A pivot must exceed rtol times its original
 * diagonal entry (rtol = 0: plain positivity). Returns 0, or 1 + the failing
 * column. */
static int chol_lower(int n, double *a, double rtol)
{
    for (int j = 0; j < n; ++j) {
        double *rj = a + (size_t)j * n;
        double s = rj[j];
        double floor = rtol * rj[j];
        for (int k = 0; k < j; ++k)
            s -= rj[k] * rj[k];
        if (!(s > floor) || !(s > 0.0) || !isfinite(s))
            return 1 + j;
        double d = sqrt(s);
        rj[j] = d;
        for (int i = j + 1; i < n; ++i) {
            double *ri = a + (size_t)i * n;
            double v = ri[j];
            for (int k = 0; k < j; ++k)
                v -= ri[k] * rj[k];
            ri[j] = v / d;
        }
    }
    return 0;
}

/* Solve L x = v in place (forward substitution), L lower, row-major n x n. */
static void forward_subst(int n, const double *l, double *v)
{
    for (int i = 0; i < n; ++i) {
        const double *ri = l + (size_t)i * n;
        double s = v[i];
        for (int k = 0; k < i; ++k)
            s -= ri[k] * v[k];
        v[i] = s / ri[i];
    }
}

static double dot(int n, const double *x, const double *y)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k)
        s += x[k] * y[k];
    return s;
}

/* Relative pivot floor for X_i^T M^{-1} X_i: a column whose part not explained
 * by the preceding columns has a (M^{-1}-weighted) squared norm below this
 * fraction of its own is treated as linearly dependent (X_i not of full rank). */
#define RANK_RTOL 1e-10

/* Solve the p x p SPD system s b = r by Cholesky (s is overwritten).
 * Returns 0, or nonzero when s is not numerically SPD. */
static int spd_solve(int p, double *s, const double *r, double *b)
{
    if (chol_lower(p, s, RANK_RTOL))
        return 1;
    for (int i = 0; i < p; ++i)
        b[i] = r[i];
    forward_subst(p, s, b);               /* L z = r   */
    for (int i = p - 1; i >= 0; --i) {    /* L^T b = z */
        double v = b[i];
        for (int k = i + 1; k < p; ++k)
            v -= s[(size_t)k * p + i] * b[k];
        b[i] = v / s[(size_t)i * p + i];
    }
    return 0;
}

/*
 * oracle_gls: solve the listed problems.
 *   n, p         samples and design width (2 <= p <= 64)
 *   phi          n x n kinship, row-major
 *   xl           X_L, (p-1) columns of n values
 *   ntraits      number of distinct traits referenced
 *   y            ntraits traits of n values
 *   h2, sigma2   per trait (sigma2 may be NULL: all ones)
 *   nprob        number of problems
 *   xr           nprob SNP columns of n values (the x_i of each problem)
 *   trait        nprob trait indices in [0, ntraits)
 *   b            out: nprob x p, FP64
 *   nthreads     OpenMP threads (<= 0: the runtime's default)
 *   non_spd      out (nullable): number of problems with a non-SPD A^T A
 * Returns 0; -1 for bad arguments; -2 - j if M_j is not SPD for trait j;
 * -3 on allocation failure.
 */
int oracle_gls(int n, int p, const double *phi, const double *xl, int ntraits,
               const double *y, const double *h2, const double *sigma2,
               int64_t nprob, const double *xr, const int32_t *trait, double *b,
               int nthreads, int64_t *non_spd)
{
    if (n <= 0 || p < 2 || p > 64 || ntraits < 0 || nprob < 0 || !phi || !xl ||
        (ntraits > 0 && (!y || !h2)) || (nprob > 0 && (!xr || !trait || !b)))
        return -1;
    for (int64_t q = 0; q < nprob; ++q)
        if (trait[q] < 0 || trait[q] >= ntraits)
            return -1;
    if (nthreads <= 0) {
#ifdef _OPENMP
        nthreads = omp_get_max_threads();
#else
        nthreads = 1;
#endif
    }
    int64_t bad_total = 0;
    int status = 0;
    /* Traits are handled in chunks of nthreads: each thread factors one M_j,
     * then all threads share the problems of the chunk. */
    size_t nn = (size_t)n * n;
    double *fac = malloc(sizeof(double) * nn * (size_t)nthreads);
    double *lxl = malloc(sizeof(double) * (size_t)n * (p - 1) * nthreads);
    double *ly = malloc(sizeof(double) * (size_t)n * nthreads);
    int *ok = malloc(sizeof(int) * nthreads);
    /* problems grouped by trait: order[] lists problem ids trait by trait */
    int64_t *start = calloc((size_t)ntraits + 1, sizeof(int64_t));
    int64_t *order = malloc(sizeof(int64_t) * (size_t)(nprob > 0 ? nprob : 1));
    if (!fac || !lxl || !ly || !ok || !start || !order) {
        free(fac); free(lxl); free(ly); free(ok); free(start); free(order);
        return -3;
    }
    for (int64_t q = 0; q < nprob; ++q)
        start[trait[q] + 1]++;
    for (int j = 0; j < ntraits; ++j)
        start[j + 1] += start[j];
    {
        int64_t *fill = malloc(sizeof(int64_t) * ((size_t)ntraits + 1));
        if (!fill) { free(fac); free(lxl); free(ly); free(ok); free(start); free(order); return -3; }
        memcpy(fill, start, sizeof(int64_t) * ((size_t)ntraits + 1));
        for (int64_t q = 0; q < nprob; ++q)
            order[fill[trait[q]]++] = q;
        free(fill);
    }

    for (int j0 = 0; j0 < ntraits && status == 0; j0 += nthreads) {
        int nj = ntraits - j0 < nthreads ? ntraits - j0 : nthreads;
        /* 1. factor M_j for each trait of the chunk; solve L^{-1} X_L, L^{-1} y_j */
        #pragma omp parallel for num_threads(nthreads) schedule(static, 1)
        for (int s = 0; s < nj; ++s) {
            int j = j0 + s;
            ok[s] = 1;
            if (start[j + 1] == start[j])
                continue;                      /* no problem uses this trait */
            double *l = fac + nn * s;
            double sg = sigma2 ? sigma2[j] : 1.0;
            double hj = h2[j];
            for (int r = 0; r < n; ++r)
                for (int c = 0; c <= r; ++c)
                    l[(size_t)r * n + c] = sg * (hj * phi[(size_t)r * n + c] + (r == c ? 1.0 - hj : 0.0));
            if (chol_lower(n, l, 0.0)) { ok[s] = 0; continue; }
            double *a = lxl + (size_t)n * (p - 1) * s;
            memcpy(a, xl, sizeof(double) * (size_t)n * (p - 1));
            for (int c = 0; c < p - 1; ++c)
                forward_subst(n, l, a + (size_t)c * n);
            double *c = ly + (size_t)n * s;
            memcpy(c, y + (size_t)j * n, sizeof(double) * n);
            forward_subst(n, l, c);
        }
        for (int s = 0; s < nj; ++s)
            if (!ok[s] && status == 0)
                status = -2 - (j0 + s);
        if (status)
            break;
        /* 2. the problems of the chunk's traits */
        int64_t q0 = start[j0], q1 = start[j0 + nj];
        int64_t bad = 0;
        #pragma omp parallel num_threads(nthreads) reduction(+:bad)
        {
            double *ax = malloc(sizeof(double) * n);
            double sm[64 * 64], r[64], bb[64];
            #pragma omp for schedule(dynamic, 4)
            for (int64_t u = q0; u < q1; ++u) {
                int64_t q = order[u];
                int s = trait[q] - j0;
                const double *l = fac + nn * s;
                const double *a = lxl + (size_t)n * (p - 1) * s;
                const double *c = ly + (size_t)n * s;
                memcpy(ax, xr + (size_t)q * n, sizeof(double) * n);
                forward_subst(n, l, ax);                 /* L^{-1} x_i */
                /* S = A^T A and r = A^T c with A = [L^{-1} X_L | L^{-1} x_i] */
                for (int u1 = 0; u1 < p; ++u1) {
                    const double *au = u1 < p - 1 ? a + (size_t)u1 * n : ax;
                    for (int u2 = 0; u2 <= u1; ++u2) {
                        const double *av = u2 < p - 1 ? a + (size_t)u2 * n : ax;
                        sm[u1 * p + u2] = dot(n, au, av);
                        sm[u2 * p + u1] = sm[u1 * p + u2];
                    }
                    r[u1] = dot(n, au, c);
                }
                double *out = b + (size_t)q * p;
                if (spd_solve(p, sm, r, bb)) {
                    for (int u1 = 0; u1 < p; ++u1)
                        out[u1] = NAN;
                    bad++;
                } else {
                    for (int u1 = 0; u1 < p; ++u1)
                        out[u1] = bb[u1];
                }
            }
            free(ax);
        }
        bad_total += bad;
    }
    free(fac); free(lxl); free(ly); free(ok); free(start); free(order);
    if (non_spd)
        *non_spd = bad_total;
    return status;
}
