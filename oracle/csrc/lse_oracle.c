/*
 * Plain C float64 oracle for the matricized least-squares polynomial fit.
 *
 * TEST INFRASTRUCTURE ONLY: linked by nothing in the product path; loaded by
 * the tests and timed by the benchmark's CPU-baseline leg.  Shares no code
 * with the HIP library.
 *
 * Route (Sec. II of the paper): t_i = (x_i - c)/s; power sums
 * S_p = sum t_i^p (p = 0..2m), T_j = sum t_i^j y_i (j = 0..m); Hankel normal
 * matrix A_jk = S_(j+k) with B_j = T_j (A_00 = S_0 = n, reading the printed
 * "1" as the zeroth power sum); Gaussian elimination with partial pivoting
 * (first row of largest magnitude; singular when |pivot| <= 2^-40 max|A|);
 * back to the x-basis a_k = sum_{j>=k} b_j C(j,k) (-c)^(j-k) s^(-j).
 *
 * Sums are Neumaier-compensated.  A single fit is cut into fixed chunks of
 * ORACLE_CHUNK points (independent of the thread count); chunk sums are added
 * in chunk order, so the result does not depend on how many threads ran.
 * Batched fits run one fit per OpenMP iteration, each fit sequentially.
 * Built without fast-math and with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAXDEG 16
#define ORACLE_CHUNK 65536
#define ST_OK 0
#define ST_INVALID 1
#define ST_SINGULAR 2
#define ST_NONFINITE 3

/* Neumaier's improvement of Kahan summation: s + c carries the sum. */
static inline void nadd(double *s, double *c, double v) {
    double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

static inline double load(const void *p, int dtype, int64_t i) {
    return dtype == 0 ? (double)((const float *)p)[i] : ((const double *)p)[i];
}

/* Compensated sums over points [lo, hi): out[0..2m] = (S, comp) pairs of S_0..S_2m,
 * out[2(2m+1)..] = pairs of T_0..T_m. */
static void range_sums(const void *x, const void *y, int dtype, int64_t lo, int64_t hi, int m,
                       double c, double s, double *sum, double *comp) {
    int ns = 2 * m + 1, nt = m + 1;
    for (int k = 0; k < ns + nt; ++k) sum[k] = comp[k] = 0.0;
    for (int64_t i = lo; i < hi; ++i) {
        double t = (load(x, dtype, i) - c) / s;
        double yv = load(y, dtype, i);
        double p = 1.0;
        for (int k = 0; k < ns; ++k) {
            nadd(&sum[k], &comp[k], p);
            if (k <= m) nadd(&sum[ns + k], &comp[ns + k], p * yv);
            p *= t;
        }
    }
}

static int gepp(int n, double *A /* n x n */, double *B, double *X) {
    double M[ORACLE_MAXDEG + 1][ORACLE_MAXDEG + 2];
    double amax = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            M[i][j] = A[i * n + j];
            if (!isfinite(M[i][j])) return ST_NONFINITE;
            if (fabs(M[i][j]) > amax) amax = fabs(M[i][j]);
        }
        M[i][n] = B[i];
        if (!isfinite(B[i])) return ST_NONFINITE;
    }
    double tiny = ldexp(amax, -40);
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(M[r][k]) > fabs(M[p][k])) p = r;
        if (!(fabs(M[p][k]) > tiny)) return ST_SINGULAR;
        if (p != k)
            for (int c = 0; c <= n; ++c) {
                double tmp = M[k][c];
                M[k][c] = M[p][c];
                M[p][c] = tmp;
            }
        for (int r = k + 1; r < n; ++r) {
            double l = M[r][k] / M[k][k];
            for (int c = k; c <= n; ++c) M[r][c] -= l * M[k][c];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double acc = M[i][n];
        for (int c = i + 1; c < n; ++c) acc -= M[i][c] * X[c];
        X[i] = acc / M[i][i];
    }
    for (int i = 0; i < n; ++i)
        if (!isfinite(X[i])) return ST_NONFINITE;
    return ST_OK;
}

static double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

static void unscale(int m, const double *b, double c, double s, double *a) {
    for (int k = 0; k <= m; ++k) {
        double acc = 0.0, comp = 0.0;
        for (int j = k; j <= m; ++j) {
            double term = b[j] * binom(j, k) * pow(-c, j - k) * pow(s, -j);
            nadd(&acc, &comp, term);
        }
        a[k] = acc + comp;
    }
}

static int solve_sums(int m, const double *S, const double *T, double c, double s, double *a, double *b) {
    double A[(ORACLE_MAXDEG + 1) * (ORACLE_MAXDEG + 1)], B[ORACLE_MAXDEG + 1], X[ORACLE_MAXDEG + 1];
    int n = m + 1;
    for (int j = 0; j < n; ++j) {
        for (int k = 0; k < n; ++k) A[j * n + k] = S[j + k];
        B[j] = T[j];
    }
    int st = gepp(n, A, B, X);
    if (st != ST_OK) {
        for (int k = 0; k < n; ++k) {
            a[k] = NAN;
            if (b) b[k] = NAN;
        }
        return st;
    }
    if (b) memcpy(b, X, sizeof(double) * n);
    unscale(m, X, c, s, a);
    return ST_OK;
}

/* Power sums of one fit: S[0..2m], T[0..m]. dtype 0 = float32, 1 = float64. */
int lse_oracle_power_sums(const void *x, const void *y, int64_t n, int dtype, int m, double c, double s,
                          double *S, double *T, int nthreads) {
    if (m < 0 || m > ORACLE_MAXDEG || n < 0 || (dtype != 0 && dtype != 1) || !(s != 0.0)) return ST_INVALID;
    int ns = 2 * m + 1, nacc = 3 * m + 2;
    int64_t nchunk = (n + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
    double *part = (double *)calloc((size_t)(nchunk > 0 ? nchunk : 1) * 2 * nacc, sizeof(double));
    if (!part) return ST_INVALID;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t ch = 0; ch < nchunk; ++ch) {
        int64_t lo = ch * ORACLE_CHUNK, hi = lo + ORACLE_CHUNK < n ? lo + ORACLE_CHUNK : n;
        range_sums(x, y, dtype, lo, hi, m, c, s, part + ch * 2 * nacc, part + ch * 2 * nacc + nacc);
    }
    for (int k = 0; k < nacc; ++k) {
        double acc = 0.0, comp = 0.0;
        for (int64_t ch = 0; ch < nchunk; ++ch) {
            nadd(&acc, &comp, part[ch * 2 * nacc + k]);
            comp += part[ch * 2 * nacc + nacc + k];
        }
        double v = acc + comp;
        if (k < ns) S[k] = v;
        else T[k - ns] = v;
    }
    free(part);
    return ST_OK;
}

/* One fit. a[m+1] x-basis; b[m+1] t-basis (nullable); S[2m+1], T[m+1] nullable. */
int lse_oracle_fit(const void *x, const void *y, int64_t n, int dtype, int m, double c, double s,
                   double *a, double *b, double *S_out, double *T_out, int nthreads) {
    double S[2 * ORACLE_MAXDEG + 1], T[ORACLE_MAXDEG + 1];
    if (m < 0 || m > ORACLE_MAXDEG) return ST_INVALID;
    int st = lse_oracle_power_sums(x, y, n, dtype, m, c, s, S, T, nthreads);
    if (st != ST_OK) return st;
    if (S_out) memcpy(S_out, S, sizeof(double) * (2 * m + 1));
    if (T_out) memcpy(T_out, T, sizeof(double) * (m + 1));
    if (n < m + 1) {
        for (int k = 0; k <= m; ++k) a[k] = NAN;
        return ST_SINGULAR;
    }
    return solve_sums(m, S, T, c, s, a, b);
}

/* Independent fits over CSR segments offsets[f]..offsets[f+1].
 * a is [B * stride] x-basis coefficients (unused tail entries left untouched);
 * centers/scales nullable (0 and 1). */
int lse_oracle_fit_batched(const void *x, const void *y, const int64_t *offsets, const int32_t *degrees,
                           int64_t B, int dtype, const double *centers, const double *scales, int stride,
                           double *a, int32_t *status, int nthreads) {
    if (B < 0 || (dtype != 0 && dtype != 1)) return ST_INVALID;
    for (int64_t f = 0; f < B; ++f)
        if (degrees[f] < 0 || degrees[f] > ORACLE_MAXDEG || degrees[f] + 1 > stride) return ST_INVALID;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t f = 0; f < B; ++f) {
        int m = degrees[f];
        int64_t lo = offsets[f], hi = offsets[f + 1];
        double c = centers ? centers[f] : 0.0, s = scales ? scales[f] : 1.0;
        double sum[3 * ORACLE_MAXDEG + 2], comp[3 * ORACLE_MAXDEG + 2];
        double S[2 * ORACLE_MAXDEG + 1], T[ORACLE_MAXDEG + 1];
        if (hi - lo < m + 1) {
            for (int k = 0; k <= m; ++k) a[f * stride + k] = NAN;
            status[f] = ST_SINGULAR;
            continue;
        }
        range_sums(x, y, dtype, lo, hi, m, c, s, sum, comp);
        for (int k = 0; k < 2 * m + 1; ++k) S[k] = sum[k] + comp[k];
        for (int j = 0; j <= m; ++j) T[j] = sum[2 * m + 1 + j] + comp[2 * m + 1 + j];
        status[f] = solve_sums(m, S, T, c, s, a + f * stride, NULL);
    }
    return ST_OK;
}

/* ---------------------------------------------------------------------------
 * Chebyshev basis (higher orders, which Sec. V leaves open): the same
 * least-squares problem with f(x) = sum_j c_j T_j(t), T_0 = 1, T_1 = t,
 * T_(k+1) = 2t T_k - T_(k-1).  Normal equations G c = D with the plain
 * definitions G_jk = sum_i T_j(t_i) T_k(t_i) and D_j = sum_i T_j(t_i) y_i,
 * every entry its own compensated sum (no product identity), then GEPP.
 * ------------------------------------------------------------------------- */
#define CHEB_NG(m) (((m) + 1) * ((m) + 2) / 2) /* upper triangle of G */

static void cheb_range_sums(const void *x, const void *y, int dtype, int64_t lo, int64_t hi, int m, double c,
                            double s, double *sum, double *comp) {
    int ng = CHEB_NG(m), nacc = ng + m + 1;
    double T[ORACLE_MAXDEG + 1];
    for (int k = 0; k < nacc; ++k) sum[k] = comp[k] = 0.0;
    for (int64_t i = lo; i < hi; ++i) {
        double t = (load(x, dtype, i) - c) / s;
        double yv = load(y, dtype, i);
        T[0] = 1.0;
        if (m >= 1) T[1] = t;
        for (int k = 1; k < m; ++k) T[k + 1] = 2.0 * t * T[k] - T[k - 1];
        int e = 0;
        for (int j = 0; j <= m; ++j)
            for (int k = j; k <= m; ++k, ++e) nadd(&sum[e], &comp[e], T[j] * T[k]);
        for (int j = 0; j <= m; ++j) nadd(&sum[ng + j], &comp[ng + j], T[j] * yv);
    }
}

static int cheb_solve(int m, const double *g, const double *D, double *cout) {
    double G[(ORACLE_MAXDEG + 1) * (ORACLE_MAXDEG + 1)], X[ORACLE_MAXDEG + 1], R[ORACLE_MAXDEG + 1];
    int n = m + 1, e = 0;
    for (int j = 0; j <= m; ++j)
        for (int k = j; k <= m; ++k, ++e) G[j * n + k] = G[k * n + j] = g[e];
    memcpy(R, D, sizeof(double) * n);
    int st = gepp(n, G, R, X);
    for (int k = 0; k < n; ++k) cout[k] = st == ST_OK ? X[k] : NAN;
    return st;
}

/* One fit: Chebyshev coefficients cout[m+1]; G_out[(m+1)^2] and D_out[m+1] nullable. */
int lse_oracle_cheb_fit(const void *x, const void *y, int64_t n, int dtype, int m, double c, double s,
                        double *cout, double *G_out, double *D_out, int nthreads) {
    if (m < 0 || m > ORACLE_MAXDEG || n < 0 || (dtype != 0 && dtype != 1) || !(s != 0.0)) return ST_INVALID;
    int ng = CHEB_NG(m), nacc = ng + m + 1;
    int64_t nchunk = (n + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
    double *part = (double *)calloc((size_t)(nchunk > 0 ? nchunk : 1) * 2 * nacc, sizeof(double));
    double tot[CHEB_NG(ORACLE_MAXDEG) + ORACLE_MAXDEG + 1];
    if (!part) return ST_INVALID;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t ch = 0; ch < nchunk; ++ch) {
        int64_t lo = ch * ORACLE_CHUNK, hi = lo + ORACLE_CHUNK < n ? lo + ORACLE_CHUNK : n;
        cheb_range_sums(x, y, dtype, lo, hi, m, c, s, part + ch * 2 * nacc, part + ch * 2 * nacc + nacc);
    }
    for (int k = 0; k < nacc; ++k) {
        double acc = 0.0, comp = 0.0;
        for (int64_t ch = 0; ch < nchunk; ++ch) {
            nadd(&acc, &comp, part[ch * 2 * nacc + k]);
            comp += part[ch * 2 * nacc + nacc + k];
        }
        tot[k] = acc + comp;
    }
    free(part);
    if (G_out) {
        int e = 0;
        for (int j = 0; j <= m; ++j)
            for (int k = j; k <= m; ++k, ++e) G_out[j * (m + 1) + k] = G_out[k * (m + 1) + j] = tot[e];
    }
    if (D_out) memcpy(D_out, tot + ng, sizeof(double) * (m + 1));
    if (n < m + 1) {
        for (int k = 0; k <= m; ++k) cout[k] = NAN;
        return ST_SINGULAR;
    }
    return cheb_solve(m, tot, tot + ng, cout);
}

/* Independent Chebyshev fits over CSR segments (layout as lse_oracle_fit_batched). */
int lse_oracle_cheb_fit_batched(const void *x, const void *y, const int64_t *offsets, const int32_t *degrees,
                                int64_t B, int dtype, const double *centers, const double *scales, int stride,
                                double *cout, int32_t *status, int nthreads) {
    if (B < 0 || (dtype != 0 && dtype != 1)) return ST_INVALID;
    for (int64_t f = 0; f < B; ++f)
        if (degrees[f] < 0 || degrees[f] > ORACLE_MAXDEG || degrees[f] + 1 > stride) return ST_INVALID;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int64_t f = 0; f < B; ++f) {
        int m = degrees[f];
        int64_t lo = offsets[f], hi = offsets[f + 1];
        double c = centers ? centers[f] : 0.0, s = scales ? scales[f] : 1.0;
        double sum[CHEB_NG(ORACLE_MAXDEG) + ORACLE_MAXDEG + 1], comp[CHEB_NG(ORACLE_MAXDEG) + ORACLE_MAXDEG + 1];
        if (hi - lo < m + 1) {
            for (int k = 0; k <= m; ++k) cout[f * stride + k] = NAN;
            status[f] = ST_SINGULAR;
            continue;
        }
        cheb_range_sums(x, y, dtype, lo, hi, m, c, s, sum, comp);
        int ng = CHEB_NG(m);
        for (int k = 0; k < ng + m + 1; ++k) sum[k] += comp[k];
        status[f] = cheb_solve(m, sum, sum + ng, cout + f * stride);
    }
    return ST_OK;
}

int lse_oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
