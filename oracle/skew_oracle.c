/*
 * Reference implementation of the dense real skew-symmetric eigensolver.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle: a plain, slow, FP64
 * host implementation that the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark compare the GPU library against.  It shares
 * no code, header or constant with the GPU library and is never called by it.
 *
 * What it computes (Penke, Marek, Vorwerk, Draxl, Benner, "High Performance
 * Solution of Skew-symmetric Eigenvalue Problems with Applications in Solving
 * the Bethe-Salpeter Eigenvalue Problem", Section 2.2, Algorithm 1):
 *
 *   A = -A^T (n x n, only the strict lower triangle is read)
 *   step 1  one-stage Householder tridiagonalization, Q_trd^T A Q_trd = A_trd,
 *           using the skew form of the rank-2 update of Section 2.3.1
 *           (A <- A + [v, -u1][u1, v]^T);
 *   step 2  Lemma 1: -i D^H A_trd D = T_sym with D = diag(i^k), k = 0..n-1, and
 *           T_sym the symmetric tridiagonal with zero diagonal whose off-
 *           diagonal is the SUPER-diagonal alpha of A_trd; its eigenpairs are
 *           found by Sturm-sequence bisection and inverse iteration (the
 *           tridiagonal method of the BSEPACK route, Section 3);
 *   step 3  Q <- D Q_diag, split into real and imaginary parts (Section 2.3);
 *   step 4  Q <- Q_trd Q, applied to the real and imaginary parts separately.
 *
 * Only the non-negative half of the spectrum is produced (Section 2.1: the
 * eigenvalues are +-i*lambda and the eigenvectors of a pair are complex
 * conjugates).  Returned: lambda[0..nev) = the nev smallest of the ceil(n/2)
 * values lambda >= 0 in ascending order, and z_k = Zre[:,k] + i Zim[:,k] with
 * A z_k = +i lambda_k z_k, ||z_k||_2 = 1.
 *
 * Pins (tests/test_oracle_pins.py): brute-force Hermitian eigensolve of -iA at
 * tiny n, prescribed spectra Q blockdiag([[0,l],[-l,0]]) Q^T with their known
 * eigenvectors, Clement and all-ones tridiagonals (closed-form spectra), the
 * bidiagonal singular-value link, brute-force Sturm counts, the odd-n null
 * vector, the Bethe-Salpeter eigenvalue identity, Frobenius invariants and the
 * special cases n = 0, 1, 2.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_NONFINITE 1
#define ORACLE_NOCONV 2
#define ORACLE_NOMEM 4

/* ------------------------------------------------------------------------ */
/* Householder reflector H = I - tau v v^T with v[0] = 1 and H x = beta e_1.
 * Convention of Golub & Van Loan (Alg. 5.1.1) / LAPACK dlarfg:
 * beta = -sign(x0) ||x||, tau = 0 (H = I) when x[1:] = 0.
 * On return x[1:] holds v[1:]; x[0] is left unchanged. */
static void house(int m, double *x, double *tau, double *beta)
{
    double alpha = x[0], sigma = 0.0;
    for (int i = 1; i < m; ++i) sigma += x[i] * x[i];
    if (m <= 1 || sigma == 0.0) {
        *tau = 0.0;
        *beta = alpha;
        for (int i = 1; i < m; ++i) x[i] = 0.0;
        return;
    }
    double norm = sqrt(alpha * alpha + sigma);
    double b = (alpha >= 0.0) ? -norm : norm;
    *tau = (b - alpha) / b;
    double scale = 1.0 / (alpha - b);
    for (int i = 1; i < m; ++i) x[i] *= scale;
    *beta = b;
}

/* ------------------------------------------------------------------------ */
/* Step 1 (Section 2.3.1): one-stage skew tridiagonalization.
 * A: strict lower triangle read (column-major, lda).
 * alpha[0..n-2]: super-diagonal of A_trd (alpha[j] = A_trd[j, j+1]).
 * V (n x n, ldv): column j holds v_j in rows j+1..n-1 (v_j[0] = 1 stored).
 * tau[0..n-1]: reflector scalars (tau[j] = 0 where no reflector is needed). */
int oracle_skew_tridiag(int n, const double *A, int lda, double *alpha,
                        double *V, int ldv, double *tau)
{
    if (n < 0) return -1;
    if (n == 0) return ORACLE_OK;
    if (!A) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    double *W = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    if (!W || !u || !x) { free(W); free(u); free(x); return ORACLE_NOMEM; }

    /* full skew working copy built from the strict lower triangle */
    for (int j = 0; j < n; ++j) {
        W[(size_t)j * n + j] = 0.0;
        for (int i = j + 1; i < n; ++i) {
            double a = A[(size_t)j * lda + i];
            W[(size_t)j * n + i] = a;
            W[(size_t)i * n + j] = -a;
        }
    }
    for (int j = 0; j < n; ++j) tau[j] = 0.0;
    if (V) for (int j = 0; j < n; ++j) memset(V + (size_t)j * ldv, 0, sizeof(double) * n);

    for (int j = 0; j + 2 < n; ++j) {
        int m = n - j - 1;                 /* trailing block rows/cols j+1..n-1 */
        double *col = W + (size_t)j * n + (j + 1);
        for (int i = 0; i < m; ++i) x[i] = col[i];
        double t, beta;
        house(m, x, &t, &beta);
        x[0] = 1.0;
        tau[j] = t;
        if (V) for (int i = 0; i < m; ++i) V[(size_t)j * ldv + j + 1 + i] = x[i];
        /* column j becomes beta e1, row j becomes -beta e1^T */
        for (int i = 0; i < m; ++i) {
            col[i] = (i == 0) ? beta : 0.0;
            W[(size_t)(j + 1 + i) * n + j] = (i == 0) ? -beta : 0.0;
        }
        alpha[j] = -beta;
        if (t == 0.0) continue;
        /* A v on the trailing block, then v^T A v */
        double *T0 = W + (size_t)(j + 1) * n + (j + 1);
        #pragma omp parallel for schedule(static)
        for (int r = 0; r < m; ++r) {
            double s = 0.0;
            for (int c = 0; c < m; ++c) s += T0[(size_t)c * n + r] * x[c];
            u[r] = s;
        }
        double vav = 0.0;
        for (int r = 0; r < m; ++r) vav += x[r] * u[r];
        /* u1 = 0.5 tau^2 (v^T A v) v - tau A^T v  with A^T = -A  (Eq. of the
         * one-stage update; the skew case has u2 = -u1) */
        for (int r = 0; r < m; ++r) u[r] = 0.5 * t * t * vav * x[r] + t * u[r];
        /* A <- A + v u1^T - u1 v^T  (skew rank-2 update) */
        #pragma omp parallel for schedule(static)
        for (int c = 0; c < m; ++c) {
            double *Tc = T0 + (size_t)c * n;
            double uc = u[c], vc = x[c];
            for (int r = 0; r < m; ++r) Tc[r] += x[r] * uc - u[r] * vc;
        }
    }
    if (n >= 2) alpha[n - 2] = W[(size_t)(n - 1) * n + (n - 2)];
    free(W); free(u); free(x);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Step 2: the symmetric tridiagonal T_sym = tridiag(alpha, 0, alpha). */

static double tri_norm(int n, const double *alpha)
{   /* infinity norm of T_sym */
    double g = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = (i > 0 ? fabs(alpha[i - 1]) : 0.0) + (i + 1 < n ? fabs(alpha[i]) : 0.0);
        if (r > g) g = r;
    }
    return g;
}

static double tri_pivmin(int n, const double *alpha)
{
    double m = 1.0;
    for (int i = 0; i + 1 < n; ++i) if (alpha[i] * alpha[i] > m) m = alpha[i] * alpha[i];
    return DBL_MIN * m;
}

/* Sturm count: number of eigenvalues of T_sym strictly below x, i.e. the
 * number of negative pivots of the LDL^T factorisation of T_sym - x I. */
int oracle_sturm_count(int n, const double *alpha, double x)
{
    if (n <= 0) return 0;
    double pivmin = tri_pivmin(n, alpha);
    int cnt = 0;
    double d = -x;
    if (fabs(d) < pivmin) d = -pivmin;
    if (d < 0.0) ++cnt;
    for (int i = 1; i < n; ++i) {
        d = -x - alpha[i - 1] * alpha[i - 1] / d;
        if (fabs(d) < pivmin) d = -pivmin;
        if (d < 0.0) ++cnt;
    }
    return cnt;
}

/* Bisection for the eigenvalues with ascending indices first..first+count-1. */
int oracle_tridiag_eigvals(int n, const double *alpha, int first, int count, double *w)
{
    if (n < 0) return -1;
    if (count <= 0) return ORACLE_OK;
    if (first < 0 || first + count > n) return -3;
    double g = tri_norm(n, alpha);
    double pivmin = tri_pivmin(n, alpha);
    double eps = DBL_EPSILON;
    double glo = -g * (1.0 + 2.0 * eps) - 2.0 * pivmin;
    double ghi = g * (1.0 + 2.0 * eps) + 2.0 * pivmin;
    double abstol = eps * g + 2.0 * pivmin;
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+:bad)
    for (int k = 0; k < count; ++k) {
        int idx = first + k;
        double lo = glo, hi = ghi;
        int it = 0;
        while (hi - lo > 2.0 * eps * fmax(fabs(lo), fabs(hi)) + abstol) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (oracle_sturm_count(n, alpha, mid) > idx) hi = mid; else lo = mid;
            if (++it > 400) { ++bad; break; }
        }
        w[k] = 0.5 * (lo + hi);
    }
    /* odd n: the middle eigenvalue of a matrix with +-symmetric spectrum is 0 */
    if (n % 2 == 1) {
        int mid = n / 2;
        if (mid >= first && mid < first + count) w[mid - first] = 0.0;
    }
    return bad ? ORACLE_NOCONV : ORACLE_OK;
}

/* splitmix64, used only to draw the start vectors of inverse iteration */
static uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Solve (T_sym - s I) y = b by Gaussian elimination with partial pivoting on
 * the tridiagonal (U gets a second super-diagonal).  Zero pivots are replaced
 * by a tiny value of the same sign, as inverse iteration requires. */
typedef struct { double *u0, *u1, *u2, *l; char *swp; } trilu;

static void tri_factor(int n, const double *alpha, double s, double tiny, trilu *f)
{
    double a = -s, b = (n > 1) ? alpha[0] : 0.0, c = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        double sub = alpha[i], dn = -s, en = (i + 2 < n) ? alpha[i + 1] : 0.0;
        if (fabs(a) >= fabs(sub)) {
            if (a == 0.0) a = tiny;
            double l = sub / a;
            f->swp[i] = 0; f->l[i] = l;
            f->u0[i] = a; f->u1[i] = b; f->u2[i] = c;
            a = dn - l * b; b = en - l * c; c = 0.0;
        } else {
            double l = a / sub;
            f->swp[i] = 1; f->l[i] = l;
            f->u0[i] = sub; f->u1[i] = dn; f->u2[i] = en;
            a = b - l * dn; b = c - l * en; c = 0.0;
        }
    }
    if (fabs(a) < tiny) a = (a < 0.0) ? -tiny : tiny;
    f->u0[n - 1] = a; f->u1[n - 1] = 0.0; f->u2[n - 1] = 0.0;
    if (n >= 2) f->u2[n - 2] = 0.0;
    for (int i = 0; i < n; ++i) if (fabs(f->u0[i]) < tiny) f->u0[i] = (f->u0[i] < 0.0) ? -tiny : tiny;
}

static void tri_solve(int n, const trilu *f, double *y)
{
    for (int i = 0; i + 1 < n; ++i) {
        if (f->swp[i]) { double t = y[i]; y[i] = y[i + 1]; y[i + 1] = t; }
        y[i + 1] -= f->l[i] * y[i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double r = y[i];
        if (i + 1 < n) r -= f->u1[i] * y[i + 1];
        if (i + 2 < n) r -= f->u2[i] * y[i + 2];
        y[i] = r / f->u0[i];
    }
}

static double nrm2(int n, const double *x)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += x[i] * x[i];
    return sqrt(s);
}

/* Eigenvectors of T_sym for the ascending eigenvalues w[0..count) (already
 * computed, non-decreasing) by inverse iteration.  Consecutive eigenvalues
 * closer than 1e-3 ||T|| form a cluster; inside a cluster each new vector is
 * re-orthogonalised (twice, classical Gram-Schmidt) against the earlier ones at
 * every iteration, as in LAPACK's dstein.  For lambda > 0 the even- and odd-
 * indexed halves of an exact eigenvector have equal norm (the mirror vector of
 * -lambda is the same vector with alternating signs), so each half is scaled
 * to 1/sqrt(2) at the end.  An exact zero eigenvalue of an odd-order unreduced
 * T_sym gets its null vector from the two-term recurrence of T q = 0 (odd
 * entries zero).  Q is n x count, column-major, ldq. */
int oracle_tridiag_eigvecs(int n, const double *alpha, int count, const double *w,
                           double *Q, int ldq, uint64_t seed)
{
    if (n < 0) return -1;
    if (count <= 0 || n == 0) return ORACLE_OK;
    if (n == 1) { Q[0] = 1.0; return ORACLE_OK; }
    double g = tri_norm(n, alpha);
    double eps = DBL_EPSILON;
    double ortol = 1e-3 * g;
    double tiny = eps * (g > 0.0 ? g : 1.0);
    int bad = 0;

    /* cluster boundaries */
    int *cstart = (int *)malloc(sizeof(int) * (count + 1));
    int ncl = 0;
    for (int k = 0; k < count; ++k)
        if (k == 0 || w[k] - w[k - 1] > ortol) cstart[ncl++] = k;
    cstart[ncl] = count;

    #pragma omp parallel reduction(+:bad)
    {
        trilu f;
        f.u0 = (double *)malloc(sizeof(double) * n);
        f.u1 = (double *)malloc(sizeof(double) * n);
        f.u2 = (double *)malloc(sizeof(double) * n);
        f.l = (double *)malloc(sizeof(double) * n);
        f.swp = (char *)malloc(n);
        double *y = (double *)malloc(sizeof(double) * n);
        #pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < ncl; ++c) {
            double prev_shift = -INFINITY;
            for (int k = cstart[c]; k < cstart[c + 1]; ++k) {
                double *q = Q + (size_t)k * ldq;
                int unreduced_odd = (n % 2 == 1) && (w[k] == 0.0);
                if (unreduced_odd)
                    for (int i = 1; i < n; i += 2) if (alpha[i] == 0.0) unreduced_odd = 0;
                if (unreduced_odd) {
                    /* T q = 0 with q_odd = 0: q_{2m+2} = -alpha_{2m} q_{2m} / alpha_{2m+1} */
                    for (int i = 0; i < n; ++i) q[i] = 0.0;
                    q[0] = 1.0;
                    for (int m2 = 0; m2 + 2 < n; m2 += 2) {
                        q[m2 + 2] = -alpha[m2] * q[m2] / alpha[m2 + 1];
                        if (fabs(q[m2 + 2]) > 1e150) for (int i = 0; i <= m2 + 2; i += 2) q[i] *= 1e-150;
                    }
                    double s = nrm2(n, q);
                    for (int i = 0; i < n; ++i) q[i] /= s;
                    continue;
                }
                /* separate coincident shifts slightly (dstein) */
                double shift = w[k];
                if (shift - prev_shift < 10.0 * eps * fabs(shift)) shift = prev_shift + 10.0 * eps * fabs(shift);
                prev_shift = shift;
                tri_factor(n, alpha, shift, tiny, &f);
                uint64_t st = seed ^ ((uint64_t)(k + 1) * 0x9e3779b97f4a7c15ULL);
                for (int i = 0; i < n; ++i) {
                    st = mix64(st);
                    y[i] = ((double)(st >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
                }
                int conv = 0;
                for (int it = 0; it < 8; ++it) {
                    double s = nrm2(n, y);
                    for (int i = 0; i < n; ++i) y[i] /= s;
                    tri_solve(n, &f, y);
                    double grow = nrm2(n, y);
                    /* re-orthogonalise against the earlier members of the cluster */
                    for (int pass = 0; pass < 2; ++pass)
                        for (int j = cstart[c]; j < k; ++j) {
                            const double *qj = Q + (size_t)j * ldq;
                            double d = 0.0;
                            for (int i = 0; i < n; ++i) d += qj[i] * y[i];
                            for (int i = 0; i < n; ++i) y[i] -= d * qj[i];
                        }
                    if (grow * tiny >= 1e-3 * 1.0) { if (++conv >= 2) break; }
                }
                if (!conv) ++bad;
                double s = nrm2(n, y);
                for (int i = 0; i < n; ++i) q[i] = y[i] / s;
                if (w[k] > 0.0) {
                    double se = 0.0, so = 0.0;
                    for (int i = 0; i < n; i += 2) se += q[i] * q[i];
                    for (int i = 1; i < n; i += 2) so += q[i] * q[i];
                    if (se > 0.0 && so > 0.0) {
                        double fe = sqrt(0.5 / se), fo = sqrt(0.5 / so);
                        for (int i = 0; i < n; i += 2) q[i] *= fe;
                        for (int i = 1; i < n; i += 2) q[i] *= fo;
                    }
                }
            }
        }
        free(f.u0); free(f.u1); free(f.u2); free(f.l); free(f.swp); free(y);
    }
    free(cstart);
    return bad ? ORACLE_NOCONV : ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* The whole solver (Algorithm 1, steps 1-4). */
int oracle_skew_evd(int n, const double *A, int lda, int nev,
                    double *lambda, double *Zre, double *Zim, int ldz)
{
    if (n < 0) return -1;
    if (n > 0 && !A) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    int half = (n + 1) / 2;
    if (nev < 0 || nev > half) return -4;
    if (nev > 0 && !lambda) return -5;
    if (nev > 0 && !Zre) return -6;
    if (nev > 0 && !Zim) return -7;
    if (ldz < (n > 1 ? n : 1)) return -8;
    if (n == 0 || nev == 0) return ORACLE_OK;
    for (int j = 0; j < n; ++j)
        for (int i = j + 1; i < n; ++i)
            if (!isfinite(A[(size_t)j * lda + i])) return ORACLE_NONFINITE;

    double *alpha = (double *)calloc((size_t)n, sizeof(double));
    double *V = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *tau = (double *)malloc(sizeof(double) * (size_t)n);
    double *Q = (double *)malloc(sizeof(double) * (size_t)n * nev);
    if (!alpha || !V || !tau || !Q) { free(alpha); free(V); free(tau); free(Q); return ORACLE_NOMEM; }

    int st = oracle_skew_tridiag(n, A, lda, alpha, V, n, tau);           /* step 1 */
    int st2 = ORACLE_OK;
    if (st == ORACLE_OK) {
        st2 = oracle_tridiag_eigvals(n, alpha, n / 2, nev, lambda);      /* step 2 */
        /* the upper half of a +-symmetric spectrum is >= 0; a bisection midpoint
         * may land a rounding error below zero */
        for (int k = 0; k < nev; ++k) if (lambda[k] < 0.0) lambda[k] = 0.0;
        if (st2 == ORACLE_OK)
            st2 = oracle_tridiag_eigvecs(n, alpha, nev, lambda, Q, n, 0x5eedULL);
    }
    if (st != ORACLE_OK || st2 != ORACLE_OK) {
        free(alpha); free(V); free(tau); free(Q);
        return st != ORACLE_OK ? st : st2;
    }
    /* step 3: Q <- D Q_diag, D_kk = i^k; real and imaginary parts apart */
    for (int c = 0; c < nev; ++c) {
        double *zr = Zre + (size_t)c * ldz, *zi = Zim + (size_t)c * ldz;
        const double *q = Q + (size_t)c * n;
        for (int k = 0; k < n; ++k) {
            switch (k & 3) {
            case 0: zr[k] = q[k];  zi[k] = 0.0;   break;
            case 1: zr[k] = 0.0;   zi[k] = q[k];  break;
            case 2: zr[k] = -q[k]; zi[k] = 0.0;   break;
            default: zr[k] = 0.0;  zi[k] = -q[k]; break;
            }
        }
    }
    /* step 4: Q <- Q_trd Q = H_0 H_1 ... H_{n-3} Q, last reflector first */
    #pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < 2 * nev; ++c) {
        double *z = (c < nev) ? Zre + (size_t)c * ldz : Zim + (size_t)(c - nev) * ldz;
        for (int j = n - 3; j >= 0; --j) {
            if (tau[j] == 0.0) continue;
            const double *v = V + (size_t)j * n;
            double s = 0.0;
            for (int i = j + 1; i < n; ++i) s += v[i] * z[i];
            s *= tau[j];
            for (int i = j + 1; i < n; ++i) z[i] -= s * v[i];
        }
    }
    free(alpha); free(V); free(tau); free(Q);
    return ORACLE_OK;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
