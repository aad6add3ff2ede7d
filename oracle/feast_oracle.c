/*
 * FEAST oracle -- a plain, slow, obviously correct FP64 CPU implementation of
 * dense Hermitian FEAST (real symmetric and complex Hermitian pencils).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library uses this file;
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no code, header or constant table with the GPU library.
 *
 * Everything is double / double complex, column-major (the guide's dense
 * storage, section "Matrix storage").  No BLAS or LAPACK is used: the LU, the
 * triangular solves, the matrix products and the Jacobi eigensolver are
 * written out below, unblocked, in the textbook order.  OpenMP only splits
 * independent columns across threads; it does not reorder any sum.
 *
 * Method (guide, section "The FEAST Algorithm"): Q = sum_j w_j Q_j where
 * (z_j B - A) Q_j = B X at the quadrature nodes z_j of a contour around
 * [Emin, Emax]; then Rayleigh-Ritz on Q gives a reduced M0 x M0 problem whose
 * solution updates X; repeat.  Readings of points the guide leaves open are
 * marked "Reading:" below.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

static double cabs1(zc v) { return fabs(creal(v)) + fabs(cimag(v)); }

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1, 1] (the default Hermitian quadrature,
 * fpm(16)=0, Table "tab_fpm").  Roots of P_n by Newton's method on the
 * three-term recurrence (k+1) P_{k+1} = (2k+1) t P_k - k P_{k-1}, started
 * from cos(pi (i + 3/4) / (n + 1/2)); weights 2 / ((1 - x^2) P_n'(x)^2).
 * Nodes are returned in ascending order.                                    */
int orc_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1) return -1;
    for (int i = 0; i < n; ++i) {
        double t = cos(M_PI * (i + 0.75) / (n + 0.5));
        double pn = 0.0, dpn = 1.0;
        for (int it = 0; it < 200; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            pn = (n == 1) ? t : p1;
            double pm = (n == 1) ? 1.0 : p0;
            dpn = n * (t * pn - pm) / (t * t - 1.0);
            double dt = pn / dpn;
            t -= dt;
            if (fabs(dt) <= 1e-16 * (1.0 + fabs(t))) break;
        }
        /* derivative at the converged root, for the weight */
        {
            double p0 = 1.0, p1 = t;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            pn = (n == 1) ? t : p1;
            double pm = (n == 1) ? 1.0 : p0;
            dpn = n * (t * pn - pm) / (t * t - 1.0);
        }
        /* descending roots, stored ascending */
        x[n - 1 - i] = t;
        w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dpn * dpn);
    }
    return 0;
}

/* Half-contour nodes and weights (section "Defining a search contour";
 * tool "[cz]feast_contour"; Table "tab_fpm" fpm(2), fpm(16), fpm(18)).
 * The contour through Emin and Emax is the ellipse
 *     z(t) = c + r cos t + i a r sin t,  c = (Emin+Emax)/2, r = (Emax-Emin)/2,
 * a = ratio/100 (vertical over horizontal semi-axis; 1 is the circle).  The
 * filter is (1/(2 pi i)) times the contour integral of dz/(z - lambda); the
 * lower half mirrors the upper one, so for real lambda it is twice the real
 * part of the upper-half integral:
 *     rho(lambda) = Re (1/pi) int_0^pi (a r cos t + i r sin t)/(z(t) - lambda) dt,
 * since dz/(2 pi i) = (a r cos t + i r sin t) dt / (2 pi).  A rule with
 * points t_j and weights dt_j on [0, pi] gives z_j = z(t_j) and
 * w_j = (dt_j/pi)(a r cos t_j + i r sin t_j):
 *   integ 0 (Gauss-Legendre): t_j = (pi/2)(1 - x_j), dt_j = (pi/2) omega_j;
 *   integ 1 (trapezoidal, midpoints): t_j = pi (ne - j - 1/2)/ne, dt_j = pi/ne.
 * Both list the nodes from t near pi down to t near 0 (increasing real part).
 * Reading: the 1/2-free form above is fixed so that the Gauss circle filter
 * equals 1 at the centre and 1/2 at both endpoints, and the trapezoidal
 * circle filter is 1/(1 + t^(2 ne)) with t = (lambda - c)/r.                */
int orc_contour(double emin, double emax, int ne, int integ, int ratio, zc *z, zc *w)
{
    if (ne < 1 || !(emin < emax) || (integ != 0 && integ != 1) || ratio < 1) return -1;
    double *t = malloc(sizeof(double) * ne), *dt = malloc(sizeof(double) * ne);
    if (integ == 0) {
        double *x = malloc(sizeof(double) * ne), *om = malloc(sizeof(double) * ne);
        orc_gauss_legendre(ne, x, om);
        for (int j = 0; j < ne; ++j) {
            t[j] = 0.5 * M_PI * (1.0 - x[j]);
            dt[j] = 0.5 * M_PI * om[j];
        }
        free(x);
        free(om);
    } else {
        for (int j = 0; j < ne; ++j) {
            t[j] = M_PI * (ne - j - 0.5) / ne;
            dt[j] = M_PI / ne;
        }
    }
    double c = 0.5 * (emin + emax), r = 0.5 * (emax - emin), a = ratio / 100.0;
    for (int j = 0; j < ne; ++j) {
        z[j] = c + r * cos(t[j]) + I * a * r * sin(t[j]);
        w[j] = (dt[j] / M_PI) * (a * r * cos(t[j]) + I * r * sin(t[j]));
    }
    free(t);
    free(dt);
    return 0;
}

/* Rational filter rho(lambda) = Re sum_j w_j / (z_j - lambda) of given
 * nodes and weights: what one contour pass multiplies each eigencomponent by
 * (tools "[sd]feast_rational", "[sd]feast_rationalx").                     */
void orc_rationalx(int ne, const zc *z, const zc *w, const double *lam, int m, double *f)
{
    for (int i = 0; i < m; ++i) {
        zc s = 0;
        for (int j = 0; j < ne; ++j) s += w[j] / (z[j] - lam[i]);
        f[i] = creal(s);
    }
}

int orc_rational(double emin, double emax, int ne, int integ, int ratio, const double *lam, int m, double *f)
{
    zc *z = malloc(sizeof(zc) * ne), *w = malloc(sizeof(zc) * ne);
    if (orc_contour(emin, emax, ne, integ, ratio, z, w)) { free(z); free(w); return -1; }
    orc_rationalx(ne, z, w, lam, m, f);
    free(z);
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* LU with partial pivoting, P A = L U, unblocked right-looking, in place
 * (the factorisation step, ijob 10 of Figure "fig_rci").  Pivot = largest
 * |re|+|im| in the column, ties to the lowest row.  ipiv[k] = row swapped
 * with row k at step k.  Returns 0, or k+1 when the k-th pivot is zero or
 * not finite.                                                              */
int orc_zgetrf(int n, zc *a, int lda, int *ipiv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = cabs1(a[IDX(k, k, lda)]);
        for (int i = k + 1; i < n; ++i) {
            double v = cabs1(a[IDX(i, k, lda)]);
            if (v > best) { best = v; p = i; }
        }
        ipiv[k] = p;
        if (!(best > 0.0) || !isfinite(best)) return k + 1;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                zc t = a[IDX(k, j, lda)];
                a[IDX(k, j, lda)] = a[IDX(p, j, lda)];
                a[IDX(p, j, lda)] = t;
            }
        zc piv = a[IDX(k, k, lda)];
        for (int i = k + 1; i < n; ++i) a[IDX(i, k, lda)] /= piv;
#pragma omp parallel for schedule(static) if (n - k > 128)
        for (int j = k + 1; j < n; ++j) {
            zc u = a[IDX(k, j, lda)];
            if (u != 0)
                for (int i = k + 1; i < n; ++i) a[IDX(i, j, lda)] -= a[IDX(i, k, lda)] * u;
        }
    }
    for (int k = 0; k < n; ++k)
        if (!isfinite(creal(a[IDX(k, k, lda)])) || !isfinite(cimag(a[IDX(k, k, lda)])))
            return k + 1;
    return 0;
}

/* Solve with the LU factors for nrhs right-hand sides (ijob 11), or with
 * their adjoint (ijob 21, reusing the same factors):
 *   trans = 'N':  A x = b   ->  b <- P b, L y = b, U x = y
 *   trans = 'C':  A^H x = b ->  U^H y = b, L^H v = y, x = P^T v           */
int orc_zgetrs(char trans, int n, int nrhs, const zc *a, int lda, const int *ipiv,
               zc *b, int ldb)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nrhs; ++c) {
        zc *x = b + (size_t)c * ldb;
        if (trans == 'N') {
            for (int k = 0; k < n; ++k)
                if (ipiv[k] != k) { zc t = x[k]; x[k] = x[ipiv[k]]; x[ipiv[k]] = t; }
            for (int k = 0; k < n; ++k)           /* unit lower, column sweep */
                for (int i = k + 1; i < n; ++i) x[i] -= a[IDX(i, k, lda)] * x[k];
            for (int k = n - 1; k >= 0; --k) {    /* upper */
                x[k] /= a[IDX(k, k, lda)];
                for (int i = 0; i < k; ++i) x[i] -= a[IDX(i, k, lda)] * x[k];
            }
        } else {
            for (int k = 0; k < n; ++k) {         /* U^H is lower: row k of U^H = conj col k of U */
                zc s = x[k];
                for (int i = 0; i < k; ++i) s -= conj(a[IDX(i, k, lda)]) * x[i];
                x[k] = s / conj(a[IDX(k, k, lda)]);
            }
            for (int k = n - 1; k >= 0; --k) {    /* L^H is unit upper */
                zc s = x[k];
                for (int i = k + 1; i < n; ++i) s -= conj(a[IDX(i, k, lda)]) * x[i];
                x[k] = s;
            }
            for (int k = n - 1; k >= 0; --k)
                if (ipiv[k] != k) { zc t = x[k]; x[k] = x[ipiv[k]]; x[ipiv[k]] = t; }
        }
    }
    return 0;
}

/* C = op(A) B, op = identity ('N') or conjugate transpose ('C').
 * op(A) is m x k, B is k x n, C is m x n; plain triple loop.               */
void orc_zgemm(char opa, int m, int n, int k, const zc *a, int lda, const zc *b, int ldb,
               zc *c, int ldc)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) {
            zc s = 0;
            if (opa == 'N')
                for (int l = 0; l < k; ++l) s += a[IDX(i, l, lda)] * b[IDX(l, j, ldb)];
            else
                for (int l = 0; l < k; ++l) s += conj(a[IDX(l, i, lda)]) * b[IDX(l, j, ldb)];
            c[IDX(i, j, ldc)] = s;
        }
}

/* ------------------------------------------------------------------------ */
/* Cyclic Jacobi for a Hermitian n x n matrix (the reduced dense eigenproblem
 * of the Rayleigh-Ritz step).  a is overwritten; on return w holds the
 * eigenvalues ascending and v (n x n) the orthonormal eigenvectors.
 * Rotation for the pair (p, q) with a_pq = b e^{i phi}:
 *   tau = (a_qq - a_pp)/(2b), t = sign(tau)/(|tau| + sqrt(1+tau^2)),
 *   c = 1/sqrt(1+t^2), s = t c,  J = [[c, s e^{i phi}], [-s e^{-i phi}, c]],
 *   A <- J^H A J,  V <- V J.
 * Sweeps p < q in row order until off(A) <= 1e-15 ||A||_F (at most 100).
 * Returns 0, or -1 without convergence.                                    */
int orc_zheev_jacobi(int n, zc *a, int lda, double *w, zc *v, int ldv)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) v[IDX(i, j, ldv)] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) fro += creal(a[IDX(i, j, lda)] * conj(a[IDX(i, j, lda)]));
    fro = sqrt(fro);
    int ok = 0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                if (i != j) off += creal(a[IDX(i, j, lda)] * conj(a[IDX(i, j, lda)]));
        if (sqrt(off) <= 1e-15 * fro || fro == 0.0) { ok = 1; break; }
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                zc apq = a[IDX(p, q, lda)];
                double b = cabs(apq);
                if (b == 0.0) continue;
                zc ph = apq / b;
                double app = creal(a[IDX(p, p, lda)]), aqq = creal(a[IDX(q, q, lda)]);
                double tau = (aqq - app) / (2.0 * b);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* columns: A <- A J */
                for (int r = 0; r < n; ++r) {
                    zc arp = a[IDX(r, p, lda)], arq = a[IDX(r, q, lda)];
                    a[IDX(r, p, lda)] = c * arp - s * conj(ph) * arq;
                    a[IDX(r, q, lda)] = s * ph * arp + c * arq;
                }
                /* rows: A <- J^H A */
                for (int col = 0; col < n; ++col) {
                    zc apc = a[IDX(p, col, lda)], aqc = a[IDX(q, col, lda)];
                    a[IDX(p, col, lda)] = c * apc - s * ph * aqc;
                    a[IDX(q, col, lda)] = s * conj(ph) * apc + c * aqc;
                }
                a[IDX(p, q, lda)] = 0.0;
                a[IDX(q, p, lda)] = 0.0;
                a[IDX(p, p, lda)] = creal(a[IDX(p, p, lda)]);
                a[IDX(q, q, lda)] = creal(a[IDX(q, q, lda)]);
                for (int r = 0; r < n; ++r) {
                    zc vrp = v[IDX(r, p, ldv)], vrq = v[IDX(r, q, ldv)];
                    v[IDX(r, p, ldv)] = c * vrp - s * conj(ph) * vrq;
                    v[IDX(r, q, ldv)] = s * ph * vrp + c * vrq;
                }
            }
    }
    for (int i = 0; i < n; ++i) w[i] = creal(a[IDX(i, i, lda)]);
    /* ascending order, vectors follow (selection sort) */
    for (int i = 0; i < n; ++i) {
        int m = i;
        for (int j = i + 1; j < n; ++j)
            if (w[j] < w[m]) m = j;
        if (m != i) {
            double t = w[i]; w[i] = w[m]; w[m] = t;
            for (int r = 0; r < n; ++r) {
                zc tv = v[IDX(r, i, ldv)];
                v[IDX(r, i, ldv)] = v[IDX(r, m, ldv)];
                v[IDX(r, m, ldv)] = tv;
            }
        }
    }
    return ok ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* Stochastic estimate of the number of eigenvalues in the interval (section
 * "Stochastic estimate"; the method of the Di Napoli-Polizzi-Saad paper it
 * cites).  One contour pass applied to probe vectors x_c gives
 * q_c = rho(B^{-1} A) x_c, whose trace is sum_i rho(lambda_i), about the count.
 * Each probe gives the sample e_c = n Re(x_c^H q_c) / (x_c^H x_c): the
 * Hutchinson estimator when x_c has entries +-1 (then x_c^H x_c = n), and
 * unbiased for any probe distribution invariant under rotations.
 *   res[c]   running average (e_0 + ... + e_c) / (c + 1), summed in order
 *   *M_out   nearest integer to res[m0 - 1], at least 0                    */
void orc_count_estimate(int n, int m0, const zc *X0, const zc *Q, double *res, int *M_out)
{
    double sum = 0.0;
    for (int c = 0; c < m0; ++c) {
        double num = 0.0, den = 0.0;
        for (int i = 0; i < n; ++i) {
            const zc x = X0[IDX(i, c, n)];
            num += creal(conj(x) * Q[IDX(i, c, n)]);
            den += creal(x) * creal(x) + cimag(x) * cimag(x);
        }
        sum += den > 0.0 ? n * num / den : 0.0;
        res[c] = sum / (c + 1);
    }
    const double est = floor(res[m0 - 1] + 0.5);
    *M_out = est > 0.0 ? (int)est : 0;
}

/* The FEAST iteration for a dense Hermitian pencil (A, B), B = NULL for the
 * standard problem.  Arguments follow Table "tab_common":
 *   herm      0: real symmetric (A, B, X0 real, stored with zero imaginary
 *             parts), 1: complex Hermitian
 *   m0_io     in: subspace size M0; out: the size actually kept
 *   X0        (n x m0) start subspace (the caller draws it, fpm(5) style)
 *   E, X, res outputs of size m0, n x m0, m0 (first M are the eigenpairs in
 *             the interval, ascending)
 *   mode      0: full iteration; 1: return Q after one contour (info 4);
 *             2: stochastic estimate of the eigenvalue count (info 5), see
 *             orc_count_estimate
 *   integ, ratio  fpm(16) (0 Gauss-Legendre, 1 trapezoidal) and fpm(18)
 *             (ellipse ratio in percent), see orc_contour
 *   zne, wne  custom nodes and weights (expert mode), or NULL
 * Returns info with the codes of Table "tab_info".                         */
#define ORC_SPURIOUS_RES 0.1
#define ORC_TRUNC 1e-14
#define ORC_INDEFINITE 1e-8

int orc_feast(int herm, int n, const zc *A, const zc *B, double emin, double emax,
              int *m0_io, int ne, double tol, int maxloop, int conv, int mode,
              const zc *X0, double *E, zc *X, double *res, int *M_out, int *loop_out,
              double *epsout_out, int integ, int ratio, const zc *zne, const zc *wne)
{
    int m0 = m0_io ? *m0_io : 0;
    /* input checks, Table "tab_info" */
    if (n < 1) return 202;
    if (m0 < 1 || m0 > n) return 201;
    if (!(emin < emax)) return 200;
    if (ne < 1) return 102;
    if (!(tol > 0.0)) return 103;
    if (maxloop < 0) return 104;
    if (conv != 0 && conv != 1) return 106;
    if (mode < 0 || mode > 2) return 114;
    if (integ != 0 && integ != 1) return 116;
    if (ratio < 1) return 118;

    const double alpha = fmax(fabs(emin), fabs(emax));
    const size_t nn = (size_t)n * n, nm = (size_t)n * m0;
    int info = 0;

    zc *z = malloc(sizeof(zc) * ne), *w = malloc(sizeof(zc) * ne);
    if (zne && wne) {   /* expert mode: the caller's nodes and weights */
        for (int j = 0; j < ne; ++j) {
            z[j] = zne[j];
            w[j] = wne[j];
        }
    } else {
        orc_contour(emin, emax, ne, integ, ratio, z, w);
    }

    zc *fac = malloc(sizeof(zc) * nn * ne);
    int *piv = malloc(sizeof(int) * (size_t)n * ne);
    zc *Xc = malloc(sizeof(zc) * nm), *R = malloc(sizeof(zc) * nm), *Y = malloc(sizeof(zc) * nm);
    zc *Q = malloc(sizeof(zc) * nm), *AQ = malloc(sizeof(zc) * nm), *BQ = malloc(sizeof(zc) * nm);
    zc *Aq = malloc(sizeof(zc) * m0 * m0), *Bq = malloc(sizeof(zc) * m0 * m0);
    zc *Wb = malloc(sizeof(zc) * m0 * m0), *T = malloc(sizeof(zc) * m0 * m0);
    zc *Cr = malloc(sizeof(zc) * m0 * m0), *V = malloc(sizeof(zc) * m0 * m0);
    zc *Phi = malloc(sizeof(zc) * m0 * m0), *tmp = malloc(sizeof(zc) * m0 * m0);
    zc *AX = malloc(sizeof(zc) * nm), *BX = malloc(sizeof(zc) * nm);
    double *beta = malloc(sizeof(double) * m0), *lam = malloc(sizeof(double) * m0);
    double *rs = malloc(sizeof(double) * m0);
    int *order = malloc(sizeof(int) * m0);
    if (!fac || !piv || !Xc || !R || !Y || !Q || !AQ || !BQ || !Aq || !Bq || !Wb || !T || !Cr ||
        !V || !Phi || !tmp || !AX || !BX || !beta || !lam || !rs || !order) {
        info = -1;
        goto done;
    }
    memcpy(Xc, X0, sizeof(zc) * nm);

    double trace_prev = 0.0, epsout = 1.0;
    int M = 0, k = 0;
    for (k = 0; k <= maxloop; ++k) {
        /* (a) right-hand sides B X (a copy for the standard problem, ijob 40) */
        if (B) orc_zgemm('N', n, m0, n, B, n, Xc, n, R, n);
        else memcpy(R, Xc, sizeof(zc) * (size_t)n * m0);

        /* (b) factor each shifted matrix once and keep the factors (fpm(10)=1);
         *     solve; accumulate the quadrature in node order.              */
        memset(Q, 0, sizeof(zc) * (size_t)n * m0);
        for (int j = 0; j < ne; ++j) {
            zc *F = fac + nn * j;
            int *pv = piv + (size_t)n * j;
            if (k == 0) {
                for (size_t e = 0; e < nn; ++e) F[e] = (B ? z[j] * B[e] : 0.0) - A[e];
                if (!B)
                    for (int i = 0; i < n; ++i) F[IDX(i, i, n)] += z[j];
                if (orc_zgetrf(n, F, n, pv)) { info = -2; goto done; }
            }
            memcpy(Y, R, sizeof(zc) * (size_t)n * m0);
            orc_zgetrs('N', n, m0, F, n, pv, Y, n);
            if (!herm) {
                /* real symmetric: Q += Re(w_j Y_j) */
                for (size_t e = 0; e < (size_t)n * m0; ++e) Q[e] += creal(w[j] * Y[e]);
            } else {
                /* Hermitian: the lower half contour uses the adjoint solve,
                 * Q += (w_j Y_j + conj(w_j) Yt_j) / 2 with A_z^H Yt_j = R  */
                for (size_t e = 0; e < (size_t)n * m0; ++e) Q[e] += 0.5 * w[j] * Y[e];
                memcpy(Y, R, sizeof(zc) * (size_t)n * m0);
                orc_zgetrs('C', n, m0, F, n, pv, Y, n);
                for (size_t e = 0; e < (size_t)n * m0; ++e) Q[e] += 0.5 * conj(w[j]) * Y[e];
            }
        }
        if (mode == 2) {
            orc_count_estimate(n, m0, X0, Q, res, M_out);
            memcpy(X, Q, sizeof(zc) * (size_t)n * m0);
            for (int c = 0; c < m0; ++c) E[c] = 0.0;
            info = 5;
            *loop_out = 0;
            *epsout_out = 1.0;
            goto done;
        }
        if (mode == 1) {
            memcpy(X, Q, sizeof(zc) * (size_t)n * m0);
            info = 4;
            *M_out = 0;
            *loop_out = 0;
            *epsout_out = 1.0;
            goto done;
        }

        /* (c) Rayleigh-Ritz: Aq = Q^H A Q, Bq = Q^H B Q, Hermitian parts */
        orc_zgemm('N', n, m0, n, A, n, Q, n, AQ, n);
        if (B) orc_zgemm('N', n, m0, n, B, n, Q, n, BQ, n);
        else memcpy(BQ, Q, sizeof(zc) * (size_t)n * m0);
        orc_zgemm('C', m0, m0, n, Q, n, AQ, n, Aq, m0);
        orc_zgemm('C', m0, m0, n, Q, n, BQ, n, Bq, m0);
        for (int j = 0; j < m0; ++j)
            for (int i = 0; i <= j; ++i) {
                zc sa = 0.5 * (Aq[IDX(i, j, m0)] + conj(Aq[IDX(j, i, m0)]));
                zc sb = 0.5 * (Bq[IDX(i, j, m0)] + conj(Bq[IDX(j, i, m0)]));
                Aq[IDX(i, j, m0)] = sa; Aq[IDX(j, i, m0)] = conj(sa);
                Bq[IDX(i, j, m0)] = sb; Bq[IDX(j, i, m0)] = conj(sb);
            }

        /* (d) reduced problem Aq phi = lambda Bq phi.
         * Reading: Bq = W diag(beta) W^H by Jacobi; directions with
         * beta_i <= 1e-14 beta_max are dropped (this is how M0 shrinks,
         * "new suitable M0" in Table "tab_common"); T = W_keep beta^{-1/2};
         * Jacobi on T^H Aq T gives lambda and V; Phi = T V.               */
        memcpy(tmp, Bq, sizeof(zc) * m0 * m0);
        if (orc_zheev_jacobi(m0, tmp, m0, beta, Wb, m0)) { info = -3; goto done; }
        double bmax = beta[m0 - 1];
        if (!(bmax > 0.0) || beta[0] < -ORC_INDEFINITE * bmax) { info = -3; goto done; }
        int keep = 0;
        for (int i = 0; i < m0; ++i)
            if (beta[i] > ORC_TRUNC * bmax) ++keep;
        int first = m0 - keep;   /* beta ascending: kept ones are the last `keep` */
        for (int c = 0; c < keep; ++c) {
            double sc = 1.0 / sqrt(beta[first + c]);
            for (int r = 0; r < m0; ++r) T[IDX(r, c, m0)] = Wb[IDX(r, first + c, m0)] * sc;
        }
        orc_zgemm('N', m0, keep, m0, Aq, m0, T, m0, tmp, m0);      /* Aq T */
        orc_zgemm('C', keep, keep, m0, T, m0, tmp, m0, Cr, keep);   /* T^H Aq T */
        for (int j = 0; j < keep; ++j)
            for (int i = 0; i <= j; ++i) {
                zc s = 0.5 * (Cr[IDX(i, j, keep)] + conj(Cr[IDX(j, i, keep)]));
                Cr[IDX(i, j, keep)] = s;
                Cr[IDX(j, i, keep)] = conj(s);
            }
        if (orc_zheev_jacobi(keep, Cr, keep, lam, V, keep)) { info = -3; goto done; }
        orc_zgemm('N', m0, keep, keep, T, m0, V, keep, Phi, m0);

        /* (e) Ritz vectors and residuals
         * res_i = ||A x_i - lambda_i B x_i||_1 / ||alpha B x_i||_1,
         * alpha = max(|Emin|, |Emax|)  (Table "tab_common", argument res) */
        orc_zgemm('N', n, keep, m0, Q, n, Phi, m0, Xc, n);
        orc_zgemm('N', n, keep, m0, AQ, n, Phi, m0, AX, n);
        orc_zgemm('N', n, keep, m0, BQ, n, Phi, m0, BX, n);
        for (int i = 0; i < keep; ++i) {
            double num = 0.0, den = 0.0;
            for (int r = 0; r < n; ++r) {
                num += cabs(AX[IDX(r, i, n)] - lam[i] * BX[IDX(r, i, n)]);
                den += cabs(BX[IDX(r, i, n)]);
            }
            rs[i] = num / (alpha * den);
        }
        m0 = keep;

        /* (f)-(h) count, spurious flag, trace, convergence */
        int inside = 0, bad = 0;
        double trace = 0.0, maxres = 0.0;
        M = 0;
        for (int i = 0; i < m0; ++i) {
            if (lam[i] < emin || lam[i] > emax) continue;
            ++inside;
            if (k >= 1 && rs[i] > ORC_SPURIOUS_RES) continue;   /* spurious */
            ++M;
            trace += lam[i];
            if (rs[i] > maxres) maxres = rs[i];
            if (!(rs[i] < tol)) ++bad;
        }
        epsout = (k == 0) ? 1.0 : fabs(trace - trace_prev) / alpha;
        trace_prev = trace;
        int converged = (M > 0) && (conv == 1 ? bad == 0 : epsout < tol);
        if (k == 0 && inside == 0) { info = 1; break; }
        if (converged) { info = 0; break; }
        if (M >= m0) { info = 3; break; }
        if (k == maxloop) { info = 2; break; }
    }
    if (k > maxloop) k = maxloop;

    /* (5) output order: non-spurious in-interval ascending, then the pairs
     * outside the interval ascending, then spurious ones with res = -1
     * (Table "tab_common", remark on E, X and res).                       */
    {
        int cnt = 0;
        for (int pass = 0; pass < 3; ++pass)
            for (int i = 0; i < m0; ++i) {
                int in = lam[i] >= emin && lam[i] <= emax;
                int sp = in && k >= 1 && rs[i] > ORC_SPURIOUS_RES;
                int cls = in ? (sp ? 2 : 0) : 1;
                if (cls == pass) order[cnt++] = i;
            }
        for (int c = 0; c < m0; ++c) {
            int i = order[c];
            int in = lam[i] >= emin && lam[i] <= emax;
            int sp = in && k >= 1 && rs[i] > ORC_SPURIOUS_RES;
            E[c] = lam[i];
            res[c] = sp ? -1.0 : rs[i];
            memcpy(X + (size_t)c * n, Xc + (size_t)i * n, sizeof(zc) * n);
        }
    }
    *M_out = M;
    *loop_out = k;
    *epsout_out = epsout;
    if (m0_io) *m0_io = m0;

done:
    free(z); free(w); free(fac); free(piv); free(Xc); free(R); free(Y); free(Q); free(AQ);
    free(BQ); free(Aq); free(Bq); free(Wb); free(T); free(Cr); free(V); free(Phi); free(tmp);
    free(AX); free(BX); free(beta); free(lam); free(rs); free(order);
    return info;
}
