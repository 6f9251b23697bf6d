/*
 * FP64 CPU oracle for the grid-based Newton-kernel convolution and TEI Gram
 * assembly (arXiv:1504.06289, Sections 2.5, 3.1, 3.2 and Appendix 3).
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark, never by the product path.  Written
 * directly from the paper's definitions, in plain loops, with no blocking,
 * fusion or reordering beyond what the definitions state.  Build flags must
 * keep IEEE semantics (-ffp-contract=off, no -ffast-math): the compensated
 * sums below rely on error-free transformations.
 *
 * Every function has a pin in tests/ that ties it to the paper or to
 * mathematics (see the header); no function here is "parity unpinned".
 */
#include "tc_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Compensated accumulation: Ogita, Rump & Oishi, "Accurate sum and dot      */
/* product", SIAM J. Sci. Comput. 26 (2005) -- algorithms Sum2 and Dot2.      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double s; /* running sum            */
    double c; /* accumulated error term */
} acc2;

static inline void two_sum(double a, double b, double *x, double *y)
{
    double s = a + b;
    double z = s - a;
    *y = (a - (s - z)) + (b - z);
    *x = s;
}

/* acc += x*y, exactly-rounded product error captured by an FMA */
static inline void acc_dot(acc2 *A, double x, double y, int comp)
{
    double p = x * y;
    if (!comp) {
        A->s += p;
        return;
    }
    double r = fma(x, y, -p);
    double s, q;
    two_sum(A->s, p, &s, &q);
    A->s = s;
    A->c += q + r;
}

static inline void acc_add(acc2 *A, double x, int comp)
{
    if (!comp) {
        A->s += x;
        return;
    }
    double s, q;
    two_sum(A->s, x, &s, &q);
    A->s = s;
    A->c += q;
}

static inline double acc_val(const acc2 *A) { return A->s + A->c; }

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1]: roots of P_npts by Newton's method on the  */
/* three-term Legendre recurrence, weights 2 / ((1-x^2) P'(x)^2).            */
/* ------------------------------------------------------------------------ */
void oracle_gauss_legendre(int npts, double *x, double *w)
{
    for (int i = 0; i < npts; ++i) {
        /* Chebyshev-like initial guess for the i-th root (descending) */
        double z = cos(M_PI * (i + 0.75) / (npts + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= npts; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            /* p1 = P_n(z), p0 = P_{n-1}(z) */
            dp = npts * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-17)
                break;
        }
        /* one more evaluation at the converged root for the weight */
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= npts; ++k) {
            double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        /* at a root P_n = 0, so (1-x^2) P_n' = n P_{n-1}: the weight
           2/((1-x^2) P_n'^2) equals 2 (1-x^2) / (n P_{n-1})^2 */
        x[i] = z;
        w[i] = 2.0 * (1.0 - z * z) / ((double)npts * npts * p0 * p0);
    }
}

#define GL_PTS 20
static double gl_x[GL_PTS], gl_w[GL_PTS];
static pthread_once_t gl_once = PTHREAD_ONCE_INIT;
static void gl_init(void) { oracle_gauss_legendre(GL_PTS, gl_x, gl_w); }

/* ------------------------------------------------------------------------ */
/* Appendix 3: sinc quadrature of the Laplace-Gauss transform of 1/r.        */
/* ------------------------------------------------------------------------ */
void oracle_sinc_rule(int R_N, double u0, double hu, double *t, double *a)
{
    const double two_over_sqrtpi = 2.0 / sqrt(M_PI);
    for (int k = 0; k < R_N; ++k) {
        double u = u0 + k * hu;
        double tk = exp(u);
        if (t)
            t[k] = tk;
        if (a)
            a[k] = two_over_sqrtpi * hu * tk; /* dt = e^u du */
    }
}

/*
 * Integral of exp(-t^2 s^2) over the cell [(m-1/2)h, (m+1/2)h].
 *   m = 0:  (sqrt(pi)/t) erf(t h / 2).
 *   The integrand's log-range over the cell is 2 t^2 |m| h^2.  Where that is
 *   at most 1 the integrand is flat and an erf/erfc difference would cancel,
 *   so integrate  exp(-t^2 x_m^2) * exp(-t^2 (2 x_m s + s^2))  over
 *   s in [-h/2, h/2] (x_m = |m| h) with a 20-point Gauss-Legendre rule;
 *   the exponent there is bounded by 5/8, so the rule is exact to rounding.
 *   Otherwise the two ends differ by a factor e or more and the difference
 *   of erfc (right tail, alpha >= 1/2) or erf (near the origin) is well
 *   conditioned.
 */
double oracle_cell_integral(double t, double h, long m)
{
    const double sqrtpi = sqrt(M_PI);
    long am = m < 0 ? -m : m;
    if (am == 0)
        return sqrtpi / t * erf(0.5 * t * h);

    double xm = (double)am * h;
    double logrange = 2.0 * t * t * (double)am * h * h;
    if (logrange <= 1.0) {
        pthread_once(&gl_once, gl_init);
        acc2 A = {0.0, 0.0};
        double half = 0.5 * h;
        for (int q = 0; q < GL_PTS; ++q) {
            double s = half * gl_x[q];
            acc_add(&A, gl_w[q] * exp(-t * t * (2.0 * xm * s + s * s)), 1);
        }
        return exp(-t * t * xm * xm) * acc_val(&A) * half;
    }
    double alpha = t * ((double)am - 0.5) * h;
    double beta = t * ((double)am + 0.5) * h;
    if (alpha >= 0.5)
        return sqrtpi / (2.0 * t) * (erfc(alpha) - erfc(beta));
    return sqrtpi / (2.0 * t) * (erf(beta) - erf(alpha));
}

void oracle_newton_kernel(int n, double h, int R_N, double u0, double hu,
                          double *t, double *a, double *c, double *p)
{
    double *tt = (double *)malloc(sizeof(double) * R_N);
    double *aa = (double *)malloc(sizeof(double) * R_N);
    oracle_sinc_rule(R_N, u0, hu, tt, aa);
    for (int k = 0; k < R_N; ++k) {
        if (t)
            t[k] = tt[k];
        if (a)
            a[k] = aa[k];
        if (c)
            c[k] = aa[k] * h * h * h; /* cell volume folded into the weight */
    }
    if (p) {
        const long L = 2L * n - 1;
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < R_N; ++k)
            for (long m = -(n - 1); m <= n - 1; ++m)
                p[k * L + m + n - 1] = oracle_cell_integral(tt[k], h, m);
    }
    free(tt);
    free(aa);
}

/* ------------------------------------------------------------------------ */
/* Section 2.5 eq. conv / Section 3.2 eq. Factor_Mk_Conv: the 1D            */
/* convolution p_k *_n u restricted to the box (aperiodic, zero outside).   */
/* ------------------------------------------------------------------------ */
void oracle_convolve(int n, int R_f, int R_N, const double *p, const double *U,
                     double *W, int compensated)
{
    const long L = 2L * n - 1;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (int k = 0; k < R_N; ++k)
        for (int j = 0; j < R_f; ++j) {
            const double *pk = p + (long)k * L;
            const double *u = U + (long)j * n;
            double *w = W + ((long)k * R_f + j) * n;
            for (long a = 0; a < n; ++a) {
                acc2 A = {0.0, 0.0};
                for (long b = 0; b < n; ++b)
                    acc_dot(&A, pk[a - b + n - 1], u[b], compensated);
                w[a] = acc_val(&A);
            }
        }
}

void oracle_gram(int n, int R_f, int R_N, const double *U, const double *W,
                 double *G, int compensated)
{
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int k = 0; k < R_N; ++k)
        for (int i = 0; i < R_f; ++i) {
            const double *ui = U + (long)i * n;
            for (int j = 0; j < R_f; ++j) {
                const double *w = W + ((long)k * R_f + j) * n;
                acc2 A = {0.0, 0.0};
                for (long a = 0; a < n; ++a)
                    acc_dot(&A, ui[a], w[a], compensated);
                G[((long)k * R_f + i) * R_f + j] = acc_val(&A);
            }
        }
}

/* Hadamard product across the three modes and sum over the kernel terms
 * (Section 3.2, the factorised TEI matrix with V = I). */
static void hadamard_sum(int R_f, int R_N, const double *c,
                         const double *const G[3], double *J, int compensated)
{
    const long F2 = (long)R_f * R_f;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < F2; ++e) {
        acc2 A = {0.0, 0.0};
        for (int k = 0; k < R_N; ++k)
            acc_add(&A, c[k] * G[0][k * F2 + e] * G[1][k * F2 + e] * G[2][k * F2 + e],
                    compensated);
        J[e] = acc_val(&A);
    }
}

void oracle_tei_gram(const int *n, int R_f, int R_N, const double *c,
                     const double *const *p, const double *const *U,
                     double *J, double *G_out, int compensated)
{
    const long F2 = (long)R_f * R_f;
    double *G[3];
    for (int l = 0; l < 3; ++l) {
        G[l] = G_out ? G_out + (long)l * R_N * F2
                     : (double *)malloc(sizeof(double) * R_N * F2);
        double *W = (double *)malloc(sizeof(double) * (long)R_N * R_f * n[l]);
        oracle_convolve(n[l], R_f, R_N, p[l], U[l], W, compensated);
        oracle_gram(n[l], R_f, R_N, U[l], W, G[l], compensated);
        free(W);
    }
    hadamard_sum(R_f, R_N, c, (const double *const *)G, J, compensated);
    if (!G_out)
        for (int l = 0; l < 3; ++l)
            free(G[l]);
}

void oracle_coulomb(const int *n, int R_f, int R_rho, int R_N, const double *c,
                    const double *const *p, const double *const *U,
                    const double *const *V, const double *d, double *Jd, int compensated)
{
    /* H[l][q][i][m] = <U^l[i], (T^l_q V^l)[m]> */
    double *H[3];
    for (int l = 0; l < 3; ++l) {
        const int nl = n[l];
        double *W = (double *)malloc(sizeof(double) * (size_t)R_N * R_rho * nl);
        oracle_convolve(nl, R_rho, R_N, p[l], V[l], W, compensated);
        H[l] = (double *)malloc(sizeof(double) * (size_t)R_N * R_f * R_rho);
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
        for (int q = 0; q < R_N; ++q)
            for (int i = 0; i < R_f; ++i) {
                const double *ui = U[l] + (long)i * nl;
                for (int m = 0; m < R_rho; ++m) {
                    const double *w = W + ((long)q * R_rho + m) * nl;
                    acc2 A = {0.0, 0.0};
                    for (long a = 0; a < nl; ++a)
                        acc_dot(&A, ui[a], w[a], compensated);
                    H[l][((long)q * R_f + i) * R_rho + m] = acc_val(&A);
                }
            }
        free(W);
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < R_f; ++i) {
        acc2 A = {0.0, 0.0};
        for (int q = 0; q < R_N; ++q)
            for (int m = 0; m < R_rho; ++m) {
                const long e = ((long)q * R_f + i) * R_rho + m;
                acc_add(&A, c[q] * d[m] * H[0][e] * H[1][e] * H[2][e], compensated);
            }
        Jd[i] = acc_val(&A);
    }
    for (int l = 0; l < 3; ++l)
        free(H[l]);
}

void oracle_tei_gram_columns(const int *n, int R_f, int R_N, const double *c,
                             const double *const *p, const double *const *U,
                             int ncols, const int *cols, double *Jcols,
                             int compensated)
{
    /* g[l][k][i] = u_i^T T_k u_j for the current column j */
    double *g = (double *)malloc(sizeof(double) * 3 * R_N * R_f);
    int nmax = n[0] > n[1] ? n[0] : n[1];
    nmax = nmax > n[2] ? nmax : n[2];
    for (int q = 0; q < ncols; ++q) {
        const int j = cols[q];
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
        for (int l = 0; l < 3; ++l)
            for (int k = 0; k < R_N; ++k) {
                const long nl = n[l], L = 2 * nl - 1;
                const double *pk = p[l] + k * L;
                const double *uj = U[l] + (long)j * nl;
                double *w = (double *)malloc(sizeof(double) * nmax);
                for (long a = 0; a < nl; ++a) {
                    acc2 A = {0.0, 0.0};
                    for (long b = 0; b < nl; ++b)
                        acc_dot(&A, pk[a - b + nl - 1], uj[b], compensated);
                    w[a] = acc_val(&A);
                }
                for (int i = 0; i < R_f; ++i) {
                    const double *ui = U[l] + (long)i * nl;
                    acc2 A = {0.0, 0.0};
                    for (long a = 0; a < nl; ++a)
                        acc_dot(&A, ui[a], w[a], compensated);
                    g[((long)l * R_N + k) * R_f + i] = acc_val(&A);
                }
                free(w);
            }
        for (int i = 0; i < R_f; ++i) {
            acc2 A = {0.0, 0.0};
            for (int k = 0; k < R_N; ++k)
                acc_add(&A,
                        c[k] * g[(0L * R_N + k) * R_f + i] * g[(1L * R_N + k) * R_f + i] *
                            g[(2L * R_N + k) * R_f + i],
                        compensated);
            Jcols[(long)q * R_f + i] = acc_val(&A);
        }
    }
    free(g);
}

/* ------------------------------------------------------------------------ */
/* Adjoint.  f = <Jbar, J>.  With E^l_k = dF/dG^l_k (entrywise) and         */
/* G = U^T T U:  df/dU = T U (E + E^T) summed over k.  Because the Grams     */
/* are symmetric, E + E^T = 2 c_k S o G^{l+1} o G^{l+2} = 2 D^l_k.           */
/* ------------------------------------------------------------------------ */
void oracle_tei_gram_backward(const int *n, int R_f, int R_N, const double *c,
                              const double *const *p, const double *const *U,
                              const double *Jbar, double *const *dU)
{
    const long F2 = (long)R_f * R_f;
    double *G = (double *)malloc(sizeof(double) * 3 * R_N * F2);
    double *W[3];
    for (int l = 0; l < 3; ++l) {
        W[l] = (double *)malloc(sizeof(double) * (long)R_N * R_f * n[l]);
        oracle_convolve(n[l], R_f, R_N, p[l], U[l], W[l], 1);
        oracle_gram(n[l], R_f, R_N, U[l], W[l], G + (long)l * R_N * F2, 1);
    }
    double *D = (double *)malloc(sizeof(double) * R_N * F2);
    for (int l = 0; l < 3; ++l) {
        const double *G1 = G + (long)((l + 1) % 3) * R_N * F2;
        const double *G2 = G + (long)((l + 2) % 3) * R_N * F2;
        for (int k = 0; k < R_N; ++k)
            for (int i = 0; i < R_f; ++i)
                for (int j = 0; j < R_f; ++j) {
                    long e = (long)i * R_f + j;
                    double s = 0.5 * (Jbar[e] + Jbar[(long)j * R_f + i]);
                    D[k * F2 + e] = c[k] * s * G1[k * F2 + e] * G2[k * F2 + e];
                }
        const long nl = n[l];
#pragma omp parallel for collapse(2) schedule(static)
        for (int i = 0; i < R_f; ++i)
            for (long a = 0; a < nl; ++a) {
                acc2 A = {0.0, 0.0};
                for (int k = 0; k < R_N; ++k)
                    for (int j = 0; j < R_f; ++j)
                        acc_dot(&A, W[l][((long)k * R_f + j) * nl + a],
                                D[k * F2 + (long)j * R_f + i], 1);
                dU[l][(long)i * nl + a] = 2.0 * acc_val(&A);
            }
    }
    free(D);
    for (int l = 0; l < 3; ++l)
        free(W[l]);
    free(G);
}

/* ------------------------------------------------------------------------ */
/* Brute-force 3D direct summation (no 1D Grams anywhere).                  */
/* ------------------------------------------------------------------------ */
void oracle_bruteforce_J(int n, double h, int R_f, int R_N, const double *a,
                         const double *p, const double *const *U, double *J)
{
    const long L = 2L * n - 1;
    const long L3 = L * L * L;
    const long N3 = (long)n * n * n;
    /* assembled 3D kernel on the lag grid */
    double *P3 = (double *)malloc(sizeof(double) * L3);
#pragma omp parallel for schedule(static)
    for (long e = 0; e < L3; ++e) {
        long m1 = e / (L * L), m2 = (e / L) % L, m3 = e % L;
        acc2 A = {0.0, 0.0};
        for (int k = 0; k < R_N; ++k)
            acc_add(&A, a[k] * p[k * L + m1] * p[k * L + m2] * p[k * L + m3], 1);
        P3[e] = acc_val(&A);
    }
    /* full 3D samples of every function */
    double *F = (double *)malloc(sizeof(double) * R_f * N3);
    for (int i = 0; i < R_f; ++i)
        for (long x = 0; x < N3; ++x) {
            long x1 = x / ((long)n * n), x2 = (x / n) % n, x3 = x % n;
            F[i * N3 + x] = U[0][(long)i * n + x1] * U[1][(long)i * n + x2] *
                            U[2][(long)i * n + x3];
        }
    double *V = (double *)malloc(sizeof(double) * N3);
    for (int j = 0; j < R_f; ++j) {
        /* V_j(x) = sum_y P(x - y) f_j(y) over the whole grid */
#pragma omp parallel for schedule(static)
        for (long x = 0; x < N3; ++x) {
            long x1 = x / ((long)n * n), x2 = (x / n) % n, x3 = x % n;
            acc2 A = {0.0, 0.0};
            const double *fj = F + j * N3;
            for (long y1 = 0; y1 < n; ++y1)
                for (long y2 = 0; y2 < n; ++y2)
                    for (long y3 = 0; y3 < n; ++y3) {
                        long e = ((x1 - y1 + n - 1) * L + (x2 - y2 + n - 1)) * L +
                                 (x3 - y3 + n - 1);
                        acc_dot(&A, P3[e], fj[(y1 * n + y2) * n + y3], 1);
                    }
            V[x] = acc_val(&A);
        }
        for (int i = 0; i < R_f; ++i) {
            acc2 A = {0.0, 0.0};
            for (long x = 0; x < N3; ++x)
                acc_dot(&A, F[i * N3 + x], V[x], 1);
            J[(long)i * R_f + j] = h * h * h * acc_val(&A);
        }
    }
    free(V);
    free(F);
    free(P3);
}
