/* Host driver for the sanitizer build of the FP64 oracle (test
 * infrastructure): every function of oracle/tc_oracle.h on tiny sizes with
 * ragged shapes, with a few consistency checks.  Built with AddressSanitizer
 * and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "tc_oracle.h"

static int failures = 0;
#define EXPECT(cond)                                                                \
    do {                                                                            \
        if (!(cond)) {                                                              \
            fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #cond);              \
            ++failures;                                                             \
        }                                                                           \
    } while (0)

int main(void)
{
    const int n[3] = {7, 5, 9};
    const int R_f = 3, R_N = 2, R_rho = 2;
    double t[2], a[2], c[2];
    double *p[3], *U[3], *V[3], *dU[3];
    oracle_sinc_rule(R_N, -1.0, 0.7, t, a);
    EXPECT(t[0] > 0.0 && a[1] > a[0]);
    EXPECT(oracle_cell_integral(0.3, 0.5, 0) > 0.0);
    EXPECT(oracle_cell_integral(0.3, 0.5, -4) == oracle_cell_integral(0.3, 0.5, 4));
    for (int l = 0; l < 3; ++l) {
        p[l] = malloc(sizeof(double) * R_N * (2 * n[l] - 1));
        U[l] = malloc(sizeof(double) * R_f * n[l]);
        V[l] = malloc(sizeof(double) * R_rho * n[l]);
        dU[l] = malloc(sizeof(double) * R_f * n[l]);
        oracle_newton_kernel(n[l], 0.5, R_N, -1.0, 0.7, NULL, NULL, c, p[l]);
        for (int j = 0; j < R_f; ++j)
            for (int x = 0; x < n[l]; ++x)
                U[l][j * n[l] + x] = exp(-0.3 * (j + 1) * (x - 2.0 - l) * (x - 2.0 - l));
        for (int j = 0; j < R_rho; ++j)
            for (int x = 0; x < n[l]; ++x)
                V[l][j * n[l] + x] = exp(-0.5 * (x - 3.0) * (x - 3.0)) * (1.0 + j);
    }
    double *W = malloc(sizeof(double) * R_N * R_f * n[0]);
    double *G = malloc(sizeof(double) * R_N * R_f * R_f);
    for (int comp = 0; comp < 2; ++comp) {
        oracle_convolve(n[0], R_f, R_N, p[0], U[0], W, comp);
        oracle_gram(n[0], R_f, R_N, U[0], W, G, comp);
    }
    double J[9], Jt[9], Gs[3 * 2 * 9], Jc[2 * 3], Jd[3];
    const double *pc[3] = {p[0], p[1], p[2]}, *Uc[3] = {U[0], U[1], U[2]},
                 *Vc[3] = {V[0], V[1], V[2]};
    oracle_tei_gram(n, R_f, R_N, c, pc, Uc, J, Gs, 1);
    oracle_tei_gram(n, R_f, R_N, c, pc, Uc, Jt, NULL, 0);
    for (int e = 0; e < 9; ++e)
        EXPECT(fabs(J[e] - Jt[e]) <= 1e-13 * fabs(J[e]) + 1e-300);
    const int cols[2] = {2, 0};
    oracle_tei_gram_columns(n, R_f, R_N, c, pc, Uc, 2, cols, Jc, 1);
    for (int q = 0; q < 2; ++q)
        for (int i = 0; i < R_f; ++i)
            EXPECT(fabs(Jc[q * R_f + i] - J[i * R_f + cols[q]]) <= 1e-14 * fabs(J[i * R_f + i]));
    const double d[2] = {0.5, 0.25};
    oracle_coulomb(n, R_f, R_rho, R_N, c, pc, Uc, Vc, d, Jd, 1);
    double Jbar[9];
    for (int e = 0; e < 9; ++e)
        Jbar[e] = 0.1 * e - 0.3;
    oracle_tei_gram_backward(n, R_f, R_N, c, pc, Uc, Jbar, dU);
    /* brute force on an isotropic grid */
    const int nb = 4;
    double pb[2 * 7], *Ub[3], Jb[9];
    oracle_newton_kernel(nb, 0.5, R_N, -1.0, 0.7, NULL, a, NULL, pb);
    for (int l = 0; l < 3; ++l) {
        Ub[l] = malloc(sizeof(double) * R_f * nb);
        for (int e = 0; e < R_f * nb; ++e)
            Ub[l][e] = 1.0 / (1.0 + e + l);
    }
    const double *Ubc[3] = {Ub[0], Ub[1], Ub[2]};
    oracle_bruteforce_J(nb, 0.5, R_f, R_N, a, pb, Ubc, Jb);
    double x[20], wq[20];
    oracle_gauss_legendre(20, x, wq);
    double sw = 0.0;
    for (int i = 0; i < 20; ++i)
        sw += wq[i];
    EXPECT(fabs(sw - 2.0) < 1e-14);
    for (int l = 0; l < 3; ++l) {
        free(p[l]);
        free(U[l]);
        free(V[l]);
        free(dU[l]);
        free(Ub[l]);
    }
    free(W);
    free(G);
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("oracle driver: all checks passed\n");
    return 0;
}
