/*
 * FP64 CPU oracle for the grid-based Newton-kernel convolution and the
 * two-electron-integral (TEI) Gram assembly of Khoromskaia & Khoromskij,
 * "Tensor numerical methods in quantum chemistry" (arXiv:1504.06289).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this code: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a plain,
 * slow, obviously correct implementation written directly from the paper.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Layouts (all row-major, FP64):
 *   U  [R_f][n]          column j of the mode side matrix U (n x R_f) is the
 *                        contiguous row U[j][*]; U[j][a] = f_j sampled at the
 *                        centre of cell a.
 *   p  [R_N][2n-1]       kernel vector of term k, lag m at index m+n-1.
 *   W  [R_N][R_f][n]     W_k = T_k U (the 1D convolutions), same layout as U.
 *   G  [R_N][R_f][R_f]   G_k = U^T T_k U.
 *   J  [R_f][R_f]        both triangles.
 *
 * Every dot product and every sum uses the Ogita-Rump-Oishi "Dot2"/"Sum2"
 * compensated algorithms (error-free TwoSum and FMA-based TwoProduct), so the
 * oracle's own rounding error is about that of a computation in twice the
 * working precision.  Passing compensated = 0 selects plain FP64 loops (same
 * loops, same order, no compensation) for speed comparisons only.
 *
 * Parity pins (the tests that tie this oracle to the paper and to
 * mathematics rather than to itself) are listed with each function.  Every
 * function here has at least one pin; none is "parity unpinned".
 */
#ifndef TC_ORACLE_H
#define TC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Sinc (trapezoid) rule for 1/r = (2/sqrt(pi)) * int_R exp(-r^2 e^{2u}) e^u du,
 * the Laplace-Gauss transform of the Newton kernel (Appendix 3, eq. sinc_Newt)
 * after the substitution t = e^u: nodes t_k = exp(u0 + k*hu) and weights
 * a_k = (2/sqrt(pi)) * hu * t_k, k = 0..R_N-1.
 * Pins: r * sum_k a_k exp(-t_k^2 r^2) -> 1 on [r_min, r_max] with error that
 * falls as R_N grows (the exponential sinc convergence stated in Appendix 3). */
void oracle_sinc_rule(int R_N, double u0, double hu, double *t, double *a);

/* Galerkin projection of exp(-t^2 x^2) onto the piecewise-constant basis
 * (Appendix 3, eqs. galten and the vector b(t_k)): the integral of
 * exp(-t^2 s^2) over the cell [(m-1/2)h, (m+1/2)h].
 * Pins: 40-digit mpmath quadrature; telescoping sum over all lags equals
 * (sqrt(pi)/t) erf(t (n-1/2) h); symmetry in m. */
double oracle_cell_integral(double t, double h, long m);

/* Canonical Newton kernel of rank R_N on an n-cell grid of width h
 * (Section 3.1 eq. NewtCan; Appendix 3 eq. sinc_general), with the weights
 * kept outside the per-mode vectors: c_k = a_k * h^3 and
 * p[k][m+n-1] = oracle_cell_integral(t_k, h, m), m = -(n-1)..(n-1).
 * t, a, c: [R_N] (any may be NULL); p: [R_N][2n-1].
 * Pins: origin-cell identity sum_k a_k p_k[0]^3 -> h^2 (3 ln(2+sqrt3) - pi/2);
 * lag entries sum_k a_k prod_l p_k[m_l] -> exact prism integral of 1/|y|. */
void oracle_newton_kernel(int n, double h, int R_N, double u0, double hu,
                          double *t, double *a, double *c, double *p);

/* Aperiodic 1D convolution of every column of U with every kernel vector,
 * restricted to the n cells of the box (Section 2.5 eq. conv; the p_k *_n U
 * of eq. Factor_Mk_Conv): W[k][j][a] = sum_b p_k[a-b] U[j][b].
 * Pins: closed-form Gaussian convolution; brute-force 3D sum. */
void oracle_convolve(int n, int R_f, int R_N, const double *p, const double *U,
                     double *W, int compensated);

/* Convolution matrices of one mode (eq. Factor_Mk_Conv):
 * G[k][i][j] = sum_a U[i][a] W[k][j][a].  W as produced by oracle_convolve. */
void oracle_gram(int n, int R_f, int R_N, const double *U, const double *W,
                 double *G, int compensated);

/* Coulomb/TEI matrix of the product functions (Section 3.2, the
 * Hadamard-across-modes sum over k with V = I):
 * J[i][j] = sum_k c_k G1_k[i][j] G2_k[i][j] G3_k[i][j].
 * n[3], p[3], U[3] per mode.  G_out: NULL or [3][R_N][R_f][R_f].
 * Pins: Boys-function closed form for s-type Gaussians (O(h^2) plus the
 * quadrature floor); brute-force 3D direct summation at small n; symmetry and
 * positive semi-definiteness. */
void oracle_tei_gram(const int *n, int R_f, int R_N, const double *c,
                     const double *const *p, const double *const *U,
                     double *J, double *G_out, int compensated);

/* Selected columns of J: Jcols[q][i] = J[i][cols[q]] for all i, computed
 * column by column (only the W columns those entries need), for sampled
 * parity checks at full problem sizes. */
void oracle_tei_gram_columns(const int *n, int R_f, int R_N, const double *c,
                             const double *const *p, const double *const *U,
                             int ncols, const int *cols, double *Jcols,
                             int compensated);

/* Coulomb entries of the product functions against a density given in
 * canonical format (Section 3.1: the Hartree potential of the density
 * Theta' = sum_m d_m v^1_m x v^2_m x v^3_m is the sum of tensor products of
 * the 1D convolutions v^l_m * p^l_q, and the Coulomb entries are its scalar
 * products with the rank-1 products of basis functions):
 *   Jd[i] = sum_q c_q sum_m d_m prod_l <U^l[i], (T^l_q V^l)[m]>,
 * with T^l_q V^l the aperiodic convolution of oracle_convolve and <.,.> the
 * plain sum over the cells (the cell volume is in c_q, as for J).
 * U[l] [R_f][n_l], V[l] [R_rho][n_l], d [R_rho], Jd [R_f].
 * Pins: with V = U the result is J d for the J of oracle_tei_gram; the Boys
 * closed form for an s-Gaussian density against s-Gaussian functions. */
void oracle_coulomb(const int *n, int R_f, int R_rho, int R_N, const double *c,
                    const double *const *p, const double *const *U,
                    const double *const *V, const double *d, double *Jd, int compensated);

/* Adjoint of f = <Jbar, J> with respect to the side matrices:
 * dU^l = 2 sum_k W^l_k D^l_k with D^l_k = c_k S o G^{l+1}_k o G^{l+2}_k and
 * S = (Jbar + Jbar^T)/2 (T_k and G symmetric).  dU[l]: [R_f][n_l].
 * Pins: central finite differences of the oracle forward (f is quadratic in
 * every entry of U, so the central difference is exact up to rounding);
 * analytic exponent/centre derivatives of the Boys closed form. */
void oracle_tei_gram_backward(const int *n, int R_f, int R_N, const double *c,
                              const double *const *p, const double *const *U,
                              const double *Jbar, double *const *dU);

/* Brute-force 3D direct summation on the full n^3 grid (isotropic grid):
 * J[i][j] = h^3 sum_x sum_y f_i(x) f_j(y) P(x - y), with the 3D kernel
 * P(m) = sum_k a_k p_k[m1] p_k[m2] p_k[m3] assembled on the (2n-1)^3 lag grid
 * and f_i(x) = U1[i][x1] U2[i][x2] U3[i][x3].  Cost O(n^6 R_f); small n only.
 * It pins the separable algebra of oracle_tei_gram (index, lag and h^3
 * conventions) by never forming a 1D Gram. */
void oracle_bruteforce_J(int n, double h, int R_f, int R_N, const double *a,
                         const double *p, const double *const *U, double *J);

/* Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on the
 * Legendre recurrence), exported for the quadrature pin. */
void oracle_gauss_legendre(int npts, double *x, double *w);

#ifdef __cplusplus
}
#endif
#endif
