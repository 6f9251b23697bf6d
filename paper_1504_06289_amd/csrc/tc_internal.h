// Internal interface between the C-ABI layer (tc_api.cpp) and the kernel
// translation units.  Every launcher enqueues on `stream` and returns the
// hipError_t of the launch; none allocates or synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tc {

// ---- kernel generation (kernel_gen.hip) ----------------------------------
// p[k][m+n-1] = integral of exp(-t_k^2 s^2) over cell m, for k < R_N.
hipError_t launch_newton_kernel(const double *t_host, int R_N, int n, double h,
                                double *p_dev, hipStream_t stream);

// ---- Toeplitz products (toeplitz.hip) -------------------------------------
// W[k][j][a] = sum_b p[k][a-b+n-1] U[j][b] in binary64 on matrix cores.
hipError_t launch_toeplitz_f64(const double *p, const double *U, double *W, int n,
                               int R_f, int R_N, hipStream_t stream);

// ---- Grams (gram.hip) -----------------------------------------------------
// G[k][i][j] = sum_a U[i][a] W[k][j][a] for all k < R_N from upper-triangle
// tiles: every Gram launcher writes the entries i <= j, and with `mirror` also
// the entries i > j (exactly symmetric); without it those entries are left
// untouched (the Hadamard sum reads only i <= j).
hipError_t launch_gram_f64(const double *U, const double *W, double *G, int n,
                           int R_f, int R_N, bool mirror, hipStream_t stream);

// Diagonal form: term k = alpha R_N + q (k < M R_N) with p_q shifted to the
// cell shift[alpha] (0 <= shift < n) in place of W_k:
// G[k][i][j] = sum_a U[i][a] U[j][a] p[q][a - shift[alpha] + n - 1].
// cls [R_N] (the term classes of launch_term_class for p, or null): groups of
// narrow terms sum only over the cells within their band of their nuclei.
hipError_t launch_diag_gram_f64(const double *U, const double *p, const int *shift,
                                const int *cls, double *G, int n, int R_f, int R_N, int M,
                                bool mirror, hipStream_t stream);

// ---- nuclear potential tables (nuclear.hip) -------------------------------
constexpr int kNuclearChunk = 64;
struct NuclearChunk {
    int base, count;                 // nuclei base .. base + count - 1
    double Z[kNuclearChunk];         // charges
    int pos[3][kNuclearChunk];       // cell of each nucleus per mode
};
// cw[alpha R_N + q] = -Z_alpha c_q inv_vol; shift[l M + alpha] = pos[alpha][l]
hipError_t launch_nuclear_table(const NuclearChunk &ch, const double *c, int R_N, int M,
                                double inv_vol, int *shift, double *cw, hipStream_t st);

// ---- binary32 matrix-core variants (fp32.hip) ------------------------------
// E[r] = exponent of the largest |X[r][.]| (max < 2^E[r]; 0 for a zero row).
hipError_t launch_row_exponents(const double *X, long rows, int len, int *E,
                                hipStream_t stream);
// Same results as launch_toeplitz_f64 / launch_gram_f64 with every operand
// row scaled by 2^-E (E from launch_row_exponents: EU per row of U, EP per
// kernel term, EW per row of W), rounded to binary32, binary32 partial sums
// over K-chunks of 64, binary64 accumulation of the chunk sums, and the
// scale put back on the binary64 result.
hipError_t launch_toeplitz_f32(const double *p, const int *EP, const double *U, const int *EU,
                               double *W, int n, int R_f, int R_N, hipStream_t stream);
hipError_t launch_gram_f32(const double *U, const int *EU, const double *W, const int *EW,
                           double *G, int n, int R_f, int R_N, bool mirror, hipStream_t stream);

// ---- split-bfloat16 matrix-core variants (bf16.hip) ------------------------
// As the binary32 variants, with each scaled binary64 entry split exactly into
// `pieces` (2 or 3) bfloat16 pieces and the piece products with index sum
// <= pieces - 1 (3 or 6 of them) on v_mfma_f32_16x16x32_bf16, binary32 sums
// over K-chunks of 64, binary64 across chunks.
hipError_t launch_toeplitz_bf16(const double *p, const int *EP, const double *U, const int *EU,
                                double *W, int n, int R_f, int R_N, int pieces,
                                hipStream_t stream);
hipError_t launch_gram_bf16(const double *U, const int *EU, const double *W, const int *EW,
                            double *G, int n, int R_f, int R_N, int pieces, bool mirror,
                            hipStream_t stream);

// ---- Hadamard product across modes and sum over k (reduce.hip) -----------
// J[e] = sum_k c[k] G0[k][e] G1[k][e] G2[k][e], e < R_f*R_f.
hipError_t launch_hadamard_sum(const double *c, const double *G0, const double *G1,
                               const double *G2, double *J, int R_f, int R_N,
                               hipStream_t stream);

// ---- Adjoint pieces (reduce.hip, gemm.hip) --------------------------------
// D[k][e] = c[k] * 0.5*(Jbar[e] + Jbar[e^T]) * Ga[k][e] * Gb[k][e]
hipError_t launch_adjoint_d(const double *c, const double *Jbar, const double *Ga,
                            const double *Gb, double *D, int R_f, int R_N,
                            hipStream_t stream);
// dU[i][a] = scale * sum_k sum_j D[k][j][i] W[k][j][a].  The contraction is
// split into adjoint_splits(n, R_f, R_N) ranges; with more than one, part
// holds the partial sums of all but the first ([S-1][R_f][n], device).
constexpr int kAdjointMaxSplit = 8;
int adjoint_splits(int n, int R_f, int R_N);
hipError_t launch_adjoint_gemm_f64(const double *D, const double *W, double *dU, int n,
                                   int R_f, int R_N, double scale, double *part,
                                   hipStream_t stream);


// ---- int8 error-free splitting path (ozaki.hip) ---------------------------
// Zero padding (bytes) in front of and behind the lag-reversed kernel slices.
constexpr int kOzakiPad = 256;
// Offset that makes every staged window of the lag-reversed slices 16-byte
// aligned: PS[.][k][x] holds lag (n-1) + off - x.
inline int ozaki_p_offset(int n) { return kOzakiPad + ((16 - n % 16) % 16); }

struct OzakiLayout {
    int n_pad;     // cells padded to the tile multiple (128)
    int R_f_pad;   // functions padded to the tile multiple (64)
    int off;       // ozaki_p_offset(n)
    int LP;        // bytes per term of the kernel slices
    long uplane;   // bytes per slice plane of the U slices  (R_f_pad * n_pad)
    long pplane;   // bytes per slice plane of the p slices  (R_N * LP)
    long wplane;   // bytes per slice plane of the W slices  (R_N * R_f_pad * n_pad)
};
OzakiLayout ozaki_layout(int n, int R_f, int R_N);

// rows of X [groups][rows][len] -> S [4][groups][rows_pad][len_pad], E [groups][rows_pad]
hipError_t launch_split_rows(const double *X, int groups, int rows, int len, int rows_pad,
                             int len_pad, long plane, int8_t *S, int *E, hipStream_t stream);
// p [R_N][2n-1] -> lag-reversed slices PS [4][R_N][LP], EP [R_N]
hipError_t launch_split_kernel_vectors(const double *p, int n, int R_N, const OzakiLayout &L,
                                       int8_t *PS, int *EP, hipStream_t stream);
// W[k][j][a] = sum_b U[j][b] p_k[a-b] from the slices (binary64 output)
hipError_t launch_toeplitz_i8(const int8_t *US, const int *EU, const int8_t *PS, const int *EP,
                              const OzakiLayout &L, double *W, int n, int R_f, int R_N,
                              hipStream_t stream);
// G[k][i][j] = sum_a U[i][a] W[k][j][a] from the slices (binary64, symmetric),
// for every k, or (cls != nullptr, device [R_N]) for the k with cls[k] != -2 only.
// tail (kOzakiTailBytes of scratch, or null): with the 128-tile kernel, the
// items of the last, partial round of each XCD are split in K and their later
// parts summed from there (bitwise the unsplit result).
constexpr int kOzakiTailSlots = 16;
constexpr size_t kOzakiTailBytes = (size_t)8 * kOzakiTailSlots * 128 * 128 * sizeof(double);
bool gram_i8_wide(int R_f, int R_f_pad);
hipError_t launch_gram_i8(const int8_t *US, const int *EU, const int8_t *WS, const int *EW,
                          const OzakiLayout &L, double *G, int R_f, int R_N, const int *cls,
                          bool mirror, double *tail, hipStream_t stream);

// ---- FFT route (fft.hip) ---------------------------------------------------
// N = smallest power of two >= 2n-1; the route needs N/2 <= 4096 (n <= 4096).
int fft_length(int n);
bool fft_supported(int n);
hipError_t launch_fft_twiddles(double2 *twN, int N, hipStream_t stream);
// half spectra [rows][N/2+1] of the zero-padded rows of X [rows][len]
hipError_t launch_rfft_rows(const double *X, int rows, int len, int N, const double2 *twN,
                            double2 *spec, hipStream_t stream);
// half spectra [R_N][N/2+1] of the circulant embeddings of p [R_N][2n-1]
hipError_t launch_rfft_kernel_embed(const double *p, int n, int R_N, int N, const double2 *twN,
                                    double2 *spec, hipStream_t stream);
// W_k[j][t] (t < n) for all j, k from the spectra; output binary64 W
// [R_N][R_f][n] (W != nullptr) or int8 slices WS [4][R_N][R_f_pad][n_pad] with
// exponents EW [R_N][R_f_pad] (W == nullptr; padding rows zeroed).  With
// band != nullptr (int8 output only; the term classes of launch_term_class),
// terms of class B >= 0 are convolved directly from U [R_f][n] and p
// [R_N][2n-1] over lags |m| <= B, and terms of class -2 are skipped.
hipError_t launch_fft_conv(const double2 *Uspec, const double2 *Cspec, int n, int N, int R_f,
                           int R_N, const double2 *twN, double *W, int8_t *WS, int *EW,
                           int R_f_pad, int n_pad, long wplane, const double *U,
                           const double *p, const int *band, hipStream_t stream);

// ---- persistent int8 Gram over a device work queue (gram_queue.hip) --------
// One job per (instance, mode); see gram_queue.hip.
struct GramJob {
    const int8_t *US;    // int8 slices of U [4][R_f_pad][n_pad]
    const int *EU;       // [R_f_pad]
    const int8_t *WS;    // int8 slices of W [4][R_N][R_f_pad][n_pad]
    const int *EW;       // [R_N][R_f_pad]
    const int *cls;      // term classes [R_N] (terms of class -2 skipped) or null
    double *G;           // Grams [R_N][R_f][R_f]
    double *slab;        // K part 1's Grams (kparts == 2) or null
    long uplane, wplane;
    int n_pad, R_f_pad, R_f, R_N;
    int ntri;            // upper-triangle tiles per term
    int tile;            // 64 or 128
    int kparts;          // 1 or 2
    int mirror;          // also write the lower triangle
    int item_begin;      // first queue item of the job
};
constexpr int kGramJobChunk = 24;  // jobs per table-writing launch (kernel arguments)
struct GramJobChunk {
    int base, count;
    GramJob job[kGramJobChunk];
};
// Writes the job table (host_jobs, sorted and with item_begin set) to
// dev_jobs, zeroes the counter and runs the queue of `total` items; then adds
// the slabs of jobs with two K parts.
hipError_t launch_gram_queue(const GramJob *host_jobs, int njobs, int total, GramJob *dev_jobs,
                             int *counter, hipStream_t st);

// ---- FFT route beyond the LDS-resident lengths (fft_large.hip) --------------
// 4096 < n <= 65536: N = fft_length(n) in 16384 .. 131072, four-step binary64
// transforms with two real rows per complex sequence.
bool fft_large_supported(int n);
struct LargeFftLayout {
    int N;           // transform length
    int P;           // complex sequences of U (pairs of rows): ceil(R_f / 2)
    int kc;          // kernel terms per inverse chunk
    long z_entries;  // complex entries of the U spectra   [P][N]
    long c_entries;  // complex entries of the kernel spectra [R_N][N]
    long t_entries;  // complex entries of the inverse scratch [kc][P][N]
};
LargeFftLayout fft_large_layout(int n, int R_f, int R_N);
// W [R_N][R_f][n] (binary64) = T_k U for all k; twN from launch_fft_twiddles(N);
// EU [R_f] from launch_row_exponents(U); Z, C, T scratch of the layout's sizes.
hipError_t launch_fft_large_W(const double *p, const double *U, const int *EU, int n, int R_f,
                              int R_N, const double2 *twN, double2 *Z, double2 *C, double2 *T,
                              double *W, hipStream_t stream);

// ---- Coulomb entries against a density (coulomb.hip) -----------------------
// H[q][i][m] = sum_a U[i][a] W[q][m][a] for i < R_f, m < R_rho, q < R_N
hipError_t launch_cross_gram_f64(const double *U, const double *W, double *H, int n, int R_f,
                                 int R_rho, int R_N, hipStream_t stream);
// Jd[i] = sum_q c_q sum_m d_m H0 H1 H2 at [q][i][m], H = [3][R_N][R_f][R_rho]
hipError_t launch_coulomb_reduce(const double *c, const double *d, const double *H, int R_f,
                                 int R_rho, int R_N, double *Jd, hipStream_t stream);

// ---- pivoted Cholesky: density fitting and the factorised TEI matrix -------
// (cholesky.hip).  stats = {max, trace}
hipError_t launch_fit_diag(const double *F, int n, int N_pair, double *d, hipStream_t st);
// part: scratch [fit_column_parts()][n]
int fit_column_parts();
hipError_t launch_fit_column(const double *F, int n, int N_pair, const int *state, double *part,
                             double *col, hipStream_t st);
// Y: scratch [3][R_N][N_pair][R] (V^l M^l_k; M symmetric)
hipError_t launch_tei_diag(const double *c, const double *const *V, const double *const *M,
                           int R, int R_N, int N_pair, double *Y, double *d, hipStream_t st);
// ispiv [N]: 1 at the pivots recorded so far (launch_chol_select sets them).
// The pivot's column comes from col [N], or from the formed matrix A [N][N]
// (A != null, symmetric: its row p).
hipError_t launch_chol_step(const double *col, const double *A, double *L, int N, int r,
                            const int *ispiv, const int *state, double *d, hipStream_t st);
// state = {pivot, done, steps}; the next pivot is recorded in piv[steps] and
// ispiv; see cholesky.hip
// step r on the formed matrix A with the selection of its pivot (from d_in,
// the previous step's residual diagonal) in one launch: records state, stats,
// piv[r] and ispiv as launch_chol_select does, then (unless done) forms L_r
// and writes the next residual diagonal to d_out (d_in and d_out distinct).
hipError_t launch_chol_select_step(const double *A, double *L, int N, int r, int *ispiv,
                                   int *state, const double *d_in, double *d_out, double thr,
                                   int R_max, double *stats, int *piv, hipStream_t st);
hipError_t launch_chol_select(double *d, int N, int clear, int steps, double thr, int R_max,
                              int *state, double *stats, int *piv, int *ispiv, hipStream_t st);
// entries of the factorised TEI matrix from V and Y = V M (Y as left by
// launch_tei_diag): the column at the pivot (state given) or the diagonal
hipError_t launch_tei_entries(const double *c, const double *const *V, const double *Y, int R,
                              int R_N, int N_pair, const int *state, double *out,
                              hipStream_t st);
// d[i] = A[i][i], A [N][N]
hipError_t launch_diag_copy(const double *A, int N, double *d, hipStream_t st);
// the factorised TEI matrix formed, B [N_pair][N_pair] = sum_k c_k o_l V^l M^l_k
// V^l^T from Y = V M (as left by launch_tei_diag), in chunks of kc terms
// through Z [3][kc][N_pair][N_pair]; d = its diagonal
hipError_t launch_tei_form_b(const double *c, const double *const *V, const double *Y, int R,
                             int R_N, int N_pair, int kc, double *Z, double *B, double *d,
                             hipStream_t st);
// A = F^T F [n][n] for F [N_pair][n]; Ft: scratch [n][N_pair]
hipError_t launch_fit_gram(const double *F, int n, int N_pair, double *Ft, double *A,
                           hipStream_t st);
hipError_t launch_fill_int(int *x, int count, int value, hipStream_t st);
// Tg: scratch [R_max][R_max]
hipError_t launch_fit_finish(const double *F, const double *L, int n, int N_pair, int R,
                             int R_max, const int *piv, double *Tg, double *U, double *V,
                             hipStream_t st);

// ---- canonical-to-Tucker pieces (tucker.hip) -------------------------------
constexpr int kTuckerMaxSub = 64;   // rows of the iterated subspace
constexpr int kTuckerMaxRank = 48;  // Tucker rank per mode
constexpr int kGemmMaxSplit = 64;   // contraction slices of launch_gemm_f64
// Slices launch_gemm_f64 uses for C [I][N] over K (part then holds
// slices x I x N doubles).
int gemm_splits(int I, int N, int K);
// nn: C[i][j] = sum_t A[i][t] B[t][j] (A [I][K], B [K][N]); otherwise
// C[i][j] = sum_t A[i][t] B[j][t] (B [N][K]).  part: split-slice scratch, or
// NULL for one slice.
// sub: C -= the product instead of C = it.
hipError_t launch_gemm_f64(bool nn, const double *A, const double *B, double *C, int I, int N,
                           int K, double *part, hipStream_t st, bool sub = false);
// rows of X [k][n] (1 <= k <= kOrthRows, k <= n) brought to an orthonormal
// basis of their span, in place, by `passes` (1 or 2) Cholesky-QR passes, with
// the Gram-Schmidt fallback on the device where a pass flags; one pass leaves
// rows orthonormal to about (condition number)^2 u, two to working precision.
// Scratch D [k][k], nrm [k], Linv [k][k], flag [1]; part as for
// launch_gemm_f64 (the product k x k over n).
constexpr int kOrthRows = kTuckerMaxSub;
hipError_t launch_orth_rows(double *X, int k, int n, int passes, double *D, double *nrm,
                            double *Linv, int *flag, double *part, unsigned long long salt,
                            hipStream_t st);
// rows i0..k-1 of X [k][n] pseudo-random in [-1, 1)
hipError_t launch_random_rows(double *X, int i0, int k, int n, unsigned long long salt,
                              hipStream_t st);
// rows i0..k-1 of X [k][n] set to zero
hipError_t launch_zero_rows(double *X, int i0, int k, int n, hipStream_t st);
// eigenpairs of the symmetric H [k][k] (k <= kTuckerMaxSub): lam decreasing,
// Vt [k][k] rows the eigenvectors
hipError_t launch_jacobi_eig(const double *H, int k, double *lam, double *Vt, hipStream_t st);
// K[(i rb + j)][t] = c[t] Ua[i][t] Ub[j][t]
hipError_t launch_khatri_rao(const double *c, const double *Ua, const double *Ub, int ra, int rb,
                             int R, double *K, hipStream_t st);
// sign of each row of Z [r][n] fixed; sv[i] = sqrt(max(lam[i], 0)) if sv
hipError_t launch_sign_rows(double *Z, int r, int n, const double *lam, double *sv,
                            hipStream_t st);

// ---- lattice sums and lattice energy (lattice.hip) -------------------------
hipError_t launch_lattice_sum(int n0, const int *L, int R_N, const double *const *p,
                              double *const *A, hipStream_t st);
// term: scratch [R_N]; E: device scalar
hipError_t launch_lattice_energy(int n0, const int *L, int R_N, const double *c,
                                 const double *h, const double *const *p, double Z,
                                 double *term, double *E, hipStream_t st);

// ---- term classes and smooth terms (lowrank.hip) ---------------------------
constexpr int kBandMax = 16;   // widest band of a narrow term
constexpr int kPolyRank = 32;  // polynomial degree < kPolyRank for a smooth term
constexpr int kPolyMinN = 128; // smooth terms only for n >= kPolyMinN
// coefficients of the orthonormal discrete Chebyshev polynomials on N points
struct PolyCoef {
    double N, c0, c1;
    double A[kPolyRank], B[kPolyRank];
};
PolyCoef poly_coef(int N);
bool smooth_terms_supported(int n);
// cls[k]: B >= 0 narrow (band B), -2 smooth (polynomial to 2^-44 relative),
// -1 general
hipError_t launch_term_class(const double *p, int n, int R_N, int *cls, hipStream_t stream);
// Q[r][a], r < kPolyRank, a < n: orthonormal polynomials on the cell grid
hipError_t launch_poly_rows(int n, double *Q, hipStream_t stream);
// X[i][r] = sum_a U[i][a] Q[r][a]; part: scratch [kProjectSplit][R_f][kPolyRank]
constexpr int kProjectSplit = 32;
hipError_t launch_poly_project(const double *U, int n, int R_f, const double *Q, double *part,
                               double *X, hipStream_t stream);
// S[k] = Q T_k Q^T (kPolyRank x kPolyRank) for the terms of class -2, from the
// half spectra of Q's rows [kPolyRank][N/2+1] and of the kernel embeddings
// [R_N][N/2+1]; partial: scratch [R_N][kSpectralSplit][kPolyRank][kPolyRank]
constexpr int kSpectralSplit = 32;
hipError_t launch_spectral_gram(const double2 *Qspec, const double2 *Cspec, int N, int R_N,
                                const int *cls, double *partial, double *S, hipStream_t stream);
// G_k = X S_k X^T for the terms of class -2 (S [R_N][kPolyRank][kPolyRank])
hipError_t launch_lowrank_gram(const double *X, const double *S, const int *cls, double *G,
                               int R_f, int R_N, bool mirror, hipStream_t stream);

}  // namespace tc

// ---- the C-ABI's TEI Gram call on a given workspace (tc_api.cpp) ----------
#include "tc.h"
namespace tc {
// the argument checks of tc_tei_gram (no device call)
tc_status tei_gram_check(const tc_instance *inst, int count, tc_precision prec);
// tc_tei_gram on the workspace ws of ws_bytes bytes (the caller's, or the
// static scratch of tc_tei_gram_noalloc): validation, plans, dispatch.
tc_status tei_gram_call(const tc_instance *inst, int count, tc_precision prec, void *ws,
                        size_t ws_bytes, void *stream);
}  // namespace tc

// ---- diagnostics (diag.hip) -------------------------------------------------
namespace tc {
bool check_finite_on();   // TC_CHECK_FINITE set (and not "0")
bool debug_sync_on();     // TC_DEBUG_SYNC set (and not "0")
bool chol_columns_on();   // TC_CHOL_COLUMNS set (and not "0")
// synchronise st after launching `kernel`; false (and a line on stderr) on error
bool debug_sync_check(const char *kernel, hipStream_t st);
struct FiniteSpan {
    const double *x;  // device
    long count;
};
// 1 if any span holds a NaN or Inf, 0 if none, -1 on a HIP error; synchronises st
int scan_nonfinite(const FiniteSpan *spans, int count, hipStream_t st);
}  // namespace tc
