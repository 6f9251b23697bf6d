/*
 * tc.h -- C ABI of the MI355X (gfx950) library for the grid-based
 * Newton-kernel convolution and two-electron-integral (TEI) Gram assembly of
 * Khoromskaia & Khoromskij, arXiv:1504.06289.
 *
 * What the library computes (notation of the paper, Sections 2.5, 3.1, 3.2
 * and Appendix 3):
 *
 *   grid          n_l cells of width h_l per mode l = 1,2,3, cell-centred;
 *   side matrix   U^l in R^{n_l x R_f}: column j is function j's mode-l
 *                 vector (the product side matrices of Section 3.2);
 *   kernel        rank-R_N canonical Newton kernel (eq. NewtCan and
 *                 Appendix 3 eq. sinc_general), term k given by the weight
 *                 c_k > 0 and the per-mode vectors p^l_k[m], lag
 *                 m = -(n_l-1)..(n_l-1), with the Toeplitz matrix
 *                 T^l_k[a][b] = p^l_k[a-b];
 *   convolution   W^l_k = T^l_k U^l  (the 1D convolutions p_k *_n U of
 *                 eq. Factor_Mk_Conv, aperiodic, restricted to the box);
 *   Grams         G^l_k = U^l^T W^l_k  (the matrices M_k^(l) of
 *                 eq. Factor_Mk_Conv);
 *   TEI matrix    J = sum_k c_k G^1_k o G^2_k o G^3_k  (the factorised TEI
 *                 matrix of Section 3.2 with V = I; o = Hadamard product).
 *
 * Conventions for every call:
 *   - All numbers crossing the ABI are IEEE binary64 (double).  The
 *     precision argument selects only the arithmetic of the Toeplitz and Gram
 *     contractions inside the library; kernel generation, the Hadamard/sum
 *     over k, and the adjoint's D formation are always binary64.
 *   - Layouts are row-major and dense:
 *       U   [R_f][n]       row j = column j of U^l (contiguous over cells)
 *       p   [R_N][2n-1]    lag m of term k at p[k*(2n-1) + m + n - 1]
 *       W   [R_N][R_f][n]
 *       G   [3][R_N][R_f][R_f]
 *       J   [R_f][R_f]     both triangles written
 *   - "device" pointers are HIP device allocations (or managed/host-mapped
 *     memory the device can read); "host" pointers are ordinary host memory.
 *   - The caller owns every buffer.  The library never allocates or frees
 *     device memory: scratch memory comes from the caller's workspace (size
 *     from tc_workspace_bytes and the other *_workspace_bytes calls), and all
 *     work is enqueued on the caller's stream (a hipStream_t passed as void*;
 *     NULL = the default stream) or, for tc_tei_gram, on internal streams
 *     forked from it and joined back into it, so that it completes in the
 *     caller's stream order.
 *   - A call synchronises the caller's stream only where its own comment
 *     says so: tc_autotune, tc_density_fit, tc_tei_cholesky,
 *     tc_lattice_energy, tc_canonical_to_tucker with eps > 0 and
 *     tc_profile_read.  Every other call only enqueues work and can be
 *     captured in a HIP graph.
 *   - Arguments are validated before anything is enqueued; on any error no
 *     output is written.  Launch failures return TC_ERR_HIP.  Faults during
 *     execution surface at the caller's next synchronisation.
 *   - Results are bitwise reproducible for a given device, precision and
 *     problem size (no floating-point atomics; fixed reduction orders).
 *   - Calls on different streams may run concurrently if their outputs and
 *     workspaces do not overlap.
 *   - Diagnostics, read from the environment at every call (both make the
 *     calls synchronise, so keep them off while capturing a graph):
 *       TC_CHECK_FINITE=1  tc_convolve, tc_tei_gram, tc_tei_gram_noalloc,
 *                          tc_tei_gram_backward, tc_coulomb and tc_nuclear
 *                          scan their binary64 device inputs (c, p, U, and
 *                          V, d, Jbar, G_saved where present) for NaN and
 *                          Inf before any other work, synchronise once to
 *                          read the result, and return TC_ERR_INVALID_ARG,
 *                          writing no output, when one is found;
 *       TC_DEBUG_SYNC=1    every kernel launch is followed by a
 *                          synchronisation of its stream; the first failing
 *                          kernel is named on stderr and the call returns
 *                          TC_ERR_HIP.
 *     and one that selects a code path:
 *       TC_CHOL_COLUMNS=1  tc_density_fit and tc_tei_cholesky form each
 *                          pivot's column from the factors at every step, the
 *                          path they take by themselves only beyond the sizes
 *                          where they form the matrix (n > 8192 cells,
 *                          N_pair > 4096 products); same workspace, same
 *                          results up to rounding.
 */
#ifndef TC_H
#define TC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TC_OK = 0,
    TC_ERR_INVALID_ARG = 1, /* null pointer, size out of range, non-finite parameter */
    TC_ERR_WORKSPACE = 2,   /* workspace missing or smaller than tc_workspace_bytes */
    TC_ERR_UNSUPPORTED = 3, /* precision or size the library does not implement */
    TC_ERR_HIP = 4,         /* a HIP launch or runtime call failed */
    /* not codes: they give the enum the range of int, so that any int a
     * caller passes is a defined value (and is rejected if unknown) */
    TC_STATUS_RANGE_MIN_ = -2147483647 - 1,
    TC_STATUS_RANGE_MAX_ = 2147483647
} tc_status;

/* Arithmetic of the Toeplitz (W = T U) and Gram (G = U^T W) contractions.
 * The values 0..3 are those of the interface's first statement (binary64,
 * binary32, split-bfloat16 with three and with six products); the int8
 * error-free splitting, the variant that meets 1e-7 on J, is appended as 4. */
typedef enum {
    TC_FP64 = 0,     /* binary64 matrix cores (v_mfma_f64_16x16x4)           */
    TC_FP32 = 1,     /* operand rows scaled by a power of two (their maximum
                        to [0.5, 1)), rounded to binary32, binary32 matrix
                        cores with binary32 partial sums over K-chunks of 64
                        and binary64 accumulation across chunks; does not
                        reach 1e-7 on J (a measured comparison point)        */
    TC_BF16X3 = 2,   /* rows scaled as for TC_FP32, each entry split exactly
                        into two bfloat16 pieces, the three leading piece
                        products on bfloat16 matrix cores with binary32
                        accumulation over K-chunks of 64, binary64 across
                        chunks (a measured comparison point)                  */
    TC_BF16X6 = 3,   /* as TC_BF16X3 with three pieces and the six products
                        of piece-index sum <= 2                               */
    TC_OZAKI_I8 = 4, /* error-free splitting of each operand into four int8
                        slices with one exponent per row (28 bits relative to
                        the row maximum), the ten leading slice products on
                        int8 matrix cores with exact int32 accumulation, and
                        binary64 recombination (Ozaki scheme)                 */
    TC_PRECISION_RANGE_MIN_ = -2147483647 - 1,  /* range of int (see tc_status) */
    TC_PRECISION_RANGE_MAX_ = 2147483647
} tc_precision;

/* How the Toeplitz products W_k = T_k U are formed.  TC_ALGO_DIRECT: the
 * implicit-Toeplitz matrix-core product in the arithmetic selected by
 * tc_precision.  TC_ALGO_FFT: aperiodic convolution through a circulant
 * embedding of length N >= 2n-1 with binary64 FFTs (LDS-resident transforms
 * for n <= 4096, four-step transforms through device memory for
 * 4096 < n <= TC_MAX_N); the Grams then use the tc_precision arithmetic.  With TC_OZAKI_I8 the route treats narrow
 * and smooth kernel terms separately (tc_term_classes).  TC_ALGO_AUTO: the
 * entry of the tuning
 * table for the mode's (n, R_f, R_N, precision), else a built-in rule. */
typedef enum {
    TC_ALGO_AUTO = 0,
    TC_ALGO_DIRECT = 1,
    TC_ALGO_FFT = 2,
    TC_ALGORITHM_RANGE_MIN_ = -2147483647 - 1,  /* range of int (see tc_status) */
    TC_ALGORITHM_RANGE_MAX_ = 2147483647
} tc_algorithm;

/* How tc_tei_gram runs a batch (count > 1).  TC_BATCH_FORK_JOIN: the
 * instances spread over internal streams, each with its own per-mode
 * launches.  TC_BATCH_QUEUE*: TC_OZAKI_I8 only: every mode of every instance
 * prepares its int8 slices on the streams, then ONE persistent launch forms
 * the int8 Grams of all of them from a device work queue of (instance, mode,
 * term, tile[, K part]) items sorted by cost (contraction length first), then
 * the Hadamard sums follow; the variants choose the tile edge (128, or 64 for
 * instances with R_f < 256) and whether each tile's contraction is split in
 * two parts (added in a fixed order; the results are bitwise those of the
 * fork-join route: the int8 sums are exact and their binary64 recombination
 * spans at most 53 bits).  TC_BATCH_AUTO: the batch's entry in the tuning
 * table (set by tc_batch_tune_set or tc_autotune), else TC_BATCH_FORK_JOIN. */
typedef enum {
    TC_BATCH_AUTO = 0,
    TC_BATCH_FORK_JOIN = 1,
    TC_BATCH_QUEUE = 2,          /* 128-tiles, one K part            */
    TC_BATCH_QUEUE_T64 = 3,      /* 64-tiles below R_f = 256         */
    TC_BATCH_QUEUE_K2 = 4,       /* 128-tiles, two K parts           */
    TC_BATCH_QUEUE_T64_K2 = 5,   /* 64-tiles below 256, two K parts  */
    TC_BATCH_ROUTE_RANGE_MIN_ = -2147483647 - 1,  /* range of int (see tc_status) */
    TC_BATCH_ROUTE_RANGE_MAX_ = 2147483647
} tc_batch_route;

/* Largest supported sizes (guards for index arithmetic). */
#define TC_MAX_N 65536
#define TC_MAX_RF 65536
#define TC_MAX_RN 256

/* One TEI problem.  Arrays of these form a batch. */
typedef struct {
    int n[3];            /* cells per mode, 1 <= n_l <= TC_MAX_N             */
    int R_f;             /* number of product functions (columns of U)       */
    int R_N;             /* number of kernel terms                           */
    const double *c;     /* [R_N] device: weights c_k = a_k h_1 h_2 h_3 > 0  */
    const double *p[3];  /* [R_N][2 n_l - 1] device; may alias across modes  */
    const double *U[3];  /* [R_f][n_l] device                                */
    double *J;           /* [R_f][R_f] device, output                        */
    double *G_saved;     /* [3][R_N][R_f][R_f] device output, or NULL        */
} tc_instance;

/* Nuclei against a set of product functions, for tc_nuclear (Section 3.3,
 * the nuclear potential operator of the core Hamiltonian). */
typedef struct {
    int n[3];            /* cells per mode, 1 <= n_l <= TC_MAX_N             */
    double h[3];         /* cell widths (> 0)                                */
    int R_f;             /* number of product functions (rows of U)          */
    int R_N;             /* number of kernel terms                           */
    int M;               /* number of nuclei, 1 <= M, M R_N <= 65535         */
    const double *c;     /* [R_N] device: weights c_q = a_q h_1 h_2 h_3      */
    const double *p[3];  /* [R_N][2 n_l - 1] device; may alias across modes  */
    const double *U[3];  /* [R_f][n_l] device: the product functions         */
    const double *Z;     /* [M] host: nuclear charges (finite)               */
    const int *pos;      /* [M][3] host: grid cell of nucleus a along mode l,
                            0 <= pos[3a + l] < n_l (nuclei at cell centres) */
    double *V;           /* [R_f][R_f] device, output, both triangles        */
} tc_nuclear_problem;

/* A density in canonical format against a set of product functions, for
 * tc_coulomb (Section 3.1, the Hartree potential and the Coulomb matrix). */
typedef struct {
    int n[3];            /* cells per mode, 1 <= n_l <= TC_MAX_N             */
    int R_f;             /* number of product functions (rows of U)          */
    int R_rho;           /* number of density terms (rows of V), >= 1        */
    int R_N;             /* number of kernel terms                           */
    const double *c;     /* [R_N] device: weights c_k = a_k h_1 h_2 h_3 > 0  */
    const double *p[3];  /* [R_N][2 n_l - 1] device; may alias across modes  */
    const double *U[3];  /* [R_f][n_l] device: the product functions         */
    const double *V[3];  /* [R_rho][n_l] device: the density factors         */
    const double *d;     /* [R_rho] device: the density weights              */
    double *Jd;          /* [R_f] device, output                             */
} tc_density;

/* Operation codes for tc_workspace_bytes. */
#define TC_OP_CONVOLVE 0
#define TC_OP_TEI_GRAM 1
#define TC_OP_TEI_GRAM_BACKWARD 2
#define TC_OP_AUTOTUNE 3   /* tc_autotune: every route of every mode may run */

/*
 * tc_newton_kernel -- rank-R_N canonical Newton kernel on an n-cell grid of
 * width h (Appendix 3).  Sinc rule for the Laplace-Gauss transform of 1/r
 * (eq. sinc_Newt) in the variable u = log t: nodes t_k = exp(u0 + k hu),
 * weights a_k = (2/sqrt(pi)) hu t_k, k = 0..R_N-1.  Kernel vectors are the
 * Galerkin projections onto the piecewise-constant cells (eq. galten and the
 * vectors b(t_k)):  p_k[m] = integral of exp(-t_k^2 s^2) over
 * [(m-1/2)h, (m+1/2)h], m = -(n-1)..(n-1).
 *   n      1..TC_MAX_N;  h > 0;  R_N 1..TC_MAX_RN;  u0, hu finite, hu > 0.
 *   t_host [R_N] host output (may be NULL): the nodes t_k.
 *   c_host [R_N] host output (may be NULL): c_k = a_k h^3 (isotropic grid;
 *          for unequal modes use a_k = c_k / h^3 times h_1 h_2 h_3).
 *   p_dev  [R_N][2n-1] device output.
 *   The nodes are computed on the host, the vectors on the device.
 */
tc_status tc_newton_kernel(int n, double h, int R_N, double u0, double hu,
                           double *t_host, double *c_host, double *p_dev,
                           void *stream);

/*
 * tc_convolve -- potential factors W_k = T_k U for one mode (Section 2.5
 * eq. conv; the factors of the canonical Hartree potential of each
 * function):  W[k][j][a] = sum_b p[k][a-b+n-1] U[j][b].
 *   p_dev [R_N][2n-1] device;  U_dev [R_f][n] device;
 *   W_dev [R_N][R_f][n] device output (must not overlap the inputs).
 *   prec  contraction arithmetic; ws/ws_bytes workspace
 *         (tc_workspace_bytes(TC_OP_CONVOLVE, ...)).
 */
tc_status tc_convolve(int n, int R_f, int R_N, const double *p_dev,
                      const double *U_dev, double *W_dev, tc_precision prec,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * tc_term_classes -- how the int8 FFT route (TC_OZAKI_I8 with TC_ALGO_FFT)
 * treats each kernel term of a mode (diagnostics; the route computes the
 * same classes internally).  cls_dev [R_N] device output:
 *   B >= 0  narrow: sum_{|m| > B} |p_k[m]| <= 2^-60 sum_m |p_k[m]| with
 *           B <= min(16, n-1) smallest; W_k by direct convolution over
 *           |m| <= B;
 *   -2      smooth (n >= 128 only): the least-squares polynomial of degree
 *           < 32 in the lag reproduces p_k to within 2^-44 max|p_k| at every
 *           lag; G_k = X S_k X^T at rank 32 from an orthonormal polynomial
 *           basis Q of the cells (X = U Q^T, S_k = Q T_k Q^T), binary64,
 *           |error of G_k[i][j]| <= 2 (2n-1) 2^-44 max|p_k| |u_i|_2 |u_j|_2;
 *   -1      general: FFT convolution and the int8 Gram.
 *   p_dev [R_N][2n-1] device.
 */
tc_status tc_term_classes(int n, int R_N, const double *p_dev, int *cls_dev, void *stream);

/*
 * tc_tei_gram -- the TEI/Coulomb matrix of every instance (Section 3.2):
 * J = sum_k c_k G^1_k o G^2_k o G^3_k with G^l_k = U^l^T T^l_k U^l.
 * Instances are independent; their output buffers must not overlap one
 * another.  When G_saved is non-NULL the Grams are also written there (the
 * backward pass can then skip recomputing them).
 *   inst  host array of count descriptors (pointers inside are device).
 *   count >= 1.   ws: tc_workspace_bytes(TC_OP_TEI_GRAM, inst, count, prec).
 * The work runs on four internal streams of default priority (created at
 * the first call and kept for the life of the process) that fork from and
 * join back into `stream` through events, so the call still completes in
 * stream order and can be captured as one graph with parallel branches.
 * With count == 1 the Grams of the three modes run concurrently (the first
 * on `stream`, the other two on internal streams), each in its own workspace
 * region, and the Hadamard sum follows on `stream`; with count > 1 the
 * instances run concurrently and the modes of each in turn.
 * Calls from several host threads are serialised while they enqueue.
 */
tc_status tc_tei_gram(const tc_instance *inst, int count, tc_precision prec,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * tc_tei_gram_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): tc_tei_gram with the workspace taken from a static device
 * array of TC_NOALLOC_SCRATCH_BYTES (256 MiB) that the library holds on each
 * GPU it runs on until the process ends.  It calls no allocating routine.
 * Same arguments, plans, kernels and results as tc_tei_gram (bitwise), less
 * the workspace.  A problem whose tc_workspace_bytes(TC_OP_TEI_GRAM, ...)
 * exceeds the array returns TC_ERR_WORKSPACE before any device call.
 * `stream` must belong to the current device: the array is looked up
 * (hipGetSymbolAddress) with that device current on its first call there.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other host threads without ordering) race; calls ordered
 * on one stream do not.  The array keeps the last call's data; nothing in
 * the computation reads workspace it has not written in the same call.
 */
#define TC_NOALLOC_SCRATCH_BYTES 268435456
tc_status tc_tei_gram_noalloc(const tc_instance *inst, int count, tc_precision prec,
                              void *stream);

/*
 * tc_tei_gram_backward -- adjoint of f = <Jbar, J> with respect to the side
 * matrices: with S = (Jbar + Jbar^T)/2 and D^l_k = c_k S o G^{l+1}_k o
 * G^{l+2}_k (modes cyclic), dU^l = 2 sum_k T^l_k U^l D^l_k = 2 sum_k W^l_k D^l_k
 * (T_k and the Grams are symmetric).  For Jbar = w w^T this is the gradient
 * of w^T J w.
 *   Jbar  host array [count] of device pointers, each [R_f][R_f].
 *   dU    host array [3*count] of device pointers: dU[3*i + l] is [R_f][n_l]
 *         output for instance i, mode l.
 *   Uses inst[i].G_saved when non-NULL (as written by tc_tei_gram with the
 *   same inputs), otherwise recomputes the Grams.  inst[i].J is not touched.
 */
tc_status tc_tei_gram_backward(const tc_instance *inst, int count,
                               const double *const *Jbar, double *const *dU,
                               tc_precision prec, void *ws, size_t ws_bytes,
                               void *stream);

/*
 * Workspace size in bytes for op (TC_OP_*) on the given problem(s); for
 * TC_OP_CONVOLVE only inst[0].n[0], R_f and R_N are read.  Returns 0 when no
 * workspace is needed and (size_t)-1 for invalid arguments.
 */
size_t tc_workspace_bytes(int op, const tc_instance *inst, int count,
                          tc_precision prec);

/*
 * Tuning table (process-wide, thread-safe): the algorithm TC_ALGO_AUTO uses
 * for a mode of n cells with R_f functions and R_N terms at precision prec.
 * tc_tune_set with TC_ALGO_AUTO removes the entry.  tc_tune_get returns the
 * algorithm a call would use now (the table entry or the built-in rule).
 */
tc_status tc_tune_set(int n, int R_f, int R_N, tc_precision prec, tc_algorithm algo);
tc_algorithm tc_tune_get(int n, int R_f, int R_N, tc_precision prec);

/*
 * Batch routes in the tuning table, keyed by the batch (precision, count and
 * every instance's n, R_f, R_N and whether it keeps its Grams).
 * tc_batch_tune_set with TC_BATCH_AUTO removes the entry; a TC_BATCH_QUEUE*
 * route for a precision other than TC_OZAKI_I8 returns TC_ERR_UNSUPPORTED.
 * tc_batch_tune_get returns the route tc_tei_gram would take now.
 */
tc_status tc_batch_tune_set(const tc_instance *inst, int count, tc_precision prec,
                            tc_batch_route route);
tc_batch_route tc_batch_tune_get(const tc_instance *inst, int count, tc_precision prec);

/*
 * tc_autotune -- measure every algorithm available for each distinct mode
 * shape of the instances (one warm-up and three timed runs of the mode's
 * Toeplitz products and Grams, HIP events on `stream`) and record the fastest
 * in the tuning table.  For a TC_OZAKI_I8 batch (count > 1) it then times the
 * whole batch on every tc_batch_route (one warm-up and two timed runs each,
 * with the J outputs in the workspace) and records the fastest route for the
 * batch.  It synchronises `stream` (it reads the timings).
 * Writes scratch data into the workspace (tc_workspace_bytes(TC_OP_AUTOTUNE,
 * ...)) and leaves inst[i].J untouched.  ms_out (host, may be NULL) receives
 * 2 entries per instance and mode: [ (i*3 + l)*2 + a ] = milliseconds of
 * algorithm a (0 = direct, 1 = FFT; negative if unavailable).
 */
tc_status tc_autotune(const tc_instance *inst, int count, tc_precision prec, void *ws,
                      size_t ws_bytes, void *stream, double *ms_out);

/*
 * Kernel timing (diagnostics).  tc_profile_enable(1) makes every kernel
 * launch of the library record a pair of HIP events on its stream (events
 * are created on demand, so do not enable it during graph capture).  While
 * it is on, tc_tei_gram runs the three modes of a lone instance in turn on
 * the caller's stream, so that every recorded duration is that of the kernel
 * alone on the device.
 * tc_profile_read synchronises the recorded events, writes up to
 * max_kernels entries (kernel name, total milliseconds, number of launches)
 * accumulated since the previous read, clears them, and returns the number
 * of distinct kernels (or -1 if an event query failed).  Any output pointer
 * may be NULL.
 */
tc_status tc_profile_enable(int on);
int tc_profile_read(int max_kernels, char (*names)[64], double *total_ms, long *calls);

/*
 * tc_coulomb -- Coulomb entries of the product functions against a density
 * given in canonical format (Section 3.1: the Hartree potential of the
 * density Theta' = sum_m d_m v^1_m x v^2_m x v^3_m is the sum over m and the
 * kernel terms q of tensor products of the 1D convolutions v^l_m * p^l_q, and
 * the Coulomb entries are its scalar products with the rank-1 products of
 * basis functions):
 *   Jd[i] = sum_q c_q sum_m d_m prod_l <U^l[i], (T^l_q V^l)[m]>,
 * the plain sum over the cells in <.,.> (the cell volume is in c_q).  With
 * V = U this is J d for the J of tc_tei_gram.
 *   prob  host descriptor, pointers inside are device.
 *   prec  TC_FP64 only (otherwise TC_ERR_UNSUPPORTED): the convolutions by
 *         the direct or FFT route (tuning table of (n_l, R_rho, R_N)), the
 *         cross Grams U (T_q V)^T on binary64 matrix cores, the sum over q and
 *         m in a fixed order (bitwise reproducible).
 *   ws    tc_coulomb_workspace_bytes(prob, prec) bytes of device memory.
 * Runs on `stream`; the modes in turn.
 */
size_t tc_coulomb_workspace_bytes(const tc_density *prob, tc_precision prec);
tc_status tc_coulomb(const tc_density *prob, tc_precision prec, void *ws, size_t ws_bytes,
                     void *stream);

/*
 * tc_density_fit -- 1D density fitting of one mode's side matrix (Section
 * 3.2): F [N_pair][n] device (row i: a product of two basis functions on the
 * mode's grid) is approximated as F ~ V U through the diagonally pivoted
 * Cholesky of A = F^T F over the grid points (never formed: diagonal and
 * pivot columns from F).  The steps run while the residual trace exceeds
 * tol^2 trace(A) and fewer than R_max columns exist; with the R pivots P,
 *   V = F[:, P]                [N_pair][R]  (the products at the pivots),
 *   U = A[P,P]^-1 A[P, :]      [R][n]       (U[:, P] = I),
 * and |F - V U|_F^2 equals the residual trace.  Pivot = first index of the
 * largest residual diagonal entry.
 *   U_dev [R_max][n], V_dev [N_pair][R_max] device outputs; rows of U and
 *   columns of V beyond R are zero (so the padded factors can be used as
 *   they are).  pivots_host [R_max] (may be NULL), R_out, residual_out
 *   (residual trace; may be NULL) host outputs.
 *   ws: tc_density_fit_workspace_bytes(n, N_pair, R_max).
 * Synchronises `stream`: once before the first step (to read trace(A)), once
 * per group of steps (16, then 32, then 64 steps a group; the stopping test
 * runs on the device, which turns the remaining steps of a group into no-ops;
 * the host reads its flag once per group), and once at the end.
 */
size_t tc_density_fit_workspace_bytes(int n, int N_pair, int R_max);
tc_status tc_density_fit(int n, int N_pair, const double *F_dev, double tol, int R_max,
                         double *U_dev, double *V_dev, int *pivots_host, int *R_out,
                         double *residual_out, void *ws, size_t ws_bytes, void *stream);

/*
 * tc_tei_cholesky -- pivoted Cholesky of the factorised TEI matrix over the
 * N_pair products (Section 3.2):
 *   B = sum_k c_k  o_l  V^l M^l_k V^l^T  ~ L L^T,
 * B never formed: its diagonal B(i,i) = sum_k c_k prod_l V^l(i,:) M^l_k
 * V^l(i,:)^T and, per step, its column at the pivot from the factors.  The
 * steps run while the residual trace exceeds tol trace(B) and fewer than
 * R_max columns exist; pivot = first index of the largest residual diagonal
 * entry.  With V^l from tc_density_fit and M^l_k = U^l T^l_k U^l^T (the Grams
 * of tc_tei_gram's G_saved for the fitted rows U^l), B approximates the TEI
 * matrix of the products.
 *   c_dev [R_N]; V_dev host array [3] of device [N_pair][R]; M_dev host array
 *   [3] of device [R_N][R][R], each M^l_k symmetric.
 *   L_dev [R_max][N_pair] device output: row r = column r of the factor.
 *   pivots_host [R_max] (may be NULL), R_out, residual_out (may be NULL).
 *   ws: tc_tei_cholesky_workspace_bytes(N_pair, R, R_N, R_max).
 * Synchronises `stream` as tc_density_fit does: before the first step and
 * once per group of steps (16, 32, then 64).
 */
size_t tc_tei_cholesky_workspace_bytes(int N_pair, int R, int R_N, int R_max);
tc_status tc_tei_cholesky(int N_pair, int R, int R_N, const double *c_dev,
                          const double *const *V_dev, const double *const *M_dev, double tol,
                          int R_max, double *L_dev, int *pivots_host, int *R_out,
                          double *residual_out, void *ws, size_t ws_bytes, void *stream);

/*
 * tc_nuclear -- Galerkin matrix of the nuclear potential operator
 * V_c(x) = -sum_a Z_a / |x - x_a| in the basis of product functions
 * (Section 3.3: the master kernel is shifted to each nucleus by a rank-1
 * windowing, the shifted kernels are summed with the charges, and the matrix
 * entries are scalar products of the rank-1 products with that sum):
 *   V[i][j] = -sum_a Z_a sum_q (c_q/(h1 h2 h3)) prod_l sum_x U^l[i][x] U^l[j][x]
 *                                                    p^l_q[x - pos[a][l] + n_l - 1],
 * i.e. the cell volume times the sum over grid cells of g_i g_j V_c, with the
 * kernel's approximation of 1/|x| (its cell average) in place of 1/|x|.
 *   prob  host descriptor; c, p, U, V device, Z and pos host (read before
 *         the call returns; the tables travel as kernel arguments).
 *   The 1D matrices U^l diag(p^l_q shifted) U^l^T of every (nucleus, term)
 *   pair on binary64 matrix cores, then the product over the modes and the
 *   sum over the pairs in a fixed order (bitwise reproducible). Groups of
 *   four pairs whose kernel vectors are all narrow (the lags beyond a band
 *   B <= 16 carry below 2^-60 of the vector's l1 norm) sum only over the
 *   cells within B of their nuclei.
 *   ws    tc_nuclear_workspace_bytes(prob) bytes of device memory
 *         (3 M R_N R_f^2 doubles for the 1D matrices, plus tables); returns
 *         (size_t)-1 for an invalid descriptor.
 * Runs on `stream`, stream-ordered, no synchronisation.
 */
size_t tc_nuclear_workspace_bytes(const tc_nuclear_problem *prob);
tc_status tc_nuclear(const tc_nuclear_problem *prob, void *ws, size_t ws_bytes, void *stream);

/*
 * tc_canonical_to_tucker -- Tucker form of a canonical tensor
 * T = sum_k c_k a^1_k x a^2_k x a^3_k (Appendix, part 1, the
 * Canonical-to-Tucker transform):
 *   (A) Z^l = the r_l dominant left singular vectors of the side matrix,
 *   (B) the side matrices projected onto them, U~^l = Z^l A^l^T,
 *   (C, D) m_max sweeps over l = 1, 2, 3: Z^l = the r_l dominant left
 *       singular vectors of the partially projected image
 *       M^l = sum_k c_k a^l_k x u~^m1_k x u~^m2_k (n_l x r_m1 r_m2), then
 *       U~^l updated,
 *   (E) the core beta = sum_k c_k u~^1_k x u~^2_k x u~^3_k,
 * so that T ~ sum beta[i][j][m] z^1_i x z^2_j x z^3_m.  Each dominant
 * subspace comes from `its` steps of orthogonal iteration on a subspace of
 * k = min(n_l, 64, max(2 r_l, r_l + 8)) vectors (pseudo-random start, or the
 * previous basis in a sweep) and a Rayleigh-Ritz step; with a gap between
 * the r_l-th and the (k+1)-th singular value the basis converges like
 * (sigma_{k+1}/sigma_{r_l})^{2 its}.  Each basis vector's entry of largest
 * magnitude is positive.
 *   eps > 0 selects the epsilon truncation of step (A): mode l keeps the
 *   singular vectors whose singular value is at least eps times the largest
 *   (at least 1, at most r_l), each rank then clamped to the product of the
 *   other two; basis rows and core entries beyond the chosen ranks are zero,
 *   and the call synchronises `stream` once to read the singular values.
 *   eps <= 0 keeps the ranks r.  r_out host [3] (or NULL): the ranks used.
 *   n host [3], 1 <= n_l <= TC_MAX_N; R >= 1 terms; c [R] device;
 *   A_dev host array [3] of device [R][n_l] (row k = the mode-l vector of
 *   term k); r host [3], 1 <= r_l <= min(48, n_l, R), and with m_max > 0
 *   r_l <= r_m1 r_m2; 0 <= m_max <= 100; 1 <= its <= 1000.
 *   Z_dev host array [3] of device [r_l][n_l] outputs (orthonormal rows);
 *   beta_dev device [r1][r2][r3] output; sv_dev device [r1 + r2 + r3] output
 *   (the singular values of the last step of each mode) or NULL.
 *   ws    tc_canonical_to_tucker_workspace_bytes(n, R, r) bytes of device
 *         memory ((size_t)-1 for invalid sizes).
 * Runs on `stream`, stream-ordered; no synchronisation unless eps > 0.
 */
size_t tc_canonical_to_tucker_workspace_bytes(const int *n, int R, const int *r);
tc_status tc_canonical_to_tucker(const int *n, int R, const double *c_dev,
                                 const double *const *A_dev, const int *r, int m_max, int its,
                                 double eps, double *const *Z_dev, double *beta_dev,
                                 double *sv_dev, int *r_out, void *ws, size_t ws_bytes,
                                 void *stream);

/*
 * tc_lattice_sum -- assembled canonical vectors of the Newton kernel summed
 * over a rectangular lattice of charges (Section 5.1, eq. CoulombLatTensCan):
 * L[l] unit cells of n0 grid cells along direction l (n_l = n0 L[l] cells of
 * width h_l), the charge of unit cell j in grid cell j n0 + n0/2 (the paper's
 * symmetric lattice, shifted so that indices start at 0).  Per direction and
 * kernel term,
 *   A^l[q][i] = sum_{j < L[l]} p^l[q][i - (j n0 + n0/2) + n_l - 1],  i < n_l,
 * so that sum_q c_q/(h1 h2 h3)^2 prod_l A^l[q][i_l] is the lattice sum of the
 * kernel's approximation of 1/|x| at grid cell (i1, i2, i3): rank R_N, the
 * rank of the kernel.
 *   n0 >= 1; L host [3], 1 <= L[l], n0 L[l] <= TC_MAX_N; R_N 1..TC_MAX_RN.
 *   p_dev host array [3] of device [R_N][2 n_l - 1] (tc_newton_kernel with
 *   n = n_l); A_dev host array [3] of device [R_N][n_l] outputs.
 */
tc_status tc_lattice_sum(int n0, const int *L, int R_N, const double *const *p_dev,
                         double *const *A_dev, void *stream);

/*
 * tc_lattice_energy -- interaction energy of equal charges Z on the lattice
 * of tc_lattice_sum (Section 5.2, eq. EnergyLattice): the kernel traced at
 * the lattice lags and summed over all ordered pairs, minus the self terms,
 *   E = Z^2/2 sum_q w_q (prod_l S^l_q - L1 L2 L3 prod_l p^l_q[0]),
 *   S^l_q = sum_{|j| < L[l]} (L[l] - |j|) p^l_q[j n0],  w_q = c_q/(h1 h2 h3)^2,
 * which is Z^2/2 sum_{k != j} K(x_k - x_j) for the kernel's approximation K
 * of 1/|x| (O(L) work per term instead of O(L^6)).
 *   c_dev [R_N] device (c_q = a_q h1 h2 h3); h host [3]; p_dev as for
 *   tc_lattice_sum; E_host host output.  ws: 8 (R_N + 1) bytes of device
 *   memory.  Synchronises `stream`.
 */
tc_status tc_lattice_energy(int n0, const int *L, int R_N, const double *c_dev, const double *h,
                            const double *const *p_dev, double Z, double *E_host, void *ws,
                            size_t ws_bytes, void *stream);

/* Static description of a status code (never NULL). */
const char *tc_status_string(tc_status s);

/* Library version as major*10000 + minor*100 + patch. */
int tc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TC_H */
