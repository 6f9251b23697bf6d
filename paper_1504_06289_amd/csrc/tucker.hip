// Canonical-to-Tucker transform (Appendix, part 1), binary64.
//
// Every step that the transform takes an SVD for needs only the r dominant
// left singular vectors of a matrix B^T given as rows B [m][n] (the side
// matrix of a mode, or the transposed partially projected image).  They are
// found by orthogonal iteration on B^T B acting on the rows of X [k][n]
// (k = a few more than r), each step X <- orth((X B^T) B), and a final
// Rayleigh-Ritz step: the k x k matrix H = (X B^T)(X B^T)^T is diagonalised
// by Jacobi rotations and the r leading Ritz vectors are rotated out of X.
//
//   gemm_f64      C = A B^T (NT: both operands contiguous along the
//                 contraction) or C = A B (NN: B contiguous along the output
//                 column), 64 x 64 tiles on binary64 matrix cores, the
//                 contraction split over blockIdx.z into fixed slices whose
//                 partial tiles are summed in order (bitwise reproducible);
//   orth_rows     Cholesky-QR of the k <= 64 rows: their Gram on matrix
//                 cores, a 64 x 64 Cholesky in one workgroup (one barrier per
//                 column) and a column-parallel forward substitution, once or
//                 twice (CholeskyQR2); where a row keeps less than about 3e-6
//                 of its norm the rows fall back, on the device, to classical
//                 Gram-Schmidt applied twice in one workgroup, and a row that
//                 keeps less than 1e-10 is replaced by pseudo-random values and
//                 orthogonalised against every earlier row;
//   jacobi_eig    cyclic Jacobi on a symmetric k x k matrix (k <= 64) held in
//                 LDS, the k/2 disjoint rotations of a round-robin round
//                 applied at once, block by block; eigenvalues sorted in
//                 decreasing order, eigenvectors as rows;
//   khatri_rao    K[(i, j)][t] = c_t Ua[i][t] Ub[j][t];
//   sign_rows     each basis vector's entry of largest magnitude positive.
#include "tc_internal.h"

namespace tc {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;  // output tile edge
constexpr int GK = 16;  // contraction step
constexpr int GPAD = 1;

template <bool NN>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const double *__restrict__ A,
                                                       const double *__restrict__ B,
                                                       double *__restrict__ C, int I, int N,
                                                       int K, int kchunk, int sub)
{
    __shared__ double As[2][GT][GK + GPAD];
    __shared__ double Bs[2][GT][GK + GPAD];

    const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    double *Cs = C + (long)blockIdx.z * I * N;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = (wave >> 1) * 32;
    const int wj = (wave & 1) * 32;
    const int l16 = lane & 15;
    const int lk = lane >> 4;

    // A (and NT B): row tid/4 of the tile, four consecutive contraction indices
    const int lrow = tid >> 2;
    const int lcol = (tid & 3) * 4;
    // NN B: contraction row tid/16 of the slice, four consecutive columns
    const int nrow = tid >> 4;
    const int ncol = (tid & 15) * 4;
    double areg[4], breg[4];

    auto load_stage = [&](int k0) {
        const int i = i0 + lrow;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = k0 + lcol + q;
            areg[q] = (i < I && kk < kend) ? A[(long)i * K + kk] : 0.0;
        }
        if constexpr (NN) {
            const int kk = k0 + nrow;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = j0 + ncol + q;
                breg[q] = (kk < kend && j < N) ? B[(long)kk * N + j] : 0.0;
            }
        } else {
            const int j = j0 + lrow;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int kk = k0 + lcol + q;
                breg[q] = (j < N && kk < kend) ? B[(long)j * K + kk] : 0.0;
            }
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            As[buf][lrow][lcol + q] = areg[q];
        if constexpr (NN) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Bs[buf][ncol + q][nrow] = breg[q];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Bs[buf][lrow][lcol + q] = breg[q];
        }
    };

    f64x4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
            acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int nsteps = kend > kbeg ? (kend - kbeg + GK - 1) / GK : 0;
    if (nsteps > 0) {
        load_stage(kbeg);
        store_stage(0);
    }
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const int buf = s & 1;
        if (s + 1 < nsteps)
            load_stage(kbeg + (s + 1) * GK);
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            double afr[2], bfr[2];
#pragma unroll
            for (int x = 0; x < 2; ++x)
                afr[x] = As[buf][wi + x * 16 + l16][kk + lk];
#pragma unroll
            for (int y = 0; y < 2; ++y)
                bfr[y] = Bs[buf][wj + y * 16 + l16][kk + lk];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[x], bfr[y], acc[x][y],
                                                                      0, 0, 0);
        }
        if (s + 1 < nsteps)
            store_stage(buf ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int j = j0 + wj + y * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + x * 16 + lk + 4 * r;
                if (i < I && j < N) {
                    if (sub)
                        Cs[(long)i * N + j] -= acc[x][y][r];
                    else
                        Cs[(long)i * N + j] = acc[x][y][r];
                }
            }
        }
}

__global__ __launch_bounds__(256) void split_sum_kernel(const double *__restrict__ part,
                                                        double *__restrict__ C, long count,
                                                        int S, int sub)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= count)
        return;
    // eight interleaved sums (eight loads in flight), combined in a fixed order
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int z = 0;
    for (; z + 8 <= S; z += 8)
#pragma unroll
        for (int q = 0; q < 8; ++q)
            a[q] += part[(long)(z + q) * count + e];
    for (; z < S; ++z)
        a[0] += part[(long)z * count + e];
    const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    C[e] = sub ? C[e] - s : s;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// pseudo-random value in [-1, 1) from (salt, row, column): splitmix64
__device__ __forceinline__ double hash_unit(unsigned long long salt, int i, int a)
{
    unsigned long long z = salt * 0x9E3779B97F4A7C15ull + ((unsigned long long)i << 32) +
                           (unsigned long long)a + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

constexpr int OT = 1024;     // threads of the orthonormalisation workgroup
constexpr int OW = OT / 64;  // its waves
constexpr int OJ = 16;       // earlier rows per pass over the row

// block-wide sum of one value per thread (every thread gets the result)
__device__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < OW; ++w)
        s += red[w];
    return s;
}

// Rows b0 .. b0+bk-1 of X, already projected against the rows before b0:
// two-pass classical Gram-Schmidt within the block.  A row left with less
// than 1e-10 of its reference norm (nrm_pre, squared: before any projection,
// or after the first Cholesky pass where the second flagged the block) lies
// in the span of the rows before it: it is refilled with pseudo-random values
// and orthogonalised against every earlier row of X.
__global__ __launch_bounds__(OT) void orth_block_kernel(double *__restrict__ X, int b0, int bk,
                                                        int n,
                                                        const double *__restrict__ nrm_pre,
                                                        const int *__restrict__ flag,
                                                        unsigned long long salt)
{
    __shared__ double red[OW][OJ + 1];
    __shared__ double dots[kTuckerMaxSub];
    if (*flag == 0)
        return;  // the Cholesky passes have orthonormalised the block
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int il = 0; il < bk; ++il) {
        const int i = b0 + il;
        double *xi = X + (long)i * n;
        double ref = nrm_pre[il];
        int jlo = b0;  // earlier rows still to project against
        for (int attempt = 0; attempt < 3; ++attempt) {
            for (int pass = 0; pass < 2; ++pass) {
                for (int j0 = jlo; j0 < i; j0 += OJ) {
                    const int jc = min(OJ, i - j0);
                    double acc[OJ];
#pragma unroll
                    for (int jj = 0; jj < OJ; ++jj)
                        acc[jj] = 0.0;
                    for (int a = tid; a < n; a += OT) {
                        const double v = xi[a];
#pragma unroll
                        for (int jj = 0; jj < OJ; ++jj)
                            if (jj < jc)
                                acc[jj] += X[(long)(j0 + jj) * n + a] * v;
                    }
                    __syncthreads();
#pragma unroll
                    for (int jj = 0; jj < OJ; ++jj) {
                        const double v = wave_sum(acc[jj]);
                        if (lane == 0)
                            red[wave][jj] = v;
                    }
                    __syncthreads();
                    if (tid < jc) {
                        double sum = 0.0;
                        for (int w = 0; w < OW; ++w)
                            sum += red[w][tid];
                        dots[j0 - jlo + tid] = sum;
                    }
                }
                __syncthreads();
                for (int a = tid; a < n; a += OT) {
                    double v = xi[a];
                    for (int j = jlo; j < i; ++j)
                        v -= dots[j - jlo] * X[(long)j * n + a];
                    xi[a] = v;
                }
                __syncthreads();
            }
            double ss = 0.0;
            for (int a = tid; a < n; a += OT)
                ss += xi[a] * xi[a];
            const double nrm = block_sum(ss, &red[0][0]);
            if ((nrm > 1e-20 * ref && nrm > 0.0) || attempt == 2) {
                const double sc = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
                for (int a = tid; a < n; a += OT)
                    xi[a] *= sc;
                __syncthreads();
                break;
            }
            // numerically in the span of the earlier rows: a fresh row,
            // projected against all of them
            ss = 0.0;
            for (int a = tid; a < n; a += OT) {
                const double v = hash_unit(salt + 7919ull * (attempt + 1), i, a);
                xi[a] = v;
                ss += v * v;
            }
            ref = block_sum(ss, &red[0][0]);
            jlo = 0;
        }
    }
}

// 1 / d for a positive normal d: the hardware reciprocal estimate refined by
// two Newton-Raphson steps r <- r + r (1 - d r), each of which squares the
// relative error (a shorter dependent chain than the IEEE division, whose
// scaling and fix-up steps only matter near the range limits)
__device__ inline double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// value of v in lane l (l uniform across the wave)
__device__ inline double lane_value(double v, int l)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)bits, l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Cholesky factor of the Gram W [k][k] of the k <= kOrthRows rows being
// orthonormalised (W = X X^T, symmetrised on load), right-looking and blocked
// by 16 columns.  Four waves: lane i holds row i, wave w its columns
// 16w .. 16w + 15, in registers.  For each panel the owning wave factors its
// 16 columns alone, column by column, broadcasting each column to its lanes
// through LDS (within one wave, no barrier); it publishes the
// finished columns to LDS, unscaled and scaled by the pivot's reciprocal, with
// the entries above the diagonal as zeros, and after one barrier every later
// wave applies the panel's 16 column steps A[i][c] -= (A[i][j] / A[j][j]) A[c][j]
// to its own columns, in column order.
// The zeros leave finished entries unchanged; entries above the diagonal take
// meaningless values but are never published or stored.
// First pass: nrm takes the squared row norms (the diagonal of W), the
// reference of the Gram-Schmidt fallback; flag = 1 when a pivot keeps less
// than 1e-11 of its row's squared norm (a row within about 3e-6 of the span of
// the rows before it).  Above that limit the row-scaled matrix has a
// condition number below about 3e5, inside the range (about 1e6 for 64 rows
// of 65536 entries) where CholeskyQR2 returns rows orthonormal to working
// precision (Yamamoto, Nakatsukasa, Yanagisawa and Fukaya 2015; the
// factorisation and the substitution are invariant to row scaling).  Second
// pass: runs only where the first did not flag; its rows are then orthonormal
// to within a few percent, so a pivot below half its row's squared norm means
// the first pass lost more than the bound allows: the rows are flagged, and
// nrm takes their squared norms.
// Lt [k][k]: L transposed (Lt[c][i] = L[i][c] for i > c), 1 / L[c][c] on the
// diagonal, zeros below it.
constexpr int CW = 16;                     // columns per wave (one panel)
constexpr int CT = 64 * (kOrthRows / CW);  // threads
static_assert(kOrthRows == 64, "one row per lane");
__global__ __launch_bounds__(CT) void chol_gram_kernel(const double *__restrict__ W, int k,
                                                       double *__restrict__ nrm, int second,
                                                       int *__restrict__ flag,
                                                       double *__restrict__ Lt)
{
    __shared__ double pf[2][CW][kOrthRows];  // A[i][j] / A[j][j] (zero for i < j)
    __shared__ double pv[2][CW][kOrthRows];  // A[i][j] (zero for i < j)
    __shared__ double d0[kOrthRows];
    __shared__ double piv[kOrthRows];
    __shared__ double pc[kOrthRows];  // the panel owner's current column
    __shared__ int sbad;
    const int tid = threadIdx.x;
    const int i = tid & 63, wave = tid >> 6, c0 = wave * CW;
    if (second && *flag)
        return;
    const bool row = i < k;
    // every load in bounds (indices clamped to k - 1), all issued before the
    // first use
    const int ic = min(i, k - 1);
    double wa[CW], wb[CW];
#pragma unroll
    for (int m = 0; m < CW; ++m) {
        const int cc = min(c0 + m, k - 1);
        wa[m] = W[ic * k + cc];
        wb[m] = W[cc * k + ic];
    }
    const double dr = W[ic * k + ic];  // row i's squared norm (lane i)
    double a[CW], lf[CW];
#pragma unroll
    for (int m = 0; m < CW; ++m) {
        a[m] = row && c0 + m < k ? 0.5 * (wa[m] + wb[m]) : 0.0;
        lf[m] = 0.0;
    }
    if (tid < k)
        d0[tid] = dr;
    if (tid == 0)
        sbad = 0;
    int bad = 0;
    for (int pb = 0; pb * CW < k; ++pb) {
        const int buf = pb & 1;
        if (wave == pb) {
            int wbad = 0;
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) {
                const int j = pb * CW + jj;
                if (j < k && !wbad) {
                    // the column through LDS (one wave: its LDS accesses
                    // complete in order, no barrier needed)
                    pc[i] = a[jj];
                    const double d = pc[j];
                    double v[CW];
#pragma unroll
                    for (int m = 0; m < CW; ++m)
                        v[m] = pc[c0 + m];
                    const double dj = lane_value(dr, j);
                    const double lim = second ? 0.5 * dj : 1e-11 * dj;
                    if (!(d > lim) || !(d > 0.0)) {
                        wbad = 1;
                    } else {
                        if (i == 0)
                            piv[j] = d;
                        const double rd = recip(d);
                        lf[jj] = a[jj];
                        const double f = i >= j ? a[jj] * rd : 0.0;
                        pf[buf][jj][i] = f;
                        pv[buf][jj][i] = i >= j ? a[jj] : 0.0;
#pragma unroll
                        for (int m = jj + 1; m < CW; ++m)
                            a[m] = fma(-f, v[m], a[m]);
                    }
                }
            }
            if (i == 0 && wbad)
                sbad = 1;
        }
        __syncthreads();
        if (sbad) {
            bad = 1;
            break;
        }
        if (wave > pb) {
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) {
                const int j = pb * CW + jj;
                if (j < k) {
                    const double f = pf[buf][jj][i];
                    double v[CW];
#pragma unroll
                    for (int m = 0; m < CW; ++m)
                        v[m] = pv[buf][jj][c0 + m];
#pragma unroll
                    for (int m = 0; m < CW; ++m)
                        a[m] = fma(-f, v[m], a[m]);
                }
            }
        }
    }
    if (tid == 0 && (!second || bad))
        *flag = bad;  // a failed second pass also hands the rows to the fallback
    if ((!second || bad) && tid < k)
        nrm[tid] = d0[tid];
    if (bad || !row)
        return;
#pragma unroll
    for (int m = 0; m < CW; ++m) {
        const int c = c0 + m;
        if (c < k)
            Lt[c * k + i] = c < i ? lf[m] / sqrt(piv[c]) : c == i ? 1.0 / sqrt(piv[c]) : 0.0;
    }
}

// X <- L^{-1} X by forward substitution, one thread per column (skipped when
// flagged); Lt as chol_gram_kernel writes it, staged in LDS.  Right-looking:
// once x_j is final every later row takes its term at once, so the dependent
// chain is two operations per row.  KB: k rounded up to a multiple of 16 (the
// rows beyond k read clamped, in-bounds entries and are never stored).  Each
// step sits behind its own (uniform) test against k, so that the reads of L
// are not all hoisted at once (which would hold the whole factor in
// registers); instead each step reads the next column while it computes.
constexpr int AT = 64;
template <int KB>
__global__ __launch_bounds__(AT) void apply_linv_kernel(double *__restrict__ X, int k, int n,
                                                        const double *__restrict__ Lt,
                                                        const int *__restrict__ flag)
{
    __shared__ double Ls[KB * KB];
    if (*flag)
        return;
    static_assert(KB * KB % AT == 0, "whole staging rounds");
    constexpr int SQ = KB * KB / AT;
    double sv[SQ];
#pragma unroll
    for (int q = 0; q < SQ; ++q) {  // every load issued before the first store
        const int e = threadIdx.x + AT * q;
        sv[q] = Lt[min(e / KB, k - 1) * k + min(e % KB, k - 1)];
    }
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
        const int e = threadIdx.x + AT * q;
        Ls[e] = e / KB < k && e % KB < k ? sv[q] : 0.0;
    }
    __syncthreads();
    const int a = blockIdx.x * AT + threadIdx.x;
    if (a >= n)
        return;
    double x[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i)
        x[i] = X[(long)min(i, k - 1) * n + a];
    // column j of L in registers, the next one read while step j computes
    double lc[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i)
        lc[i] = Ls[i];
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        if (j < k) {
            double ln[KB];
#pragma unroll
            for (int i = j + 1; i < KB; ++i)
                ln[i] = j + 1 < KB ? Ls[(j + 1) * KB + i] : 0.0;
            x[j] *= lc[j];
#pragma unroll
            for (int i = j + 1; i < KB; ++i)
                x[i] = fma(-lc[i], x[j], x[i]);
#pragma unroll
            for (int i = j + 1; i < KB; ++i)
                lc[i] = ln[i];
        }
    }
#pragma unroll
    for (int i = 0; i < KB; ++i)
        if (i < k)
            X[(long)i * n + a] = x[i];
}

__global__ __launch_bounds__(256) void zero_rows_kernel(double *__restrict__ X, int i0, int k,
                                                        int n)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e < (long)(k - i0) * n)
        X[(long)i0 * n + e] = 0.0;
}

__global__ __launch_bounds__(256) void random_rows_kernel(double *__restrict__ X, int i0, int k,
                                                          int n, unsigned long long salt)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    const long count = (long)(k - i0) * n;
    if (e >= count)
        return;
    const int i = i0 + (int)(e / n), a = (int)(e % n);
    X[(long)i * n + a] = hash_unit(salt, i, a);
}

// 1 / sqrt(x) for a positive normal x: the hardware estimate refined by two
// Newton-Raphson steps r <- r (3 - x r^2) / 2
__device__ inline double rsqrt_nr(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    r = r * fma(-0.5 * x, r * r, 1.5);
    return r * fma(-0.5 * x, r * r, 1.5);
}

// Cyclic Jacobi on the symmetric H [k][k] in LDS.  Each round-robin round
// rotates k/2 disjoint pairs (p, q); since the pairs partition the indices,
// the 2 x 2 blocks (rows of one pair, columns of another) partition H, and
// each block becomes R1 B R2^T in one pass, one thread per block, with
// R = [[c, -s], [s, c]] (the identity for a pair that is not rotated); the
// columns of V take the same rotations in that pass.  A round in which no
// pair rotates (all of the last, confirming sweep) skips that pass and its
// barrier.
constexpr int JT = 1024;

__global__ __launch_bounds__(JT) void jacobi_eig_kernel(const double *__restrict__ Hin, int k,
                                                        double *__restrict__ lam,
                                                        double *__restrict__ Vt)
{
    __shared__ double H[kTuckerMaxSub][kTuckerMaxSub + 1];
    __shared__ double V[kTuckerMaxSub][kTuckerMaxSub + 1];
    __shared__ double cs[kTuckerMaxSub / 2], sn[kTuckerMaxSub / 2];
    __shared__ int pp[kTuckerMaxSub / 2], qq[kTuckerMaxSub / 2];
    __shared__ int rotated, live[2];
    const int tid = threadIdx.x;
    const int kk = k + (k & 1);  // an odd k gets one padding index, never rotated
    const int half = kk / 2;
    for (int e = tid; e < kk * kk; e += JT) {
        const int i = e / kk, j = e % kk;
        H[i][j] = i < k && j < k ? 0.5 * (Hin[(long)i * k + j] + Hin[(long)j * k + i]) : 0.0;
        V[i][j] = i == j ? 1.0 : 0.0;
    }
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (tid == 0) {
            rotated = 0;
            live[0] = 0;  // round 0's flag (the previous sweep ended with a barrier)
        }
        __syncthreads();
        for (int rnd = 0; rnd < kk - 1; ++rnd) {
            if (tid < half) {
                // round-robin pairing: position 0 fixed, the rest rotate
                const int m1 = tid, m2 = kk - 1 - tid;
                int p = m1 == 0 ? 0 : 1 + (m1 - 1 + rnd) % (kk - 1);
                int q = 1 + (m2 - 1 + rnd) % (kk - 1);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, sv = 0.0;
                if (q < k) {
                    const double hpq = H[p][q], hpp = H[p][p], hqq = H[q][q];
                    // |h_pq| > 1e-17 sqrt(|h_pp h_qq|), squared
                    if (hpq != 0.0 && hpq * hpq > 1e-34 * fabs(hpp * hqq)) {
                        const double th = (hqq - hpp) * recip(2.0 * hpq);
                        const double u = fma(th, th, 1.0);
                        const double t =
                            th != 0.0 ? copysign(recip(fabs(th) + u * rsqrt_nr(u)), th) : 1.0;
                        c = rsqrt_nr(fma(t, t, 1.0));
                        sv = t * c;
                        rotated = 1;
                        live[rnd & 1] = 1;
                    }
                }
                pp[tid] = p;
                qq[tid] = q;
                cs[tid] = c;
                sn[tid] = sv;
            }
            if (tid == JT - 1)
                live[(rnd + 1) & 1] = 0;  // the next round's flag (read two barriers ago)
            __syncthreads();
            if (live[rnd & 1]) {
                for (int e = tid; e < half * half; e += JT) {
                    const int r1 = e / half, r2 = e % half;
                    const int p1 = pp[r1], q1 = qq[r1], p2 = pp[r2], q2 = qq[r2];
                    const double c1 = cs[r1], s1 = sn[r1], c2 = cs[r2], s2 = sn[r2];
                    const double h00 = H[p1][p2], h01 = H[p1][q2], h10 = H[q1][p2],
                                 h11 = H[q1][q2];
                    // rows: R1 B
                    const double a00 = c1 * h00 - s1 * h10, a01 = c1 * h01 - s1 * h11;
                    const double a10 = s1 * h00 + c1 * h10, a11 = s1 * h01 + c1 * h11;
                    // columns: (R1 B) R2^T
                    H[p1][p2] = c2 * a00 - s2 * a01;
                    H[p1][q2] = s2 * a00 + c2 * a01;
                    H[q1][p2] = c2 * a10 - s2 * a11;
                    H[q1][q2] = s2 * a10 + c2 * a11;
                }
                for (int e = tid; e < half * kk; e += JT) {
                    const int r = e / kk, row = e % kk;
                    const int p = pp[r], q = qq[r];
                    const double c = cs[r], sv = sn[r];
                    const double vp = V[row][p], vq = V[row][q];
                    V[row][p] = c * vp - sv * vq;
                    V[row][q] = sv * vp + c * vq;
                }
                __syncthreads();
            }
        }
        if (!rotated)
            break;
        __syncthreads();
    }
    // decreasing order: the rank of eigenvalue i among all (ties by index)
    if (tid < k) {
        const double li = H[tid][tid];
        int rank = 0;
        for (int j = 0; j < k; ++j) {
            const double lj = H[j][j];
            rank += (lj > li) || (lj == li && j < tid);
        }
        lam[rank] = li;
        for (int j = 0; j < k; ++j)
            Vt[(long)rank * k + j] = V[j][tid];
    }
}

__global__ __launch_bounds__(256) void khatri_rao_kernel(const double *__restrict__ c,
                                                         const double *__restrict__ Ua,
                                                         const double *__restrict__ Ub, int ra,
                                                         int rb, int R, double *__restrict__ K)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    const long count = (long)ra * rb * R;
    if (e >= count)
        return;
    const int t = (int)(e % R);
    const long ij = e / R;
    const int i = (int)(ij / rb), j = (int)(ij % rb);
    K[e] = c[t] * Ua[(long)i * R + t] * Ub[(long)j * R + t];
}

__global__ __launch_bounds__(256) void sign_rows_kernel(double *__restrict__ Z, int n,
                                                        const double *__restrict__ lam,
                                                        double *__restrict__ sv, int r)
{
    __shared__ double bv[256];
    __shared__ int bi[256];
    const int i = blockIdx.x, tid = threadIdx.x;
    double *z = Z + (long)i * n;
    double best = -1.0;
    int idx = n;
    for (int a = tid; a < n; a += 256) {
        const double v = fabs(z[a]);
        if (v > best) {
            best = v;
            idx = a;
        }
    }
    bv[tid] = best;
    bi[tid] = idx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            const double v2 = bv[tid + w];
            const int i2 = bi[tid + w];
            if (v2 > bv[tid] || (v2 == bv[tid] && i2 < bi[tid])) {
                bv[tid] = v2;
                bi[tid] = i2;
            }
        }
        __syncthreads();
    }
    const double sg = (bi[0] < n && z[bi[0]] < 0.0) ? -1.0 : 1.0;
    __syncthreads();
    if (sg < 0.0)
        for (int a = tid; a < n; a += 256)
            z[a] = -z[a];
    if (tid == 0 && sv)
        sv[i] = sqrt(fmax(lam[i], 0.0));
}

}  // namespace

int gemm_splits(int I, int N, int K)
{
    const long tiles = (long)((I + GT - 1) / GT) * ((N + GT - 1) / GT);
    int S = (int)((512 + tiles - 1) / tiles);
    const int kmax = (K + 63) / 64;
    S = std::min(S, std::min(kGemmMaxSplit, kmax));
    return std::max(S, 1);
}

hipError_t launch_gemm_f64(bool nn, const double *A, const double *B, double *C, int I, int N,
                           int K, double *part, hipStream_t st, bool sub)
{
    const int S = part ? gemm_splits(I, N, K) : 1;
    int kchunk = (K + S - 1) / S;
    kchunk = (kchunk + GK - 1) / GK * GK;
    const int Sused = (K + kchunk - 1) / kchunk > 0 ? (K + kchunk - 1) / kchunk : 1;
    dim3 grid((N + GT - 1) / GT, (I + GT - 1) / GT, Sused);
    double *out = Sused > 1 ? part : C;
    const int sub_here = Sused > 1 ? 0 : (int)sub;
    if (nn)
        hipLaunchKernelGGL(gemm_f64_kernel<true>, grid, dim3(256), 0, st, A, B, out, I, N, K,
                           kchunk, sub_here);
    else
        hipLaunchKernelGGL(gemm_f64_kernel<false>, grid, dim3(256), 0, st, A, B, out, I, N, K,
                           kchunk, sub_here);
    if (Sused > 1) {
        const long count = (long)I * N;
        hipLaunchKernelGGL(split_sum_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256),
                           0, st, part, C, count, Sused, (int)sub);
    }
    return hipGetLastError();
}

hipError_t launch_orth_rows(double *X, int k, int n, int passes, double *D, double *nrm,
                            double *Linv, int *flag, double *part, unsigned long long salt,
                            hipStream_t st)
{
    if (k < 1 || k > kOrthRows || k > n || passes < 1 || passes > 2)
        return hipErrorInvalidValue;
    for (int pass = 0; pass < passes; ++pass) {
        // W = X X^T on matrix cores, its Cholesky factor, X <- L^{-1} X
        hipError_t e = launch_gemm_f64(false, X, X, D, k, k, n, part, st, false);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(chol_gram_kernel, dim3(1), dim3(CT), 0, st, D, k, nrm, pass, flag,
                           Linv);
        const dim3 grid((n + AT - 1) / AT);
        if (k <= 16)
            hipLaunchKernelGGL(apply_linv_kernel<16>, grid, dim3(AT), 0, st, X, k, n, Linv, flag);
        else if (k <= 32)
            hipLaunchKernelGGL(apply_linv_kernel<32>, grid, dim3(AT), 0, st, X, k, n, Linv, flag);
        else if (k <= 48)
            hipLaunchKernelGGL(apply_linv_kernel<48>, grid, dim3(AT), 0, st, X, k, n, Linv, flag);
        else
            hipLaunchKernelGGL(apply_linv_kernel<64>, grid, dim3(AT), 0, st, X, k, n, Linv, flag);
    }
    hipLaunchKernelGGL(orth_block_kernel, dim3(1), dim3(OT), 0, st, X, 0, k, n, nrm, flag, salt);
    return hipGetLastError();
}

hipError_t launch_random_rows(double *X, int i0, int k, int n, unsigned long long salt,
                              hipStream_t st)
{
    const long count = (long)(k - i0) * n;
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(random_rows_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                       st, X, i0, k, n, salt);
    return hipGetLastError();
}

hipError_t launch_zero_rows(double *X, int i0, int k, int n, hipStream_t st)
{
    const long count = (long)(k - i0) * n;
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                       X, i0, k, n);
    return hipGetLastError();
}

hipError_t launch_jacobi_eig(const double *H, int k, double *lam, double *Vt, hipStream_t st)
{
    hipLaunchKernelGGL(jacobi_eig_kernel, dim3(1), dim3(JT), 0, st, H, k, lam, Vt);
    return hipGetLastError();
}

hipError_t launch_khatri_rao(const double *c, const double *Ua, const double *Ub, int ra, int rb,
                             int R, double *K, hipStream_t st)
{
    const long count = (long)ra * rb * R;
    hipLaunchKernelGGL(khatri_rao_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                       st, c, Ua, Ub, ra, rb, R, K);
    return hipGetLastError();
}

hipError_t launch_sign_rows(double *Z, int r, int n, const double *lam, double *sv,
                            hipStream_t st)
{
    hipLaunchKernelGGL(sign_rows_kernel, dim3(r), dim3(256), 0, st, Z, n, lam, sv, r);
    return hipGetLastError();
}

}  // namespace tc
