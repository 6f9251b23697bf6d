// 1D density fitting of a side matrix and the pivoted Cholesky of the
// factorised TEI matrix (Section 3.2), binary64.
//
// Both run the diagonally pivoted Cholesky of a positive semi-definite
// matrix A (N x N) that is never formed: its diagonal and, per step, the
// column at the pivot come from the factors.
//   fit:  A = F^T F over the n grid points of one mode, F [N_pair][n]
//         (rows: products of basis functions);
//   TEI:  A = B = sum_k c_k o_l V^l M^l_k V^l^T over the N_pair products.
// A step r with pivot p: col = A[:, p] - sum_{s<r} L_s L_s[p];
// L_r = col / sqrt(d[p]), zero on the earlier pivots; d -= L_r^2, d[p] = 0;
// then the next pivot is the first index of the largest residual diagonal
// entry, and the residual trace decides whether to go on.  L is stored by
// columns: L [R_max][N], row r = column r of the factor.  The stopping test
// runs on the device (a `done` flag that turns the later kernels into no-ops),
// so the host enqueues several steps between synchronisations.
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int CT = 256;  // threads of the elementwise kernels

// d[a] = sum_i F[i][a]^2
__global__ __launch_bounds__(CT) void fit_diag_kernel(const double *__restrict__ F, int n,
                                                      int N_pair, double *__restrict__ d)
{
    const int a = blockIdx.x * CT + threadIdx.x;
    if (a >= n)
        return;
    double s = 0.0;
    for (int i = 0; i < N_pair; ++i) {
        const double f = F[(long)i * n + a];
        s = fma(f, f, s);
    }
    d[a] = s;
}

// col[a] = sum_i F[i][a] F[i][p]  (p read from the device state), rows split
// into kFitSplit contiguous chunks (blockIdx.y); part[z][a] the chunk sums
constexpr int kFitSplit = 16;

__global__ __launch_bounds__(CT) void fit_column_kernel(const double *__restrict__ F, int n,
                                                        int N_pair,
                                                        const int *__restrict__ state,
                                                        double *__restrict__ part)
{
    const int a = blockIdx.x * CT + threadIdx.x;
    if (a >= n || state[1])
        return;
    const int p = state[0];
    const int z = blockIdx.y;
    const int ib = (int)((long)z * N_pair / kFitSplit), ie = (int)((long)(z + 1) * N_pair / kFitSplit);
    double s = 0.0;
    for (int i = ib; i < ie; ++i)
        s = fma(F[(long)i * n + a], F[(long)i * n + p], s);
    part[(long)z * n + a] = s;
}

__global__ __launch_bounds__(CT) void fit_column_reduce(const double *__restrict__ part, int n,
                                                        const int *__restrict__ state,
                                                        double *__restrict__ col)
{
    const int a = blockIdx.x * CT + threadIdx.x;
    if (a >= n || state[1])
        return;
    double s = 0.0;
    for (int z = 0; z < kFitSplit; ++z)
        s += part[(long)z * n + a];
    col[a] = s;
}

// step r: L_r = (col - sum_{s<r} L_s L_s[p]) / sqrt(d[p]), zero on the
// earlier pivots; d -= L_r^2; d[p] = 0
// One step: column r of L at every index a, with the sum over the earlier
// columns split over 16 waves (64 indices per workgroup) and added in a fixed
// order; the earlier pivots (ispiv) get zero; the residual diagonal drops by
// l^2 except at the pivot itself.
constexpr int kStepA = 64;
constexpr int kStepG = 16;

__global__ __launch_bounds__(kStepA * kStepG) void chol_step_kernel(
    const double *__restrict__ col, const double *__restrict__ A, double *__restrict__ L, int N,
    int r, const int *__restrict__ ispiv, const int *__restrict__ state, double *__restrict__ d)
{
    __shared__ double red[kStepG][kStepA + 1];
    if (state[1])
        return;
    const int al = threadIdx.x & (kStepA - 1), g = threadIdx.x / kStepA;
    const int a = blockIdx.x * kStepA + al;
    const int p = state[0];
    double sum = 0.0;
    if (a < N)
        for (int q = g; q < r; q += kStepG)
            sum = fma(L[(long)q * N + a], L[(long)q * N + p], sum);
    red[g][al] = sum;
    __syncthreads();
    if (g == 0 && a < N) {
        // the pivot's column of A: from the formed matrix (symmetric, so its
        // row p), or as computed by the column kernels
        double v = A ? A[(long)p * N + a] : col[a];
        for (int h = 0; h < kStepG; ++h)
            v -= red[h][al];
        double l = v / sqrt(d[p]);
        if (ispiv[a] && a != p)
            l = 0.0;
        L[(long)r * N + a] = l;
        // every thread reads d[p], so the pivot's own entry is cleared by the
        // next kernel (chol_select), not here
        if (a != p)
            d[a] -= l * l;
    }
}

// One step on a formed matrix, with the selection of its pivot in the same
// launch.  Every workgroup scans the residual diagonal d_in (the previous
// step's output, earlier pivots already zero) with chol_select's loop and
// reduction order, so each finds the same pivot, trace and stopping decision
// without communicating; workgroup 0 records them (state, stats, piv, ispiv).
// Unless the factorisation is done, each workgroup then forms its kStepA
// entries of L_r as chol_step does and writes the next residual diagonal to
// d_out (the pivot's entry zero), so no workgroup reads an entry that another
// is updating.  The steps alternate the two diagonal buffers.
__global__ __launch_bounds__(kStepA * kStepG) void chol_select_step_kernel(
    const double *__restrict__ A, double *__restrict__ L, int N, int r, int *__restrict__ ispiv,
    int *__restrict__ state, const double *__restrict__ d_in, double *__restrict__ d_out,
    double thr, int R_max, double *__restrict__ stats, int *__restrict__ piv)
{
    constexpr int TT = kStepA * kStepG;
    static_assert(TT == 1024, "chol_select's reduction order");
    __shared__ double smax[TT], ssum[TT];
    __shared__ int sidx[TT];
    __shared__ double red[kStepG][kStepA + 1];
    if (state[1])
        return;
    const int tid = threadIdx.x;
    {
        double m = -1.0, sm = 0.0;
        int idx = 0x7fffffff;
        for (int a = tid; a < N; a += TT) {
            const double v = d_in[a];
            sm += v;
            if (v > m) {
                m = v;
                idx = a;
            }
        }
        smax[tid] = m;
        ssum[tid] = sm;
        sidx[tid] = idx;
    }
    __syncthreads();
    for (int w = TT / 2; w > 0; w >>= 1) {
        if (tid < w) {
            const double m2 = smax[tid + w];
            const int i2 = sidx[tid + w];
            if (m2 > smax[tid] || (m2 == smax[tid] && i2 < sidx[tid])) {
                smax[tid] = m2;
                sidx[tid] = i2;
            }
            ssum[tid] += ssum[tid + w];
        }
        __syncthreads();
    }
    const double mx = smax[0], tr = ssum[0];
    const int p = sidx[0];
    const bool done = r >= R_max || !(tr > thr) || !(mx > 0.0);
    if (blockIdx.x == 0 && tid == 0) {
        stats[0] = mx;
        stats[1] = tr;
        if (done) {
            state[1] = 1;
            state[2] = r;
        } else {
            state[0] = p;
            piv[r] = p;
            ispiv[p] = 1;  // read below only at a != p
        }
    }
    if (done)
        return;
    const int al = tid & (kStepA - 1), g = tid / kStepA;
    const int a = blockIdx.x * kStepA + al;
    double sum = 0.0;
    if (a < N)
        for (int q = g; q < r; q += kStepG)
            sum = fma(L[(long)q * N + a], L[(long)q * N + p], sum);
    red[g][al] = sum;
    __syncthreads();
    if (g == 0 && a < N) {
        double v = A[(long)p * N + a];
        for (int h = 0; h < kStepG; ++h)
            v -= red[h][al];
        double l = v / sqrt(d_in[p]);
        if (a != p && ispiv[a])
            l = 0.0;
        L[(long)r * N + a] = l;
        d_out[a] = a == p ? 0.0 : d_in[a] - l * l;
    }
}

// The largest residual diagonal entry (first index among equals) and the
// residual trace; one workgroup.  state = {pivot, done, steps}, stats = {max,
// trace}.  Nothing happens once done is set.  `clear`: the last pivot's entry
// is set to zero first; `steps`: the steps completed so far.  The process is
// done when steps >= R_max, the trace is at most thr or the maximum is not
// positive; otherwise the maximum's index is the next pivot.
__global__ __launch_bounds__(1024) void chol_select_kernel(double *__restrict__ d, int N,
                                                           int clear, int steps, double thr,
                                                           int R_max, int *__restrict__ state,
                                                           double *__restrict__ stats,
                                                           int *__restrict__ piv,
                                                           int *__restrict__ ispiv)
{
    __shared__ double smax[1024], ssum[1024];
    __shared__ int sidx[1024];
    const int tid = threadIdx.x;
    if (state[1])
        return;
    if (clear) {
        const int p = state[0];
        if (tid == 0)
            d[p] = 0.0;
        __syncthreads();
    }
    double m = -1.0, s = 0.0;
    int idx = 0x7fffffff;
    for (int a = tid; a < N; a += 1024) {
        const double v = d[a];
        s += v;
        if (v > m) {
            m = v;
            idx = a;
        }
    }
    smax[tid] = m;
    ssum[tid] = s;
    sidx[tid] = idx;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) {
            const double m2 = smax[tid + w];
            const int i2 = sidx[tid + w];
            if (m2 > smax[tid] || (m2 == smax[tid] && i2 < sidx[tid])) {
                smax[tid] = m2;
                sidx[tid] = i2;
            }
            ssum[tid] += ssum[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        stats[0] = smax[0];
        stats[1] = ssum[0];
        if (steps >= R_max || !(ssum[0] > thr) || !(smax[0] > 0.0)) {
            state[1] = 1;
            state[2] = steps;
        } else {
            // the next pivot, recorded as step `steps`
            state[0] = sidx[0];
            piv[steps] = sidx[0];
            ispiv[sidx[0]] = 1;
        }
    }
}

__global__ void fill_int_kernel(int *__restrict__ x, int count, int value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        x[i] = value;
}

// fit result: T[r][s] = L_s[P[r]] is lower triangular (pivot order); for each
// grid point a solve T^T u_a = (L_0[a], ..., L_{R-1}[a]) by back substitution
// and store U[s][a] = u_a[s] (rows s >= R of U zero).  fit_t gathers T into
// Tg[s][r] first, so that the substitution reads it at addresses common to
// the whole wave; one thread per grid point, 64 per workgroup.
__global__ __launch_bounds__(CT) void fit_t_kernel(const double *__restrict__ L, int n, int R,
                                                   const int *__restrict__ piv,
                                                   double *__restrict__ Tg)
{
    const long e = (long)blockIdx.x * CT + threadIdx.x;
    if (e >= (long)R * R)
        return;
    const int s = (int)(e / R), r = (int)(e % R);
    Tg[e] = L[(long)s * n + piv[r]];
}

constexpr int kFitUThreads = 64;

__global__ __launch_bounds__(kFitUThreads) void fit_u_kernel(const double *__restrict__ L, int n,
                                                             int R, int R_max,
                                                             const double *__restrict__ Tg,
                                                             double *__restrict__ U)
{
    const int a = blockIdx.x * kFitUThreads + threadIdx.x;
    if (a >= n)
        return;
    for (int s = R - 1; s >= 0; --s) {
        const double *ts = Tg + (long)s * R;
        double v = L[(long)s * n + a];
        for (int r = s + 1; r < R; ++r)
            v -= ts[r] * U[(long)r * n + a];  // T[r][s] u[r]
        U[(long)s * n + a] = v / ts[s];       // T[s][s]
    }
    for (int s = R; s < R_max; ++s)
        U[(long)s * n + a] = 0.0;
}

// The same solve, blocked by eight unknowns, for R <= kFitMaxR: the solved
// entries of the workgroup's 64 columns stay in LDS (ush[r][lane]), and so do
// the rows of T that a block needs (Tsh[r][q] = T[r][top - q], eight
// contiguous values per r).  For a block s = top - 7 .. top, each of four
// waves sums T[r][s] u_r over its share of the rows solved before the block
// (r > top), every u_r read once for eight products; after one barrier wave
// 0 adds the four partial sums in fixed order and solves the 8 x 8 triangle
// in registers.  The next block's rows of T and of L are loaded into
// registers while the current block is solved.  (fit_u_kernel above
// re-reads every solved entry from global memory in its inner loop.)
constexpr int kFitMaxR = 240;
constexpr int kFitBlk = 8;
constexpr int kFitW = 4;                 // waves
constexpr int kFitT = 64 * kFitW;        // threads
constexpr int kFitTQ = (kFitMaxR * kFitBlk + kFitT - 1) / kFitT;  // staged T entries per thread

__global__ __launch_bounds__(kFitT) void fit_u_blk_kernel(const double *__restrict__ L, int n,
                                                          int R, int R_max,
                                                          const double *__restrict__ Tg,
                                                          double *__restrict__ U)
{
    __shared__ double ush[kFitMaxR][64];
    __shared__ __align__(16) double Tsh[kFitMaxR][kFitBlk];
    __shared__ double red[kFitW][kFitBlk][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int a = blockIdx.x * 64 + lane;
    const int ac = min(a, n - 1);  // loads stay in bounds; results of a >= n are not stored
    // rows top, top - 1, ..., top - 7 of L (zero below row 0)
    auto load_l = [&](int top, double(&dst)[kFitBlk]) {
#pragma unroll
        for (int q = 0; q < kFitBlk; ++q) {
            const int sr = top - q;
            dst[q] = sr >= 0 ? L[(long)sr * n + ac] : 0.0;
        }
    };
    // T[r][top - q] for r < R (Tg[s][r] = T[r][s]), entry e = r * 8 + q
    auto load_t = [&](int top, double(&dst)[kFitTQ]) {
#pragma unroll
        for (int e = 0; e < kFitTQ; ++e) {
            const int idx = tid + kFitT * e;
            const int r = idx / kFitBlk, q = idx % kFitBlk;
            const int sr = top - q;
            dst[e] = idx < kFitMaxR * kFitBlk && r < R && sr >= 0 ? Tg[(long)sr * R + r] : 0.0;
        }
    };
    double lcur[kFitBlk], lnxt[kFitBlk], tnxt[kFitTQ];
    load_l(R - 1, lnxt);
    load_t(R - 1, tnxt);
    for (int top = R - 1; top >= 0; top -= kFitBlk) {
        __syncthreads();  // the previous block's solved entries are stored, its T no longer read
#pragma unroll
        for (int e = 0; e < kFitTQ; ++e) {
            const int idx = tid + kFitT * e;
            if (idx < kFitMaxR * kFitBlk)
                Tsh[idx / kFitBlk][idx % kFitBlk] = tnxt[e];
        }
#pragma unroll
        for (int q = 0; q < kFitBlk; ++q)
            lcur[q] = lnxt[q];
        __syncthreads();
        if (top - kFitBlk >= 0) {
            load_l(top - kFitBlk, lnxt);
            load_t(top - kFitBlk, tnxt);
        }
        // this wave's share of the rows solved before the block
        double acc[kFitBlk];
#pragma unroll
        for (int q = 0; q < kFitBlk; ++q)
            acc[q] = 0.0;
        for (int r = top + 1 + w; r < R; r += kFitW) {
            const double ur = ush[r][lane];
            const double2 *tp = reinterpret_cast<const double2 *>(Tsh[r]);
#pragma unroll
            for (int h = 0; h < kFitBlk / 2; ++h) {
                const double2 t = tp[h];
                acc[2 * h] = fma(t.x, ur, acc[2 * h]);
                acc[2 * h + 1] = fma(t.y, ur, acc[2 * h + 1]);
            }
        }
#pragma unroll
        for (int q = 0; q < kFitBlk; ++q)
            red[w][q][lane] = acc[q];
        __syncthreads();
        if (w == 0) {
            double us[kFitBlk];
#pragma unroll
            for (int q = 0; q < kFitBlk; ++q) {
                const int sr = top - q;
                us[q] = 0.0;
                if (sr >= 0) {
                    double v = lcur[q] - (((red[0][q][lane] + red[1][q][lane]) + red[2][q][lane]) +
                                          red[3][q][lane]);
#pragma unroll
                    for (int q2 = 0; q2 < q; ++q2)
                        v = fma(-Tsh[top - q2][q], us[q2], v);  // T[top - q2][sr] u
                    us[q] = v / Tsh[sr][q];                    // T[sr][sr]
                    ush[sr][lane] = us[q];
                    if (a < n)
                        U[(long)sr * n + a] = us[q];
                }
            }
        }
    }
    if (w == 0 && a < n)
        for (int sr = R; sr < R_max; ++sr)
            U[(long)sr * n + a] = 0.0;
}

// V[i][r] = F[i][P[r]] for r < R, zero for R <= r < R_max
__global__ __launch_bounds__(CT) void fit_v_kernel(const double *__restrict__ F, int n,
                                                   int N_pair, int R, int R_max,
                                                   const int *__restrict__ piv,
                                                   double *__restrict__ V)
{
    const long e = (long)blockIdx.x * CT + threadIdx.x;
    if (e >= (long)N_pair * R_max)
        return;
    const long i = e / R_max;
    const int r = (int)(e % R_max);
    V[e] = r < R ? F[i * n + piv[r]] : 0.0;
}

// Entries of B from V and Y = V M (M symmetric): for the pivot p (state
// given) the column col[i] = B(i, p) = sum_k c_k prod_l V^l[i] . Y^l_k[p], else
// the diagonal d[i] = B(i, i) = sum_k c_k prod_l V^l[i] . Y^l_k[i].  One
// thread per (i, k mod KP) (KP = R_N rounded up to a power of two, at most
// 64): it forms the three dot products of its terms k, k + KP, ... and sums
// c_k times their product; the KP lanes of an index i then add their sums by
// a shuffle tree, and lane k = 0 (fixed order) writes the entry.
__global__ __launch_bounds__(256) void tei_entries_kernel(
    const double *__restrict__ c, const double *__restrict__ V0, const double *__restrict__ V1,
    const double *__restrict__ V2, const double *__restrict__ Y, int R, int R_N, int N_pair,
    int KP, const int *__restrict__ state, double *__restrict__ out)
{
    if (state && state[1])
        return;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    const int i = (int)(t / KP), k0 = (int)(t % KP);
    const bool live = i < N_pair;
    const int row = state ? state[0] : i;
    const long plane = (long)R_N * N_pair * R;
    double s = 0.0;
    if (live)
        for (int k = k0; k < R_N; k += KP) {
            double prod = c[k];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const double *v = (l == 0 ? V0 : l == 1 ? V1 : V2) + (long)i * R;
                const double *y = Y + l * plane + ((long)k * N_pair + row) * R;
                double dd = 0.0;
                for (int a = 0; a < R; ++a)
                    dd = fma(v[a], y[a], dd);
                prod *= dd;
            }
            s += prod;
        }
    for (int o = KP / 2; o > 0; o >>= 1)
        s += __shfl_xor(s, o);
    if (live && k0 == 0)
        out[i] = s;
}

// B += sum_{k < kc} c_k Z^0_k o Z^1_k o Z^2_k over the N x N entries (Z^l
// [kc][N][N], the terms of one chunk; first: B = that sum), in term order
__global__ __launch_bounds__(256) void tei_b_accum_kernel(const double *__restrict__ c,
                                                          const double *__restrict__ Z, long NN,
                                                          int kc, int first,
                                                          double *__restrict__ B)
{
    const long plane = (long)kc * NN;
    for (long e = blockIdx.x * 256L + threadIdx.x; e < NN; e += (long)gridDim.x * 256) {
        double v = first ? 0.0 : B[e];
        for (int k = 0; k < kc; ++k) {
            const long o = (long)k * NN + e;
            v += c[k] * (Z[o] * Z[plane + o] * Z[2 * plane + o]);
        }
        B[e] = v;
    }
}

// d[i] = A[i][i]
__global__ __launch_bounds__(256) void diag_copy_kernel(const double *__restrict__ A, int N,
                                                        double *__restrict__ d)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < N)
        d[i] = A[(long)i * N + i];
}

// T [cols][rows] = X^T for X [rows][cols] (32 x 32 tiles through LDS)
__global__ __launch_bounds__(256) void transpose_kernel(const double *__restrict__ X, int rows,
                                                        int cols, double *__restrict__ T)
{
    __shared__ double tile[32][33];
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows per pass
    for (int y = ty; y < 32; y += 8)
        if (r0 + y < rows && c0 + tx < cols)
            tile[y][tx] = X[(long)(r0 + y) * cols + c0 + tx];
    __syncthreads();
    for (int y = ty; y < 32; y += 8)
        if (c0 + y < cols && r0 + tx < rows)
            T[(long)(c0 + y) * rows + r0 + tx] = tile[tx][y];
}

}  // namespace

hipError_t launch_fit_diag(const double *F, int n, int N_pair, double *d, hipStream_t st)
{
    hipLaunchKernelGGL(fit_diag_kernel, dim3((n + CT - 1) / CT), dim3(CT), 0, st, F, n, N_pair,
                       d);
    return hipGetLastError();
}

hipError_t launch_fit_column(const double *F, int n, int N_pair, const int *state, double *part,
                             double *col, hipStream_t st)
{
    hipLaunchKernelGGL(fit_column_kernel, dim3((n + CT - 1) / CT, kFitSplit), dim3(CT), 0, st, F,
                       n, N_pair, state, part);
    hipLaunchKernelGGL(fit_column_reduce, dim3((n + CT - 1) / CT), dim3(CT), 0, st, part, n,
                       state, col);
    return hipGetLastError();
}

int fit_column_parts() { return kFitSplit; }

hipError_t launch_tei_diag(const double *c, const double *const *V, const double *const *M,
                           int R, int R_N, int N_pair, double *Y, double *d, hipStream_t st)
{
    const long plane = (long)R_N * N_pair * R;
    for (int l = 0; l < 3; ++l) {
        // Y^l[k][i][m] = sum_a V^l[i][a] M^l_k[m][a] = (V^l M^l_k)[i][m]
        const hipError_t e = launch_cross_gram_f64(V[l], M[l], Y + l * plane, R, N_pair, R, R_N,
                                                   st);
        if (e != hipSuccess)
            return e;
    }
    return launch_tei_entries(c, V, Y, R, R_N, N_pair, nullptr, d, st);
}

hipError_t launch_chol_step(const double *col, const double *A, double *L, int N, int r,
                            const int *ispiv, const int *state, double *d, hipStream_t st)
{
    hipLaunchKernelGGL(chol_step_kernel, dim3((N + kStepA - 1) / kStepA), dim3(kStepA * kStepG),
                       0, st, col, A, L, N, r, ispiv, state, d);
    return hipGetLastError();
}

hipError_t launch_chol_select_step(const double *A, double *L, int N, int r, int *ispiv,
                                   int *state, const double *d_in, double *d_out, double thr,
                                   int R_max, double *stats, int *piv, hipStream_t st)
{
    hipLaunchKernelGGL(chol_select_step_kernel, dim3((N + kStepA - 1) / kStepA),
                       dim3(kStepA * kStepG), 0, st, A, L, N, r, ispiv, state, d_in, d_out, thr,
                       R_max, stats, piv);
    return hipGetLastError();
}

hipError_t launch_chol_select(double *d, int N, int clear, int steps, double thr, int R_max,
                              int *state, double *stats, int *piv, int *ispiv, hipStream_t st)
{
    hipLaunchKernelGGL(chol_select_kernel, dim3(1), dim3(1024), 0, st, d, N, clear, steps, thr,
                       R_max, state, stats, piv, ispiv);
    return hipGetLastError();
}

hipError_t launch_tei_entries(const double *c, const double *const *V, const double *Y, int R,
                              int R_N, int N_pair, const int *state, double *out, hipStream_t st)
{
    int KP = 1;
    while (KP < R_N && KP < 64)
        KP *= 2;
    const long threads = (long)N_pair * KP;
    hipLaunchKernelGGL(tei_entries_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                       st, c, V[0], V[1], V[2], Y, R, R_N, N_pair, KP, state, out);
    return hipGetLastError();
}

hipError_t launch_diag_copy(const double *A, int N, double *d, hipStream_t st)
{
    hipLaunchKernelGGL(diag_copy_kernel, dim3((N + 255) / 256), dim3(256), 0, st, A, N, d);
    return hipGetLastError();
}

hipError_t launch_tei_form_b(const double *c, const double *const *V, const double *Y, int R,
                             int R_N, int N_pair, int kc, double *Z, double *B, double *d,
                             hipStream_t st)
{
    const long NN = (long)N_pair * N_pair;
    const long plane = (long)R_N * N_pair * R;  // of Y
    for (int k0 = 0; k0 < R_N; k0 += kc) {
        const int kn = R_N - k0 < kc ? R_N - k0 : kc;
        for (int l = 0; l < 3; ++l) {
            // Z^l[k][i][j] = sum_a V^l[i][a] Y^l[k0 + k][j][a] = (V M V^T)[i][j]
            const hipError_t e = launch_cross_gram_f64(V[l], Y + l * plane + (long)k0 * N_pair * R,
                                                       Z + (long)l * kn * NN, R, N_pair, N_pair,
                                                       kn, st);
            if (e != hipSuccess)
                return e;
        }
        long blocks = (NN + 255) / 256;
        if (blocks > 4096)
            blocks = 4096;
        hipLaunchKernelGGL(tei_b_accum_kernel, dim3((unsigned)blocks), dim3(256), 0, st, c + k0, Z,
                           NN, kn, k0 == 0 ? 1 : 0, B);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(diag_copy_kernel, dim3((N_pair + 255) / 256), dim3(256), 0, st, B, N_pair,
                       d);
    return hipGetLastError();
}

hipError_t launch_fit_gram(const double *F, int n, int N_pair, double *Ft, double *A,
                           hipStream_t st)
{
    hipLaunchKernelGGL(transpose_kernel, dim3((n + 31) / 32, (N_pair + 31) / 32), dim3(256), 0,
                       st, F, N_pair, n, Ft);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    // A[a][b] = sum_i Ft[a][i] Ft[b][i]
    return launch_cross_gram_f64(Ft, Ft, A, N_pair, n, n, 1, st);
}

hipError_t launch_fill_int(int *x, int count, int value, hipStream_t st)
{
    hipLaunchKernelGGL(fill_int_kernel, dim3((count + 255) / 256), dim3(256), 0, st, x, count,
                       value);
    return hipGetLastError();
}


hipError_t launch_fit_finish(const double *F, const double *L, int n, int N_pair, int R,
                             int R_max, const int *piv, double *Tg, double *U, double *V,
                             hipStream_t st)
{
    if (R > 0) {
        const long e = (long)R * R;
        hipLaunchKernelGGL(fit_t_kernel, dim3((unsigned)((e + CT - 1) / CT)), dim3(CT), 0, st, L,
                           n, R, piv, Tg);
    }
    if (R <= kFitMaxR)
        hipLaunchKernelGGL(fit_u_blk_kernel, dim3((n + 63) / 64), dim3(kFitT), 0, st, L, n, R,
                           R_max, Tg, U);
    else
        hipLaunchKernelGGL(fit_u_kernel, dim3((n + kFitUThreads - 1) / kFitUThreads),
                           dim3(kFitUThreads), 0, st, L, n, R, R_max, Tg, U);
    const long e = (long)N_pair * R_max;
    hipLaunchKernelGGL(fit_v_kernel, dim3((unsigned)((e + CT - 1) / CT)), dim3(CT), 0, st, F, n,
                       N_pair, R, R_max, piv, V);
    return hipGetLastError();
}

}  // namespace tc
