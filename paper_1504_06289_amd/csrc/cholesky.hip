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

// y[l][k][s] = sum_t M^l_k[s][t] V^l[j][t] for the pivot j (one workgroup per
// (l, k), threads over s)
// y^l_k = M^l_k v_j (v_j the pivot's row of V^l): workgroup (l k, row block)
// takes 64 rows s, its 4 waves the t = g mod 4 terms of each, summed in a
// fixed order.  M is symmetric: row s is read as column s, so that the
// lanes' loads are contiguous.
constexpr int kYRows = 64;
constexpr int kYGroups = 4;

__global__ __launch_bounds__(kYRows * kYGroups) void tei_y_kernel(
    const double *__restrict__ V0, const double *__restrict__ V1, const double *__restrict__ V2,
    const double *__restrict__ M0, const double *__restrict__ M1, const double *__restrict__ M2,
    int R, int R_N, const int *__restrict__ state, double *__restrict__ y)
{
    __shared__ double red[kYGroups][kYRows + 1];
    if (state[1])
        return;
    const int l = blockIdx.x / R_N, k = blockIdx.x % R_N;
    const double *V = l == 0 ? V0 : (l == 1 ? V1 : V2);
    const double *M = (l == 0 ? M0 : (l == 1 ? M1 : M2)) + (long)k * R * R;
    const double *vj = V + (long)state[0] * R;
    const int sl = threadIdx.x % kYRows, g = threadIdx.x / kYRows;
    const int s = blockIdx.y * kYRows + sl;
    double acc = 0.0;
    if (s < R)
        for (int t = g; t < R; t += kYGroups)
            acc = fma(M[(long)t * R + s], vj[t], acc);
    red[g][sl] = acc;
    __syncthreads();
    if (g == 0 && s < R) {
        double v = red[0][sl];
        for (int h = 1; h < kYGroups; ++h)
            v += red[h][sl];
        y[((long)l * R_N + k) * R + s] = v;
    }
}

// col[i] = sum_k c_k prod_l Z^l[i][k] with Z^l = V^l y^l^T (the column of B
// at the pivot; Z from cross_gram_f64)
__global__ __launch_bounds__(CT) void tei_column_kernel(const double *__restrict__ c,
                                                        const double *__restrict__ Z, int R_N,
                                                        int N_pair,
                                                        const int *__restrict__ state,
                                                        double *__restrict__ col)
{
    const int i = blockIdx.x * CT + threadIdx.x;
    if (i >= N_pair || state[1])
        return;
    const long plane = (long)N_pair * R_N;
    double s = 0.0;
    for (int k = 0; k < R_N; ++k) {
        const long o = (long)i * R_N + k;
        s += c[k] * (Z[o] * Z[plane + o] * Z[2 * plane + o]);
    }
    col[i] = s;
}

// d[i] = B(i, i) = sum_k c_k prod_l V^l[i] . Y^l[k][i] with Y^l_k = V^l M^l_k
// (from cross_gram_f64; M symmetric)
__global__ __launch_bounds__(CT) void tei_diag_kernel(const double *__restrict__ c,
                                                      const double *__restrict__ V0,
                                                      const double *__restrict__ V1,
                                                      const double *__restrict__ V2,
                                                      const double *__restrict__ Y, int R,
                                                      int R_N, int N_pair,
                                                      double *__restrict__ d)
{
    const int i = blockIdx.x * CT + threadIdx.x;
    if (i >= N_pair)
        return;
    const double *v[3] = {V0 + (long)i * R, V1 + (long)i * R, V2 + (long)i * R};
    const long plane = (long)R_N * N_pair * R;
    double s = 0.0;
    for (int k = 0; k < R_N; ++k) {
        double prod = c[k];
        for (int l = 0; l < 3; ++l) {
            const double *yk = Y + l * plane + ((long)k * N_pair + i) * R;
            double q = 0.0;
            for (int a = 0; a < R; ++a)
                q = fma(v[l][a], yk[a], q);
            prod *= q;
        }
        s += prod;
    }
    d[i] = s;
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
    const double *__restrict__ col, double *__restrict__ L, int N, int r,
    const int *__restrict__ ispiv, const int *__restrict__ state, double *__restrict__ d)
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
        double v = col[a];
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

// The largest residual diagonal entry (first index among equals) and the
// residual trace; one workgroup.  state = {pivot, done, steps}, stats = {max,
// trace}.  Nothing happens once done is set.  `clear`: the last pivot's entry
// is set to zero first; `steps`: the steps completed so far.  The process is
// done when steps >= R_max, the trace is at most thr or the maximum is not
// positive; otherwise the maximum's index is the next pivot.
__global__ __launch_bounds__(1024) void chol_select_kernel(double *__restrict__ d, int N,
                                                           int clear, int steps, double thr,
                                                           int R_max, int *__restrict__ state,
                                                           double *__restrict__ stats)
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
            state[0] = sidx[0];
        }
    }
}

__global__ void fill_int_kernel(int *__restrict__ x, int count, int value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        x[i] = value;
}

// piv[r] = the current pivot (unless done)
__global__ void chol_record_kernel(int r, const int *__restrict__ state, int *__restrict__ piv,
                                   int *__restrict__ ispiv)
{
    if (threadIdx.x == 0 && !state[1]) {
        piv[r] = state[0];
        ispiv[state[0]] = 1;
    }
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
    hipLaunchKernelGGL(tei_diag_kernel, dim3((N_pair + CT - 1) / CT), dim3(CT), 0, st, c, V[0],
                       V[1], V[2], Y, R, R_N, N_pair, d);
    return hipGetLastError();
}

hipError_t launch_tei_column(const double *c, const double *const *V, const double *const *M,
                             int R, int R_N, int N_pair, const int *state, double *y, double *Z,
                             double *col, hipStream_t st)
{
    hipLaunchKernelGGL(tei_y_kernel, dim3(3 * R_N, (R + kYRows - 1) / kYRows),
                       dim3(kYRows * kYGroups), 0, st, V[0], V[1], V[2], M[0],
                       M[1], M[2], R, R_N, state, y);
    const long plane = (long)N_pair * R_N;
    for (int l = 0; l < 3; ++l) {
        // Z^l[i][k] = sum_a V^l[i][a] y^l[k][a]
        const hipError_t e = launch_cross_gram_f64(V[l], y + (long)l * R_N * R, Z + l * plane, R,
                                                   N_pair, R_N, 1, st);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(tei_column_kernel, dim3((N_pair + CT - 1) / CT), dim3(CT), 0, st, c, Z,
                       R_N, N_pair, state, col);
    return hipGetLastError();
}

hipError_t launch_chol_step(const double *col, double *L, int N, int r, const int *ispiv,
                            const int *state, double *d, hipStream_t st)
{
    hipLaunchKernelGGL(chol_step_kernel, dim3((N + kStepA - 1) / kStepA), dim3(kStepA * kStepG),
                       0, st, col, L, N, r, ispiv, state, d);
    return hipGetLastError();
}

hipError_t launch_chol_select(double *d, int N, int clear, int steps, double thr, int R_max,
                              int *state, double *stats, hipStream_t st)
{
    hipLaunchKernelGGL(chol_select_kernel, dim3(1), dim3(1024), 0, st, d, N, clear, steps, thr,
                       R_max, state, stats);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *x, int count, int value, hipStream_t st)
{
    hipLaunchKernelGGL(fill_int_kernel, dim3((count + 255) / 256), dim3(256), 0, st, x, count,
                       value);
    return hipGetLastError();
}

hipError_t launch_chol_record(int r, const int *state, int *piv, int *ispiv, hipStream_t st)
{
    hipLaunchKernelGGL(chol_record_kernel, dim3(1), dim3(64), 0, st, r, state, piv, ispiv);
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
    hipLaunchKernelGGL(fit_u_kernel, dim3((n + kFitUThreads - 1) / kFitUThreads),
                       dim3(kFitUThreads), 0, st, L, n, R, R_max, Tg, U);
    const long e = (long)N_pair * R_max;
    hipLaunchKernelGGL(fit_v_kernel, dim3((unsigned)((e + CT - 1) / CT)), dim3(CT), 0, st, F, n,
                       N_pair, R, R_max, piv, V);
    return hipGetLastError();
}

}  // namespace tc
