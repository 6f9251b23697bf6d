// Assembled lattice sums of the Newton kernel (Section 5.1, eq. CoulombLatTensCan)
// and the pair energy of a charge lattice (Section 5.2, eq. EnergyLattice),
// binary64.
//
// The lattice has L_l unit cells of n0 grid cells along direction l
// (n_l = n0 L_l); the charge of unit cell j sits in grid cell j n0 + n0/2.
// Kernel vectors p^l [R_N][2 n_l - 1] are indexed by lag (lag m at m + n - 1).
//
//   lattice_sum:    A^l[q][i] = sum_{j < L_l} p^l_q[i - (j n0 + n0/2)], i < n_l,
//                   the shifted and windowed kernel vectors summed over the
//                   lattice, one direction at a time (the 3D lattice sum of
//                   the rank-R_N kernel is the rank-R_N tensor of the A^l_q);
//   lattice_energy: E = Z^2/2 sum_q w_q (prod_l S^l_q - L1 L2 L3 prod_l p^l_q[0]),
//                   S^l_q = sum_{|j| < L_l} (L_l - |j|) p^l_q[j n0],
//                   w_q = c_q / (h1 h2 h3)^2: the kernel summed over all
//                   ordered pairs of charges, minus the self terms.  With
//                   a_l = L_l p^l_q[0] and s_l the off-centre part of S^l_q, the
//                   difference of products is taken in the telescoped form
//                   s_1 S_2 S_3 + a_1 s_2 S_3 + a_1 a_2 s_3, which holds no
//                   cancellation of the (largest) self term.
// Sums run in a fixed order (bitwise reproducible).  The lattice sum has two
// forms: one thread per output summing its L terms (O(n L) per term), and
// running sums over the stride-n0 subsequences (O(n) per term).
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int LT = 256;
// (r, q) pairs from which the running-sum form is used (fewer: one thread per
// output, L terms each, for parallelism)
constexpr long kLatticeScanThreads = 2048;

// one thread per (i, q): the L terms in increasing j; blockIdx.z = direction
__global__ __launch_bounds__(LT) void lattice_sum_kernel(const double *__restrict__ p0,
                                                         const double *__restrict__ p1,
                                                         const double *__restrict__ p2,
                                                         double *__restrict__ A0,
                                                         double *__restrict__ A1,
                                                         double *__restrict__ A2, int n0,
                                                         int L0, int L1, int L2, int R_N)
{
    const int l = blockIdx.z, q = blockIdx.y;
    const int L = l == 0 ? L0 : (l == 1 ? L1 : L2);
    const int n = n0 * L;
    const int i = blockIdx.x * LT + threadIdx.x;
    if (i >= n)
        return;
    const double *p = (l == 0 ? p0 : (l == 1 ? p1 : p2)) + (long)q * (2L * n - 1) + (n - 1);
    double *A = (l == 0 ? A0 : (l == 1 ? A1 : A2)) + (long)q * n;
    double s = 0.0;
    for (int j = 0; j < L; ++j)
        s += p[i - (j * n0 + n0 / 2)];
    A[i] = s;
}

// The same sums in O(n_l) per term: with i = r + k n0 (r < n0, k < L) and
// s_r[m] = p_q[r - n0/2 + m n0], A[i] is the sum of s_r over the window
// m = k-L+1..k, and every such window holds m = 0, so
//   A[r + k n0] = SL(k-L+1) + PR(k),  SL(a) = sum_{a <= m < 0} s_r[m],
//                                      PR(k) = sum_{0 <= m <= k} s_r[m],
// two running sums without cancellation.  One thread per (r, q): a
// descending pass writes SL into A, an ascending pass adds PR.
__global__ __launch_bounds__(LT) void lattice_scan_kernel(const double *__restrict__ p0,
                                                          const double *__restrict__ p1,
                                                          const double *__restrict__ p2,
                                                          double *__restrict__ A0,
                                                          double *__restrict__ A1,
                                                          double *__restrict__ A2, int n0,
                                                          int L0, int L1, int L2)
{
    const int l = blockIdx.z, q = blockIdx.y;
    const int L = l == 0 ? L0 : (l == 1 ? L1 : L2);
    const int n = n0 * L;
    const int r = blockIdx.x * LT + threadIdx.x;
    if (r >= n0)
        return;
    // s[m] at s + m n0, m in [-(L-1), L-1]
    const double *s = (l == 0 ? p0 : (l == 1 ? p1 : p2)) + (long)q * (2L * n - 1) + (n - 1) +
                      (r - n0 / 2);
    double *A = (l == 0 ? A0 : (l == 1 ? A1 : A2)) + (long)q * n + r;
    double acc = 0.0;
    A[(long)(L - 1) * n0] = 0.0;
    for (int k = L - 2; k >= 0; --k) {
        acc += s[(long)(k - L + 1) * n0];
        A[(long)k * n0] = acc;
    }
    acc = 0.0;
    for (int k = 0; k < L; ++k) {
        acc += s[(long)k * n0];
        A[(long)k * n0] += acc;
    }
}

// one workgroup per q: term[q] = w_q (prod_l S^l_q - L1 L2 L3 prod_l p^l_q[0]),
// telescoped
__global__ __launch_bounds__(LT) void lattice_energy_kernel(const double *__restrict__ c,
                                                            const double *__restrict__ p0,
                                                            const double *__restrict__ p1,
                                                            const double *__restrict__ p2,
                                                            int n0, int L0, int L1, int L2,
                                                            double vol2,
                                                            double *__restrict__ term)
{
    __shared__ double red[LT];
    const int q = blockIdx.x;
    const int tid = threadIdx.x;
    double s_off[3], a[3];
    for (int l = 0; l < 3; ++l) {
        const int L = l == 0 ? L0 : (l == 1 ? L1 : L2);
        const int n = n0 * L;
        const double *p = (l == 0 ? p0 : (l == 1 ? p1 : p2)) + (long)q * (2L * n - 1) + (n - 1);
        double s = 0.0;
        for (int j = tid - (L - 1); j <= L - 1; j += LT)
            if (j != 0)
                s += (double)(L - (j < 0 ? -j : j)) * p[j * n0];
        red[tid] = s;
        __syncthreads();
        for (int w = LT / 2; w > 0; w >>= 1) {
            if (tid < w)
                red[tid] += red[tid + w];
            __syncthreads();
        }
        s_off[l] = red[0];
        a[l] = (double)L * p[0];
        __syncthreads();
    }
    if (tid == 0) {
        const double S1 = a[1] + s_off[1], S2 = a[2] + s_off[2];
        term[q] = c[q] / vol2 * (s_off[0] * S1 * S2 + a[0] * s_off[1] * S2 + a[0] * a[1] * s_off[2]);
    }
}

__global__ void lattice_energy_sum_kernel(const double *__restrict__ term, int R_N, double Z,
                                          double *__restrict__ E)
{
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < R_N; ++q)
            s += term[q];
        *E = 0.5 * Z * Z * s;
    }
}

}  // namespace

hipError_t launch_lattice_sum(int n0, const int *L, int R_N, const double *const *p,
                              double *const *A, hipStream_t st)
{
    if ((long)n0 * R_N >= kLatticeScanThreads) {
        // enough (r, q) pairs to fill the chip: the O(n) running sums
        dim3 grid((n0 + LT - 1) / LT, R_N, 3);
        hipLaunchKernelGGL(lattice_scan_kernel, grid, dim3(LT), 0, st, p[0], p[1], p[2], A[0],
                           A[1], A[2], n0, L[0], L[1], L[2]);
        return hipGetLastError();
    }
    int nmax = 0;
    for (int l = 0; l < 3; ++l)
        nmax = n0 * L[l] > nmax ? n0 * L[l] : nmax;
    dim3 grid((nmax + LT - 1) / LT, R_N, 3);
    hipLaunchKernelGGL(lattice_sum_kernel, grid, dim3(LT), 0, st, p[0], p[1], p[2], A[0], A[1],
                       A[2], n0, L[0], L[1], L[2], R_N);
    return hipGetLastError();
}

hipError_t launch_lattice_energy(int n0, const int *L, int R_N, const double *c,
                                 const double *h, const double *const *p, double Z,
                                 double *term, double *E, hipStream_t st)
{
    const double vol = h[0] * h[1] * h[2];
    hipLaunchKernelGGL(lattice_energy_kernel, dim3(R_N), dim3(LT), 0, st, c, p[0], p[1], p[2],
                       n0, L[0], L[1], L[2], vol * vol, term);
    hipLaunchKernelGGL(lattice_energy_sum_kernel, dim3(1), dim3(64), 0, st, term, R_N, Z, E);
    return hipGetLastError();
}

}  // namespace tc
