// Grams of one mode (the matrices M_k^(l) of eq. Factor_Mk_Conv), binary64
// on matrix cores:
//   G[k][i][j] = sum_a U[i][a] W[k][j][a]        (G_k = U^T W_k)
//
// G_k is symmetric (T_k is), so only upper-triangle tiles (ti <= tj) are
// computed; each computed entry with i <= j is written to (i, j) and (j, i),
// which makes the stored Gram exactly symmetric.
//
// The diagonal form (nuclear potential matrices) takes a diagonal operator in
// place of T_k: term t = alpha R_N + q has the kernel vector p_q shifted to the
// cell shift[alpha],
//   G[t][i][j] = sum_a U[i][a] U[j][a] p_q[a - shift[alpha]].
// Its workgroups stage the two U tiles once and apply the shifted vectors of
// kDiagTerms terms while reading the fragments (one accumulator set per
// term), so the U tiles are read once per kDiagTerms terms.
//
// Both operands are contiguous along the contraction index a.  Tiles:
// 64 x 64 per workgroup, 4 waves as 2 x 2 wave tiles of 32 x 32, K-step 16,
// v_mfma_f64_16x16x4_f64 (lane l supplies A[l%16][l/16], B[l/16][l%16];
// result lane l holds D[l/16 + 4r][l%16]).
#include "tc_internal.h"

namespace tc {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int BT = 64;  // tile edge (i and j)
constexpr int BK = 16;
constexpr int PAD = 1;

__global__ __launch_bounds__(256) void gram_f64_kernel(const double *__restrict__ U,
                                                       const double *__restrict__ W,
                                                       double *__restrict__ G, int n, int R_f,
                                                       int ntiles, int mirror)
{
    __shared__ double As[2][BT][BK + PAD];
    __shared__ double Bs[2][BT][BK + PAD];

    // upper-triangle tile index -> (ti, tj), ti <= tj, row-major over ti
    int t = blockIdx.x;
    int ti = 0;
    while (t >= ntiles - ti) {
        t -= ntiles - ti;
        ++ti;
    }
    const int tj = ti + t;
    const int k = blockIdx.y;
    const int i0 = ti * BT, j0 = tj * BT;
    const double *Wk = W + (long)k * R_f * n;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = (wave >> 1) * 32;
    const int wj = (wave & 1) * 32;
    const int l16 = lane & 15;
    const int lk = lane >> 4;

    const int lrow = tid >> 2;
    const int lcol = (tid & 3) * 4;
    double areg[4], breg[4];

    auto load_stage = [&](int a0) {
        const int i = i0 + lrow, j = j0 + lrow;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int a = a0 + lcol + q;
            areg[q] = (i < R_f && a < n) ? U[(long)i * n + a] : 0.0;
            breg[q] = (j < R_f && a < n) ? Wk[(long)j * n + a] : 0.0;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[buf][lrow][lcol + q] = areg[q];
            Bs[buf][lrow][lcol + q] = breg[q];
        }
    };

    f64x4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
            acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int nsteps = (n + BK - 1) / BK;
    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const int buf = s & 1;
        if (s + 1 < nsteps)
            load_stage((s + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
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

    double *Gk = G + (long)k * R_f * R_f;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int j = j0 + wj + y * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + x * 16 + lk + 4 * r;
                if (i < R_f && j < R_f && i <= j) {
                    Gk[(long)i * R_f + j] = acc[x][y][r];
                    if (mirror)
                        Gk[(long)j * R_f + i] = acc[x][y][r];
                }
            }
        }
}

constexpr int kDiagTerms = 4;

__global__ __launch_bounds__(256) void diag_gram_f64_kernel(const double *__restrict__ U,
                                                            const double *__restrict__ p,
                                                            const int *__restrict__ shift,
                                                            const int *__restrict__ cls,
                                                            double *__restrict__ G, int n,
                                                            int R_f, int ntiles, int T, int R_N,
                                                            int mirror)
{
    __shared__ double As[2][BT][BK + PAD];
    __shared__ double Bs[2][BT][BK + PAD];
    __shared__ double Ss[2][kDiagTerms][BK];

    int t = blockIdx.x;
    int ti = 0;
    while (t >= ntiles - ti) {
        t -= ntiles - ti;
        ++ti;
    }
    const int tj = ti + t;
    const int t0 = blockIdx.y * kDiagTerms;
    const int nt = min(kDiagTerms, T - t0);
    const int i0 = ti * BT, j0 = tj * BT;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = (wave >> 1) * 32;
    const int wj = (wave & 1) * 32;
    const int l16 = lane & 15;
    const int lk = lane >> 4;

    const int lrow = tid >> 2;
    const int lcol = (tid & 3) * 4;
    // the shifted kernel vector of term t0 + u: sv(u)[a] = p_q[a - shift[alpha]]
    // (lag a - shift in [-(n-1), n-1]); thread tid < kDiagTerms * BK stages
    // entry (u, c) = (tid / BK, tid % BK) of each K-step
    const int su = tid / BK, sc = tid % BK;
    const double *srow = nullptr;
    if (tid < kDiagTerms * BK && su < nt) {
        const int tt = t0 + su;
        const int alpha = tt / R_N, q = tt - alpha * R_N;
        srow = p + (long)q * (2L * n - 1) + (n - 1) - shift[alpha];
    }
    double areg[4], breg[4], sreg = 0.0;

    auto load_stage = [&](int a0) {
        const int i = i0 + lrow, j = j0 + lrow;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int a = a0 + lcol + q;
            areg[q] = (i < R_f && a < n) ? U[(long)i * n + a] : 0.0;
            breg[q] = (j < R_f && a < n) ? U[(long)j * n + a] : 0.0;
        }
        if (srow) {
            const int a = a0 + sc;
            sreg = a < n ? srow[a] : 0.0;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[buf][lrow][lcol + q] = areg[q];
            Bs[buf][lrow][lcol + q] = breg[q];
        }
        if (tid < kDiagTerms * BK)
            Ss[buf][su][sc] = sreg;  // zero for terms past the end
    };

    f64x4 acc[kDiagTerms][2][2];
#pragma unroll
    for (int u = 0; u < kDiagTerms; ++u)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
                acc[u][x][y] = f64x4{0.0, 0.0, 0.0, 0.0};

    // K steps: every cell, or, when every term of the group is narrow (class
    // B >= 0: the lags beyond B carry less than 2^-60 of the kernel vector's
    // l1 norm), only the cells within B of the group's nuclei
    int sbeg = 0, send = (n + BK - 1) / BK;
    if (cls) {
        int lo = n, hi = -1;
        bool narrow = true;
        for (int u = 0; u < nt && narrow; ++u) {
            const int tt = t0 + u;
            const int alpha = tt / R_N, q = tt - alpha * R_N;
            const int b = cls[q];
            narrow = b >= 0;
            lo = min(lo, shift[alpha] - b);
            hi = max(hi, shift[alpha] + b);
        }
        if (narrow) {
            lo = max(lo, 0);
            hi = min(hi, n - 1);
            sbeg = lo / BK;
            send = hi >= lo ? hi / BK + 1 : sbeg;
        }
    }
    const int nsteps = send - sbeg;
    load_stage(sbeg * BK);
    store_stage(0);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const int buf = s & 1;
        if (s + 1 < nsteps)
            load_stage((sbeg + s + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double afr[2], bfr[2];
#pragma unroll
            for (int x = 0; x < 2; ++x)
                afr[x] = As[buf][wi + x * 16 + l16][kk + lk];
#pragma unroll
            for (int y = 0; y < 2; ++y)
                bfr[y] = Bs[buf][wj + y * 16 + l16][kk + lk];
#pragma unroll
            for (int u = 0; u < kDiagTerms; ++u) {
                const double su_k = Ss[buf][u][kk + lk];
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        acc[u][x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            afr[x], bfr[y] * su_k, acc[u][x][y], 0, 0, 0);
            }
        }
        if (s + 1 < nsteps)
            store_stage(buf ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int u = 0; u < kDiagTerms; ++u) {
        if (u >= nt)
            break;
        double *Gt = G + (long)(t0 + u) * R_f * R_f;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int j = j0 + wj + y * 16 + l16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + wi + x * 16 + lk + 4 * r;
                    if (i < R_f && j < R_f && i <= j) {
                        Gt[(long)i * R_f + j] = acc[u][x][y][r];
                        if (mirror)
                            Gt[(long)j * R_f + i] = acc[u][x][y][r];
                    }
                }
            }
    }
}

}  // namespace

hipError_t launch_gram_f64(const double *U, const double *W, double *G, int n, int R_f,
                           int R_N, bool mirror, hipStream_t stream)
{
    const int nt = (R_f + BT - 1) / BT;
    dim3 grid(nt * (nt + 1) / 2, R_N);
    hipLaunchKernelGGL(gram_f64_kernel, grid, dim3(256), 0, stream, U, W, G, n, R_f, nt,
                       (int)mirror);
    return hipGetLastError();
}

hipError_t launch_diag_gram_f64(const double *U, const double *p, const int *shift,
                                const int *cls, double *G, int n, int R_f, int R_N, int M,
                                bool mirror, hipStream_t stream)
{
    const int nt = (R_f + BT - 1) / BT;
    const int T = M * R_N;
    dim3 grid(nt * (nt + 1) / 2, (T + kDiagTerms - 1) / kDiagTerms);
    hipLaunchKernelGGL(diag_gram_f64_kernel, grid, dim3(256), 0, stream, U, p, shift, cls, G, n,
                       R_f, nt, T, R_N, (int)mirror);
    return hipGetLastError();
}

}  // namespace tc
