// Coulomb entries against a density in canonical format (Section 3.1: the
// Hartree potential of Theta' = sum_m d_m v^1_m x v^2_m x v^3_m is a sum of
// tensor products of the 1D convolutions v^l_m * p^l_q, and the Coulomb
// entries are its scalar products with the rank-1 products of basis
// functions), binary64:
//
//   H^l[q][i][m] = sum_a U^l[i][a] W^l[q][m][a]     (W^l_q = T^l_q V^l)
//   Jd[i]        = sum_q c_q sum_m d_m H^1[q][i][m] H^2[q][i][m] H^3[q][i][m]
//
// cross_gram_f64: H^l_q = U^l (W^l_q)^T on matrix cores, 64 x 64 tiles over
// (i, m), four waves of 32 x 32, K-step 16, v_mfma_f64_16x16x4_f64 (lane l
// supplies A[l%16][l/16], B[l/16][l%16]; result lane l holds D[l/16+4r][l%16]).
// coulomb_reduce: one workgroup per i, the R_N R_rho products summed in a
// fixed order (per-thread strided sums, then a fixed tree), so the result is
// bitwise reproducible.
#include "tc_internal.h"

namespace tc {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int CT = 64;  // tile edge (i and m)
constexpr int CK = 16;
constexpr int CPAD = 1;

__global__ __launch_bounds__(256) void cross_gram_f64_kernel(const double *__restrict__ U,
                                                             const double *__restrict__ W,
                                                             double *__restrict__ H, int n,
                                                             int R_f, int R_rho)
{
    __shared__ double As[2][CT][CK + CPAD];
    __shared__ double Bs[2][CT][CK + CPAD];

    const int i0 = blockIdx.x * CT, m0 = blockIdx.y * CT;
    const int q = blockIdx.z;
    const double *Wq = W + (long)q * R_rho * n;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = (wave >> 1) * 32;
    const int wm = (wave & 1) * 32;
    const int l16 = lane & 15;
    const int lk = lane >> 4;

    // staging: row tid/4 of each tile, four consecutive a
    const int lrow = tid >> 2;
    const int lcol = (tid & 3) * 4;
    double areg[4], breg[4];
    auto load_stage = [&](int a0) {
        const int i = i0 + lrow, m = m0 + lrow;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int a = a0 + lcol + r;
            areg[r] = (i < R_f && a < n) ? U[(long)i * n + a] : 0.0;
            breg[r] = (m < R_rho && a < n) ? Wq[(long)m * n + a] : 0.0;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            As[buf][lrow][lcol + r] = areg[r];
            Bs[buf][lrow][lcol + r] = breg[r];
        }
    };

    f64x4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
            acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int nsteps = (n + CK - 1) / CK;
    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const int buf = s & 1;
        if (s + 1 < nsteps)
            load_stage((s + 1) * CK);
#pragma unroll
        for (int kk = 0; kk < CK; kk += 4) {
            double afr[2], bfr[2];
#pragma unroll
            for (int x = 0; x < 2; ++x)
                afr[x] = As[buf][wi + x * 16 + l16][kk + lk];
#pragma unroll
            for (int y = 0; y < 2; ++y)
                bfr[y] = Bs[buf][wm + y * 16 + l16][kk + lk];
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

    double *Hq = H + (long)q * R_f * R_rho;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int m = m0 + wm + y * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + x * 16 + lk + 4 * r;
                if (i < R_f && m < R_rho)
                    Hq[(long)i * R_rho + m] = acc[x][y][r];
            }
        }
}

constexpr int RT = 256;  // threads of the reduction workgroup

__global__ __launch_bounds__(RT) void coulomb_reduce_kernel(const double *__restrict__ c,
                                                            const double *__restrict__ d,
                                                            const double *__restrict__ H0,
                                                            const double *__restrict__ H1,
                                                            const double *__restrict__ H2,
                                                            double *__restrict__ Jd, int R_f,
                                                            int R_rho, int R_N)
{
    __shared__ double red[RT];
    const int i = blockIdx.x;
    const int tid = threadIdx.x;
    const long terms = (long)R_N * R_rho;
    double s = 0.0;
    for (long e = tid; e < terms; e += RT) {
        const int q = (int)(e / R_rho), m = (int)(e % R_rho);
        const long o = ((long)q * R_f + i) * R_rho + m;
        s += c[q] * d[m] * (H0[o] * H1[o] * H2[o]);
    }
    red[tid] = s;
    __syncthreads();
    for (int w = RT / 2; w > 0; w >>= 1) {
        if (tid < w)
            red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0)
        Jd[i] = red[0];
}

}  // namespace

hipError_t launch_cross_gram_f64(const double *U, const double *W, double *H, int n, int R_f,
                                 int R_rho, int R_N, hipStream_t stream)
{
    dim3 grid((R_f + CT - 1) / CT, (R_rho + CT - 1) / CT, R_N);
    hipLaunchKernelGGL(cross_gram_f64_kernel, grid, dim3(256), 0, stream, U, W, H, n, R_f,
                       R_rho);
    return hipGetLastError();
}

hipError_t launch_coulomb_reduce(const double *c, const double *d, const double *H, int R_f,
                                 int R_rho, int R_N, double *Jd, hipStream_t stream)
{
    const long plane = (long)R_N * R_f * R_rho;
    hipLaunchKernelGGL(coulomb_reduce_kernel, dim3(R_f), dim3(RT), 0, stream, c, d, H,
                       H + plane, H + 2 * plane, Jd, R_f, R_rho, R_N);
    return hipGetLastError();
}

}  // namespace tc
