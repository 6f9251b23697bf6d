// Adjoint contraction of one mode, binary64 on matrix cores:
//   dU[i][a] = scale * sum_k sum_j D_k[j][i] W_k[j][a]      (dU = 2 sum_k W_k D_k)
//
// With the contraction index K = k*R_f + j both operands are plain row-major
// [K][R_f] and [K][n] slabs (D and W as stored), so this is one GEMM
// dU = scale * D_flat^T W_flat with K = R_N R_f.  Both LDS tiles are kept as
// [K][row]: the MFMA fragment reads (16 consecutive rows for one K) are then
// contiguous.  Tiles 64 (i) x 64 (a), 4 waves of 32 x 32, K-step 16,
// v_mfma_f64_16x16x4_f64 (lane l supplies A[l%16][l/16], B[l/16][l%16];
// result lane l holds D[l/16 + 4r][l%16]).
//
// When the output has few tiles, K is split into S contiguous ranges
// (blockIdx.z) so that about 1024 workgroups run: range 0 writes its raw sum
// to dU, range z > 0 to part[z-1], and adjoint_reduce forms
// dU = scale (((dU + part[0]) + part[1]) + ...) in that fixed order.
#include "tc_internal.h"

namespace tc {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int BT = 64;
constexpr int BK = 16;
constexpr int PAD = 2;

__global__ __launch_bounds__(256) void adjoint_gemm_f64_kernel(const double *__restrict__ D,
                                                               const double *__restrict__ W,
                                                               double *__restrict__ dU, int n,
                                                               int R_f, long Ktot,
                                                               double scale,
                                                               double *__restrict__ part)
{
    __shared__ double As[2][BK][BT + PAD];
    __shared__ double Bs[2][BK][BT + PAD];

    const int a0 = blockIdx.x * BT;
    const int i0 = blockIdx.y * BT;
    // this workgroup's K range [Kb, Ke): split on multiples of BK
    const long nstep_all = (Ktot + BK - 1) / BK;
    const long Kb = (long)blockIdx.z * nstep_all / gridDim.z * BK;
    const long Ke0 = (long)(blockIdx.z + 1) * nstep_all / gridDim.z * BK;
    const long Ke = Ke0 < Ktot ? Ke0 : Ktot;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = (wave >> 1) * 32;
    const int wa = (wave & 1) * 32;
    const int l16 = lane & 15;
    const int lk = lane >> 4;

    // staging: BK x BT = 1024 doubles per operand; thread -> row tid/16, cols (tid%16)*4..+3
    const int srow = tid >> 4;
    const int scol = (tid & 15) * 4;
    double areg[4], breg[4];
    auto load_stage = [&](long K0) {
        const long K = K0 + srow;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + scol + q;
            const int a = a0 + scol + q;
            areg[q] = (K < Ke && i < R_f) ? D[K * R_f + i] : 0.0;
            breg[q] = (K < Ke && a < n) ? W[K * n + a] : 0.0;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[buf][srow][scol + q] = areg[q];
            Bs[buf][srow][scol + q] = breg[q];
        }
    };

    f64x4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
            acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};

    const long nsteps = (Ke - Kb + BK - 1) / BK;
    load_stage(Kb);
    store_stage(0);
    __syncthreads();
    for (long s = 0; s < nsteps; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < nsteps)
            load_stage(Kb + (s + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double afr[2], bfr[2];
#pragma unroll
            for (int x = 0; x < 2; ++x)
                afr[x] = As[buf][kk + lk][wi + x * 16 + l16];
#pragma unroll
            for (int y = 0; y < 2; ++y)
                bfr[y] = Bs[buf][kk + lk][wa + y * 16 + l16];
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

    // one K range: the scaled result; several: raw partial sums
    double *out = blockIdx.z == 0 ? dU : part + (long)(blockIdx.z - 1) * R_f * n;
    const double sc = gridDim.z == 1 ? scale : 1.0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int a = a0 + wa + y * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + x * 16 + lk + 4 * r;
                if (i < R_f && a < n)
                    out[(long)i * n + a] = sc * acc[x][y][r];
            }
        }
}

__global__ __launch_bounds__(256) void adjoint_reduce_kernel(double *__restrict__ dU,
                                                             const double *__restrict__ part,
                                                             long len, int nparts, double scale)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= len)
        return;
    double v = dU[e];
    for (int z = 0; z < nparts; ++z)
        v += part[(long)z * len + e];
    dU[e] = scale * v;
}

}  // namespace

int adjoint_splits(int n, int R_f, int R_N)
{
    const long tiles = (long)((n + BT - 1) / BT) * ((R_f + BT - 1) / BT);
    const long ksteps = ((long)R_N * R_f + BK - 1) / BK;
    long S = (1024 + tiles - 1) / tiles;
    if (S > kAdjointMaxSplit)
        S = kAdjointMaxSplit;
    if (S > ksteps / 32)  // at least 32 K-steps (512 products) per range
        S = ksteps / 32;
    return S < 1 ? 1 : (int)S;
}

hipError_t launch_adjoint_gemm_f64(const double *D, const double *W, double *dU, int n, int R_f,
                                   int R_N, double scale, double *part, hipStream_t stream)
{
    const int S = adjoint_splits(n, R_f, R_N);
    if (S > 1 && !part)
        return hipErrorInvalidValue;
    dim3 grid((n + BT - 1) / BT, (R_f + BT - 1) / BT, S);
    hipLaunchKernelGGL(adjoint_gemm_f64_kernel, grid, dim3(256), 0, stream, D, W, dU, n, R_f,
                       (long)R_N * R_f, scale, part);
    if (S > 1) {
        const long len = (long)R_f * n;
        hipLaunchKernelGGL(adjoint_reduce_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256),
                           0, stream, dU, part, len, S - 1, scale);
    }
    return hipGetLastError();
}

}  // namespace tc
