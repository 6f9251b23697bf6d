// Binary32 matrix-core variants of the Toeplitz product and the Gram
// (precision TC_FP32): operands rounded to binary32 when they are staged in
// LDS, v_mfma_f32_16x16x4_f32 with binary32 partial sums over K-chunks of
// 64, and binary64 accumulation of the chunk sums.
//
// Every operand row is first scaled by a power of two, 2^-e with e the
// exponent of its largest magnitude, so that binary32's narrow exponent range
// only loses entries far below the row maximum; the power is put back on the
// binary64 result.  Without it, functions or kernel terms whose values sit
// below about 1e-38 would be flushed to zero outright.
//
//   W[k][j][a] = sum_b U[j][b] p_k[a-b]          (implicit Toeplitz operand)
//   G[k][i][j] = sum_a U[i][a] W[k][j][a]        (upper-triangle tiles, mirrored)
//
// v_mfma_f32_16x16x4_f32: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// the result lane l holds D[4(l/16)+r][l%16], r = 0..3.
// Tiles 64 x 64, 4 waves of 32 x 32 (2 x 2 MFMA blocks), K-step 16.
#include "tc_internal.h"

namespace tc {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int BT = 64;
constexpr int BK = 16;
constexpr int CHUNK_STEPS = 4;  // K-steps of 16 per binary32 chunk (64 products)
constexpr int PW = BT + BK - 1;

__device__ inline void flush(f32x4 (&acc)[2][2], f64x4 (&sum)[2][2])
{
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sum[x][y][r] += (double)acc[x][y][r];
            acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
}

// E[r] = exponent e of the largest |X[r][.]| (frexp convention: max < 2^e),
// 0 for an all-zero row, at least -1000 so that 2^-e stays finite for rows of
// subnormal numbers.  One wave per row.
__global__ __launch_bounds__(256) void row_exponent_kernel(const double *__restrict__ X,
                                                           long rows, int len,
                                                           int *__restrict__ E)
{
    const long r = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows)
        return;
    const double *x = X + r * len;
    double m = 0.0;
    for (int i = lane; i < len; i += 64)
        m = fmax(m, fabs(x[i]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        m = fmax(m, __shfl_xor(m, off, 64));
    if (lane == 0) {
        int e = 0;
        if (m > 0.0)
            frexp(m, &e);
        E[r] = e < -1000 ? -1000 : e;
    }
}

__global__ __launch_bounds__(256) void toeplitz_f32_kernel(const double *__restrict__ p,
                                                           const int *__restrict__ EP,
                                                           const double *__restrict__ U,
                                                           const int *__restrict__ EU,
                                                           double *__restrict__ W, int n,
                                                           int R_f)
{
    __shared__ float Us[2][BT][BK + 1];
    __shared__ float Ps[2][PW + 1];

    const int k = blockIdx.z;
    const int a0 = blockIdx.x * BT;
    const int j0 = blockIdx.y * BT;
    const long L = 2L * n - 1;
    const double *pk = p + (long)k * L + (n - 1);

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wj = (wave >> 1) * 32, wa = (wave & 1) * 32;
    const int l16 = lane & 15, lk = lane >> 4;
    const int urow = tid >> 2, ucol = (tid & 3) * 4;
    float ureg[4], preg = 0.f;
    const double uscale = (j0 + urow < R_f) ? ldexp(1.0, -EU[j0 + urow]) : 0.0;
    const double pscale = ldexp(1.0, -EP[k]);

    auto load_stage = [&](int b0) {
        const int j = j0 + urow;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = b0 + ucol + q;
            ureg[q] = (j < R_f && b < n) ? (float)(U[(long)j * n + b] * uscale) : 0.f;
        }
        if (tid < PW) {
            const int lag = a0 - b0 - (BK - 1) + tid;
            preg = (lag > -n && lag < n) ? (float)(pk[lag] * pscale) : 0.f;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            Us[buf][urow][ucol + q] = ureg[q];
        if (tid < PW)
            Ps[buf][tid] = preg;
    };

    f32x4 acc[2][2];
    f64x4 sum[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
            sum[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
        }

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
            float afr[2], bfr[2];
#pragma unroll
            for (int x = 0; x < 2; ++x)
                afr[x] = Us[buf][wj + x * 16 + l16][kk + lk];
#pragma unroll
            for (int y = 0; y < 2; ++y)
                bfr[y] = Ps[buf][(wa + y * 16 + l16) - (kk + lk) + (BK - 1)];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] =
                        __builtin_amdgcn_mfma_f32_16x16x4f32(afr[x], bfr[y], acc[x][y], 0, 0, 0);
        }
        if ((s + 1) % CHUNK_STEPS == 0 || s + 1 == nsteps)
            flush(acc, sum);
        if (s + 1 < nsteps)
            store_stage(buf ^ 1);
        __syncthreads();
    }

    double *Wk = W + (long)k * R_f * n;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int a = a0 + wa + y * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 + wj + x * 16 + 4 * lk + r;
                if (j < R_f && a < n)
                    Wk[(long)j * n + a] = ldexp(sum[x][y][r], EU[j] + EP[k]);
            }
        }
}

__global__ __launch_bounds__(256) void gram_f32_kernel(const double *__restrict__ U,
                                                       const int *__restrict__ EU,
                                                       const double *__restrict__ W,
                                                       const int *__restrict__ EW,
                                                       double *__restrict__ G, int n, int R_f,
                                                       int ntiles, int mirror)
{
    __shared__ float As[2][BT][BK + 1];
    __shared__ float Bs[2][BT][BK + 1];

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
    const int lane = tid & 63, wave = tid >> 6;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    const int l16 = lane & 15, lk = lane >> 4;
    const int lrow = tid >> 2, lcol = (tid & 3) * 4;
    float areg[4], breg[4];
    const int *EWk = EW + (long)k * R_f;
    const double ascale = (i0 + lrow < R_f) ? ldexp(1.0, -EU[i0 + lrow]) : 0.0;
    const double bscale = (j0 + lrow < R_f) ? ldexp(1.0, -EWk[j0 + lrow]) : 0.0;

    auto load_stage = [&](int a0) {
        const int i = i0 + lrow, j = j0 + lrow;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int a = a0 + lcol + q;
            areg[q] = (i < R_f && a < n) ? (float)(U[(long)i * n + a] * ascale) : 0.f;
            breg[q] = (j < R_f && a < n) ? (float)(Wk[(long)j * n + a] * bscale) : 0.f;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[buf][lrow][lcol + q] = areg[q];
            Bs[buf][lrow][lcol + q] = breg[q];
        }
    };

    f32x4 acc[2][2];
    f64x4 sum[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
            sum[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
        }

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
            float afr[2], bfr[2];
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
                    acc[x][y] =
                        __builtin_amdgcn_mfma_f32_16x16x4f32(afr[x], bfr[y], acc[x][y], 0, 0, 0);
        }
        if ((s + 1) % CHUNK_STEPS == 0 || s + 1 == nsteps)
            flush(acc, sum);
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
                const int i = i0 + wi + x * 16 + 4 * lk + r;
                if (i < R_f && j < R_f && i <= j) {
                    const double g = ldexp(sum[x][y][r], EU[i] + EWk[j]);
                    Gk[(long)i * R_f + j] = g;
                    if (mirror)
                        Gk[(long)j * R_f + i] = g;
                }
            }
        }
}

}  // namespace

hipError_t launch_row_exponents(const double *X, long rows, int len, int *E, hipStream_t stream)
{
    hipLaunchKernelGGL(row_exponent_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0,
                       stream, X, rows, len, E);
    return hipGetLastError();
}

hipError_t launch_toeplitz_f32(const double *p, const int *EP, const double *U, const int *EU,
                               double *W, int n, int R_f, int R_N, hipStream_t stream)
{
    dim3 grid((n + BT - 1) / BT, (R_f + BT - 1) / BT, R_N);
    hipLaunchKernelGGL(toeplitz_f32_kernel, grid, dim3(256), 0, stream, p, EP, U, EU, W, n, R_f);
    return hipGetLastError();
}

hipError_t launch_gram_f32(const double *U, const int *EU, const double *W, const int *EW,
                           double *G, int n, int R_f, int R_N, bool mirror,
                           hipStream_t stream)
{
    const int nt = (R_f + BT - 1) / BT;
    dim3 grid(nt * (nt + 1) / 2, R_N);
    hipLaunchKernelGGL(gram_f32_kernel, grid, dim3(256), 0, stream, U, EU, W, EW, G, n, R_f, nt,
                       (int)mirror);
    return hipGetLastError();
}

}  // namespace tc
