// Implicit-Toeplitz products on matrix cores (binary64):
//   W[k][j][a] = sum_b p_k[a-b] U[j][b]     (W_k = T_k U, Section 3.2)
//
// The Toeplitz operand is never materialised.  For a K-step covering cells
// b0..b0+BK-1 and an output tile covering cells a0..a0+BA-1, every entry
// T[a][b] = p[a-b] lies in the contiguous lag window
// p[a0-b0-BK+1 .. a0-b0+BA-1] (BA+BK-1 values), which is staged into LDS;
// the MFMA B-fragments are then read from that window at offset
// (a - b) - (a0 - b0 - BK + 1), i.e. each fragment row is the window
// shifted by one entry per K index.
//
// GEMM orientation: D[j][a] = sum_b A[j][b] * B[b][a] with A = U (rows j,
// K = b contiguous in memory) and B[b][a] = p[a-b], so the MFMA output rows
// are functions j and the columns are cells a, and each output row segment is
// contiguous in W.
//
// Matrix-core instruction: v_mfma_f64_16x16x4_f64 (D 16x16, K = 4).
// Operand layout per 64-wide wave: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; the result lane l holds D[l/16 + 4r][l%16], r = 0..3.
//
// Tiles: workgroup 64 (j) x 64 (a), 4 waves in a 2 x 2 arrangement of 32x32
// wave tiles (2 x 2 MFMA blocks each), K-step 16, double-buffered LDS.
#include "tc_internal.h"

namespace tc {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int BJ = 64;   // functions per workgroup tile
constexpr int BA = 64;   // cells per workgroup tile
constexpr int BK = 16;   // K-step (cells b)
constexpr int UPAD = 1;  // LDS row padding (doubles) against bank conflicts
constexpr int PW = BA + BK - 1;

__global__ __launch_bounds__(256) void toeplitz_f64_kernel(const double *__restrict__ p,
                                                           const double *__restrict__ U,
                                                           double *__restrict__ W, int n,
                                                           int R_f)
{
    __shared__ double Us[2][BJ][BK + UPAD];
    __shared__ double Ps[2][PW + 1];

    const int k = blockIdx.z;
    const int a0 = blockIdx.x * BA;
    const int j0 = blockIdx.y * BJ;
    const long L = 2L * n - 1;
    const double *pk = p + (long)k * L + (n - 1);  // pk[m], m in [-(n-1), n-1]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wj = (wave >> 1) * 32;
    const int wa = (wave & 1) * 32;
    const int l16 = lane & 15;
    const int lk = lane >> 4;

    // global -> register staging for one K-step
    // U tile: BJ x BK = 1024 doubles, 4 per thread: row tid/4, cols (tid%4)*4..+3
    const int urow = tid >> 2;
    const int ucol = (tid & 3) * 4;
    double ureg[4];
    double preg;  // window entry tid (PW = 79 < 256)

    auto load_stage = [&](int b0) {
        const int j = j0 + urow;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = b0 + ucol + q;
            ureg[q] = (j < R_f && b < n) ? U[(long)j * n + b] : 0.0;
        }
        if (tid < PW) {
            const int lag = a0 - b0 - (BK - 1) + tid;
            preg = (lag > -n && lag < n) ? pk[lag] : 0.0;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            Us[buf][urow][ucol + q] = ureg[q];
        if (tid < PW)
            Ps[buf][tid] = preg;
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
                afr[x] = Us[buf][wj + x * 16 + l16][kk + lk];
#pragma unroll
            for (int y = 0; y < 2; ++y)
                bfr[y] = Ps[buf][(wa + y * 16 + l16) - (kk + lk) + (BK - 1)];
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

    double *Wk = W + (long)k * R_f * n;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int a = a0 + wa + y * 16 + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 + wj + x * 16 + lk + 4 * r;
                if (j < R_f && a < n)
                    Wk[(long)j * n + a] = acc[x][y][r];
            }
        }
}

}  // namespace

hipError_t launch_toeplitz_f64(const double *p, const double *U, double *W, int n, int R_f,
                               int R_N, hipStream_t stream)
{
    dim3 grid((n + BA - 1) / BA, (R_f + BJ - 1) / BJ, R_N);
    hipLaunchKernelGGL(toeplitz_f64_kernel, grid, dim3(256), 0, stream, p, U, W, n, R_f);
    return hipGetLastError();
}

}  // namespace tc
