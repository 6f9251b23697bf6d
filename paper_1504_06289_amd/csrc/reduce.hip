// Binary64 elementwise stages (memory-bound):
//
//   J[e] = sum_k c_k G1_k[e] G2_k[e] G3_k[e]
//       the Hadamard product across the three modes and the sum over the
//       kernel terms (Section 3.2, factorised TEI matrix with V = I).  The
//       Grams are symmetric, so only the upper triangle is read: one
//       workgroup per 32 x 32 tile (I <= J), written to (I, J) and, through
//       LDS, transposed to (J, I); on diagonal tiles the entries with i > j
//       are the mirrors of those with i < j, so J is exactly symmetric;
//   D_k[e] = c_k S[e] Ga_k[e] Gb_k[e],  S = (Jbar + Jbar^T)/2
//       the adjoint weights of one mode (Ga, Gb = the other two modes), one
//       thread per entry.
//
// The sum over k runs in a fixed order (k = 0, 1, ...) for every entry, so the
// result is bitwise reproducible.  Loads are coalesced: consecutive threads
// take consecutive entries of each [R_f][R_f] slice.
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int HT = 32;  // Hadamard tile edge

// 256 threads, each 4 entries of the tile: rows (tid >> 4) + 16 q, q = 0, 1,
// columns 2 (tid & 15) + {0, 1} (one 16-byte load when VEC2)
template <bool VEC2>
__global__ __launch_bounds__(256) void hadamard_sum_kernel(const double *__restrict__ c,
                                                           const double *__restrict__ G0,
                                                           const double *__restrict__ G1,
                                                           const double *__restrict__ G2,
                                                           double *__restrict__ J, int R_f,
                                                           int nt, int R_N)
{
    __shared__ double tile[HT][HT + 1];
    int t = blockIdx.x, ti = 0;
    while (t >= nt - ti) {
        t -= nt - ti;
        ++ti;
    }
    const int tj = ti + t;
    const int i0 = ti * HT, j0 = tj * HT;
    const int tid = threadIdx.x;
    const int cc = 2 * (tid & 15), r0 = tid >> 4;
    const long F2 = (long)R_f * R_f;
    double s[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    bool in[2][2];
    long off[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int i = i0 + r0 + 16 * q, j = j0 + cc;
        in[q][0] = i < R_f && j < R_f;
        in[q][1] = i < R_f && j + 1 < R_f;
        off[q] = (long)i * R_f + j;
    }
#pragma unroll 4
    for (int k = 0; k < R_N; ++k) {
        const double ck = c[k];
        const long o = (long)k * F2;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            double a[3][2];
            if (VEC2 && in[q][1]) {
                const double2 x = *(const double2 *)(G0 + o + off[q]);
                const double2 y = *(const double2 *)(G1 + o + off[q]);
                const double2 z = *(const double2 *)(G2 + o + off[q]);
                a[0][0] = x.x; a[0][1] = x.y;
                a[1][0] = y.x; a[1][1] = y.y;
                a[2][0] = z.x; a[2][1] = z.y;
            } else {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    a[0][e] = in[q][e] ? G0[o + off[q] + e] : 0.0;
                    a[1][e] = in[q][e] ? G1[o + off[q] + e] : 0.0;
                    a[2][e] = in[q][e] ? G2[o + off[q] + e] : 0.0;
                }
            }
#pragma unroll
            for (int e = 0; e < 2; ++e)
                s[q][e] += ck * (a[0][e] * a[1][e] * a[2][e]);
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        tile[r0 + 16 * q][cc] = s[q][0];
        tile[r0 + 16 * q][cc + 1] = s[q][1];
    }
    __syncthreads();
    // (I, J): on a diagonal tile the lower entries mirror the upper ones
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int r = r0 + 16 * q, col = cc + e;
            if (in[q][e])
                J[off[q] + e] = (ti == tj && r > col) ? tile[col][r] : tile[r][col];
        }
    if (ti == tj)
        return;
    // (J, I): row j0 + r of J holds column r of the tile
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int r = r0 + 16 * q, col = cc + e;  // output row j0 + r, column i0 + col
            if (j0 + r < R_f && i0 + col < R_f)
                J[(long)(j0 + r) * R_f + i0 + col] = tile[col][r];
        }
}

__global__ __launch_bounds__(256) void adjoint_d_kernel(const double *__restrict__ c,
                                                        const double *__restrict__ Jbar,
                                                        const double *__restrict__ Ga,
                                                        const double *__restrict__ Gb,
                                                        double *__restrict__ D, int R_f, int R_N)
{
    const long F2 = (long)R_f * R_f;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= F2)
        return;
    const long i = e / R_f, j = e - i * R_f;
    const double s = 0.5 * (Jbar[e] + Jbar[j * R_f + i]);
    for (int k = 0; k < R_N; ++k) {
        const long o = (long)k * F2 + e;
        D[o] = c[k] * s * (Ga[o] * Gb[o]);
    }
}

}  // namespace

hipError_t launch_hadamard_sum(const double *c, const double *G0, const double *G1,
                               const double *G2, double *J, int R_f, int R_N,
                               hipStream_t stream)
{
    const int nt = (R_f + HT - 1) / HT;
    const unsigned blocks = (unsigned)(nt * (nt + 1) / 2);
    // 16-byte loads need even row lengths (and 16-byte aligned Grams)
    const bool vec2 = R_f % 2 == 0 && ((uintptr_t)G0 | (uintptr_t)G1 | (uintptr_t)G2) % 16 == 0;
    if (vec2)
        hipLaunchKernelGGL(hadamard_sum_kernel<true>, dim3(blocks), dim3(256), 0, stream, c, G0,
                           G1, G2, J, R_f, nt, R_N);
    else
        hipLaunchKernelGGL(hadamard_sum_kernel<false>, dim3(blocks), dim3(256), 0, stream, c, G0,
                           G1, G2, J, R_f, nt, R_N);
    return hipGetLastError();
}

hipError_t launch_adjoint_d(const double *c, const double *Jbar, const double *Ga,
                            const double *Gb, double *D, int R_f, int R_N, hipStream_t stream)
{
    const long F2 = (long)R_f * R_f;
    const unsigned blocks = (unsigned)((F2 + 255) / 256);
    hipLaunchKernelGGL(adjoint_d_kernel, dim3(blocks), dim3(256), 0, stream, c, Jbar, Ga, Gb, D,
                       R_f, R_N);
    return hipGetLastError();
}

}  // namespace tc
