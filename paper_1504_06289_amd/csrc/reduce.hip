// Binary64 elementwise stages (memory-bound, one thread per matrix entry):
//
//   J[e] = sum_k c_k G1_k[e] G2_k[e] G3_k[e]
//       the Hadamard product across the three modes and the sum over the
//       kernel terms (Section 3.2, factorised TEI matrix with V = I);
//   D_k[e] = c_k S[e] Ga_k[e] Gb_k[e],  S = (Jbar + Jbar^T)/2
//       the adjoint weights of one mode (Ga, Gb = the other two modes).
//
// The sum over k runs in a fixed order (k = 0, 1, ...) in every thread, so the
// result is bitwise reproducible.  Loads are coalesced: consecutive threads
// take consecutive entries of each [R_f][R_f] slice.
#include "tc_internal.h"

namespace tc {

namespace {

__global__ __launch_bounds__(256) void hadamard_sum_kernel(const double *__restrict__ c,
                                                           const double *__restrict__ G0,
                                                           const double *__restrict__ G1,
                                                           const double *__restrict__ G2,
                                                           double *__restrict__ J, long F2,
                                                           int R_N)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= F2)
        return;
    double s = 0.0;
    for (int k = 0; k < R_N; ++k) {
        const long o = (long)k * F2 + e;
        s += c[k] * (G0[o] * G1[o] * G2[o]);
    }
    J[e] = s;
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
    const long F2 = (long)R_f * R_f;
    const unsigned blocks = (unsigned)((F2 + 255) / 256);
    hipLaunchKernelGGL(hadamard_sum_kernel, dim3(blocks), dim3(256), 0, stream, c, G0, G1, G2,
                       J, F2, R_N);
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
