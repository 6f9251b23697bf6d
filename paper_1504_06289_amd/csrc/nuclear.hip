// Tables of the nuclear potential matrix (Section 3.3): the master kernel
// shifted to each nucleus and weighted by its charge.  Term t = alpha R_N + q
// has weight -Z_alpha c_q / (h1 h2 h3) (c_q = a_q h1 h2 h3, so the weight is
// -Z_alpha a_q) and, along mode l, the shift pos[alpha][l]; the 1D matrices
// U^l diag(p^l_q[. - pos]) U^l^T come from the diagonal form of the Gram
// kernel and the product over modes and the sum over t from the Hadamard sum.
//
// The charges and cells arrive as kernel arguments (a chunk of nuclei per
// launch), so the call moves no host memory and stays stream-ordered.
#include "tc_internal.h"

namespace tc {

namespace {

__global__ __launch_bounds__(256) void nuclear_table_kernel(NuclearChunk ch,
                                                            const double *__restrict__ c,
                                                            int R_N, int M, double inv_vol,
                                                            int *__restrict__ shift,
                                                            double *__restrict__ cw)
{
    const int a = blockIdx.x;  // nucleus within the chunk
    const int alpha = ch.base + a;
    for (int q = threadIdx.x; q < R_N; q += blockDim.x)
        cw[(long)alpha * R_N + q] = -ch.Z[a] * c[q] * inv_vol;
    if (threadIdx.x < 3)
        shift[threadIdx.x * M + alpha] = ch.pos[threadIdx.x][a];
}

}  // namespace

hipError_t launch_nuclear_table(const NuclearChunk &ch, const double *c, int R_N, int M,
                                double inv_vol, int *shift, double *cw, hipStream_t st)
{
    hipLaunchKernelGGL(nuclear_table_kernel, dim3(ch.count), dim3(256), 0, st, ch, c, R_N, M,
                       inv_vol, shift, cw);
    return hipGetLastError();
}

}  // namespace tc
