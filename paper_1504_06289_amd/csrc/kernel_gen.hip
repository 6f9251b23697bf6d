// Kernel generation: the per-mode vectors of the rank-R_N canonical Newton
// kernel (Appendix 3, eq. sinc_general with the Galerkin vectors b(t_k) of
// eq. galten).  One thread per (term, lag); binary64 throughout.
//
//   p_k[m] = integral of exp(-t_k^2 s^2) over [(m-1/2)h, (m+1/2)h].
//
// Evaluation by regime (z = t |m| h is the scaled cell centre, q = t h / 2):
//   m = 0                    (sqrt(pi)/t) erf(q)
//   t^2 |m| h^2 <= 1/2       the integrand is nearly flat over the cell and an
//                            erf difference would cancel; use the midpoint
//                            Taylor series of exp(-s^2) in Hermite form,
//                            h exp(-z^2) sum_{k even} H_k(z) q^k / (k+1)!,
//                            whose terms are bounded by (2zq)^k/(k+1)! <= 2^-k/(k+1)!
//   otherwise                the cell ends differ by a factor e or more:
//                            difference of erfc (tail) or erf (near origin).
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kMaxTermsPerLaunch = 128;

struct NodeBlock {
    double t[kMaxTermsPerLaunch];
};

__device__ double cell_integral(double t, double h, long m)
{
    const double kSqrtPi = 1.7724538509055160273;
    const long am = m < 0 ? -m : m;
    const double q = 0.5 * t * h;
    if (am == 0)
        return kSqrtPi / t * erf(q);

    const double z = t * (double)am * h;
    if (2.0 * z * q <= 0.5) {
        // sum over even k of H_k(z) q^k / (k+1)!, Hermite recurrence
        // H_{k+1} = 2 z H_k - 2 k H_{k-1}
        double hkm1 = 1.0;       // H_0
        double hk = 2.0 * z;     // H_1
        double qk = 1.0;         // q^k / (k+1)! for k = 0
        double sum = 1.0;        // k = 0 term
        for (int k = 1; k < 30; ++k) {
            // advance qk to k
            qk *= q / (double)(k + 1);
            if ((k & 1) == 0)
                sum += hk * qk;    // hk holds H_k at step k
            double hn = 2.0 * z * hk - 2.0 * (double)k * hkm1;
            hkm1 = hk;
            hk = hn;
        }
        return h * exp(-z * z) * sum;
    }
    const double lo = t * ((double)am - 0.5) * h;
    const double hi = t * ((double)am + 0.5) * h;
    if (lo >= 0.5)
        return kSqrtPi / (2.0 * t) * (erfc(lo) - erfc(hi));
    return kSqrtPi / (2.0 * t) * (erf(hi) - erf(lo));
}

__global__ __launch_bounds__(256) void newton_kernel_gen(NodeBlock nodes, int nk, int n,
                                                          double h, double *__restrict__ p)
{
    const long L = 2L * n - 1;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nk * L)
        return;
    const int k = (int)(idx / L);
    const long mi = idx - (long)k * L;
    p[(long)k * L + mi] = cell_integral(nodes.t[k], h, mi - (n - 1));
}

}  // namespace

hipError_t launch_newton_kernel(const double *t_host, int R_N, int n, double h,
                                double *p_dev, hipStream_t stream)
{
    const long L = 2L * n - 1;
    for (int k0 = 0; k0 < R_N; k0 += kMaxTermsPerLaunch) {
        const int nk = R_N - k0 < kMaxTermsPerLaunch ? R_N - k0 : kMaxTermsPerLaunch;
        NodeBlock nodes;
        for (int k = 0; k < nk; ++k)
            nodes.t[k] = t_host[k0 + k];
        const long total = (long)nk * L;
        const unsigned blocks = (unsigned)((total + 255) / 256);
        hipLaunchKernelGGL(newton_kernel_gen, dim3(blocks), dim3(256), 0, stream, nodes, nk, n,
                           h, p_dev + (long)k0 * L);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace tc
