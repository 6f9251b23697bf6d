// Term classes of the int8 FFT route and the low-rank Grams of smooth terms.
//
// A kernel term is
//   narrow  (class B >= 0) when |p_k[m]|, |m| > B <= 16, carry at most 2^-60
//           of sum_m |p_k[m]| (convolved directly inside the FFT kernel);
//   smooth  (class -2) when p_k is a polynomial of degree < kPolyRank in the
//           lag to within 2^-44 max|p_k| (least squares on the 2n-1 lags);
//   general (class -1) otherwise (FFT convolution and int8 Gram).
// For a smooth term the Toeplitz matrix is T_k = T_poly + E with T_poly[a][b]
// = P(a-b), P of degree < kPolyRank, |E| <= delta.  The rows and columns of
// T_poly lie in the span of the polynomials of degree < kPolyRank on the cell
// grid, with orthonormal basis Q (rows Q[r][a]), so T_poly = Q^T Q T_poly Q^T Q
// and
//   G_k = U T_k U^T ~ X S_k X^T,   X = U Q^T [R_f][R],   S_k = Q T_k Q^T [R][R],
// with |dG_ij| <= 2 (2n-1) delta |u_i|_2 |u_j|_2.  S_k comes from the half
// spectra of Q's rows and of the kernel embedding (Parseval); the Gram costs
// 2 R_f^2 R flops instead of an FFT convolution plus an int8 Gram over n.
//
// The basis is the orthonormal discrete Chebyshev (Gram) polynomials on the
// points x = 0..N-1, from the three-term recurrence
//   phi_0 = N^-1/2,  phi_1 = (3 / (N (N^2-1)))^1/2 z,  z = 2x - N + 1,
//   phi_{r+1} = A_r z phi_r - B_r phi_{r-1},
//   A_r = ((2r+1)(2r+3) / (N^2-(r+1)^2))^1/2 / (r+1),
//   B_r = r/(r+1) ((2r+3)(N^2-r^2) / ((2r-1)(N^2-(r+1)^2)))^1/2,
// evaluated point by point (coefficients from the host).
#include "tc_internal.h"

namespace tc {

namespace {

constexpr int RQ = kPolyRank;

__device__ inline void poly_eval(const PolyCoef &pc, int x, double (&ph)[RQ])
{
    const double z = 2.0 * x - pc.N + 1.0;
    ph[0] = pc.c0;
    ph[1] = pc.c1 * z;
#pragma unroll
    for (int r = 1; r < RQ - 1; ++r)
        ph[r + 1] = pc.A[r] * z * ph[r] - pc.B[r] * ph[r - 1];
}

constexpr int TCT = 256;        // threads of the term-class workgroup
constexpr int TCW = TCT / 64;   // its waves

// sum over the TCT threads of a block, for RQ values at once (result in every
// thread; fixed order)
__device__ inline void block_sum(double (&v)[RQ], double (*red)[RQ])
{
#pragma unroll
    for (int r = 0; r < RQ; ++r)
        for (int o = 32; o > 0; o >>= 1)
            v[r] += __shfl_xor(v[r], o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < RQ) {
        double w = 0.0;
#pragma unroll
        for (int r = 0; r < RQ; ++r)
            w = lane == r ? v[r] : w;
        red[wave][lane] = w;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
        double t = 0.0;
        for (int wv = 0; wv < TCW; ++wv)
            t += red[wv][r];
        v[r] = t;
    }
    __syncthreads();
}

__device__ inline double block_max(double v, double *redw)
{
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0)
        redw[threadIdx.x >> 6] = v;
    __syncthreads();
    v = redw[0];
    for (int wv = 1; wv < TCW; ++wv)
        v = fmax(v, redw[wv]);
    __syncthreads();
    return v;
}

// one workgroup (TCT threads) per term
__global__ __launch_bounds__(TCT) void term_class_kernel(const double *__restrict__ p, int n,
                                                         PolyCoef lag, int smooth_ok,
                                                         int *__restrict__ cls)
{
    __shared__ double red[TCW][RQ];
    __shared__ double redw[TCW];
    __shared__ double part[2][TCW];
    __shared__ double cA[RQ], cB[RQ];
    const int k = blockIdx.x;
    const int tid = threadIdx.x;
    const double *pk = p + (long)k * (2L * n - 1) + (n - 1);  // pk[lag]
    const int L = 2 * n - 1;

    // narrow: smallest B <= min(16, n-1) with the tail beyond B below 2^-60 of the sum
    const int cap = n - 1 < kBandMax ? n - 1 : kBandMax;
    double tot = 0.0, out = 0.0;
    for (int m = tid; m < n; m += TCT) {
        const double a = fabs(pk[m]) + (m > 0 ? fabs(pk[-m]) : 0.0);
        tot += a;
        if (m > cap)
            out += a;
    }
    for (int o = 32; o > 0; o >>= 1) {
        tot += __shfl_xor(tot, o);
        out += __shfl_xor(out, o);
    }
    if ((tid & 63) == 0) {
        part[0][tid >> 6] = tot;
        part[1][tid >> 6] = out;
    }
    __syncthreads();
    tot = 0.0;
    out = 0.0;
    for (int wv = 0; wv < TCW; ++wv) {
        tot += part[0][wv];
        out += part[1][wv];
    }
    const double thr = ldexp(tot, -60);
    if (out <= thr) {
        if (tid == 0) {
            int B = cap;
            double tail = out;
            while (B > 0) {
                const double add = fabs(pk[B]) + fabs(pk[-B]);
                if (tail + add > thr)
                    break;
                tail += add;
                --B;
            }
            cls[k] = B;
        }
        return;  // uniform: every thread saw the same out and thr
    }
    if (!smooth_ok) {
        if (tid == 0)
            cls[k] = -1;
        return;
    }

    // smooth: least-squares polynomial fit on the lags x = m + n - 1 = 0..L-1.
    // The basis values are produced by the recurrence as they are consumed
    // (two live values), with its coefficients in LDS.
    if (tid < RQ) {
        cA[tid] = lag.A[tid];
        cB[tid] = lag.B[tid];
    }
    __syncthreads();
    double c[RQ];
#pragma unroll
    for (int r = 0; r < RQ; ++r)
        c[r] = 0.0;
    double pmax = 0.0;
    for (int x = tid; x < L; x += TCT) {
        const double v = pk[x - (n - 1)];
        pmax = fmax(pmax, fabs(v));
        const double z = 2.0 * x - lag.N + 1.0;
        double f0 = lag.c0, f1 = lag.c1 * z;
        c[0] = fma(f0, v, c[0]);
        c[1] = fma(f1, v, c[1]);
#pragma unroll
        for (int r = 1; r < RQ - 1; ++r) {
            const double f2 = cA[r] * z * f1 - cB[r] * f0;
            c[r + 1] = fma(f2, v, c[r + 1]);
            f0 = f1;
            f1 = f2;
        }
    }
    block_sum(c, red);
    pmax = block_max(pmax, redw);
    double res = 0.0;
    for (int x = tid; x < L; x += TCT) {
        const double z = 2.0 * x - lag.N + 1.0;
        double f0 = lag.c0, f1 = lag.c1 * z;
        double fit = fma(c[1], f1, c[0] * f0);
#pragma unroll
        for (int r = 1; r < RQ - 1; ++r) {
            const double f2 = cA[r] * z * f1 - cB[r] * f0;
            fit = fma(c[r + 1], f2, fit);
            f0 = f1;
            f1 = f2;
        }
        res = fmax(res, fabs(pk[x - (n - 1)] - fit));
    }
    res = block_max(res, redw);
    if (tid == 0)
        cls[k] = (pmax > 0.0 && res <= ldexp(pmax, -44)) ? -2 : -1;
}

// Q[r][a] = phi_r(a) on the cell grid
__global__ __launch_bounds__(256) void poly_rows_kernel(int n, PolyCoef cell,
                                                        double *__restrict__ Q)
{
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a >= n)
        return;
    double ph[RQ];
    poly_eval(cell, a, ph);
#pragma unroll
    for (int r = 0; r < RQ; ++r)
        Q[(long)r * n + a] = ph[r];
}

// X[i][r] = sum_a U[i][a] Q[r][a]: workgroup (row block, cell split) takes 32
// rows of U and one of PKS ranges of cells, in chunks of 64 cells staged in LDS
// with the matching columns of Q; each thread accumulates 4 outputs.  The
// splits are added in a fixed order by poly_project_reduce.
constexpr int PRT = 32, PKC = 64, PKS = kProjectSplit;
__global__ __launch_bounds__(256) void poly_project_kernel(const double *__restrict__ U, int n,
                                                           int R_f, const double *__restrict__ Q,
                                                           double *__restrict__ part)
{
    __shared__ double Us[PRT][PKC + 1];
    __shared__ double Qs[RQ][PKC + 1];
    const int i0 = blockIdx.x * PRT;
    const int ks = blockIdx.y;
    const int c0 = (int)((long)ks * n / PKS), c1 = (int)((long)(ks + 1) * n / PKS);
    const int tid = threadIdx.x;
    const int row = tid >> 3, r0 = (tid & 7) * 4;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int a0 = c0; a0 < c1; a0 += PKC) {
        for (int e = tid; e < PRT * PKC; e += 256) {
            const int rr = e / PKC, aa = e % PKC;
            Us[rr][aa] = (i0 + rr < R_f && a0 + aa < c1) ? U[(long)(i0 + rr) * n + a0 + aa] : 0.0;
        }
        for (int e = tid; e < RQ * PKC; e += 256) {
            const int rr = e / PKC, aa = e % PKC;
            Qs[rr][aa] = a0 + aa < c1 ? Q[(long)rr * n + a0 + aa] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int aa = 0; aa < PKC; ++aa) {
            const double u = Us[row][aa];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[q] = fma(u, Qs[r0 + q][aa], acc[q]);
        }
        __syncthreads();
    }
    if (i0 + row < R_f) {
        double *out = part + ((long)ks * R_f + i0 + row) * RQ + r0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            out[q] = acc[q];
    }
}

__global__ __launch_bounds__(256) void poly_project_reduce(const double *__restrict__ part,
                                                           int R_f, double *__restrict__ X)
{
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)R_f * RQ)
        return;
    double v = 0.0;
    for (int ks = 0; ks < PKS; ++ks)
        v += part[(long)ks * R_f * RQ + e];
    X[e] = v;
}

// S_k = Q T_k Q^T for the smooth terms from the half spectra (real signals of
// length N = 2M, zero-padded, so the circular product is the aperiodic one on
// the cells):  S_k[r][s] = (1/N) sum_{w=0}^{M} m_w Re(conj(Qh_r(w)) Ch_k(w) Qh_s(w)),
// m_0 = m_M = 1, else 2.  Workgroup (k, split) sums one range of frequencies in
// chunks staged in LDS; its four waves take every fourth frequency and each
// thread a 4 x 4 block of (r, s), and the waves' sums are added in LDS.
// spectral_reduce adds the splits in a fixed order (one thread per entry).
constexpr int SW = 64;  // frequencies per LDS chunk
__global__ __launch_bounds__(256) void spectral_gram_kernel(const double2 *__restrict__ Qspec,
                                                            const double2 *__restrict__ Cspec,
                                                            int M, const int *__restrict__ cls,
                                                            double *__restrict__ partial)
{
    __shared__ double2 Qs[RQ][SW + 1];
    __shared__ double2 Cs[SW];
    __shared__ double red[4][RQ * RQ / 2];
    const int k = blockIdx.x, sp = blockIdx.y;
    if (cls[k] != -2)
        return;
    const int tot = M + 1;
    const int w0 = (int)((long)sp * tot / gridDim.y);
    const int w1 = (int)((long)(sp + 1) * tot / gridDim.y);
    const int tid = threadIdx.x;
    const int grp = tid >> 6, t64 = tid & 63;
    const int rb = (t64 >> 3) * 4, sb = (t64 & 7) * 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            acc[a][b] = 0.0;
    const double2 *Ck = Cspec + (long)k * (M + 1);
    for (int wb = w0; wb < w1; wb += SW) {
        const int cnt = w1 - wb < SW ? w1 - wb : SW;
        for (int e = tid; e < RQ * SW; e += 256) {
            const int rr = e / SW, ww = e % SW;
            Qs[rr][ww] = ww < cnt ? Qspec[(long)rr * (M + 1) + wb + ww] : make_double2(0.0, 0.0);
        }
        if (tid < SW)
            Cs[tid] = tid < cnt ? Ck[wb + tid] : make_double2(0.0, 0.0);
        __syncthreads();
        for (int ww = grp; ww < cnt; ww += 4) {
            const int w = wb + ww;
            const double m = (w == 0 || w == M) ? 1.0 : 2.0;
            const double2 c = Cs[ww];
            double2 ar[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double2 q = Qs[rb + a][ww];
                // m conj(q) c
                ar[a] = make_double2(m * (q.x * c.x + q.y * c.y), m * (q.x * c.y - q.y * c.x));
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double2 qs = Qs[sb + b][ww];
#pragma unroll
                for (int a = 0; a < 4; ++a)
                    acc[a][b] = fma(ar[a].x, qs.x, fma(-ar[a].y, qs.y, acc[a][b]));
            }
        }
        __syncthreads();
    }
    // add the four waves' sums: two halves of the 32 x 32 block through LDS
    double *out = partial + ((long)k * gridDim.y + sp) * RQ * RQ;
    for (int half = 0; half < 2; ++half) {
        const bool mine = (rb >= 16 * half) && (rb < 16 * half + 16);
        if (mine) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    red[grp][(rb - 16 * half + a) * RQ + sb + b] = acc[a][b];
        }
        __syncthreads();
        for (int e = tid; e < RQ * RQ / 2; e += 256)
            out[16 * half * RQ + e] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void spectral_reduce_kernel(const double *__restrict__ partial,
                                                              const int *__restrict__ cls,
                                                              int nsplit, double inv_n,
                                                              double *__restrict__ S)
{
    const int k = blockIdx.x;
    if (cls[k] != -2)
        return;
    for (int e = blockIdx.y * 256 + threadIdx.x; e < RQ * RQ; e += 256 * gridDim.y) {
        double v = 0.0;
        for (int sp = 0; sp < nsplit; ++sp)
            v += partial[((long)k * nsplit + sp) * RQ * RQ + e];
        S[(long)k * RQ * RQ + e] = v * inv_n;
    }
}

// G_k = X S_k X^T for the smooth terms: upper-triangle 64 x 64 tiles,
// mirrored.  A workgroup stages the row blocks X_i and X_j (64 x RQ) and S_k
// in LDS, forms Y_i = X_i S_k (each wave 16 rows) into X_i's place, then
// contracts Y_i X_j^T with four waves of 32 x 32 (2 x 2 blocks of 16 x 16).
// Both products run on v_mfma_f64_16x16x4_f64 (lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; result lane l holds D[l/16 + 4r][l%16]).
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int LT = 64;
static_assert(LT == 4 * 16 && RQ % 16 == 0, "four waves of 16 rows form Y_i");
__global__ __launch_bounds__(256) void lowrank_gram_kernel(const double *__restrict__ X,
                                                           const double *__restrict__ S,
                                                           const int *__restrict__ cls,
                                                           double *__restrict__ G, int R_f,
                                                           int ntiles, int mirror)
{
    __shared__ double Ys[LT][RQ + 1];  // X_i, then Y_i
    __shared__ double Xs[LT][RQ + 1];  // X_j
    __shared__ double Ss[RQ][RQ + 1];
    const int k = blockIdx.y;
    if (cls[k] != -2)
        return;
    int t = blockIdx.x;
    int ti = 0;
    while (t >= ntiles - ti) {
        t -= ntiles - ti;
        ++ti;
    }
    const int tj = ti + t;
    const int i0 = ti * LT, j0 = tj * LT;
    const int tid = threadIdx.x;
    const double *Sk = S + (long)k * RQ * RQ;
    for (int e = tid; e < LT * RQ; e += 256) {
        const int row = e / RQ, r = e % RQ;
        Ys[row][r] = i0 + row < R_f ? X[(long)(i0 + row) * RQ + r] : 0.0;
        Xs[row][r] = j0 + row < R_f ? X[(long)(j0 + row) * RQ + r] : 0.0;
    }
    for (int e = tid; e < RQ * RQ; e += 256)
        Ss[e / RQ][e % RQ] = Sk[e];
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int l16 = lane & 15, lk = lane >> 4;

    // Y_i rows 16 wave .. 16 wave + 15: Y[i][s] = sum_r X[i][r] S_k[r][s]
    {
        f64x4 ay[RQ / 16];
#pragma unroll
        for (int y = 0; y < RQ / 16; ++y)
            ay[y] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < RQ; kk += 4) {
            const double afr = Ys[16 * wave + l16][kk + lk];
#pragma unroll
            for (int y = 0; y < RQ / 16; ++y)
                ay[y] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr, Ss[kk + lk][16 * y + l16],
                                                             ay[y], 0, 0, 0);
        }
        __syncthreads();  // every wave has read its rows of X_i
#pragma unroll
        for (int y = 0; y < RQ / 16; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Ys[16 * wave + lk + 4 * r][16 * y + l16] = ay[y][r];
        __syncthreads();
    }

    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    f64x4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
            acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < RQ; kk += 4) {
        double afr[2], bfr[2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
            afr[x] = Ys[wi + 16 * x + l16][kk + lk];
#pragma unroll
        for (int y = 0; y < 2; ++y)
            bfr[y] = Xs[wj + 16 * y + l16][kk + lk];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[x], bfr[y], acc[x][y], 0, 0, 0);
    }
    double *Gk = G + (long)k * R_f * R_f;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int j = j0 + wj + 16 * y + l16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wi + 16 * x + lk + 4 * r;
                if (i < R_f && j < R_f && i <= j) {
                    Gk[(long)i * R_f + j] = acc[x][y][r];
                    if (mirror)
                        Gk[(long)j * R_f + i] = acc[x][y][r];
                }
            }
        }
}

}  // namespace

PolyCoef poly_coef(int N)
{
    PolyCoef pc{};
    const double Nd = N;
    pc.N = Nd;
    pc.c0 = 1.0 / std::sqrt(Nd);
    pc.c1 = std::sqrt(3.0 / (Nd * (Nd * Nd - 1.0)));
    for (int r = 1; r < kPolyRank - 1; ++r) {
        const double rr = r;
        const double den = Nd * Nd - (rr + 1.0) * (rr + 1.0);
        pc.A[r] = std::sqrt((2.0 * rr + 1.0) * (2.0 * rr + 3.0) / den) / (rr + 1.0);
        pc.B[r] = rr / (rr + 1.0) *
                  std::sqrt((2.0 * rr + 3.0) * (Nd * Nd - rr * rr) / ((2.0 * rr - 1.0) * den));
    }
    return pc;
}

bool smooth_terms_supported(int n) { return n >= kPolyMinN; }

hipError_t launch_term_class(const double *p, int n, int R_N, int *cls, hipStream_t stream)
{
    const int smooth = smooth_terms_supported(n) ? 1 : 0;
    const PolyCoef lag = smooth ? poly_coef(2 * n - 1) : PolyCoef{};
    hipLaunchKernelGGL(term_class_kernel, dim3(R_N), dim3(TCT), 0, stream, p, n, lag, smooth, cls);
    return hipGetLastError();
}


hipError_t launch_poly_rows(int n, double *Q, hipStream_t stream)
{
    hipLaunchKernelGGL(poly_rows_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n,
                       poly_coef(n), Q);
    return hipGetLastError();
}

hipError_t launch_poly_project(const double *U, int n, int R_f, const double *Q, double *part,
                               double *X, hipStream_t stream)
{
    // on the binary64 matrix cores (X = U Q^T, contraction split into fixed
    // slices summed in order) where its slices fit part: the vector form below
    // is bound by LDS instruction issue (five 8-byte reads per four FMAs)
    if (gemm_splits(R_f, RQ, n) <= PKS)
        return launch_gemm_f64(false, U, Q, X, R_f, RQ, n, part, stream);
    hipLaunchKernelGGL(poly_project_kernel, dim3((R_f + PRT - 1) / PRT, PKS), dim3(256), 0,
                       stream, U, n, R_f, Q, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(poly_project_reduce, dim3((unsigned)(((long)R_f * RQ + 255) / 256)),
                       dim3(256), 0, stream, part, R_f, X);
    return hipGetLastError();
}

hipError_t launch_spectral_gram(const double2 *Qspec, const double2 *Cspec, int N, int R_N,
                                const int *cls, double *partial, double *S, hipStream_t stream)
{
    const int M = N / 2;
    hipLaunchKernelGGL(spectral_gram_kernel, dim3(R_N, kSpectralSplit), dim3(256), 0, stream,
                       Qspec, Cspec, M, cls, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(spectral_reduce_kernel, dim3(R_N, RQ * RQ / 256), dim3(256), 0, stream,
                       partial, cls, kSpectralSplit, 1.0 / (double)N, S);
    return hipGetLastError();
}

hipError_t launch_lowrank_gram(const double *X, const double *S, const int *cls, double *G,
                               int R_f, int R_N, bool mirror, hipStream_t stream)
{
    const int nt = (R_f + LT - 1) / LT;
    dim3 grid(nt * (nt + 1) / 2, R_N);
    hipLaunchKernelGGL(lowrank_gram_kernel, grid, dim3(256), 0, stream, X, S, cls, G, R_f, nt,
                       (int)mirror);
    return hipGetLastError();
}

}  // namespace tc
