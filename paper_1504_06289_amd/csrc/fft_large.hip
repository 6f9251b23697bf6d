// FFT route for grids longer than the LDS-resident route (4096 < n <= 65536):
// the same aperiodic convolution W_k[j] = p_k *_n u_j through a circulant
// embedding of length N = 2^ceil(log2(2n-1)) (16384 .. 131072), computed with
// binary64 transforms that are too long for one workgroup's LDS.
//
// Two real sequences share one complex transform: z_q = u_{2q} 2^-E_{2q} +
// i u_{2q+1} 2^-E_{2q+1} (the kernel vector is real, so p *_N z_q is the pair
// of convolutions of the scaled rows, and the scales are exact).  Each row is
// scaled by the power of two that brings its maximum to [1/2, 1): the
// rounding error of a transform is spread over the whole sequence in
// proportion to its norm, so without the scaling a row paired with a much
// larger one would carry the larger row's absolute error (measured: 9e-12
// relative to the smaller row's maximum for a ratio of 4e4).
// Each length-N transform is split into N = N1 N2 (four-step): with
// m = m1 + N1 m2 and frequency f = f2 + N2 f1,
//
//   X[f2 + N2 f1] = sum_m1 w_N1^(m1 f1) w_N^(m1 f2) sum_m2 x[m1 + N1 m2] w_N2^(m2 f2),
//
// so a sequence stored as N2 rows of N1 entries (natural order, entry m at
// m) is transformed by a column pass (length-N2 DFTs of the columns m1, then
// the twiddle w_N^(m1 f2)) and a row pass (length-N1 DFTs of the rows f2).
// The spectrum stays in that "transposed" order (entry f2 N1 + f1 holds
// X[f2 + N2 f1]); the pointwise products pair equal positions, and the
// inverse runs the passes in the reverse order (row pass, conjugate twiddle,
// column pass), which returns the natural order.  Each pass keeps a block of
// rows or columns in LDS and transforms them with radix-4 Stockham passes
// (one radix-2 pass when log2 of the length is odd).
//
// Kernels (T = 256 threads):
//   lfft_col_fwd   columns of the zero-padded pairs of U rows, or of the
//                  circulant embeddings of the p_k, forward, times the twiddle
//   lfft_row       rows, forward in place, or inverse of the spectral product
//                  C_k . Z_q into a scratch sequence
//   lfft_col_inv   columns of that scratch (conjugate twiddle first), inverse,
//                  1/N, the first n samples written as W_k[2q], W_k[2q+1]
#include "tc_internal.h"

namespace tc {

namespace {

typedef double2 cplx;

constexpr int kT = 256;       // threads per workgroup
constexpr int kCB = 16;       // columns per column-pass workgroup
constexpr int kLdsEntries = 4096;  // complex entries of LDS per workgroup (64 KB)

__device__ inline cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline cplx cmul(cplx a, cplx b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline cplx cconj(cplx a) { return make_double2(a.x, -a.y); }

// e^(SIGN 2 pi i t / N) from the table twN[t] = e^(-2 pi i t / N)
template <int SIGN> __device__ inline cplx tw(const cplx *__restrict__ twN, long t, int N)
{
    const cplx x = twN[t & (N - 1)];
    return SIGN > 0 ? cconj(x) : x;
}

// LDS position of entry i of sequence b (an XOR permutation inside aligned
// groups of 16 spreads the strided accesses of the passes over the banks)
template <int L> __device__ inline int lpos(int b, int i) { return b * L + (i ^ ((i >> 4) & 15)); }

// In-place Stockham FFT of B sequences of length L held in LDS (sequence b at
// lpos<L>(b, .)), direction SIGN (-1 forward, +1 inverse, unscaled).  A pass
// of radix R with sub-transform size Ns reads entries j + r L/R, multiplies
// entry r by e^(SIGN 2 pi i (j mod Ns) r / (Ns R)), does an R-point DFT and
// writes entries (j/Ns) Ns R + (j mod Ns) + r Ns.
template <int L, int R, int SIGN>
__device__ inline void stockham_pass(cplx *buf, int B, int Ns, const cplx *__restrict__ twN,
                                     int N)
{
    constexpr int NB = L / R;  // butterflies per sequence
    const int total = B * NB;
    constexpr int MAXPER = (kLdsEntries / R + kT - 1) / kT;
    cplx v[MAXPER][R];
#pragma unroll
    for (int s = 0; s < MAXPER; ++s) {
        const int idx = threadIdx.x + kT * s;
        if (idx < total) {
            const int b = idx / NB, j = idx % NB;
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[s][r] = buf[lpos<L>(b, j + r * NB)];
            if (Ns > 1) {
                const int jm = j % Ns;
                const long step = (long)jm * (N / (Ns * R));
#pragma unroll
                for (int r = 1; r < R; ++r)
                    v[s][r] = cmul(v[s][r], tw<SIGN>(twN, step * r, N));
            }
            if (R == 4) {
                const cplx a0 = cadd(v[s][0], v[s][2]), a1 = csub(v[s][0], v[s][2]);
                const cplx b0 = cadd(v[s][1], v[s][3]);
                const cplx d = csub(v[s][1], v[s][3]);
                // SIGN i d
                const cplx b1 = SIGN > 0 ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);
                v[s][0] = cadd(a0, b0);
                v[s][2] = csub(a0, b0);
                v[s][1] = cadd(a1, b1);
                v[s][3] = csub(a1, b1);
            } else {
                const cplx a = v[s][0], c = v[s][1];
                v[s][0] = cadd(a, c);
                v[s][1] = csub(a, c);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < MAXPER; ++s) {
        const int idx = threadIdx.x + kT * s;
        if (idx < total) {
            const int b = idx / NB, j = idx % NB;
            const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
            for (int r = 0; r < R; ++r)
                buf[lpos<L>(b, base + r * Ns)] = v[s][r];
        }
    }
    __syncthreads();
}

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

template <int L, int SIGN>
__device__ inline void lds_fft(cplx *buf, int B, const cplx *__restrict__ twN, int N)
{
    constexpr int LOG = ilog2c(L);
    int Ns = 1;
#pragma unroll 1
    for (int p = 0; p < LOG / 2; ++p) {
        stockham_pass<L, 4, SIGN>(buf, B, Ns, twN, N);
        Ns *= 4;
    }
    if (LOG % 2)
        stockham_pass<L, 2, SIGN>(buf, B, Ns, twN, N);
}

// Forward column pass.  Sequence s (blockIdx.y) of the batch is, in natural
// order, either the pair z_s = X[2s] + i X[2s+1] of zero-padded rows of X
// [rows][len] (p == nullptr), or the circulant embedding of kernel vector s of
// p [R][2n-1] (X == nullptr): c[t] = p[t + n - 1] for t < n, c[N - m] =
// p[n - 1 - m] for 1 <= m < n, 0 otherwise.  Columns c0 .. c0 + kCB - 1
// (c0 = blockIdx.x kCB) of the N2 x N1 arrangement are transformed over their
// N2 entries and multiplied by w_N^(m1 f2); output: out[s][f2 N1 + m1].
template <int N2>
__global__ __launch_bounds__(kT) void lfft_col_fwd(const double *__restrict__ X,
                                                   const int *__restrict__ E, int rows,
                                                   int len, const double *__restrict__ p,
                                                   int n, const cplx *__restrict__ twN, int N,
                                                   int N1, cplx *__restrict__ out)
{
    __shared__ cplx buf[kCB * N2];
    const int s = blockIdx.y;
    const int c0 = blockIdx.x * kCB;
    const int e0 = X ? -E[2 * s] : 0;
    const int e1 = X && 2 * s + 1 < rows ? -E[2 * s + 1] : 0;
    for (int e = threadIdx.x; e < kCB * N2; e += kT) {
        const int cb = e % kCB, m2 = e / kCB;
        const long m = c0 + cb + (long)N1 * m2;
        cplx z = make_double2(0.0, 0.0);
        if (p) {
            const double *pk = p + (long)s * (2 * n - 1);
            if (m < n)
                z.x = pk[m + n - 1];
            else if (m > N - n)
                z.x = pk[n - 1 - (N - m)];
        } else if (m < len) {
            const int r0 = 2 * s, r1 = 2 * s + 1;
            z.x = ldexp(X[(long)r0 * len + m], e0);
            if (r1 < rows)
                z.y = ldexp(X[(long)r1 * len + m], e1);
        }
        buf[lpos<N2>(cb, m2)] = z;
    }
    __syncthreads();
    lds_fft<N2, -1>(buf, kCB, twN, N);
    cplx *o = out + (long)s * N;
    for (int e = threadIdx.x; e < kCB * N2; e += kT) {
        const int cb = e % kCB, f2 = e / kCB;
        const int m1 = c0 + cb;
        o[(long)f2 * N1 + m1] = cmul(buf[lpos<N2>(cb, f2)], tw<-1>(twN, (long)m1 * f2, N));
    }
}

// Row pass over RB rows (f2 = blockIdx.x RB ..) of length N1.
//   forward (SIGN = -1): in place on spec[s] (s = blockIdx.y);
//   inverse (SIGN = +1): the product C[k0 + kk] . Z[q] (q = blockIdx.y,
//   kk = blockIdx.z) transformed into out[kk][q], each entry then multiplied
//   by w_N^(-m1 f2).
template <int N1, int SIGN>
__global__ __launch_bounds__(kT) void lfft_row(const cplx *__restrict__ C, int k0,
                                               const cplx *__restrict__ Z, int P,
                                               const cplx *__restrict__ twN, int N,
                                               cplx *__restrict__ spec)
{
    constexpr int RB = kLdsEntries / N1;
    __shared__ cplx buf[RB * N1];
    const int f20 = blockIdx.x * RB;
    const int q = blockIdx.y;
    if (SIGN < 0) {
        cplx *row = spec + (long)q * N + (long)f20 * N1;
        for (int e = threadIdx.x; e < RB * N1; e += kT)
            buf[lpos<N1>(e / N1, e % N1)] = row[e];
    } else {
        const int kk = blockIdx.z;
        const cplx *c = C + (long)(k0 + kk) * N + (long)f20 * N1;
        const cplx *z = Z + (long)q * N + (long)f20 * N1;
        for (int e = threadIdx.x; e < RB * N1; e += kT)
            buf[lpos<N1>(e / N1, e % N1)] = cmul(c[e], z[e]);
    }
    __syncthreads();
    lds_fft<N1, SIGN>(buf, RB, twN, N);
    if (SIGN < 0) {
        cplx *row = spec + (long)q * N + (long)f20 * N1;
        for (int e = threadIdx.x; e < RB * N1; e += kT)
            row[e] = buf[lpos<N1>(e / N1, e % N1)];
    } else {
        cplx *o = spec + ((long)blockIdx.z * P + q) * N + (long)f20 * N1;
        for (int e = threadIdx.x; e < RB * N1; e += kT) {
            const int f2 = f20 + e / N1, m1 = e % N1;
            o[e] = cmul(buf[lpos<N1>(e / N1, m1)], tw<+1>(twN, (long)m1 * f2, N));
        }
    }
}

// Inverse column pass of tmp[kk][q] (kk = blockIdx.z, q = blockIdx.y): the
// columns c0 .. c0 + kCB - 1 over their N2 entries, scaled by 1/N; natural
// position m = m1 + N1 m2 < n goes to W[k0 + kk][2q][m] (real part) and
// W[k0 + kk][2q + 1][m] (imaginary part, if 2q + 1 < R_f).
template <int N2>
__global__ __launch_bounds__(kT) void lfft_col_inv(const cplx *__restrict__ tmp, int P, int k0,
                                                   const cplx *__restrict__ twN, int N, int N1,
                                                   int n, int R_f, const int *__restrict__ E,
                                                   double *__restrict__ W)
{
    __shared__ cplx buf[kCB * N2];
    const int q = blockIdx.y, kk = blockIdx.z;
    const int c0 = blockIdx.x * kCB;
    const cplx *t = tmp + ((long)kk * P + q) * N;
    for (int e = threadIdx.x; e < kCB * N2; e += kT) {
        const int cb = e % kCB, f2 = e / kCB;
        buf[lpos<N2>(cb, f2)] = t[(long)f2 * N1 + c0 + cb];
    }
    __syncthreads();
    lds_fft<N2, +1>(buf, kCB, twN, N);
    // 1/N and the rows' scales, both powers of two
    const int lgN = 31 - __clz(N);
    const bool second = 2 * q + 1 < R_f;
    const int s0 = E[2 * q] - lgN, s1 = second ? E[2 * q + 1] - lgN : 0;
    double *w0 = W + ((long)(k0 + kk) * R_f + 2 * q) * n;
    for (int e = threadIdx.x; e < kCB * N2; e += kT) {
        const int cb = e % kCB, m2 = e / kCB;
        const long m = c0 + cb + (long)N1 * m2;
        if (m < n) {
            const cplx v = buf[lpos<N2>(cb, m2)];
            w0[m] = ldexp(v.x, s0);
            if (second)
                w0[n + m] = ldexp(v.y, s1);
        }
    }
}

template <int N2>
hipError_t col_fwd(const double *X, const int *E, int rows, int len, const double *p, int n,
                   int count, const cplx *twN, int N, int N1, cplx *out, hipStream_t st)
{
    hipLaunchKernelGGL(lfft_col_fwd<N2>, dim3(N1 / kCB, count), dim3(kT), 0, st, X, E, rows,
                       len, p, n, twN, N, N1, out);
    return hipGetLastError();
}

template <int N1, int SIGN>
hipError_t row(const cplx *C, int k0, int kc, const cplx *Z, int P, const cplx *twN, int N,
               cplx *spec, int count, hipStream_t st)
{
    constexpr int RB = kLdsEntries / N1;
    const int N2 = N / N1;
    hipLaunchKernelGGL((lfft_row<N1, SIGN>), dim3(N2 / RB, count, SIGN < 0 ? 1 : kc), dim3(kT),
                       0, st, C, k0, Z, P, twN, N, spec);
    return hipGetLastError();
}

template <int N2>
hipError_t col_inv(const cplx *tmp, int P, int k0, int kc, const cplx *twN, int N, int N1, int n,
                   int R_f, const int *E, double *W, hipStream_t st)
{
    hipLaunchKernelGGL(lfft_col_inv<N2>, dim3(N1 / kCB, P, kc), dim3(kT), 0, st, tmp, P, k0, twN,
                       N, N1, n, R_f, E, W);
    return hipGetLastError();
}

// N = N1 N2 with N1 >= N2, both in {128, 256, 512}
void split_length(int N, int &N1, int &N2)
{
    int lg = 0;
    while ((1 << lg) < N)
        ++lg;
    N1 = 1 << ((lg + 1) / 2);
    N2 = N / N1;
}

}  // namespace

bool fft_large_supported(int n) { return n > 4096 && n <= 65536; }

int fft_large_terms_per_chunk(int n, int R_f, int R_N)
{
    // the inverse scratch holds kc x P sequences of N complex entries; keep it
    // near 512 MiB (at least one term)
    const long P = (R_f + 1) / 2;
    const long per = P * (long)fft_length(n) * 16;
    long kc = (512L << 20) / (per > 0 ? per : 1);
    if (kc < 1)
        kc = 1;
    if (kc > R_N)
        kc = R_N;
    return (int)kc;
}

LargeFftLayout fft_large_layout(int n, int R_f, int R_N)
{
    LargeFftLayout L;
    L.N = fft_length(n);
    L.P = (R_f + 1) / 2;
    L.kc = fft_large_terms_per_chunk(n, R_f, R_N);
    L.z_entries = (long)L.P * L.N;
    L.c_entries = (long)R_N * L.N;
    L.t_entries = (long)L.kc * L.P * L.N;
    return L;
}

hipError_t launch_fft_large_W(const double *p, const double *U, const int *EU, int n, int R_f,
                              int R_N, const cplx *twN, cplx *Z, cplx *C, cplx *T, double *W,
                              hipStream_t st)
{
    const LargeFftLayout L = fft_large_layout(n, R_f, R_N);
    const int N = L.N, P = L.P;
    int N1, N2;
    split_length(N, N1, N2);
    hipError_t e;
    auto colf = [&](const double *X, int rows, int len, const double *pp, int count, cplx *out) {
        switch (N2) {
        case 128: return col_fwd<128>(X, EU, rows, len, pp, n, count, twN, N, N1, out, st);
        case 256: return col_fwd<256>(X, EU, rows, len, pp, n, count, twN, N, N1, out, st);
        default: return hipErrorInvalidValue;
        }
    };
    auto rowk = [&](bool inv, int k0, int kc, cplx *spec, const cplx *Zs, int count) {
        if (inv) {
            switch (N1) {
            case 128: return row<128, +1>(C, k0, kc, Zs, P, twN, N, spec, count, st);
            case 256: return row<256, +1>(C, k0, kc, Zs, P, twN, N, spec, count, st);
            case 512: return row<512, +1>(C, k0, kc, Zs, P, twN, N, spec, count, st);
            default: return hipErrorInvalidValue;
            }
        }
        switch (N1) {
        case 128: return row<128, -1>(nullptr, 0, 1, nullptr, P, twN, N, spec, count, st);
        case 256: return row<256, -1>(nullptr, 0, 1, nullptr, P, twN, N, spec, count, st);
        case 512: return row<512, -1>(nullptr, 0, 1, nullptr, P, twN, N, spec, count, st);
        default: return hipErrorInvalidValue;
        }
    };
    auto coli = [&](int k0, int kc) {
        switch (N2) {
        case 128: return col_inv<128>(T, P, k0, kc, twN, N, N1, n, R_f, EU, W, st);
        case 256: return col_inv<256>(T, P, k0, kc, twN, N, N1, n, R_f, EU, W, st);
        default: return hipErrorInvalidValue;
        }
    };
    // spectra of the pairs of U rows and of the kernel embeddings
    if ((e = colf(U, R_f, n, nullptr, P, Z)) != hipSuccess)
        return e;
    if ((e = rowk(false, 0, 1, Z, nullptr, P)) != hipSuccess)
        return e;
    if ((e = colf(nullptr, 0, 0, p, R_N, C)) != hipSuccess)
        return e;
    if ((e = rowk(false, 0, 1, C, nullptr, R_N)) != hipSuccess)
        return e;
    // per chunk of terms: products, inverse row pass, inverse column pass
    for (int k0 = 0; k0 < R_N; k0 += L.kc) {
        const int kc = R_N - k0 < L.kc ? R_N - k0 : L.kc;
        if ((e = rowk(true, k0, kc, T, Z, P)) != hipSuccess)
            return e;
        if ((e = coli(k0, kc)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace tc
