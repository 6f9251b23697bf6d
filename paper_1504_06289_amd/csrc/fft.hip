// FFT route for the Toeplitz products (binary64):  W_k = T_k U  computed as
// the aperiodic convolution p_k *_n u_j through a circulant embedding of
// length N >= 2n-1 (power of two), i.e. the 1D FFT convolution that the
// d-dimensional FFT of Section 2.3 factors into, applied per mode.
//
//   c_k[t] = p_k[t] (0 <= t < n),  c_k[N-m] = p_k[-m] (1 <= m < n),  0 else
//   W_k[j][t] = (IDFT_N(DFT_N(c_k) . DFT_N(u_j zero-padded)))[t],  t < n
//
// Real transforms of length N use one complex transform of length M = N/2
// (even samples as real part, odd as imaginary part) plus the standard
// split/merge step with the twiddles e^(-2 pi i f / N).  The complex
// transform runs in LDS with 512 threads as a Stockham autosort FFT whose
// pass structure is fixed at compile time (radix 8, last pass radix 8/4/2);
// after each pass the sub-transform size Ns grows by the radix R, butterfly j
// reads entries j + r M/R, multiplies entry r by
// e^(sign 2 pi i (j mod Ns) r / (Ns R)), does an R-point DFT and writes
// entries (j/Ns) Ns R + (j mod Ns) + r Ns.  Each thread keeps the twiddle
// bases of its butterflies in registers.  LDS entry i is stored at
// i ^ ((i >> 4) & 15) (a permutation inside each aligned group of 16), which
// makes the strided reads and writes of every pass hit distinct banks and
// keeps the buffer at exactly M entries (64 KB for M = 4096).
//
// Kernels:
//   fft_twiddles       e^(-2 pi i t / N), t < N, for one N (sincospi)
//   rfft_batch         half spectra of the zero-padded rows of U, or of the
//                      circulant embeddings of the p_k
//   fft_conv           for one function j and every term k: product of the
//                      spectra, inverse transform, first n samples written
//                      either as binary64 W or directly as the int8 slices
//                      (one exponent per row) that the Gram consumes.
#include "tc_internal.h"

namespace tc {

namespace {

typedef double2 cplx;
typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kMaxM = 4096;  // complex length: N <= 8192, n <= 4096

__device__ inline cplx cadd(cplx a, cplx b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline cplx csub(cplx a, cplx b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline cplx cmul(cplx a, cplx b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline cplx cconj(cplx a) { return make_double2(a.x, -a.y); }
__device__ inline cplx cscale(cplx a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by SIGN * i
template <int SIGN> __device__ inline cplx mul_si(cplx a)
{
    return SIGN > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

__device__ inline int pad(int i) { return i ^ ((i >> 4) & 15); }

// ---- small DFTs: X[q] = sum_r v[r] exp(SIGN 2 pi i r q / R) ----------------
template <int SIGN> __device__ inline void dft2(cplx *v)
{
    const cplx a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int SIGN> __device__ inline void dft4(cplx *v)
{
    const cplx a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const cplx b0 = cadd(v[1], v[3]), b1 = mul_si<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
}

template <int SIGN> __device__ inline void dft8(cplx *v)
{
    const double h = 0.70710678118654752440;  // cos(pi/4)
    cplx e[4] = {v[0], v[2], v[4], v[6]};
    cplx o[4] = {v[1], v[3], v[5], v[7]};
    dft4<SIGN>(e);
    dft4<SIGN>(o);
    // w8^q = exp(SIGN 2 pi i q / 8)
    const cplx w[4] = {make_double2(1.0, 0.0), make_double2(h, SIGN * h),
                       make_double2(0.0, (double)SIGN), make_double2(-h, SIGN * h)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const cplx t = cmul(w[q], o[q]);
        v[q] = cadd(e[q], t);
        v[q + 4] = csub(e[q], t);
    }
}

template <int SIGN> __device__ inline void dft16(cplx *v)
{
    const double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;  // pi/8
    const double h = 0.70710678118654752440;
    cplx e[8], o[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        e[r] = v[2 * r];
        o[r] = v[2 * r + 1];
    }
    dft8<SIGN>(e);
    dft8<SIGN>(o);
    // w16^q = cos(2 pi q/16) + SIGN i sin(2 pi q/16)
    const double cs[8] = {1.0, c1, h, s1, 0.0, -s1, -h, -c1};
    const double sn[8] = {0.0, s1, h, c1, 1.0, c1, h, s1};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const cplx t = cmul(make_double2(cs[q], SIGN * sn[q]), o[q]);
        v[q] = cadd(e[q], t);
        v[q + 8] = csub(e[q], t);
    }
}

template <int R, int SIGN> __device__ inline void dft_small(cplx *v)
{
    if constexpr (R == 16)
        dft16<SIGN>(v);
    else if constexpr (R == 8)
        dft8<SIGN>(v);
    else if constexpr (R == 4)
        dft4<SIGN>(v);
    else if constexpr (R == 2)
        dft2<SIGN>(v);
}

// ---- FFT with the pass structure fixed at compile time ----------------------
// Used by the per-term inverse transforms, where the same transform runs for
// every kernel term: each thread loads the twiddle bases of its butterfly in
// every pass once (e^(SIGN 2 pi i s/M) for s = step, 2 step, 4 step, 8 step)
// and keeps them in registers, so the passes touch only LDS.
constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

template <int M, int RMAX> struct FftShape {
    static constexpr int LOG = ilog2c(M);
    static constexpr int LR = ilog2c(RMAX);
    static constexpr int NFULL = LOG / LR;
    static constexpr int REM = LOG % LR;
    static constexpr int NP = NFULL + (REM ? 1 : 0);
    static constexpr int radix(int p) { return p < NFULL ? RMAX : (1 << REM); }
    static constexpr int ns(int p) { return p == 0 ? 1 : ns(p - 1) * radix(p - 1); }
};

template <int M, int RMAX> struct FftTwiddles {
    cplx w[FftShape<M, RMAX>::NP > 0 ? FftShape<M, RMAX>::NP : 1][4];
};

template <int M, int RMAX, int T, int SIGN, int P>
__device__ inline void load_twiddles_pass(FftTwiddles<M, RMAX> &Tw, const cplx *__restrict__ twN)
{
    using F = FftShape<M, RMAX>;
    if constexpr (P < F::NP) {
        constexpr int R = F::radix(P), Ns = F::ns(P);
        if constexpr (Ns > 1) {
            const int j = threadIdx.x;
            if (j < M / R) {
                const int step = (j % Ns) * (M / (Ns * R));
                auto tw = [&](int s) {
                    const cplx x = twN[2 * s];
                    return SIGN > 0 ? cconj(x) : x;
                };
                Tw.w[P][0] = tw(step);
                if constexpr (R >= 4)
                    Tw.w[P][1] = tw(2 * step);
                if constexpr (R >= 8)
                    Tw.w[P][2] = tw(4 * step);
                if constexpr (R >= 16)
                    Tw.w[P][3] = tw(8 * step);
            }
        }
        load_twiddles_pass<M, RMAX, T, SIGN, P + 1>(Tw, twN);
    }
}

// the butterfly of thread j (< M/R) in one Stockham pass: entries j + r M/R of
// buf, twiddled and transformed into v (outputs base + r Ns of the pass)
template <int M, int R, int Ns, int SIGN>
__device__ inline void butterfly_fixed(const cplx *buf, const cplx *wb, cplx (&v)[R])
{
    constexpr int nb = M / R;
    const int j = threadIdx.x;
#pragma unroll
    for (int r = 0; r < R; ++r)
        v[r] = buf[pad(j + r * nb)];
    if constexpr (Ns > 1) {
        // w^r from the bases w^1, w^2, w^4, w^8 (binary digits of r),
        // applied as soon as it is formed to keep few values live
#pragma unroll
        for (int r = 1; r < R; ++r) {
            cplx w = (r & 1) ? wb[0] : make_double2(1.0, 0.0);
            if constexpr (R >= 4)
                if (r & 2)
                    w = (r & 1) ? cmul(w, wb[1]) : wb[1];
            if constexpr (R >= 8)
                if (r & 4)
                    w = (r & 3) ? cmul(w, wb[2]) : wb[2];
            if constexpr (R >= 16)
                if (r & 8)
                    w = (r & 7) ? cmul(w, wb[3]) : wb[3];
            v[r] = cmul(v[r], w);
        }
    }
    dft_small<R, SIGN>(v);
}

// one in-place Stockham pass with T threads (M/R <= T butterflies); outputs
// at indices >= keep are not stored (the caller reads only [0, keep))
template <int M, int R, int Ns, int T, int SIGN>
__device__ inline void pass_fixed(cplx *buf, const cplx *wb, int keep)
{
    constexpr int nb = M / R;
    static_assert(nb <= T, "one butterfly per thread");
    const int j = threadIdx.x;
    const bool active = nb >= T || j < nb;
    cplx v[R];
    if (active)
        butterfly_fixed<M, R, Ns, SIGN>(buf, wb, v);
    __syncthreads();
    if (active) {
        const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (base + r * Ns < keep)
                buf[pad(base + r * Ns)] = v[r];
    }
    __syncthreads();
}

// The whole transform; only outputs [0, keep) of the last pass are stored.
template <int M, int RMAX, int T, int SIGN, int P>
__device__ inline void fft_fixed(cplx *buf, const FftTwiddles<M, RMAX> &Tw, int keep)
{
    using F = FftShape<M, RMAX>;
    if constexpr (P < F::NP) {
        pass_fixed<M, F::radix(P), F::ns(P), T, SIGN>(buf, Tw.w[P], P + 1 == F::NP ? keep : M);
        fft_fixed<M, RMAX, T, SIGN, P + 1>(buf, Tw, keep);
    }
}

// The whole transform with the last pass kept in registers: thread j ends
// with the outputs j + r Ns (r < R, R and Ns the last pass's radix and
// sub-transform size) in v and buf holds the last pass's inputs.  Needs one
// last-pass butterfly per thread (M / R == T), so that Ns == T.
template <int M, int RMAX> struct FftLast {
    using F = FftShape<M, RMAX>;
    static constexpr int R = F::radix(F::NP - 1);
    static constexpr int Ns = F::ns(F::NP - 1);
};
template <int M, int RMAX, int T, int SIGN, int P>
__device__ inline void fft_fixed_regs(cplx *buf, const FftTwiddles<M, RMAX> &Tw,
                                      cplx (&v)[FftLast<M, RMAX>::R])
{
    using F = FftShape<M, RMAX>;
    static_assert(M / FftLast<M, RMAX>::R == T, "one last-pass butterfly per thread");
    if constexpr (P + 1 < F::NP) {
        pass_fixed<M, F::radix(P), F::ns(P), T, SIGN>(buf, Tw.w[P], M);
        fft_fixed_regs<M, RMAX, T, SIGN, P + 1>(buf, Tw, v);
    } else {
        butterfly_fixed<M, F::radix(P), F::ns(P), SIGN>(buf, Tw.w[P], v);
    }
}

__global__ __launch_bounds__(256) void fft_twiddles_kernel(cplx *twN, int N)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N) {
        double s, c;
        sincospi(2.0 * (double)t / (double)N, &s, &c);
        twN[t] = make_double2(c, -s);
    }
}

__device__ inline int row_exp(double amax)
{
    if (!(amax > 0.0))
        return 0;
    int E = ilogb(amax) - 6;
    if (ldexp(amax, -E) > 127.0)
        ++E;
    return E;
}

// Four int8 digits of x 2^-E (|x 2^-E| <= 127) at weights 1, 2^-7, 2^-14,
// 2^-21: round x 2^(21-E) to the integer q (|q| < 2^28, error <= 2^(E-22)),
// then split q exactly into balanced base-128 digits (the leading digit in
// [-127, 127], the others in [-64, 64]) with integer shifts.
__device__ inline void split4_i8(double x, int E, int8_t s[4])
{
    int q = (int)rint(ldexp(x, 21 - E));
    const int d0 = (q + (1 << 20)) >> 21;
    q -= d0 << 21;
    const int d1 = (q + (1 << 13)) >> 14;
    q -= d1 << 14;
    const int d2 = (q + (1 << 6)) >> 7;
    q -= d2 << 7;
    s[0] = (int8_t)d0;
    s[1] = (int8_t)d1;
    s[2] = (int8_t)d2;
    s[3] = (int8_t)q;
}

// For function j (blockIdx.x) and every term k: W_k[j][t], t < n, from the
// product of the spectra.  Output either binary64 rows (W != nullptr, layout
// [R_N][R_f][n]) or int8 slices (WS != nullptr, layout [4][R_N][R_f_pad][n_pad]
// with exponents EW [R_N][R_f_pad]); blocks with j >= R_f write zero slices.
//
// Each thread owns the frequency pairs (f, M - f), f = tid + 512 q <= M/2.
// The spectrum of u_j and the split twiddles e^(-2 pi i f/N), f <= M/4, stay
// in LDS for all terms (with the transform buffer: 144 KB at M = 4096),
// and the kernel spectrum of the next transformed term is loaded into
// registers while the current one is transformed, so the inner loop waits on
// no global load.
//
// Term classes (band != nullptr, int8 output only; see launch_term_class): a
// narrow term, band[k] = B >= 0 (all of |p_k[m]|, |m| > B, together below
// 2^-60 of sum_m |p_k[m]|), is convolved directly as
// sum_{|m| <= B} p_k[m] u_j[t - m] in binary64 from u_j staged in LDS, after
// the transformed terms (the dropped tail is far below the 28-bit split); a
// smooth term, band[k] = -2, is skipped (its Gram is formed at low rank).
constexpr int kConvThreads = 512;  // 8 waves: two per SIMD with one workgroup per CU
constexpr int kConvRadix = 8;      // M/8 <= 512 butterflies per pass
constexpr int kBandPad = 32;       // zeros around u_j in LDS: >= kBandMax + 15

template <int M, bool F64>
__global__ __launch_bounds__(kConvThreads) void fft_conv_kernel(
    const cplx *__restrict__ Uspec, const cplx *__restrict__ Cspec, int n, int R_f, int R_N,
    const cplx *__restrict__ twN, double *__restrict__ W, int8_t *__restrict__ WS,
    int *__restrict__ EW, int R_f_pad, int n_pad, long wplane, const double *__restrict__ U,
    const double *__restrict__ p, const int *__restrict__ band, int narrow_here)
{
    constexpr int TT = kConvThreads;
    constexpr int PAIRS = (M / 2 + 1 + TT - 1) / TT;
    constexpr int QUART = M / 4 + 1;  // twiddles w^f, f <= M/4 (the rest by symmetry)
    __shared__ cplx buf[M];
    __shared__ cplx Ush[M];
    __shared__ cplx twsh[QUART];
    __shared__ double red[2][TT / 64];  // per-wave maxima, alternating between terms
    const int j = blockIdx.x;
    const int tid = threadIdx.x;

    // the terms of this workgroup: [kb, ke) (a split over blockIdx.y when there
    // are few rows)
    const int kb = (int)((long)blockIdx.y * R_N / gridDim.y);
    const int ke = (int)((long)(blockIdx.y + 1) * R_N / gridDim.y);

    if (j >= R_f) {  // zero padding rows of the slices
        for (int k = kb; k < ke; ++k) {
            int8_t *row = WS + ((long)k * R_f_pad + j) * n_pad;
            for (int t = tid; t < n_pad; t += blockDim.x)
                for (int s = 0; s < 4; ++s)
                    row[s * wplane + t] = 0;
            if (tid == 0)
                EW[(long)k * R_f_pad + j] = 0;
        }
        return;
    }

    FftTwiddles<M, kConvRadix> Tw;
    load_twiddles_pass<M, kConvRadix, TT, +1, 0>(Tw, twN);

    const cplx *Uj = Uspec + (long)j * (M + 1);
    for (int f = tid; f < M; f += TT)
        Ush[f] = Uj[f];
    for (int f = tid; f < QUART && f < M / 2; f += TT)
        twsh[f] = twN[f];
    const cplx uM = Uj[M];  // only the pair (0, M) uses it
    constexpr double invM = 1.0 / (double)M;

    // kernel spectrum of a term at this thread's pairs
    cplx cf[PAIRS], cg[PAIRS];
    auto load_c = [&](int k) {
        const cplx *Ck = Cspec + (long)k * (M + 1);
#pragma unroll
        for (int q = 0; q < PAIRS; ++q) {
            const int f = tid + TT * q;
            if (f <= M / 2) {
                cf[q] = Ck[f];
                cg[q] = Ck[M - f];
            }
        }
    };
    // the next transformed term at or after k
    auto next_fft = [&](int k) {
        while (k < ke && band && band[k] != -1)
            ++k;
        return k;
    };

    // int8 slices of W_k[j] from the samples t = 8 tid .. 8 tid + 7 (zero at
    // t >= n): block maximum, row exponent, split, one 8-byte store per slice.
    // The maxima alternate between two arrays, so the next term's writes
    // cannot meet this term's reads.  n_pad <= 8 TT on this route.
    int nemit = 0;
    auto emit = [&](int k, const double (&zs)[8]) {
        const bool own = 8 * tid < n_pad;
        double amax = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            amax = fmax(amax, fabs(zs[q]));
        for (int o = 32; o > 0; o >>= 1)
            amax = fmax(amax, __shfl_xor(amax, o));
        double *rd = red[nemit & 1];
        ++nemit;
        if ((tid & 63) == 0)
            rd[tid >> 6] = amax;
        __syncthreads();
        amax = rd[0];
#pragma unroll
        for (int wv = 1; wv < TT / 64; ++wv)
            amax = fmax(amax, rd[wv]);
        const int E = row_exp(amax);
        if (tid == 0)
            EW[(long)k * R_f_pad + j] = E;
        if (own) {
            unsigned long long packed[4] = {0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                int8_t d[4];
                split4_i8(zs[q], E, d);
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    packed[s] |= (unsigned long long)(unsigned char)d[s] << (8 * q);
            }
            int8_t *row = WS + ((long)k * R_f_pad + j) * n_pad + 8 * tid;
#pragma unroll
            for (int s = 0; s < 4; ++s)
                *reinterpret_cast<unsigned long long *>(row + s * wplane) = packed[s];
        }
    };

    // With one last-pass butterfly per thread, thread tid ends the transform
    // holding the complex outputs m = tid + r TT (r < LR), i.e. the samples
    // t = 2m, 2m + 1, and splits them from registers: two bytes per slice and
    // output, consecutive across the lanes of a wave.  Same values, maximum
    // and digits as emit.  Only r < LR/2 (m < M/2) can hold samples t < n or
    // slice bytes t < n_pad, since n <= M and n_pad <= M, so the other half of
    // the last butterfly is never formed.
    using Last = FftLast<M, kConvRadix>;
    constexpr int LR = Last::R;
    constexpr int RU = LR / 2;
    constexpr bool kLastInRegs = M / LR == TT;
    auto emit_regs = [&](int k, const cplx (&v)[LR]) {
        double za[RU], zb[RU];
        double amax = 0.0;
#pragma unroll
        for (int r = 0; r < RU; ++r) {
            const int t = 2 * (tid + r * TT);
            za[r] = t < n ? v[r].x * invM : 0.0;
            zb[r] = t + 1 < n ? v[r].y * invM : 0.0;
            amax = fmax(amax, fmax(fabs(za[r]), fabs(zb[r])));
        }
        for (int o = 32; o > 0; o >>= 1)
            amax = fmax(amax, __shfl_xor(amax, o));
        double *rd = red[nemit & 1];
        ++nemit;
        if ((tid & 63) == 0)
            rd[tid >> 6] = amax;
        __syncthreads();
        amax = rd[0];
#pragma unroll
        for (int wv = 1; wv < TT / 64; ++wv)
            amax = fmax(amax, rd[wv]);
        const int E = row_exp(amax);
        if (tid == 0)
            EW[(long)k * R_f_pad + j] = E;
        int8_t *row = WS + ((long)k * R_f_pad + j) * n_pad;
#pragma unroll
        for (int r = 0; r < RU; ++r) {
            const int t = 2 * (tid + r * TT);
            if (t < n_pad) {  // n_pad is even: t + 1 < n_pad too
                int8_t da[4], db[4];
                split4_i8(za[r], E, da);
                split4_i8(zb[r], E, db);
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    *reinterpret_cast<unsigned short *>(row + s * wplane + t) =
                        (unsigned short)((unsigned char)da[s] | ((unsigned)(unsigned char)db[s] << 8));
            }
        }
    };

    int k = next_fft(kb);
    if (k < ke)
        load_c(k);
    __syncthreads();

    while (k < ke) {
#pragma unroll
        for (int q = 0; q < PAIRS; ++q) {
            const int f = tid + TT * q;
            if (f <= M / 2) {
                const int g = M - f;
                // w^f = e^(-i pi f/M); for M/4 < f < M/2, w^f = -i conj(w^(M/2-f));
                // w^(M/2) = -i
                cplx wf = make_double2(0.0, -1.0);
                if (f <= M / 4 && f < M / 2) {
                    wf = twsh[f];
                } else if (f < M / 2) {
                    const cplx v = twsh[M / 2 - f];
                    wf = make_double2(-v.y, -v.x);
                }
                const cplx yf = cmul(cf[q], Ush[f]);
                const cplx yg = cmul(cg[q], g < M ? Ush[g] : uM);
                // Z[f] = E + i O,  E = (Y[f] + conj Y[g]) / 2,  O = (Y[f] - conj Y[g]) conj(w^f) / 2
                {
                    const cplx E = cscale(cadd(yf, cconj(yg)), 0.5);
                    const cplx O = cscale(cmul(csub(yf, cconj(yg)), cconj(wf)), 0.5);
                    buf[pad(f)] = make_double2(E.x - O.y, E.y + O.x);
                }
                if (g < M && g != f) {
                    const cplx wg = make_double2(-wf.x, wf.y);  // w^(M-f) = -conj(w^f)
                    const cplx E = cscale(cadd(yg, cconj(yf)), 0.5);
                    const cplx O = cscale(cmul(csub(yg, cconj(yf)), cconj(wg)), 0.5);
                    buf[pad(g)] = make_double2(E.x - O.y, E.y + O.x);
                }
            }
        }
        const int kn = next_fft(k + 1);
        if (kn < ke)
            load_c(kn);  // in flight during the transform
        __syncthreads();
        if constexpr (kLastInRegs && !F64) {
            // the last pass's outputs go to the split from registers; buf's
            // last reads end before the barrier inside emit_regs
            cplx v[LR];
            fft_fixed_regs<M, kConvRadix, TT, +1, 0>(buf, Tw, v);
            emit_regs(k, v);
            k = kn;
            continue;
        }
        // outputs m hold the samples 2m, 2m + 1: only m < ceil(n/2) are used
        fft_fixed<M, kConvRadix, TT, +1, 0>(buf, Tw, (n + 1) / 2);

        if constexpr (F64) {
            double *Wrow = W + ((long)k * R_f + j) * n;
            for (int m = tid; m < M; m += TT) {
                const cplx z = buf[pad(m)];
                const int t = 2 * m;
                if (t < n)
                    Wrow[t] = z.x * invM;
                if (t + 1 < n)
                    Wrow[t + 1] = z.y * invM;
            }
            __syncthreads();  // buf is rewritten by the next term
        } else {
            // thread tid owns the eight samples t = 8 tid .. 8 tid + 7 (the
            // complex outputs m = 4 tid .. 4 tid + 3); all reads of buf for this
            // term happen before the barrier inside emit, so the next term may
            // overwrite buf without another barrier
            double zs[8];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = 4 * tid + q;
                const int t = 2 * m;
                cplx z = make_double2(0.0, 0.0);
                if (8 * tid < n_pad && m < M)
                    z = buf[pad(m)];
                zs[2 * q] = t < n ? z.x * invM : 0.0;
                zs[2 * q + 1] = t + 1 < n ? z.y * invM : 0.0;
            }
            emit(k, zs);
        }
        k = kn;
    }

    if (!F64 && band && narrow_here) {
        // narrow terms: u_j in LDS with kBandPad zeros on both sides (buf is
        // free: the last transform's reads ended before the barrier in its
        // emit; 2M >= 9/8 (n + 2 kBandPad) is checked at launch).  Entry x of
        // the padded row sits at x + x/8, so the lanes' windows (eight entries
        // apart) fall on different banks.
        double *ush = reinterpret_cast<double *>(buf);
        const double *urow = U + (long)j * n;
        for (int t = tid; t < n + 2 * kBandPad; t += TT) {
            const int x = t - kBandPad;
            ush[t + (t >> 3)] = (x >= 0 && x < n) ? urow[x] : 0.0;
        }
        __syncthreads();
        const int t0 = 8 * tid;
        const double *uw = ush + 9 * tid;  // entry 8 tid + c of the padded row at uw[c + c/8]
        for (int kt = kb; kt < ke; ++kt) {
            const int b = band[kt];
            if (b < 0)
                continue;
            const double *pk = p + (long)kt * (2L * n - 1) + (n - 1);  // pk[lag]
            double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (t0 < n) {
                // chunks of eight lags m0 .. m0 + 7 over the window
                // u[t0 - m0 - 7 .. t0 - m0 + 7]
                for (int m0 = -b; m0 <= b; m0 += 8) {
                    double pm[8], win[15];
#pragma unroll
                    for (int r = 0; r < 8; ++r)
                        pm[r] = m0 + r <= b ? pk[m0 + r] : 0.0;
#pragma unroll
                    for (int q = 0; q < 15; ++q) {
                        // u[t0 - m0 + q - 7] = padded entry 8 tid + c, c >= 0
                        const int c = kBandPad - 7 + q - m0;
                        win[q] = uw[c + (c >> 3)];
                    }
#pragma unroll
                    for (int i = 0; i < 8; ++i)
#pragma unroll
                        for (int r = 0; r < 8; ++r)
                            acc[i] = fma(pm[r], win[i - r + 7], acc[i]);
                }
            }
            double zs[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                zs[i] = t0 + i < n ? acc[i] : 0.0;
            emit(kt, zs);
        }
    }
}

// The narrow terms of fft_conv_kernel in a launch of their own: for row j
// (blockIdx.x < R_f) and every narrow term k (band[k] >= 0) in [0, R_N),
// W_k[j][t] = sum_{|m| <= B} p_k[m] u_j[t - m] in binary64 and its int8
// slices, exactly as fft_conv_kernel's direct loop and split output compute
// them.  With only the padded row of u_j in LDS (37 KB at n = 4096) and no
// transform registers, several workgroups share a CU, which hides the
// latency of the direct loops and of the split output that the transform
// kernel's one workgroup per CU cannot.  Rows j >= R_f are zeroed by the
// transform kernel.
__global__ __launch_bounds__(kConvThreads) void narrow_conv_kernel(
    const double *__restrict__ U, const double *__restrict__ p, const int *__restrict__ band,
    int n, int R_N, int8_t *__restrict__ WS, int *__restrict__ EW, int R_f_pad, int n_pad,
    long wplane)
{
    constexpr int TT = kConvThreads;
    constexpr int NU = (4096 + 2 * kBandPad) * 9 / 8 + 1;  // padded row, entry x at x + x/8
    __shared__ double ush[NU];
    __shared__ double red[2][TT / 64];
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    const double *urow = U + (long)j * n;
    for (int t = tid; t < n + 2 * kBandPad; t += TT) {
        const int x = t - kBandPad;
        ush[t + (t >> 3)] = (x >= 0 && x < n) ? urow[x] : 0.0;
    }
    __syncthreads();
    int nemit = 0;
    auto emit = [&](int k, const double (&zs)[8]) {
        const bool own = 8 * tid < n_pad;
        double amax = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            amax = fmax(amax, fabs(zs[q]));
        for (int o = 32; o > 0; o >>= 1)
            amax = fmax(amax, __shfl_xor(amax, o));
        double *rd = red[nemit & 1];
        ++nemit;
        if ((tid & 63) == 0)
            rd[tid >> 6] = amax;
        __syncthreads();
        amax = rd[0];
#pragma unroll
        for (int wv = 1; wv < TT / 64; ++wv)
            amax = fmax(amax, rd[wv]);
        const int E = row_exp(amax);
        if (tid == 0)
            EW[(long)k * R_f_pad + j] = E;
        if (own) {
            unsigned long long packed[4] = {0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                int8_t d[4];
                split4_i8(zs[q], E, d);
#pragma unroll
                for (int sl = 0; sl < 4; ++sl)
                    packed[sl] |= (unsigned long long)(unsigned char)d[sl] << (8 * q);
            }
            int8_t *row = WS + ((long)k * R_f_pad + j) * n_pad + 8 * tid;
#pragma unroll
            for (int sl = 0; sl < 4; ++sl)
                *reinterpret_cast<unsigned long long *>(row + sl * wplane) = packed[sl];
        }
    };
    const int t0 = 8 * tid;
    const double *uw = ush + 9 * tid;  // entry 8 tid + c of the padded row at uw[c + c/8]
    for (int kt = 0; kt < R_N; ++kt) {
        const int b = band[kt];
        if (b < 0)
            continue;
        const double *pk = p + (long)kt * (2L * n - 1) + (n - 1);  // pk[lag]
        double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (t0 < n) {
            for (int m0 = -b; m0 <= b; m0 += 8) {
                double pm[8], win[15];
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    pm[r] = m0 + r <= b ? pk[m0 + r] : 0.0;
#pragma unroll
                for (int q = 0; q < 15; ++q) {
                    const int c = kBandPad - 7 + q - m0;
                    win[q] = uw[c + (c >> 3)];
                }
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int r = 0; r < 8; ++r)
                        acc[i] = fma(pm[r], win[i - r + 7], acc[i]);
            }
        }
        double zs[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            zs[i] = t0 + i < n ? acc[i] : 0.0;
        emit(kt, zs);
    }
}

// Forward real FFTs (half spectra [rows][M+1]) of either the rows of X
// [rows][len] zero-padded to N = 2M (X != nullptr) or the circulant
// embeddings of the kernel vectors p [rows][2n-1] (X == nullptr).  Each
// workgroup takes rows blockIdx.x, blockIdx.x + gridDim.x, ...: the twiddles
// stay in registers across its rows and the next row's samples are loaded
// while the current one is transformed.
template <int M>
__global__ __launch_bounds__(kConvThreads) void rfft_batch_kernel(
    const double *__restrict__ X, int len, const double *__restrict__ p, int n, int rows,
    const cplx *__restrict__ twN, cplx *__restrict__ spec)
{
    constexpr int TT = kConvThreads;
    constexpr int PER = (M + TT - 1) / TT;      // packed inputs per thread
    constexpr int FIN = (M + 1 + TT - 1) / TT;  // outputs per thread
    __shared__ cplx buf[M];
    const int tid = threadIdx.x;

    FftTwiddles<M, kConvRadix> Tw;
    load_twiddles_pass<M, kConvRadix, TT, -1, 0>(Tw, twN);

    auto sample = [&](int r, int t) -> double {
        if (X)
            return t < len ? X[(long)r * len + t] : 0.0;
        const double *pk = p + (long)r * (2L * n - 1) + (n - 1);  // pk[lag]
        if (t < n)
            return pk[t];
        if (t > 2 * M - n)
            return pk[t - 2 * M];
        return 0.0;
    };
    cplx nxt[PER];
    auto load_row = [&](int r) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int m = tid + TT * q;
            if (m < M)
                nxt[q] = make_double2(sample(r, 2 * m), sample(r, 2 * m + 1));
        }
    };

    int r = blockIdx.x;
    if (r < rows)
        load_row(r);
    for (; r < rows; r += gridDim.x) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int m = tid + TT * q;
            if (m < M)
                buf[pad(m)] = nxt[q];
        }
        if (r + (int)gridDim.x < rows)
            load_row(r + gridDim.x);  // in flight during the transform
        __syncthreads();
        fft_fixed<M, kConvRadix, TT, -1, 0>(buf, Tw, M);
        // X[f] = E + w^f O from the packed transform Z: E = (Z[f] + conj Z[M-f]) / 2,
        // O = (Z[f] - conj Z[M-f]) / (2i)
        cplx *out = spec + (long)r * (M + 1);
#pragma unroll
        for (int q = 0; q < FIN; ++q) {
            const int f = tid + TT * q;
            if (f <= M) {
                const cplx a = buf[pad(f % M)];
                const cplx b = cconj(buf[pad((M - f) % M)]);
                const cplx E = cscale(cadd(a, b), 0.5);
                const cplx d = csub(a, b);
                const cplx O = make_double2(0.5 * d.y, -0.5 * d.x);
                out[f] = cadd(E, cmul(twN[f], O));
            }
        }
        __syncthreads();  // buf is rewritten by the next row
    }
}


}  // namespace

int fft_length(int n)
{
    int N = 2;
    while (N < 2 * n - 1)
        N *= 2;
    return N;
}

bool fft_supported(int n) { return n >= 1 && fft_length(n) / 2 <= kMaxM; }

hipError_t launch_fft_twiddles(cplx *twN, int N, hipStream_t stream)
{
    hipLaunchKernelGGL(fft_twiddles_kernel, dim3((N + 255) / 256), dim3(256), 0, stream, twN, N);
    return hipGetLastError();
}

static hipError_t launch_rfft_batch(const double *X, int len, const double *p, int n, int rows,
                                    int N, const cplx *twN, cplx *spec, hipStream_t stream)
{
    const int M = N / 2;
    const int blocks = rows < 512 ? rows : 512;  // two 64 KB workgroups per CU
#define TC_RFFT_CASE(MM)                                                                        \
    case MM:                                                                                    \
        hipLaunchKernelGGL(rfft_batch_kernel<MM>, dim3(blocks), dim3(kConvThreads), 0, stream,  \
                           X, len, p, n, rows, twN, spec);                                      \
        break;
    switch (M) {
        TC_RFFT_CASE(1)
        TC_RFFT_CASE(2)
        TC_RFFT_CASE(4)
        TC_RFFT_CASE(8)
        TC_RFFT_CASE(16)
        TC_RFFT_CASE(32)
        TC_RFFT_CASE(64)
        TC_RFFT_CASE(128)
        TC_RFFT_CASE(256)
        TC_RFFT_CASE(512)
        TC_RFFT_CASE(1024)
        TC_RFFT_CASE(2048)
        TC_RFFT_CASE(4096)
    default:
        return hipErrorInvalidValue;
    }
#undef TC_RFFT_CASE
    return hipGetLastError();
}

hipError_t launch_rfft_rows(const double *X, int rows, int len, int N, const cplx *twN,
                            cplx *spec, hipStream_t stream)
{
    return launch_rfft_batch(X, len, nullptr, 0, rows, N, twN, spec, stream);
}

hipError_t launch_rfft_kernel_embed(const double *p, int n, int R_N, int N, const cplx *twN,
                                    cplx *spec, hipStream_t stream)
{
    return launch_rfft_batch(nullptr, 0, p, n, R_N, N, twN, spec, stream);
}

hipError_t launch_fft_conv(const cplx *Uspec, const cplx *Cspec, int n, int N, int R_f, int R_N,
                           const cplx *twN, double *W, int8_t *WS, int *EW, int R_f_pad,
                           int n_pad, long wplane, const double *U, const double *p,
                           const int *band, hipStream_t stream)
{
    const int M = N / 2;
    const int blocks = W ? R_f : R_f_pad;
    // few rows: split the terms over blockIdx.y so that ~512 workgroups run
    int ysplit = (512 + blocks - 1) / blocks;
    ysplit = ysplit < 1 ? 1 : (ysplit > R_N ? R_N : ysplit);
    if (W || 2 * M < (n + 2 * kBandPad) * 9 / 8 + 1)
        band = nullptr;  // the direct path is for int8 output with room for the padded row
    if (!W && (n_pad > 8 * kConvThreads || n_pad % 8 != 0))
        return hipErrorInvalidValue;  // one 8-byte slice chunk per thread
    // the narrow terms in a launch of their own (its padded row holds n <= 4096)
    const int narrow_apart = band && n <= 4096 && R_f >= 256;
    // the int8 output of the last pass's registers covers the bytes t < M
    if (!W && M >= 128 && n_pad > M)
        return hipErrorInvalidValue;
#define TC_FFT_CONV_CASE(MM)                                                                    \
    case MM:                                                                                    \
        if (W)                                                                                  \
            hipLaunchKernelGGL((fft_conv_kernel<MM, true>), dim3(blocks, ysplit),                 \
                               dim3(kConvThreads), 0, stream, Uspec, Cspec, n, R_f, R_N, twN,   \
                               W, WS, EW, R_f_pad, n_pad, wplane, U, p, band, 0);               \
        else                                                                                    \
            hipLaunchKernelGGL((fft_conv_kernel<MM, false>), dim3(blocks, ysplit),                \
                               dim3(kConvThreads), 0, stream, Uspec, Cspec, n, R_f, R_N, twN,   \
                               W, WS, EW, R_f_pad, n_pad, wplane, U, p, band, !narrow_apart);   \
        break;
    switch (M) {
        TC_FFT_CONV_CASE(1)
        TC_FFT_CONV_CASE(2)
        TC_FFT_CONV_CASE(4)
        TC_FFT_CONV_CASE(8)
        TC_FFT_CONV_CASE(16)
        TC_FFT_CONV_CASE(32)
        TC_FFT_CONV_CASE(64)
        TC_FFT_CONV_CASE(128)
        TC_FFT_CONV_CASE(256)
        TC_FFT_CONV_CASE(512)
        TC_FFT_CONV_CASE(1024)
        TC_FFT_CONV_CASE(2048)
        TC_FFT_CONV_CASE(4096)
    default:
        return hipErrorInvalidValue;
    }
#undef TC_FFT_CONV_CASE
    if (narrow_apart)
        hipLaunchKernelGGL(narrow_conv_kernel, dim3(R_f), dim3(kConvThreads), 0, stream, U, p,
                           band, n, R_N, WS, EW, R_f_pad, n_pad, wplane);
    return hipGetLastError();
}

}  // namespace tc
