// Error-free int8 splitting (Ozaki scheme on integer matrix cores) for the
// Toeplitz products and the Grams.
//
// Splitting.  Each row r of an operand gets one exponent E_r chosen so that
// max_b |x_rb| 2^-E_r lies in [63.5, 127]; every entry is then written as
//   x = 2^E_r (s1 + s2 2^-7 + s3 2^-14 + s4 2^-21) + residual,
// s1 in [-127, 127], s2..s4 in [-64, 64] (each a rounding of the scaled
// residual), |residual| <= 2^(E_r - 22), i.e. 28 bits relative to the row
// maximum.  Every step of the split is exact in binary64.
//
// Products.  With A = 2^Ea sum_i a_i 2^-7(i-1) and B likewise, the slice
// products a_i b_j with i + j <= 5 (ten of them) are summed on
// v_mfma_i32_16x16x64_i8 into four int32 accumulators, one per d = i+j-2
// (all pairs with equal d share the scale 2^-7d).  Integer accumulation is
// exact: |acc_d| <= 24448 K < 2^31 for K <= 65536.  The binary64 result is
//   2^(Ea+Eb) (acc_0 + acc_1 2^-7 + acc_2 2^-14 + acc_3 2^-21).
//
// The Toeplitz operand keeps the implicit form: the kernel vector p_k is
// split once with one exponent per term (its maximum, p_k[0], appears in
// every row of T_k), stored lag-reversed, and each K-step stages the
// contiguous window of lags the tile needs; a lane's 16-byte B-fragment is a
// byte-shifted run of that window, assembled with v_alignbyte_b32 from
// dword-aligned LDS reads.
//
// v_mfma_i32_16x16x64_i8: lane l supplies A[l%16][k in 16(l/16)+0..15] and
// B[k in 16(l/16)+0..15][l%16] (any k order works as long as A and B agree),
// and receives D[4(l/16)+r][l%16], r = 0..3.
#include "tc_internal.h"

namespace tc {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// splitting
// ---------------------------------------------------------------------------
__device__ inline int row_exponent(double amax)
{
    if (!(amax > 0.0))
        return 0;
    int E = ilogb(amax) - 6;  // amax 2^-E in [64, 128)
    if (ldexp(amax, -E) > 127.0)
        ++E;  // then in [63.5, 64)
    return E;
}

__device__ inline void split4(double x, int E, int8_t s[4])
{
    double y = ldexp(x, -E);
    double q = rint(y);
    s[0] = (int8_t)q;
    y = (y - q) * 128.0;
    q = rint(y);
    s[1] = (int8_t)q;
    y = (y - q) * 128.0;
    q = rint(y);
    s[2] = (int8_t)q;
    y = (y - q) * 128.0;
    q = rint(y);
    s[3] = (int8_t)q;
}

__device__ inline double block_max_abs(double v, double *red)
{
    // 256 threads
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    v = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return v;
}

// Rows of a [groups][rows][len] FP64 array (row stride len) -> slices
// S[4][groups][rows_pad][len_pad] int8 and exponents E[groups][rows_pad].
// One workgroup per output row; rows >= rows and columns >= len are zero.
__global__ __launch_bounds__(256) void split_rows_kernel(const double *__restrict__ X, int rows,
                                                         int len, int rows_pad, int len_pad,
                                                         long plane, int8_t *__restrict__ S,
                                                         int *__restrict__ E)
{
    __shared__ double red[4];
    const int grp = blockIdx.y;
    const int r = blockIdx.x;  // < rows_pad
    const long orow = (long)grp * rows_pad + r;
    int8_t *s0 = S + orow * len_pad;
    if (r >= rows) {
        for (int b = threadIdx.x; b < len_pad; b += 256)
            for (int q = 0; q < 4; ++q)
                s0[q * plane + b] = 0;
        if (threadIdx.x == 0)
            E[orow] = 0;
        return;
    }
    const double *x = X + ((long)grp * rows + r) * len;
    double m = 0.0;
    for (int b = threadIdx.x; b < len; b += 256)
        m = fmax(m, fabs(x[b]));
    m = block_max_abs(m, red);
    const int e = row_exponent(m);
    if (threadIdx.x == 0)
        E[orow] = e;
    for (int b = threadIdx.x; b < len_pad; b += 256) {
        int8_t s[4] = {0, 0, 0, 0};
        if (b < len)
            split4(x[b], e, s);
        for (int q = 0; q < 4; ++q)
            s0[q * plane + b] = s[q];
    }
}

// Kernel vectors p [R_N][2n-1] -> lag-reversed slices PS[4][R_N][LP] with
// PS[.][k][x] holding lag m = (n-1) + off - x, off = ozaki_p_offset(n), zero
// outside the lag range; exponents EP[R_N].  One workgroup per term.
__global__ __launch_bounds__(256) void split_kernel_vectors(const double *__restrict__ p, int n,
                                                            int LP, int off, long plane,
                                                            int8_t *__restrict__ PS,
                                                            int *__restrict__ EP)
{
    __shared__ double red[4];
    const int k = blockIdx.x;
    const long L = 2L * n - 1;
    const double *pk = p + k * L;  // pk[m + n - 1]
    double m = 0.0;
    for (long i = threadIdx.x; i < L; i += 256)
        m = fmax(m, fabs(pk[i]));
    m = block_max_abs(m, red);
    const int e = row_exponent(m);
    if (threadIdx.x == 0)
        EP[k] = e;
    int8_t *out = PS + (long)k * LP;
    for (int x = threadIdx.x; x < LP; x += 256) {
        const long lag = (long)(n - 1) + off - x;
        int8_t s[4] = {0, 0, 0, 0};
        if (lag > -n && lag < n)
            split4(pk[lag + n - 1], e, s);
        for (int q = 0; q < 4; ++q)
            out[q * plane + x] = s[q];
    }
}

// ---------------------------------------------------------------------------
// implicit-Toeplitz product on int8 matrix cores
//   W[k][j][a] = sum_b U[j][b] p_k[a-b]
// Workgroup tile 64 (j) x 128 (a), K-step 64; waves 2 x 2 with 32 x 64 wave
// tiles (2 x 4 MFMA blocks, four int32 accumulators each).
// ---------------------------------------------------------------------------
constexpr int TJ = 64, TA = 128, TK = 64;
constexpr int AROW = 80;                  // LDS row stride (bytes): conflict-free b128 reads
constexpr int WLEN = 256;                 // window bytes per slice (>= TA + TK - 1 + 16)
constexpr int A_BYTES = 4 * TJ * AROW;    // 20480
constexpr int W_BYTES = 4 * WLEN;         // 1024

__device__ inline double combine16(const v16i *acc, int r, int E)
{
    // as combine, for the 16-register accumulators of the 32 x 32 products
    double v = ldexp((double)acc[3][r], -21);
    v += ldexp((double)acc[2][r], -14);
    v += ldexp((double)acc[1][r], -7);
    v += (double)acc[0][r];
    return ldexp(v, E);
}

__device__ inline double combine(const v4i *acc, int r, int E)
{
    // sum from the smallest scale up; each term is exact
    double v = ldexp((double)acc[3][r], -21);
    v += ldexp((double)acc[2][r], -14);
    v += ldexp((double)acc[1][r], -7);
    v += (double)acc[0][r];
    return ldexp(v, E);
}

__global__ __launch_bounds__(256) void toeplitz_i8_kernel(
    const int8_t *__restrict__ US, const int *__restrict__ EU, long uplane, int n_pad,
    const int8_t *__restrict__ PS, const int *__restrict__ EP, long pplane, int LP, int off,
    double *__restrict__ W, int n, int R_f)
{
    __shared__ __attribute__((aligned(16))) int8_t As[2][A_BYTES];
    __shared__ __attribute__((aligned(16))) int8_t Pw[2][W_BYTES];

    const int k = blockIdx.z;
    const int a0 = blockIdx.x * TA;
    const int j0 = blockIdx.y * TJ;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wj = (wave >> 1) * 32, wa = (wave & 1) * 64;
    const int l16 = lane & 15, g = lane >> 4;

    // reversed-window start for K-step b0: x = off + n - TA - a0 + b0 (16-aligned)
    const long xs0 = (long)off + n - TA - a0;
    const int8_t *pk = PS + (long)k * LP;

    // staging registers: A = 1024 chunks of 16 B (4 per thread); window 4 x 16 chunks
    v4i areg[4];
    v4i preg;
    auto load_stage = [&](int b0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tid + 256 * q;  // slice = c/256, row = (c%256)/4, col16 = c%4
            const int sl = c >> 8, row = (c & 255) >> 2, c16 = c & 3;
            areg[q] = *reinterpret_cast<const v4i *>(US + sl * uplane + (long)(j0 + row) * n_pad +
                                                     b0 + 16 * c16);
        }
        if (tid < 64) {
            const int sl = tid >> 4, c16 = tid & 15;
            preg = *reinterpret_cast<const v4i *>(pk + sl * pplane + xs0 + b0 + 16 * c16);
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tid + 256 * q;
            const int sl = c >> 8, row = (c & 255) >> 2, c16 = c & 3;
            *reinterpret_cast<v4i *>(As[buf] + sl * (TJ * AROW) + row * AROW + 16 * c16) =
                areg[q];
        }
        if (tid < 64) {
            const int sl = tid >> 4, c16 = tid & 15;
            *reinterpret_cast<v4i *>(Pw[buf] + sl * WLEN + 16 * c16) = preg;
        }
    };

    v4i acc[2][4][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int d = 0; d < 4; ++d)
                acc[x][y][d] = v4i{0, 0, 0, 0};

    // window offsets of this lane: frag y starts at o_y = o3 + 16 (3 - y)
    const int o3 = TA - 1 - wa - l16 + 16 * g - 48;  // >= 0
    const int dw0 = o3 >> 2, sh = o3 & 3;

    const int nsteps = n_pad / TK;
    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const int cur = s & 1;
        if (s + 1 < nsteps)
            load_stage((s + 1) * TK);

        v4i afr[2][4];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int sl = 0; sl < 4; ++sl)
                afr[x][sl] = *reinterpret_cast<const v4i *>(
                    As[cur] + sl * (TJ * AROW) + (wj + 16 * x + l16) * AROW + 16 * g);

#pragma unroll
        for (int sl = 0; sl < 4; ++sl) {
            const unsigned *w32 = reinterpret_cast<const unsigned *>(Pw[cur] + sl * WLEN);
            unsigned dw[17];
#pragma unroll
            for (int i = 0; i < 17; ++i)
                dw[i] = w32[dw0 + i];
            v4i bfr[4];
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const int base = 4 * (3 - y);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    bfr[y][q] = (int)__builtin_amdgcn_alignbyte(dw[base + q + 1], dw[base + q],
                                                                (unsigned)sh);
            }
            // slice sl of B pairs with A slices i such that i + sl <= 3
#pragma unroll
            for (int i = 0; i + sl <= 3; ++i)
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y)
                        acc[x][y][i + sl] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            afr[x][i], bfr[y], acc[x][y][i + sl], 0, 0, 0);
        }
        if (s + 1 < nsteps)
            store_stage(cur ^ 1);
        __syncthreads();
    }

    const int Ep = EP[k];
    double *Wk = W + (long)k * R_f * n;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = j0 + wj + 16 * x + 4 * g + r;
            if (j >= R_f)
                continue;
            const int Ej = EU[j] + Ep;
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const int a = a0 + wa + 16 * y + l16;
                if (a < n)
                    Wk[(long)j * n + a] = combine(acc[x][y], r, Ej);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Grams on int8 matrix cores: G[k][i][j] = sum_a U[i][a] W[k][j][a]
// Upper-triangle 64 x 64 tiles, waves 2 x 2 of 32 x 32, K-step 64.
// ---------------------------------------------------------------------------
constexpr int GT = 64;
constexpr int G_BYTES = 4 * GT * AROW;  // 20480 per operand

// the kk-th term (in increasing k) whose class is not -2, or -1 if there are
// fewer; uniform over the workgroup
__device__ inline int nth_listed_term(const int *__restrict__ cls, int R_N, int kk)
{
    for (int k = 0; k < R_N; ++k)
        if (cls[k] != -2 && kk-- == 0)
            return k;
    return -1;
}

__global__ __launch_bounds__(256) void gram_i8_kernel(
    const int8_t *__restrict__ US, const int *__restrict__ EU, long uplane,
    const int8_t *__restrict__ WS, const int *__restrict__ EW, long wplane, int n_pad,
    int R_f_pad, double *__restrict__ G, int R_f, int ntiles, int R_N,
    const int *__restrict__ cls, int mirror)
{
    __shared__ __attribute__((aligned(16))) int8_t As[G_BYTES];
    __shared__ __attribute__((aligned(16))) int8_t Bs[G_BYTES];

    const int k = cls ? nth_listed_term(cls, R_N, blockIdx.y) : (int)blockIdx.y;
    if (k < 0)
        return;
    int t = blockIdx.x;
    int ti = 0;
    while (t >= ntiles - ti) {
        t -= ntiles - ti;
        ++ti;
    }
    const int tj = ti + t;
    const int i0 = ti * GT, j0 = tj * GT;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    const int l16 = lane & 15, g = lane >> 4;
    const int8_t *Wk = WS + (long)k * R_f_pad * n_pad;

    v4i areg[4], breg[4];
    auto load_stage = [&](int a0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tid + 256 * q;
            const int sl = c >> 8, row = (c & 255) >> 2, c16 = c & 3;
            areg[q] = *reinterpret_cast<const v4i *>(US + sl * uplane + (long)(i0 + row) * n_pad +
                                                     a0 + 16 * c16);
            breg[q] = *reinterpret_cast<const v4i *>(Wk + sl * wplane + (long)(j0 + row) * n_pad +
                                                     a0 + 16 * c16);
        }
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = tid + 256 * q;
            const int sl = c >> 8, row = (c & 255) >> 2, c16 = c & 3;
            const int o = sl * (GT * AROW) + row * AROW + 16 * c16;
            *reinterpret_cast<v4i *>(As + o) = areg[q];
            *reinterpret_cast<v4i *>(Bs + o) = breg[q];
        }
    };

    v4i acc[2][2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int d = 0; d < 4; ++d)
                acc[x][y][d] = v4i{0, 0, 0, 0};

    const int nsteps = n_pad / TK;
    load_stage(0);
    for (int s = 0; s < nsteps; ++s) {
        __syncthreads();
        store_stage();
        __syncthreads();
        if (s + 1 < nsteps)
            load_stage((s + 1) * TK);
        v4i afr[2][4], bfr[2][4];
#pragma unroll
        for (int sl = 0; sl < 4; ++sl)
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                afr[x][sl] = *reinterpret_cast<const v4i *>(
                    As + sl * (GT * AROW) + (wi + 16 * x + l16) * AROW + 16 * g);
                bfr[x][sl] = *reinterpret_cast<const v4i *>(
                    Bs + sl * (GT * AROW) + (wj + 16 * x + l16) * AROW + 16 * g);
            }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; i + j <= 3; ++j)
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        acc[x][y][i + j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            afr[x][i], bfr[y][j], acc[x][y][i + j], 0, 0, 0);
    }

    double *Gk = G + (long)k * R_f * R_f;
    const int *EWk = EW + (long)k * R_f_pad;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + wi + 16 * x + 4 * g + r;
            if (i >= R_f)
                continue;
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int j = j0 + wj + 16 * y + l16;
                if (j < R_f && i <= j) {
                    const double v = combine(acc[x][y], r, EU[i] + EWk[j]);
                    Gk[(long)i * R_f + j] = v;
                    if (mirror)
                        Gk[(long)j * R_f + i] = v;
                }
            }
        }
}

// Large-tile variant for R_f >= 256: 128 x 128 tiles, K-step 64, sixteen
// waves (1024 threads) in 4 x 4 of 32 x 32 blocks on v_mfma_i32_32x32x32_i8
// (four 16-register accumulators, one per scale group; 124 VGPRs), so four
// waves share each SIMD and hide each other's LDS and barrier waits.  The
// 32 x 32 x 32 form sustains 1.7 times the int8 rate of the 16 x 16 x 64
// form on gfx950 (which occupies the matrix pipe 32 cycles per product).
// The per-workgroup operand traffic per multiply-add halves compared with the
// 64 x 64 tiles.
//
// Work items are (k, tile) with k grouped by XCD (work item w runs on XCD
// w mod 8), and the tiles of one term are enumerated column by column
// (tj outer, ti <= tj inner), so the workgroups in flight on one XCD share
// the W slices of one column block and re-read them from that XCD's L2.
//
// LDS rows are unpadded (64 B) with the 16-byte chunks of row r permuted by
// c ^ swz(r): then the staging writes (four lanes per row) and the fragment
// reads (consecutive rows, one chunk) hit distinct banks in every group of
// sixteen lanes.
constexpr int GT2 = 128;
constexpr int kTailSlots = kOzakiTailSlots;  // slots per XCD for later K parts of tail items
constexpr int GW_ROW = 64;
constexpr int GW_PLANE = GT2 * GW_ROW;    // one slice of one operand
constexpr int GW_BYTES = 4 * GW_PLANE;    // 32768 per operand
__device__ inline int gw_offset(int sl, int row, int c16)
{
    const int swz = ((row >> 1) ^ (row >> 2)) & 3;
    return sl * GW_PLANE + row * GW_ROW + 16 * (c16 ^ swz);
}

// The (term, tile) items of XCD x, in the order its workgroups take them:
// with term classes (FFT route) the items of the nk listed terms in term
// order, cut into eight contiguous chunks; otherwise the terms x, x + 8, ...
// with all their tiles.  Of the list's Ix items, the first
// floor(Ix / cux) cux are whole (full rounds of the XCD's cux CUs); the rem
// items of the last, partial round are split into P K ranges each (P at most
// kTailParts, cux / rem and 1 + kTailSlots / rem), so that round holds
// rem P <= cux shorter items.  Part 0 of a split item writes the Gram tile,
// parts 1 .. P-1 write partial tiles to slots of the tail slab, and
// gram_i8_tail_sum adds them in part order.  Each part's binary64
// recombination of its exact int32 sums is exact (it spans at most 53
// bits), and so is every partial sum of the parts: the result is bitwise
// that of the unsplit tile.
constexpr int kTailParts = 4;
struct XcdList {
    int Ix, full, rem, P, start;
};
__device__ inline XcdList xcd_list(int x, const int *__restrict__ cls, int R_N, int ntri, int cux)
{
    XcdList L;
    if (cls) {
        int nk = 0;
        for (int kk = 0; kk < R_N; ++kk)
            nk += cls[kk] != -2;
        const int tot = nk * ntri, per = (tot + 7) / 8;
        L.start = x * per;
        L.Ix = tot - L.start < per ? tot - L.start : per;
        if (L.Ix < 0)
            L.Ix = 0;
    } else {
        L.start = 0;
        L.Ix = x < R_N ? ((R_N - x + 7) / 8) * ntri : 0;
    }
    L.full = (L.Ix / cux) * cux;
    L.rem = L.Ix - L.full;
    L.P = 1;
    if (L.rem > 0) {
        L.P = cux / L.rem;
        if (L.P > 1 + kTailSlots / L.rem)
            L.P = 1 + kTailSlots / L.rem;
        L.P = L.P < 1 ? 1 : L.P > kTailParts ? kTailParts : L.P;
    }
    return L;
}
// term and tile of list index li of XCD x (k < 0: nothing to do)
__device__ inline void xcd_item(const XcdList &L, int x, int li, const int *__restrict__ cls,
                                int R_N, int ntri, int &k, int &t)
{
    if (cls) {
        const int gi = L.start + li;
        t = gi % ntri;
        k = nth_listed_term(cls, R_N, gi / ntri);
    } else {
        k = x + 8 * (li / ntri);
        t = li % ntri;
    }
}

// slot of part p >= 1 of tail item r of XCD x: [8][kTailSlots] slots of
// GT2 x GT2 doubles
__device__ inline double *tail_slot(double *slab, int x, int r, int p, int P)
{
    return slab + ((long)x * kTailSlots + r * (P - 1) + (p - 1)) * GT2 * GT2;
}

constexpr int kWideThreads = 1024;
__global__ __launch_bounds__(kWideThreads) void gram_i8_wide_kernel(
    const int8_t *__restrict__ US, const int *__restrict__ EU, long uplane,
    const int8_t *__restrict__ WS, const int *__restrict__ EW, long wplane, int n_pad,
    int R_f_pad, double *__restrict__ G, int R_f, int R_N, int ntri,
    const int *__restrict__ cls, int mirror, int cux, double *__restrict__ slab)
{
    __shared__ __attribute__((aligned(16))) int8_t As[2][GW_BYTES];
    __shared__ __attribute__((aligned(16))) int8_t Bs[2][GW_BYTES];

    // work item w runs on XCD w mod 8; local = w / 8 indexes that XCD's list
    const int w = blockIdx.x;
    const int xcd = w & 7, local = w >> 3;
    const XcdList XL = xcd_list(xcd, cls, R_N, ntri, slab ? cux : 1 << 30);
    int li, part = 0, parts = 1, tail = 0;
    if (local < XL.full || !slab) {
        li = local;
    } else {
        const int j = local - XL.full;
        if (j >= XL.rem * XL.P)
            return;
        tail = j / XL.P;
        li = XL.full + tail;
        part = j % XL.P;
        parts = XL.P;
    }
    if (li >= XL.Ix)
        return;
    int k, t;
    xcd_item(XL, xcd, li, cls, R_N, ntri, k, t);
    if (k < 0 || k >= R_N)
        return;
    int tj = 0;
    while ((tj + 1) * (tj + 2) / 2 <= t)
        ++tj;
    const int ti = t - tj * (tj + 1) / 2;
    const int i0 = ti * GT2, j0 = tj * GT2;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // sixteen waves in 4 x 4 of 32 x 32 blocks, four per SIMD
    const int wi = (wave >> 2) * 32, wj = (wave & 3) * 32;
    const int l32 = lane & 31, h = lane >> 5;
    const int8_t *Wk = WS + (long)k * R_f_pad * n_pad;

    // staging: per operand 2048 chunks of 16 B, 2 per thread
    v4i areg[2], breg[2];
    auto load_stage = [&](int a0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + kWideThreads * q;  // slice = c/512, row = (c%512)/4, col16 = c%4
            const int sl = c >> 9, row = (c & 511) >> 2, c16 = c & 3;
            areg[q] = *reinterpret_cast<const v4i *>(US + sl * uplane + (long)(i0 + row) * n_pad +
                                                     a0 + 16 * c16);
            breg[q] = *reinterpret_cast<const v4i *>(Wk + sl * wplane + (long)(j0 + row) * n_pad +
                                                     a0 + 16 * c16);
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = tid + kWideThreads * q;
            const int sl = c >> 9, row = (c & 511) >> 2, c16 = c & 3;
            const int o = gw_offset(sl, row, c16);
            *reinterpret_cast<v4i *>(As[buf] + o) = areg[q];
            *reinterpret_cast<v4i *>(Bs[buf] + o) = breg[q];
        }
    };

    // one accumulator per scale group d = s + t of the slice products
    v16i acc[4];
#pragma unroll
    for (int d = 0; d < 4; ++d)
        acc[d] = v16i{};

    // this item's K steps [s0, s0 + nsteps)
    const int ktot = n_pad / TK;
    const int s0 = (int)((long)part * ktot / parts);
    const int nsteps = (int)((long)(part + 1) * ktot / parts) - s0;

    // Each 64-byte K step is two 32-byte halves kc; lane l reads row l mod 32
    // of its block, bytes 16 (l / 32) .. + 16 of the half (chunk 2 kc + l / 32)
    auto read_a = [&](int buf, int kc, v4i (&A)[4]) {
#pragma unroll
        for (int sl = 0; sl < 4; ++sl)
            A[sl] = *reinterpret_cast<const v4i *>(As[buf] + gw_offset(sl, wi + l32, 2 * kc + h));
    };
    auto read_b = [&](int buf, int kc, int sl) {
        return *reinterpret_cast<const v4i *>(Bs[buf] + gw_offset(sl, wj + l32, 2 * kc + h));
    };
    // products of B slice j against A slices i <= 3 - j
    auto products = [&](int j, const v4i (&A)[4], v4i B) {
#pragma unroll
        for (int i = 0; i + j <= 3; ++i)
            acc[i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i], B, acc[i + j], 0, 0, 0);
    };

    // Stage s+1 is written to LDS at the start of step s (from registers
    // loaded during step s-1), and stage s+2 is then loaded into those
    // registers, so the LDS writes overlap this step's matrix-core work.
    load_stage(s0 * TK);
    store_stage(0);
    if (nsteps > 1)
        load_stage((s0 + 1) * TK);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const int cur = s & 1;
        v4i a[4];
        read_a(cur, 0, a);
        v4i b0 = read_b(cur, 0, 0);
        // the other buffer was last read in step s-1, before the barrier that ended it
        if (s + 1 < nsteps)
            store_stage(cur ^ 1);
        if (s + 2 < nsteps)
            load_stage((s0 + s + 2) * TK);
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
            if (kc == 1) {
                read_a(cur, 1, a);
                b0 = read_b(cur, 1, 0);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                products(j, a, j == 0 ? b0 : read_b(cur, kc, j));
        }
        __syncthreads();
    }

    // register r of lane l holds row 8 (r / 4) + 4 (l / 32) + r mod 4 and
    // column l mod 32 of the wave's block
    const int *EWk = EW + (long)k * R_f_pad;
    if (part > 0) {
        // a later K part of a split tail item: the partial tile to its slot
        double *sl = tail_slot(slab, xcd, tail, part, parts);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int a = wi + 8 * (r >> 2) + 4 * h + (r & 3), b = wj + l32;
            const int i = i0 + a, j = j0 + b;
            if (i < R_f && j < R_f && i <= j)
                sl[a * GT2 + b] = combine16(acc, r, EU[i] + EWk[j]);
        }
        return;
    }
    double *Gk = G + (long)k * R_f * R_f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = i0 + wi + 8 * (r >> 2) + 4 * h + (r & 3), j = j0 + wj + l32;
        if (i < R_f && j < R_f && i <= j) {
            const double v = combine16(acc, r, EU[i] + EWk[j]);
            Gk[(long)i * R_f + j] = v;
            if (mirror && parts == 1)
                Gk[(long)j * R_f + i] = v;
        }
    }
}

// The split tail items: part 0's tile in G plus the later parts' slots, in
// part order; then the mirrored entries.  Workgroup (x, r): tail item r of
// XCD x.
// one workgroup per (XCD x, tail item r, block of kTailRows rows of the tile)
constexpr int kTailRows = 8;
__global__ __launch_bounds__(256) void gram_i8_tail_sum(double *__restrict__ G, int R_f, int R_N,
                                                        int ntri, const int *__restrict__ cls,
                                                        int mirror, int cux,
                                                        const double *__restrict__ slab)
{
    const int x = blockIdx.x, r = blockIdx.y, a0 = blockIdx.z * kTailRows;
    const XcdList XL = xcd_list(x, cls, R_N, ntri, cux);
    if (XL.P < 2 || r >= XL.rem)
        return;
    int k, t;
    xcd_item(XL, x, XL.full + r, cls, R_N, ntri, k, t);
    if (k < 0 || k >= R_N)
        return;
    int tj = 0;
    while ((tj + 1) * (tj + 2) / 2 <= t)
        ++tj;
    const int ti = t - tj * (tj + 1) / 2;
    double *Gk = G + (long)k * R_f * R_f;
#pragma unroll
    for (int e = threadIdx.x; e < kTailRows * GT2; e += 256) {
        const int a = a0 + e / GT2, b = e % GT2;
        const int i = ti * GT2 + a, j = tj * GT2 + b;
        if (i >= R_f || j >= R_f || i > j)
            continue;
        double v = Gk[(long)i * R_f + j];
        for (int p = 1; p < XL.P; ++p)
            v += tail_slot(const_cast<double *>(slab), x, r, p, XL.P)[a * GT2 + b];
        Gk[(long)i * R_f + j] = v;
        if (mirror)
            Gk[(long)j * R_f + i] = v;
    }
}

}  // namespace

OzakiLayout ozaki_layout(int n, int R_f, int R_N)
{
    OzakiLayout L;
    L.n_pad = (n + TA - 1) / TA * TA;  // multiple of both TA and TK
    L.R_f_pad = (R_f + TJ - 1) / TJ * TJ;
    L.off = ozaki_p_offset(n);
    L.LP = ((2 * n - 1 + 2 * kOzakiPad + 16) + 15) / 16 * 16;
    L.uplane = (long)L.R_f_pad * L.n_pad;
    L.pplane = (long)R_N * L.LP;
    L.wplane = (long)R_N * L.R_f_pad * L.n_pad;
    return L;
}

hipError_t launch_split_rows(const double *X, int groups, int rows, int len, int rows_pad,
                             int len_pad, long plane, int8_t *S, int *E, hipStream_t stream)
{
    hipLaunchKernelGGL(split_rows_kernel, dim3(rows_pad, groups), dim3(256), 0, stream, X, rows,
                       len, rows_pad, len_pad, plane, S, E);
    return hipGetLastError();
}

hipError_t launch_split_kernel_vectors(const double *p, int n, int R_N, const OzakiLayout &L,
                                       int8_t *PS, int *EP, hipStream_t stream)
{
    hipLaunchKernelGGL(split_kernel_vectors, dim3(R_N), dim3(256), 0, stream, p, n, L.LP, L.off,
                       L.pplane, PS, EP);
    return hipGetLastError();
}

hipError_t launch_toeplitz_i8(const int8_t *US, const int *EU, const int8_t *PS, const int *EP,
                              const OzakiLayout &L, double *W, int n, int R_f, int R_N,
                              hipStream_t stream)
{
    dim3 grid(L.n_pad / TA, L.R_f_pad / TJ, R_N);
    hipLaunchKernelGGL(toeplitz_i8_kernel, grid, dim3(256), 0, stream, US, EU, L.uplane, L.n_pad,
                       PS, EP, L.pplane, L.LP, L.off, W, n, R_f);
    return hipGetLastError();
}

bool gram_i8_wide(int R_f, int R_f_pad) { return R_f >= 256 && R_f_pad % GT2 == 0; }

static int cus_per_xcd()
{
    static int cux[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 32;
    if (!cux[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v < 8)
            v = 256;
        cux[dev] = v / 8;
    }
    return cux[dev];
}

hipError_t launch_gram_i8(const int8_t *US, const int *EU, const int8_t *WS, const int *EW,
                          const OzakiLayout &L, double *G, int R_f, int R_N, const int *cls,
                          bool mirror, double *tail, hipStream_t stream)
{
    if (gram_i8_wide(R_f, L.R_f_pad)) {
        const int nt = L.R_f_pad / GT2;
        const int ntri = nt * (nt + 1) / 2;
        // all terms: for every XCD x, the terms k = x, x + 8, ... each with ntri
        // tiles; classes given: the items of the listed terms in eight
        // contiguous chunks, one per XCD; with a tail slab, up to kTailSlots
        // more workgroups per XCD for the later K parts of the last round
        // (a multiple of 8 workgroups, the excess exits)
        const int per = cls ? (R_N * ntri + 7) / 8 : ((R_N + 7) / 8) * ntri;
        const int cux = cus_per_xcd();
        const int items = 8 * (per + (tail ? kTailSlots : 0));
        hipLaunchKernelGGL(gram_i8_wide_kernel, dim3(items), dim3(kWideThreads), 0, stream, US, EU,
                           L.uplane, WS, EW, L.wplane, L.n_pad, L.R_f_pad, G, R_f, R_N, ntri,
                           cls, (int)mirror, cux, tail);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !tail)
            return e;
        hipLaunchKernelGGL(gram_i8_tail_sum, dim3(8, cux, GT2 / kTailRows), dim3(256), 0, stream,
                           G, R_f, R_N, ntri, cls, (int)mirror, cux, tail);
        return hipGetLastError();
    }
    const int nt = L.R_f_pad / GT;
    dim3 grid(nt * (nt + 1) / 2, R_N);
    hipLaunchKernelGGL(gram_i8_kernel, grid, dim3(256), 0, stream, US, EU, L.uplane, WS, EW,
                       L.wplane, L.n_pad, L.R_f_pad, G, R_f, nt, R_N, cls, (int)mirror);
    return hipGetLastError();
}

}  // namespace tc
