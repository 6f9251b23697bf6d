// Split-bfloat16 matrix-core variants of the Toeplitz product and the Gram
// (precisions TC_BF16X3 and TC_BF16X6).
//
// Every operand row is scaled by 2^-e (e from launch_row_exponents, as on the
// binary32 path) and each binary64 entry x is split, exactly in binary64, into
// NP bfloat16 pieces x = x_0 + x_1 + ... + x_{NP-1} + r (x_0 = bf16(x),
// x_i = bf16(x - x_0 - ... - x_{i-1})), |r| <= 2^(-8 NP) |x|.  The products
// x_i y_j with i + j <= NP - 1 (three for NP = 2, six for NP = 3) run on
// v_mfma_f32_16x16x32_bf16 into one binary32 accumulator per output; the
// binary32 sums are flushed into binary64 every 64 contraction indices.
//
//   W[k][j][a] = sum_b U[j][b] p_k[a-b]          (implicit Toeplitz operand)
//   G[k][i][j] = sum_a U[i][a] W[k][j][a]        (upper-triangle tiles, mirrored)
//
// v_mfma_f32_16x16x32_bf16: lane l supplies eight consecutive contraction
// indices of row l%16 of A and of column l%16 of B (the same eight for A and
// B, group l/16), and receives D[4(l/16)+r][l%16], r = 0..3.
// Tiles 64 x 64, four waves of 32 x 32 (2 x 2 blocks), K-step 32.
#include "tc_internal.h"

namespace tc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BT = 64;
constexpr int BK = 32;
constexpr int FLUSH_STEPS = 2;   // binary32 chunks of 64 contraction indices
constexpr int ROWB = 40;         // bf16 per LDS row: 32 + 8 padding (80 bytes)
constexpr int PW = BT + BK - 1;  // 95 lags per K-step
constexpr int PWA = 104;         // window entries incl. the zero tail the 5-dword reads touch

// binary32 -> bfloat16 bits, round to nearest even (finite inputs)
__device__ inline unsigned short bf16_bits(float f)
{
    const unsigned u = __float_as_uint(f);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ inline double bf16_value(unsigned short b)
{
    return (double)__uint_as_float((unsigned)b << 16);
}

// pieces of x (already scaled, |x| < 1): each piece is the bfloat16 nearest
// the binary64 remainder (through binary32; the remainder stays exact)
template <int NP> __device__ inline void split_bf16(double x, unsigned short (&s)[NP])
{
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        s[i] = bf16_bits((float)x);
        x -= bf16_value(s[i]);
    }
}

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

__device__ inline bf16x8 as_bf16x8(u32x4 v)
{
    return __builtin_bit_cast(bf16x8, v);
}

// Implicit-Toeplitz product.  Per K-step the tile needs the lags
// a - b in [a0 - b0 - 31, a0 - b0 + 63]; they are staged lag-reversed,
// Pr[i] = p[a0 - b0 + 63 - i], so that the eight entries a lane needs
// (b = b0 + 8g + e, e = 0..7, at fixed a) are Pr[i0 .. i0 + 7] with
// i0 = 63 - (a - a0) + 8g, read as five dwords and shifted by i0 mod 2.
template <int NP>
__global__ __launch_bounds__(256) void toeplitz_bf16_kernel(const double *__restrict__ p,
                                                            const int *__restrict__ EP,
                                                            const double *__restrict__ U,
                                                            const int *__restrict__ EU,
                                                            double *__restrict__ W, int n, int R_f)
{
    __shared__ __attribute__((aligned(16))) unsigned short Us[2][NP][BT * ROWB];
    __shared__ __attribute__((aligned(16))) unsigned short Pr[2][NP][PWA];

    const int k = blockIdx.z;
    const int a0 = blockIdx.x * BT;
    const int j0 = blockIdx.y * BT;
    const long L = 2L * n - 1;
    const double *pk = p + (long)k * L + (n - 1);

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wj = (wave >> 1) * 32, wa = (wave & 1) * 32;
    const int l16 = lane & 15, g = lane >> 4;
    const int urow = tid >> 2, ucol = (tid & 3) * 8;
    const double uscale = (j0 + urow < R_f) ? ldexp(1.0, -EU[j0 + urow]) : 0.0;
    const double pscale = ldexp(1.0, -EP[k]);

    double ureg[8], preg = 0.0;
    auto load_stage = [&](int b0) {
        const int j = j0 + urow;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int b = b0 + ucol + q;
            ureg[q] = (j < R_f && b < n) ? U[(long)j * n + b] * uscale : 0.0;
        }
        if (tid < PWA) {
            const int lag = a0 - b0 + (BT - 1) - tid;
            preg = (tid < PW && lag > -n && lag < n) ? pk[lag] * pscale : 0.0;
        }
    };
    auto store_stage = [&](int buf) {
        unsigned short s[8][NP];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            unsigned short t[NP];
            split_bf16<NP>(ureg[q], t);
#pragma unroll
            for (int i = 0; i < NP; ++i)
                s[q][i] = t[i];
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            u32x4 v;
#pragma unroll
            for (int h = 0; h < 4; ++h)
                v[h] = (unsigned)s[2 * h][i] | ((unsigned)s[2 * h + 1][i] << 16);
            *reinterpret_cast<u32x4 *>(&Us[buf][i][urow * ROWB + ucol]) = v;
        }
        if (tid < PWA) {
            unsigned short t[NP];
            split_bf16<NP>(preg, t);
#pragma unroll
            for (int i = 0; i < NP; ++i)
                Pr[buf][i][tid] = t[i];
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
        bf16x8 afr[2][NP], bfr[2][NP];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int i = 0; i < NP; ++i)
                afr[x][i] = as_bf16x8(*reinterpret_cast<const u32x4 *>(
                    &Us[buf][i][(wj + 16 * x + l16) * ROWB + 8 * g]));
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int i0 = (BT - 1) - (wa + 16 * y + l16) + 8 * g;
            const int sh = (i0 & 1) * 2;  // byte shift
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const unsigned *w32 = reinterpret_cast<const unsigned *>(Pr[buf][i]) + (i0 >> 1);
                unsigned d[5];
#pragma unroll
                for (int h = 0; h < 5; ++h)
                    d[h] = w32[h];
                u32x4 v;
#pragma unroll
                for (int h = 0; h < 4; ++h)
                    v[h] = __builtin_amdgcn_alignbyte(d[h + 1], d[h], sh);
                bfr[y][i] = as_bf16x8(v);
            }
        }
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int jp = 0; i + jp < NP; ++jp)
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[x][i], bfr[y][jp],
                                                                            acc[x][y], 0, 0, 0);
        if ((s + 1) % FLUSH_STEPS == 0 || s + 1 == nsteps)
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
                const int j = j0 + wj + x * 16 + 4 * g + r;
                if (j < R_f && a < n)
                    Wk[(long)j * n + a] = ldexp(sum[x][y][r], EU[j] + EP[k]);
            }
        }
}

template <int NP>
__global__ __launch_bounds__(256) void gram_bf16_kernel(const double *__restrict__ U,
                                                        const int *__restrict__ EU,
                                                        const double *__restrict__ W,
                                                        const int *__restrict__ EW,
                                                        double *__restrict__ G, int n, int R_f,
                                                        int ntiles, int mirror)
{
    __shared__ __attribute__((aligned(16))) unsigned short As[2][NP][BT * ROWB];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][NP][BT * ROWB];

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
    const int *EWk = EW + (long)k * R_f;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    const int l16 = lane & 15, g = lane >> 4;
    const int lrow = tid >> 2, lcol = (tid & 3) * 8;
    const double ascale = (i0 + lrow < R_f) ? ldexp(1.0, -EU[i0 + lrow]) : 0.0;
    const double bscale = (j0 + lrow < R_f) ? ldexp(1.0, -EWk[j0 + lrow]) : 0.0;

    double areg[8], breg[8];
    auto load_stage = [&](int a0) {
        const int i = i0 + lrow, j = j0 + lrow;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int a = a0 + lcol + q;
            areg[q] = (i < R_f && a < n) ? U[(long)i * n + a] * ascale : 0.0;
            breg[q] = (j < R_f && a < n) ? Wk[(long)j * n + a] * bscale : 0.0;
        }
    };
    auto put = [&](unsigned short (*dst)[BT * ROWB], const double (&src)[8]) {
        unsigned short s[8][NP];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            unsigned short t2[NP];
            split_bf16<NP>(src[q], t2);
#pragma unroll
            for (int i = 0; i < NP; ++i)
                s[q][i] = t2[i];
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            u32x4 v;
#pragma unroll
            for (int h = 0; h < 4; ++h)
                v[h] = (unsigned)s[2 * h][i] | ((unsigned)s[2 * h + 1][i] << 16);
            *reinterpret_cast<u32x4 *>(&dst[i][lrow * ROWB + lcol]) = v;
        }
    };
    auto store_stage = [&](int buf) {
        put(As[buf], areg);
        put(Bs[buf], breg);
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
        bf16x8 afr[2][NP], bfr[2][NP];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int i = 0; i < NP; ++i)
                afr[x][i] = as_bf16x8(*reinterpret_cast<const u32x4 *>(
                    &As[buf][i][(wi + 16 * x + l16) * ROWB + 8 * g]));
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int i = 0; i < NP; ++i)
                bfr[y][i] = as_bf16x8(*reinterpret_cast<const u32x4 *>(
                    &Bs[buf][i][(wj + 16 * y + l16) * ROWB + 8 * g]));
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int jp = 0; i + jp < NP; ++jp)
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[x][i], bfr[y][jp],
                                                                            acc[x][y], 0, 0, 0);
        if ((s + 1) % FLUSH_STEPS == 0 || s + 1 == nsteps)
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
                const int i = i0 + wi + x * 16 + 4 * g + r;
                if (i < R_f && j < R_f && i <= j) {
                    const double v = ldexp(sum[x][y][r], EU[i] + EWk[j]);
                    Gk[(long)i * R_f + j] = v;
                    if (mirror)
                        Gk[(long)j * R_f + i] = v;
                }
            }
        }
}

}  // namespace

hipError_t launch_toeplitz_bf16(const double *p, const int *EP, const double *U, const int *EU,
                                double *W, int n, int R_f, int R_N, int pieces, hipStream_t stream)
{
    dim3 grid((n + BT - 1) / BT, (R_f + BT - 1) / BT, R_N);
    if (pieces == 2)
        hipLaunchKernelGGL(toeplitz_bf16_kernel<2>, grid, dim3(256), 0, stream, p, EP, U, EU, W,
                           n, R_f);
    else if (pieces == 3)
        hipLaunchKernelGGL(toeplitz_bf16_kernel<3>, grid, dim3(256), 0, stream, p, EP, U, EU, W,
                           n, R_f);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_gram_bf16(const double *U, const int *EU, const double *W, const int *EW,
                            double *G, int n, int R_f, int R_N, int pieces, bool mirror,
                            hipStream_t stream)
{
    const int nt = (R_f + BT - 1) / BT;
    dim3 grid(nt * (nt + 1) / 2, R_N);
    if (pieces == 2)
        hipLaunchKernelGGL(gram_bf16_kernel<2>, grid, dim3(256), 0, stream, U, EU, W, EW, G, n,
                           R_f, nt, (int)mirror);
    else if (pieces == 3)
        hipLaunchKernelGGL(gram_bf16_kernel<3>, grid, dim3(256), 0, stream, U, EU, W, EW, G, n,
                           R_f, nt, (int)mirror);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace tc
