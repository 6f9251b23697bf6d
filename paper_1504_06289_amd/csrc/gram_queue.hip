// Persistent int8 Gram over a device work queue: the Grams of every mode of
// every instance of a batch in one launch.
//
// The host lists one job per (instance, mode): the int8 slices of U and W
// with their exponents, the Gram destination, the term classes (terms of
// class -2 are skipped: their Grams come from the low-rank path), the tile
// edge (64 or 128) and the number of K parts.  Jobs are sorted by cost (the
// padded cell count, i.e. the contraction length, then the padded R_f), and
// the queue is the concatenation of their items: for each term, each K part
// and each upper-triangle tile (column by column), one item.  The table goes
// to device memory through kernel arguments (gq_write_jobs), so the whole
// batch can be captured in a graph without host buffers that must outlive
// it.
//
// One 512-thread workgroup per CU takes items from an atomic counter until
// the queue is exhausted, so long items start first and the short ones fill
// the tail.  An item is the int8 Gram tile of the Ozaki scheme (ten slice
// products accumulated exactly in int32, binary64 recombination; see
// ozaki.hip) over its K range: for 128-tiles eight waves of 32 x 64, for
// 64-tiles eight waves of 16 x 32, double-buffered LDS with XOR-permuted
// 16-byte chunks.  Rows beyond a job's padded R_f (128-tiles over slices
// padded to 64) are staged as zeros.  With two K parts, part 0 writes the
// Gram and part 1 a slab of the same layout; gq_add_slab then adds the slab
// (fixed order, so the result is bitwise reproducible).
#include "tc_internal.h"

namespace tc {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;
constexpr int TKQ = 64;                 // K-step (bytes of one row per slice)
constexpr int kRowBytes = 64;
constexpr int kOperandBytes = 4 * 128 * kRowBytes;  // 4 slices x 128 rows

__device__ inline int lds_off(int sl, int row, int c16, int GT)
{
    const int swz = ((row >> 1) ^ (row >> 2)) & 3;
    return sl * GT * kRowBytes + row * kRowBytes + 16 * (c16 ^ swz);
}

__device__ inline double combine4(const v4i *acc, int r, int E)
{
    // smallest scale first; each term is exact
    double v = ldexp((double)acc[3][r], -21);
    v += ldexp((double)acc[2][r], -14);
    v += ldexp((double)acc[1][r], -7);
    v += (double)acc[0][r];
    return ldexp(v, E);
}

// One item: tile (ti, tj) of term k of job J, K steps [s0, s1).
template <int GT>
__device__ void gram_tile(const GramJob &J, int k, int ti, int tj, int s0, int s1, bool to_slab,
                          int8_t *lds)
{
    constexpr int XI = GT / 64;         // 16-row blocks per wave (4 wave rows)
    constexpr int YJ = GT / 32;         // 16-column blocks per wave (2 wave columns)
    constexpr int CH = GT * 4 * 4;      // 16-byte chunks per operand and stage
    constexpr int PER = CH / kThreads;  // per thread
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wi = (wave >> 1) * (GT / 4), wj = (wave & 1) * (GT / 2);
    const int l16 = lane & 15, g = lane >> 4;
    const int i0 = ti * GT, j0 = tj * GT;
    const int8_t *Wk = J.WS + (long)k * J.R_f_pad * J.n_pad;
    int8_t *As[2] = {lds, lds + 2 * kOperandBytes};
    int8_t *Bs[2] = {lds + kOperandBytes, lds + 3 * kOperandBytes};

    v4i areg[PER], breg[PER];
    auto load_stage = [&](int a0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int c = tid + kThreads * q;
            const int sl = c / (GT * 4), row = (c % (GT * 4)) >> 2, c16 = c & 3;
            const v4i z = v4i{0, 0, 0, 0};
            areg[q] = i0 + row < J.R_f_pad
                          ? *reinterpret_cast<const v4i *>(J.US + sl * J.uplane +
                                                           (long)(i0 + row) * J.n_pad + a0 +
                                                           16 * c16)
                          : z;
            breg[q] = j0 + row < J.R_f_pad
                          ? *reinterpret_cast<const v4i *>(Wk + sl * J.wplane +
                                                           (long)(j0 + row) * J.n_pad + a0 +
                                                           16 * c16)
                          : z;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int c = tid + kThreads * q;
            const int sl = c / (GT * 4), row = (c % (GT * 4)) >> 2, c16 = c & 3;
            const int o = lds_off(sl, row, c16, GT);
            *reinterpret_cast<v4i *>(As[buf] + o) = areg[q];
            *reinterpret_cast<v4i *>(Bs[buf] + o) = breg[q];
        }
    };

    v4i acc[XI][YJ][4];
#pragma unroll
    for (int x = 0; x < XI; ++x)
#pragma unroll
        for (int y = 0; y < YJ; ++y)
#pragma unroll
            for (int d = 0; d < 4; ++d)
                acc[x][y][d] = v4i{0, 0, 0, 0};

    const int nsteps = s1 - s0;
    load_stage(s0 * TKQ);
    store_stage(0);
    if (nsteps > 1)
        load_stage((s0 + 1) * TKQ);
    __syncthreads();
    for (int s = 0; s < nsteps; ++s) {
        const int cur = s & 1;
        if (s + 1 < nsteps)
            store_stage(cur ^ 1);
        if (s + 2 < nsteps)
            load_stage((s0 + s + 2) * TKQ);
        v4i afr[XI][4];
#pragma unroll
        for (int sl = 0; sl < 4; ++sl)
#pragma unroll
            for (int x = 0; x < XI; ++x)
                afr[x][sl] = *reinterpret_cast<const v4i *>(
                    As[cur] + lds_off(sl, wi + 16 * x + l16, g, GT));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v4i bfr[YJ];
#pragma unroll
            for (int y = 0; y < YJ; ++y)
                bfr[y] = *reinterpret_cast<const v4i *>(Bs[cur] +
                                                        lds_off(j, wj + 16 * y + l16, g, GT));
#pragma unroll
            for (int i = 0; i + j <= 3; ++i)
#pragma unroll
                for (int x = 0; x < XI; ++x)
#pragma unroll
                    for (int y = 0; y < YJ; ++y)
                        acc[x][y][i + j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                            afr[x][i], bfr[y], acc[x][y][i + j], 0, 0, 0);
        }
        __syncthreads();
    }

    const long F2 = (long)J.R_f * J.R_f;
    double *Gk = (to_slab ? J.slab : J.G) + (long)k * F2;
    const int *EWk = J.EW + (long)k * J.R_f_pad;
#pragma unroll
    for (int x = 0; x < XI; ++x)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + wi + 16 * x + 4 * g + r;
            if (i >= J.R_f)
                continue;
#pragma unroll
            for (int y = 0; y < YJ; ++y) {
                const int j = j0 + wj + 16 * y + l16;
                if (j < J.R_f && i <= j) {
                    const double v = combine4(acc[x][y], r, J.EU[i] + EWk[j]);
                    Gk[(long)i * J.R_f + j] = v;
                    if (J.mirror)
                        Gk[(long)j * J.R_f + i] = v;
                }
            }
        }
}

__global__ __launch_bounds__(kThreads) void gq_gram_kernel(const GramJob *__restrict__ jobs,
                                                           int njobs, int total,
                                                           int *__restrict__ counter)
{
    __shared__ __attribute__((aligned(16))) int8_t lds[4 * kOperandBytes];
    __shared__ int item_sh;
    for (;;) {
        if (threadIdx.x == 0)
            item_sh = atomicAdd(counter, 1);
        __syncthreads();
        const int item = item_sh;
        __syncthreads();  // item_sh is rewritten only after every thread read it
        if (item >= total)
            break;
        // the job holding this item: the last with item_begin <= item
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].item_begin <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const GramJob &J = jobs[lo];
        int local = item - J.item_begin;
        const int per_term = J.ntri * J.kparts;
        const int k = local / per_term;
        local -= k * per_term;
        const int part = local / J.ntri;
        const int t = local - part * J.ntri;
        if (J.cls && J.cls[k] == -2)
            continue;  // smooth term: its Gram is formed at low rank
        int tj = 0;
        while ((tj + 1) * (tj + 2) / 2 <= t)
            ++tj;
        const int ti = t - tj * (tj + 1) / 2;
        const int nsteps = J.n_pad / TKQ;
        const int s0 = (int)((long)part * nsteps / J.kparts);
        const int s1 = (int)((long)(part + 1) * nsteps / J.kparts);
        if (J.tile == 128)
            gram_tile<128>(J, k, ti, tj, s0, s1, part > 0, lds);
        else
            gram_tile<64>(J, k, ti, tj, s0, s1, part > 0, lds);
    }
}

__global__ void gq_write_jobs_kernel(GramJobChunk ch, GramJob *jobs)
{
    const int i = threadIdx.x;
    if (i < ch.count)
        jobs[ch.base + i] = ch.job[i];
}

__global__ void gq_counter_kernel(int *counter) { *counter = 0; }

// G[k][e] += slab[k][e] over the upper triangle (both triangles when the job
// mirrors) of the terms the queue processed
__global__ __launch_bounds__(256) void gq_add_slab_kernel(GramJob J)
{
    const int k = blockIdx.y;
    if (J.cls && J.cls[k] == -2)
        return;
    const long F2 = (long)J.R_f * J.R_f;
    double *G = J.G + (long)k * F2;
    const double *S = J.slab + (long)k * F2;
    for (long e = blockIdx.x * 256L + threadIdx.x; e < F2; e += (long)gridDim.x * 256) {
        const int i = (int)(e / J.R_f), j = (int)(e % J.R_f);
        if (i <= j || J.mirror)
            G[e] = G[e] + S[e];
    }
}

int device_cus()
{
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    if (!cus[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            v <= 0)
            v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

}  // namespace

hipError_t launch_gram_queue(const GramJob *host_jobs, int njobs, int total, GramJob *dev_jobs,
                             int *counter, hipStream_t st)
{
    for (int base = 0; base < njobs; base += kGramJobChunk) {
        GramJobChunk ch;
        ch.base = base;
        ch.count = njobs - base < kGramJobChunk ? njobs - base : kGramJobChunk;
        for (int i = 0; i < ch.count; ++i)
            ch.job[i] = host_jobs[base + i];
        hipLaunchKernelGGL(gq_write_jobs_kernel, dim3(1), dim3(kGramJobChunk), 0, st, ch,
                           dev_jobs);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(gq_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || total == 0)
        return e;
    const int grid = total < device_cus() ? total : device_cus();
    hipLaunchKernelGGL(gq_gram_kernel, dim3(grid), dim3(kThreads), 0, st, dev_jobs, njobs, total,
                       counter);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    for (int i = 0; i < njobs; ++i) {
        const GramJob &J = host_jobs[i];
        if (J.kparts < 2)
            continue;
        const long F2 = (long)J.R_f * J.R_f;
        long blocks = (F2 + 255) / 256;
        if (blocks > 1024)
            blocks = 1024;
        hipLaunchKernelGGL(gq_add_slab_kernel, dim3((unsigned)blocks, J.R_N), dim3(256), 0, st,
                           J);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace tc
