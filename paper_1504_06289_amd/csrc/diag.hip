// Diagnostics behind environment switches (read at every call):
//   TC_CHECK_FINITE=1  the binary64 inputs of a call are scanned for NaN and
//                      Inf before any work is enqueued; the call then
//                      synchronises its stream once to read the result.
//   TC_DEBUG_SYNC=1    every kernel launch is followed by a synchronisation
//                      of its stream, and the first failing kernel is named
//                      on stderr.
// Both synchronise, so neither may be on while a call is captured in a graph.
//   TC_CHOL_COLUMNS=1  the pivoted Cholesky drivers form each pivot's column
//                      from the factors, the path they take on their own only
//                      beyond the sizes where the matrix is formed (a check
//                      of that path at small sizes).
#include <stdio.h>
#include <stdlib.h>

#include <mutex>

#include "tc_internal.h"

namespace tc {

namespace {

// one flag per device: set to 1 by any thread that meets a non-finite value
static __device__ int nonfinite_flag;

constexpr int kMaxDevices = 64;
std::mutex g_flag_mu;
int *g_flag_ptr[kMaxDevices] = {};

int *device_flag()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_flag_mu);
    if (!g_flag_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(nonfinite_flag)) != hipSuccess || !ptr)
            return nullptr;
        g_flag_ptr[dev] = (int *)ptr;
    }
    return g_flag_ptr[dev];
}

__global__ __launch_bounds__(256) void flag_nonfinite_kernel(const double *__restrict__ x,
                                                             long count, int *flag)
{
    bool bad = false;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < count; i += (long)gridDim.x * 256)
        bad |= !isfinite(x[i]);
    if (bad)
        *flag = 1;  // every writer stores the same value
}

__global__ void set_flag_kernel(int *flag, int v) { *flag = v; }

bool env_on(const char *name)
{
    const char *v = getenv(name);
    return v && v[0] && !(v[0] == '0' && v[1] == 0);
}

}  // namespace

bool check_finite_on() { return env_on("TC_CHECK_FINITE"); }
bool debug_sync_on() { return env_on("TC_DEBUG_SYNC"); }
bool chol_columns_on() { return env_on("TC_CHOL_COLUMNS"); }

bool debug_sync_check(const char *kernel, hipStream_t st)
{
    const hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess)
        return true;
    fprintf(stderr, "tc: kernel %s failed: %s\n", kernel, hipGetErrorString(e));
    return false;
}

int scan_nonfinite(const FiniteSpan *spans, int count, hipStream_t st)
{
    int *flag = device_flag();
    if (!flag)
        return -1;
    hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(1), 0, st, flag, 0);
    if (hipGetLastError() != hipSuccess)
        return -1;
    for (int i = 0; i < count; ++i) {
        if (!spans[i].x || spans[i].count <= 0)
            continue;
        long blocks = (spans[i].count + 255) / 256;
        if (blocks > 4096)
            blocks = 4096;
        hipLaunchKernelGGL(flag_nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                           spans[i].x, spans[i].count, flag);
        if (hipGetLastError() != hipSuccess)
            return -1;
    }
    int h = 0;
    if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return -1;
    return h ? 1 : 0;
}

}  // namespace tc
