// tc_tei_gram_noalloc: tc_tei_gram for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  The workspace is a file-scope device array of
// TC_NOALLOC_SCRATCH_BYTES, one copy per GPU, held until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress (with
// that device current) and only that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tc.h"
#include "tc_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[TC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device), or nullptr on failure.
void *device_scratch(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" tc_status tc_tei_gram_noalloc(const tc_instance *inst, int count, tc_precision prec,
                                         void *stream)
{
    // arguments and sizes first: a problem beyond the static scratch is
    // rejected before any device call
    const tc_status chk = tc::tei_gram_check(inst, count, prec);
    if (chk != TC_OK)
        return chk;
    const size_t need = tc_workspace_bytes(TC_OP_TEI_GRAM, inst, count, prec);
    if (need > (size_t)TC_NOALLOC_SCRATCH_BYTES)
        return TC_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return TC_ERR_HIP;
    void *ws = device_scratch(dev);
    if (!ws)
        return TC_ERR_HIP;
    return tc::tei_gram_call(inst, count, prec, ws, TC_NOALLOC_SCRATCH_BYTES, stream);
}
