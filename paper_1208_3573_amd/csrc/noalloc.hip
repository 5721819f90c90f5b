// Fixed device scratch for the allocation-free apply (diaf_apply_noalloc):
// a file-scope device array that every GPU the library runs on holds until
// the process ends, its per-device address, and a fill kernel that clears a
// part of it without hipMemsetAsync (a memset node misbehaves on replays of a
// captured graph; a kernel does not).
//
// Layout: bytes [0, 256) hold the triangular solve's control words
// (TrsvCtl, cleared before every use); bytes [256, NOALLOC_SCRATCH_BYTES)
// hold the intermediate vector t of the apply.
#include <mutex>

#include "dcommon.h"
#include "factor_kernels.h"
#include "noalloc.h"

namespace diaf {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

__global__ void clear_words_kernel(uint32_t* p, int nwords)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nwords) p[i] = 0u;
}

}  // namespace

Err noalloc_init(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return {DIAF_EINVAL, "allocation-free scratch: device index out of range"};
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return {};
    int cur = -1;
    DIAF_HIP_TRY(hipGetDevice(&cur));
    if (cur != device) return {DIAF_EINVAL, "allocation-free scratch: device not current"};
    void* p = nullptr;
    DIAF_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return {DIAF_EDEVICE, "allocation-free scratch: no device address"};
    g_ptr[device] = p;
    return {};
}

Err noalloc_scratch(int device, void** ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return {DIAF_EINVAL, "allocation-free scratch: device index out of range"};
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device])
        return {DIAF_EDEVICE, "allocation-free scratch: not set up on this device"};
    *ptr = g_ptr[device];
    return {};
}

Err noalloc_clear(void* p, size_t bytes, hipStream_t st)
{
    const int nwords = (int)((bytes + 3) / 4);
    if (nwords == 0) return {};
    hipLaunchKernelGGL(clear_words_kernel, dim3((nwords + 255) / 256), dim3(256), 0, st,
                       (uint32_t*)p, nwords);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

}  // namespace diaf
