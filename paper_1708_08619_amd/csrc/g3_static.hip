// Static device scratch of libg3 for g3_accumulate_noalloc, the entry point
// for callers that cannot allocate device memory, and the small kernel that
// writes its tables (passed by value as kernel arguments, so no host staging
// buffer is needed either).
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy, of kStaticScratchBytes, from the moment the module is loaded
// until the process ends.  In host code its name only stands in for the
// symbol; the device address of each GPU's copy is looked up once per device
// with hipGetSymbolAddress (static_scratch), and only that address is ever
// passed to kernels or used for device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "g3_device.h"

namespace g3 {

namespace {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_done[kMaxDevices] = {};
void* g_addr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

struct PutArgs {
    uint32_t n;
    uint32_t w[kPutWords];
};

__global__ void __launch_bounds__(256) k_put_words(uint32_t* __restrict__ dst, PutArgs a)
{
    for (uint32_t i = threadIdx.x; i < a.n; i += 256) dst[i] = a.w[i];
}

}  // namespace

void* static_scratch(int device, hipError_t* err)
{
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[device]) {
        // the caller has made `device` current: this is its copy's address
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_addr[device] = e == hipSuccess ? p : nullptr;
        g_err[device] = e;
        g_done[device] = true;
    }
    *err = g_err[device];
    return g_addr[device];
}

void launch_put_words(uint32_t* dst, const uint32_t* src, size_t n_words, hipStream_t s)
{
    PutArgs a;
    for (size_t o = 0; o < n_words; o += kPutWords) {
        const size_t n = n_words - o < (size_t)kPutWords ? n_words - o : (size_t)kPutWords;
        a.n = (uint32_t)n;
        for (size_t i = 0; i < n; ++i) a.w[i] = src[o + i];
        hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s, dst + o, a);
    }
}

}  // namespace g3
