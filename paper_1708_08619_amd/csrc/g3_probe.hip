// LDS rate probe of libg3: the measured ceilings behind the triplet kernel's
// roofline.  That kernel's LDS work per candidate pair is one ds_read_b32
// (the bin table) and one ds_add_u32 (the histogram slab, or the lane's own
// trash word for a rejected candidate); the probe times each pattern alone
// and the read+add pair, with one 1024-thread workgroup per CU as the
// triplet kernel runs, each lane cycling through 16 addresses held in
// registers so that nothing but the LDS instructions limits the loop.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "g3.h"

namespace {

constexpr int kProbeThreads = 1024;
constexpr int kProbeAddrs = 16;

typedef __attribute__((address_space(3))) uint32_t lds_u32;

#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wint-to-pointer-cast"
__device__ __forceinline__ void lds_add(uint32_t a)
{
    __hip_atomic_fetch_add((lds_u32*)a, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t lds_read(uint32_t a) { return *(volatile lds_u32*)a; }
__device__ __forceinline__ void lds_store(uint32_t a, uint32_t v) { *(lds_u32*)a = v; }
#pragma clang diagnostic pop

// pattern: 0 add to the lane's own word, 1 add at random words, 2 read at
// random words, 3 read (random) + add (random) per step.  Byte addresses
// from 0 (the kernel declares no static LDS); words = slab size.
__global__ void __launch_bounds__(kProbeThreads) k_lds_probe(int pattern, int words, int iters,
                                                             uint32_t* sink)
{
    const int tid = threadIdx.x;
    for (int x = tid; x < words; x += kProbeThreads) lds_store(4u * (uint32_t)x, 0u);
    __syncthreads();
    uint32_t r = 0x9e3779b9u ^ (uint32_t)(blockIdx.x * kProbeThreads + tid) * 0x85ebca6bu;
    uint32_t a[kProbeAddrs], b[kProbeAddrs];
#pragma unroll
    for (int k = 0; k < kProbeAddrs; ++k) {
        r ^= r << 13; r ^= r >> 17; r ^= r << 5;
        a[k] = 4u * (r % (uint32_t)words);
        r ^= r << 13; r ^= r >> 17; r ^= r << 5;
        b[k] = 4u * (r % (uint32_t)words);
        if (pattern == 0) a[k] = 4u * (uint32_t)(tid & 63) + 256u * (uint32_t)(tid >> 6);
    }
    uint32_t acc = 0;
    if (pattern == 0 || pattern == 1) {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kProbeAddrs; ++k) lds_add(a[k]);
        }
    } else if (pattern == 2) {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kProbeAddrs; ++k) acc += lds_read(a[k]);
        }
    } else {
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kProbeAddrs; ++k) {
                acc += lds_read(b[k]);
                lds_add(a[k]);
            }
        }
    }
    __syncthreads();
    if (tid == 0) acc += lds_read(0u);
    sink[blockIdx.x * kProbeThreads + tid] = acc;
}

}  // namespace

extern "C" g3_status g3_lds_rate(int32_t pattern, int32_t words, double* lane_ops_per_s)
{
    if (!lane_ops_per_s || pattern < 0 || pattern > 3) return G3_EINVAL;
    // pattern 0 uses 64 words per wave of the workgroup
    if (words < 1 || words > 36 * 1024 || (pattern == 0 && words < 16 * 64)) return G3_EINVAL;
    *lane_ops_per_s = 0.0;
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return G3_EDEVICE;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
        return G3_EDEVICE;
    const size_t lds = (size_t)words * 4;
    if (hipFuncSetAttribute((const void*)k_lds_probe, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))
        return G3_EDEVICE;
    uint32_t* sink = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    g3_status status = G3_EDEVICE;
    const int iters = 2048;
    double best = 0.0;
    if (hipMalloc((void**)&sink, sizeof(uint32_t) * (size_t)n_cu * kProbeThreads) == hipSuccess &&
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        status = G3_OK;
        for (int rep = 0; rep < 4 && status == G3_OK; ++rep) {
            (void)hipEventRecord(e0, st);
            hipLaunchKernelGGL(k_lds_probe, dim3(n_cu), dim3(kProbeThreads), lds, st, pattern, words, iters,
                               sink);
            (void)hipEventRecord(e1, st);
            if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                status = G3_EDEVICE;
                break;
            }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double ops = (double)n_cu * kProbeThreads * (double)iters * kProbeAddrs;
            if (rep > 0 && ms > 0) best = std::max(best, ops / (ms * 1e-3));   // first launch warms up
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (sink) (void)hipFree(sink);
    *lane_ops_per_s = best;
    return status;
}
