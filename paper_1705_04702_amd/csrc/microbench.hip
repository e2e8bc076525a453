// microbench.hip -- memory-system microbenchmarks that give the transport
// kernel its roofline denominators on the device it runs on: random 4-byte
// gathers, random FP64/FP32 atomic additions (device or workgroup scope, one
// or several consecutive elements per lane) and a streaming copy, each over
// a chosen working-set size.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/mcrt.h"

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    // splitmix64 finaliser (Steele, Lea & Flood 2014): a cheap bijective hash
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__global__ void gather_kernel(const float *__restrict__ src, uint64_t n, uint64_t iters, float *sink)
{
    uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.0f;
    for (uint64_t i = 0; i < iters; ++i) acc += src[mix64(tid * iters + i) % n];
    if (acc == 1234.5f) sink[0] = acc; // keeps the loads alive
}

template <int SCOPE, int RUN>
__global__ void atomic_f64_kernel(double *dst, uint64_t n, uint64_t iters)
{
    uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = 0; i < iters; i += RUN) {
        uint64_t base = (mix64(tid * iters + i) % (n / RUN)) * RUN;
#pragma unroll
        for (int r = 0; r < RUN; ++r) __hip_atomic_fetch_add(dst + base + r, 1.0, __ATOMIC_RELAXED, SCOPE);
    }
}

// GROUP consecutive lanes add to GROUP consecutive elements (one random
// base per group and iteration): how the L2 handles atomics that arrive
// together for one cache line.
template <int GROUP>
__global__ void atomic_f64_group_kernel(double *dst, uint64_t n, uint64_t iters)
{
    uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t gid = tid / GROUP;
    int r = (int)(tid % GROUP);
    for (uint64_t i = 0; i < iters; ++i) {
        uint64_t base = (mix64(gid * iters + i) % (n / GROUP)) * GROUP;
        __hip_atomic_fetch_add(dst + base + r, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void atomic_f32_kernel(float *dst, uint64_t n, uint64_t iters)
{
    uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = 0; i < iters; ++i) unsafeAtomicAdd(dst + mix64(tid * iters + i) % n, 1.0f);
}

__global__ void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst, uint64_t n16)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) dst[i] = src[i];
}

thread_local std::string g_mb_err;

} // namespace

extern "C" const char *mcrt_microbench_error(void) { return g_mb_err.c_str(); }

// kind: 0 random 4-byte gathers, 1 random FP64 atomics (device scope),
// 2 random FP64 atomics (workgroup scope), 3 random FP32 atomics (device
// scope), 4 streaming copy (bytes read + written), 5 FP64 atomics (device
// scope) in runs of 4 consecutive elements, 6 FP64 atomics (device scope)
// by groups of 8 lanes on 8 consecutive elements (one 64-byte line), 7 the
// same by whole waves on 64 consecutive elements.  bytes = working set; n_ops =
// operations (ignored for the copy).  *rate = operations/s (bytes/s for the
// copy), timed with HIP events on the default stream.
extern "C" int mcrt_microbench(int device, int kind, uint64_t bytes, uint64_t n_ops, double *rate)
{
    if (!rate || bytes < 4096 || kind < 0 || kind > 7) {
        g_mb_err = "microbench: bad arguments";
        return MCRT_EINVAL;
    }
    if (hipSetDevice(device) != hipSuccess) {
        g_mb_err = "microbench: hipSetDevice failed";
        return MCRT_EDEVICE;
    }
    void *buf = nullptr, *buf2 = nullptr;
    if (hipMalloc(&buf, bytes) != hipSuccess) {
        g_mb_err = "microbench: allocation failed";
        return MCRT_ENOMEM;
    }
    if (kind == 4 && hipMalloc(&buf2, bytes) != hipSuccess) {
        (void)hipFree(buf);
        g_mb_err = "microbench: allocation failed";
        return MCRT_ENOMEM;
    }
    hipError_t err = hipMemset(buf, 0, bytes);
    const int block = 256, grid = 256 * 32;
    const uint64_t threads = (uint64_t)block * grid;
    uint64_t iters = (n_ops + threads - 1) / threads;
    if (kind == 5) iters = (iters + 3) / 4 * 4;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) { // first pass warms up
        (void)hipEventRecord(e0, 0);
        switch (kind) {
        case 0:
            hipLaunchKernelGGL(gather_kernel, dim3(grid), dim3(block), 0, 0, (const float *)buf, bytes / 4, iters,
                               (float *)buf);
            break;
        case 1:
            hipLaunchKernelGGL((atomic_f64_kernel<__HIP_MEMORY_SCOPE_AGENT, 1>), dim3(grid), dim3(block), 0, 0,
                               (double *)buf, bytes / 8, iters);
            break;
        case 2:
            hipLaunchKernelGGL((atomic_f64_kernel<__HIP_MEMORY_SCOPE_WORKGROUP, 1>), dim3(grid), dim3(block), 0, 0,
                               (double *)buf, bytes / 8, iters);
            break;
        case 3:
            hipLaunchKernelGGL(atomic_f32_kernel, dim3(grid), dim3(block), 0, 0, (float *)buf, bytes / 4, iters);
            break;
        case 4:
            hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(block), 0, 0, (const uint4 *)buf, (uint4 *)buf2,
                               bytes / 16);
            break;
        case 5:
            hipLaunchKernelGGL((atomic_f64_kernel<__HIP_MEMORY_SCOPE_AGENT, 4>), dim3(grid), dim3(block), 0, 0,
                               (double *)buf, bytes / 8, iters);
            break;
        case 6:
            hipLaunchKernelGGL((atomic_f64_group_kernel<8>), dim3(grid), dim3(block), 0, 0, (double *)buf, bytes / 8,
                               iters);
            break;
        case 7:
            hipLaunchKernelGGL((atomic_f64_group_kernel<64>), dim3(grid), dim3(block), 0, 0, (double *)buf,
                               bytes / 8, iters);
            break;
        }
        err = hipGetLastError();
        if (err == hipSuccess) err = hipEventRecord(e1, 0);
    }
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (buf2) (void)hipFree(buf2);
    if (err != hipSuccess) {
        g_mb_err = std::string("microbench: ") + hipGetErrorString(err);
        return MCRT_EDEVICE;
    }
    double secs = ms * 1e-3;
    if (kind == 4) *rate = 2.0 * (double)bytes / secs;
    else *rate = (double)(iters * threads) / secs;
    return MCRT_OK;
}
