// Streaming-bandwidth kernels: the measured ceiling that the solver's
// bandwidth-bound kernels are compared with, beside the nominal HBM peak.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ns_api.h"

namespace {

constexpr int kStreamBlock = 256;

// One 16-byte vector per thread over the whole buffer (a grid of bytes/4096
// workgroups): measured the fastest of the shapes tried on MI355X (6.8 TB/s
// read-only over 4 GiB, against 5.2-6.2 TB/s for grid-stride loops with 4-32
// workgroups per CU and 1-8 loads in flight per thread, 6.3-6.7 TB/s with
// non-temporal loads).
__global__ __launch_bounds__(kStreamBlock) void k_stream_read(const uint4* __restrict__ src, int64_t n16,
                                                              uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x;
    uint32_t acc = 0;
    if (i < n16) {
        const uint4 v = src[i];
        acc = v.x ^ v.y ^ v.z ^ v.w;
    }
    // fold what was read into one word per workgroup, written only when it
    // matches a sentinel (so the loads stay and the writes cost nothing)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0 && acc == 0x9e3779b9u) out[blockIdx.x & 1023] = acc;
}

__global__ __launch_bounds__(kStreamBlock) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                              int64_t n16) {
    const int64_t i = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

}  // namespace

extern "C" ns_status ns_stream_bench(int32_t mode, const void* d_src, void* d_dst, size_t bytes, int32_t reps,
                                     double* h_ms) {
    if ((mode != 0 && mode != 1) || !d_src || !d_dst || !h_ms || reps < 1 || bytes < 16 || bytes % 16 != 0 ||
        reinterpret_cast<uintptr_t>(d_src) % 16 != 0 || reinterpret_cast<uintptr_t>(d_dst) % 16 != 0)
        return NS_ERR_ARG;
    const int64_t n16 = (int64_t)(bytes / 16);
    const int64_t blocks = (n16 + kStreamBlock - 1) / kStreamBlock;
    if (blocks > 0x7fffffff) return NS_ERR_ARG;
    const int grid = (int)blocks;
    // the read kernel may write into the first 1024 words of d_dst
    if (mode == 0 && bytes < 1024 * sizeof(uint32_t)) return NS_ERR_ARG;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return NS_ERR_HIP;
    ns_status rc = NS_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = NS_ERR_HIP;
    for (int r = 0; rc == NS_OK && r <= reps; ++r) {  // r == 0 is an untimed warm-up launch
        if (r == 1 && hipEventRecord(e0, st) != hipSuccess) rc = NS_ERR_HIP;
        if (mode == 0)
            hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(kStreamBlock), 0, st,
                               static_cast<const uint4*>(d_src), n16, static_cast<uint32_t*>(d_dst));
        else
            hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(kStreamBlock), 0, st,
                               static_cast<const uint4*>(d_src), static_cast<uint4*>(d_dst), n16);
        if (hipGetLastError() != hipSuccess) rc = NS_ERR_HIP;
    }
    float ms = 0.f;
    if (rc == NS_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = NS_ERR_HIP;
    if (rc == NS_OK) *h_ms = (double)ms / reps;
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    return rc;
}
