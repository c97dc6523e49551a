// Streaming-bandwidth kernels: the measured ceiling that the solver's
// bandwidth-bound kernels are compared with, beside the nominal HBM peak.
// Both move 16-byte vectors with a grid-stride loop, four loads in flight per
// thread; the read-only kernel folds what it reads into one word per
// workgroup so no load can be dropped.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ns_api.h"

namespace {

constexpr int kStreamBlock = 256;
constexpr int kUnroll = 4;

__global__ __launch_bounds__(kStreamBlock) void k_stream_read(const uint4* __restrict__ src, int64_t n16,
                                                              uint32_t* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kStreamBlock;
    int64_t i = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x;
    uint32_t acc = 0;
    for (; i + (kUnroll - 1) * stride < n16; i += kUnroll * stride) {
        uint4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n16; i += stride) {
        const uint4 v = src[i];
        acc += v.x ^ v.y ^ v.z ^ v.w;
    }
    __shared__ uint32_t lds[kStreamBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kStreamBlock / 64; ++w) s += lds[w];
        out[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kStreamBlock) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                              int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * kStreamBlock;
    int64_t i = (int64_t)blockIdx.x * kStreamBlock + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n16; i += kUnroll * stride) {
        uint4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) dst[i + u * stride] = v[u];
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" ns_status ns_stream_bench(int32_t mode, const void* d_src, void* d_dst, size_t bytes, int32_t reps,
                                     double* h_ms) {
    if ((mode != 0 && mode != 1) || !d_src || !d_dst || !h_ms || reps < 1 || bytes < 16 || bytes % 16 != 0 ||
        reinterpret_cast<uintptr_t>(d_src) % 16 != 0 || reinterpret_cast<uintptr_t>(d_dst) % 16 != 0)
        return NS_ERR_ARG;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return NS_ERR_HIP;
    const int64_t n16 = (int64_t)(bytes / 16);
    // eight workgroups per CU keep every CU streaming; the read kernel's
    // per-workgroup words go to the start of d_dst
    const int64_t want = (int64_t)cus * 8;
    const int64_t need = (n16 + kStreamBlock - 1) / kStreamBlock;
    const int grid = (int)(want < need ? want : need);
    if (mode == 0 && (size_t)grid * sizeof(uint32_t) > bytes) return NS_ERR_ARG;
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
