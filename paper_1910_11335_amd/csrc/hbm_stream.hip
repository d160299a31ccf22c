// Plain HBM streaming kernels (read only, write only, copy) that show the
// bandwidth a kernel on this device reaches when it does nothing but stream:
// the measured ceiling beside the published 8 TB/s, against which the
// sweep's and the contractions' rates are read.  Not part of the solver.
//
// Each lane moves 16 bytes per access (one buffer_load/store_dwordx4), four
// accesses in flight per loop trip, grid-stride over the buffer; NT = 1 adds
// the non-temporal hint (the data is not kept in the caches).
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hbm_stream.h"

namespace {

typedef unsigned V4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ V4 ld(const V4 *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT>
__device__ __forceinline__ void st(V4 *p, V4 v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

constexpr int kUnroll = 4;

// n: 16-byte vectors; every kernel covers [0, n) exactly once.
template <bool NT>
__global__ __launch_bounds__(256) void k_stream_read(const V4 *src, long n, unsigned *sink)
{
    const long stride = (long)gridDim.x * 256;
    long i = blockIdx.x * 256L + threadIdx.x;
    unsigned acc = 0;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        V4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = ld<NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n; i += stride) {
        const V4 v = ld<NT>(src + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9E3779B9u) sink[0] = acc;  // keeps the loads; practically never stores
}

template <bool NT>
__global__ __launch_bounds__(256) void k_stream_write(V4 *dst, long n)
{
    const long stride = (long)gridDim.x * 256;
    long i = blockIdx.x * 256L + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const unsigned x = (unsigned)(i + u * stride);
            st<NT>(dst + i + u * stride, V4{x, x + 1u, x + 2u, x + 3u});
        }
    }
    for (; i < n; i += stride) {
        const unsigned x = (unsigned)i;
        st<NT>(dst + i, V4{x, x + 1u, x + 2u, x + 3u});
    }
}

template <bool NT>
__global__ __launch_bounds__(256) void k_stream_copy(V4 *dst, const V4 *src, long n)
{
    const long stride = (long)gridDim.x * 256;
    long i = blockIdx.x * 256L + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        V4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = ld<NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) st<NT>(dst + i + u * stride, v[u]);
    }
    for (; i < n; i += stride) st<NT>(dst + i, ld<NT>(src + i));
}

void launch(int kind, int nt, void *dst, const void *src, long n, int blocks, unsigned *sink, hipStream_t s)
{
    const dim3 g((unsigned)blocks), b(256);
    if (kind == HBM_STREAM_READ) {
        if (nt) hipLaunchKernelGGL(k_stream_read<true>, g, b, 0, s, (const V4 *)src, n, sink);
        else hipLaunchKernelGGL(k_stream_read<false>, g, b, 0, s, (const V4 *)src, n, sink);
    } else if (kind == HBM_STREAM_WRITE) {
        if (nt) hipLaunchKernelGGL(k_stream_write<true>, g, b, 0, s, (V4 *)dst, n);
        else hipLaunchKernelGGL(k_stream_write<false>, g, b, 0, s, (V4 *)dst, n);
    } else {
        if (nt) hipLaunchKernelGGL(k_stream_copy<true>, g, b, 0, s, (V4 *)dst, (const V4 *)src, n);
        else hipLaunchKernelGGL(k_stream_copy<false>, g, b, 0, s, (V4 *)dst, (const V4 *)src, n);
    }
}

}  // namespace

extern "C" int hbm_stream_run(int kind, int nt, void *dst, const void *src, size_t bytes, int blocks, int reps,
                              void *stream, float *ms)
{
    if (kind < HBM_STREAM_READ || kind > HBM_STREAM_COPY || (nt != 0 && nt != 1) || bytes % 16 || bytes == 0 ||
        blocks < 1 || reps < 1 || !ms)
        return 1;
    if (!dst || (kind != HBM_STREAM_WRITE && !src)) return 1;
    if (((uintptr_t)dst | (uintptr_t)src) % 16) return 1;
    hipStream_t s = (hipStream_t)stream;
    const long n = (long)(bytes / 16);
    unsigned *sink = (unsigned *)dst;  // the read kernel's guard store (never taken in practice)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 2;
    int rc = 0;
    launch(kind, nt, dst, src, n, blocks, sink, s);  // untimed warm-up
    if (hipEventRecord(e0, s) != hipSuccess) rc = 2;
    for (int r = 0; r < reps && !rc; ++r) launch(kind, nt, dst, src, n, blocks, sink, s);
    if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = 2;
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = 2;
    if (!rc && hipGetLastError() != hipSuccess) rc = 2;
    float t = 0.0f;
    if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = 2;
    *ms = t / (float)reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
