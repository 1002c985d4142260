// Streaming ceilings of the device, measured with hand-written kernels: the
// bandwidth a plain grid sweep reaches with 16-byte accesses, against which
// the streaming steps of the unwrapper (residues, edge costs, integration)
// are judged.  Not part of the unwrapping path.
#include <algorithm>

#include "ww_internal.h"

namespace ww {

constexpr int PR_THREADS = 256;
constexpr int PR_UNROLL = 4;      // 16-byte words in flight per thread
constexpr int PR_GRID = 2048;     // workgroups (8 per CU)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte word

// dst[k] = src[k] over n 16-byte words: every load of an iteration issued
// before its stores.
template <bool NT>
__global__ __launch_bounds__(PR_THREADS) void k_probe_copy(const u32x4 *__restrict__ src,
                                                           u32x4 *__restrict__ dst, long long n) {
    const long long stride = (long long)gridDim.x * PR_THREADS * PR_UNROLL;
    for (long long base = (long long)blockIdx.x * PR_THREADS * PR_UNROLL + threadIdx.x; base < n;
         base += stride) {
        u32x4 v[PR_UNROLL];
#pragma unroll
        for (int u = 0; u < PR_UNROLL; ++u) {
            const long long k = base + (long long)u * PR_THREADS;
            if (k < n) v[u] = NT ? __builtin_nontemporal_load(src + k) : src[k];
        }
#pragma unroll
        for (int u = 0; u < PR_UNROLL; ++u) {
            const long long k = base + (long long)u * PR_THREADS;
            if (k < n) {
                if (NT)
                    __builtin_nontemporal_store(v[u], dst + k);
                else
                    dst[k] = v[u];
            }
        }
    }
}

// Reads n 16-byte words; each workgroup writes the XOR of what it read
// (so that no load is dead) to out[blockIdx.x].
__global__ __launch_bounds__(PR_THREADS) void k_probe_read(const u32x4 *__restrict__ src, long long n,
                                                           u32x4 *__restrict__ out) {
    const long long stride = (long long)gridDim.x * PR_THREADS * PR_UNROLL;
    u32x4 acc = u32x4{0u, 0u, 0u, 0u};
    for (long long base = (long long)blockIdx.x * PR_THREADS * PR_UNROLL + threadIdx.x; base < n;
         base += stride) {
        u32x4 v[PR_UNROLL];
#pragma unroll
        for (int u = 0; u < PR_UNROLL; ++u) {
            const long long k = base + (long long)u * PR_THREADS;
            v[u] = k < n ? src[k] : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < PR_UNROLL; ++u) {
            acc.x ^= v[u].x;
            acc.y ^= v[u].y;
            acc.z ^= v[u].z;
            acc.w ^= v[u].w;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc.x ^= __shfl_xor(acc.x, off, 64);
        acc.y ^= __shfl_xor(acc.y, off, 64);
        acc.z ^= __shfl_xor(acc.z, off, 64);
        acc.w ^= __shfl_xor(acc.w, off, 64);
    }
    __shared__ u32x4 part[PR_THREADS / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        u32x4 s = part[0];
        for (int w = 1; w < PR_THREADS / 64; ++w) {
            s.x ^= part[w].x;
            s.y ^= part[w].y;
            s.z ^= part[w].z;
            s.w ^= part[w].w;
        }
        out[blockIdx.x] = s;
    }
}

}  // namespace ww

using namespace ww;

extern "C" ww_status ww_stream_probe(const void *src, void *dst, int64_t bytes, int32_t mode,
                                     int32_t reps, float *ms_host, void *stream) {
    clear_error();
    if (!src || !dst || !ms_host || bytes <= 0 || bytes % 16 != 0 || reps < 1 || mode < 0 ||
        mode > 2 || ((uintptr_t)src % 16) != 0 || ((uintptr_t)dst % 16) != 0)
        return fail(WW_E_INVALID_ARG,
                    "stream probe: need 16-byte aligned buffers, bytes a positive multiple of 16, "
                    "reps >= 1 and mode 0, 1 or 2");
    hipStream_t st = (hipStream_t)stream;
    const long long n = bytes / 16;
    const int grid = (int)std::min<long long>(PR_GRID, std::max<long long>(1, (n + PR_THREADS * PR_UNROLL - 1) /
                                                                                  (PR_THREADS * PR_UNROLL)));
    hipEvent_t e0, e1;
    WW_HIP(hipEventCreate(&e0));
    WW_HIP(hipEventCreate(&e1));
    auto launch = [&]() {
        if (mode == 0)
            hipLaunchKernelGGL(k_probe_copy<false>, dim3(grid), dim3(PR_THREADS), 0, st,
                               (const u32x4 *)src, (u32x4 *)dst, n);
        else if (mode == 2)
            hipLaunchKernelGGL(k_probe_copy<true>, dim3(grid), dim3(PR_THREADS), 0, st,
                               (const u32x4 *)src, (u32x4 *)dst, n);
        else
            hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(PR_THREADS), 0, st, (const u32x4 *)src,
                               n, (u32x4 *)dst);
    };
    launch();  // warm
    ww_status rc = WW_OK;
    if (hipGetLastError() != hipSuccess) rc = fail(WW_E_DEVICE, "stream probe launch failed");
    if (rc == WW_OK) {
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps; ++r) launch();
        (void)hipEventRecord(e1, st);
        float ms = 0.f;
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = fail(WW_E_DEVICE, "stream probe timing failed");
        else
            *ms_host = ms / (float)reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
