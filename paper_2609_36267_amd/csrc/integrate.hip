// Integration of the corrected gradients into the integer cycle field K and
// the unwrapped phase (Sections II-A and II-C).
//
// Along every edge K_v - K_u = dk_e - w_e (w_e = wrap count of psi), exact
// in integers, so any integration order gives the same K when the corrected
// gradients are curl-free.  K is fixed by K(ref) = 0.
//
//   k_first_valid : reference pixel = first valid pixel, row-major (atomicMin)
//   k_col0        : one workgroup; column-0 prefix sums K0[i] and K(ref)
//   k_rows        : one workgroup per row; chunked workgroup scan of the
//                   row's x-edge increments, then K and
//                   phi = (float)((double)psi + 2 pi K) (nodata if invalid).
// Bytes per pixel: psi 4 + valid 1 + dk_x 1 read, K 4 + phi 4 written.
#pragma clang fp contract(off)

#include "ww_internal.h"

namespace ww {

constexpr int IT_THREADS = 256;
constexpr int IT_PER = 4;
constexpr int IT_CHUNK = IT_THREADS * IT_PER;

struct IntegState {
    long long first_valid;
    int kref;
    int pad;
};

// First valid pixel (row-major).  One workgroup scans chunks from the start
// and stops at the first chunk holding a valid pixel: typical masks end the
// search in the first chunk, an all-invalid image reads the mask once.
__global__ __launch_bounds__(1024) void k_first_valid(const uint8_t *__restrict__ valid, int64_t N,
                                                     IntegState *st) {
    __shared__ unsigned long long best;
    if (threadIdx.x == 0) best = (unsigned long long)N;
    __syncthreads();
    for (int64_t base = 0; base < N; base += 1024 * 16) {
        const int64_t k0 = base + (int64_t)threadIdx.x * 16;
        for (int q = 0; q < 16; ++q) {
            const int64_t k = k0 + q;
            if (k < N && valid[k]) {
                atomicMin(&best, (unsigned long long)k);
                break;
            }
        }
        __syncthreads();
        if (best < (unsigned long long)N) break;
        __syncthreads();
    }
    if (threadIdx.x == 0) st->first_valid = (long long)best;
}

// Block-wide exclusive scan of one int per thread; returns the exclusive
// prefix and writes the block total to *total.
__device__ int block_exclusive_scan(int v, int *total) {
    __shared__ int wsum[IT_THREADS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        int o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < IT_THREADS / 64; ++w) {
        if (w < wid) before += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

__device__ __forceinline__ int gx_at(const float *psi, const uint8_t *valid, const int8_t *dkx,
                                     int n, int i, int j) {
    const int64_t a = (int64_t)i * n + j;
    return (int)dkx[(int64_t)i * (n - 1) + j] -
           wrap_cycles(phase_at(psi, valid, a + 1) - phase_at(psi, valid, a));
}

__global__ __launch_bounds__(IT_THREADS) void k_col0(const float *__restrict__ psi,
                                                    const uint8_t *__restrict__ valid,
                                                    const int8_t *__restrict__ dkx,
                                                    const int8_t *__restrict__ dky, int m, int n,
                                                    int ref_i, int ref_j, IntegState *st,
                                                    int *__restrict__ K0) {
    int ri = ref_i, rj = ref_j;
    if (ri < 0) {
        long long fv = st->first_valid;
        if (fv >= (long long)m * n) fv = 0;
        ri = (int)(fv / n);
        rj = (int)(fv % n);
    }
    // K0[i] = sum_{i' < i} (dk_y(i',0) - w_y(i',0))
    int carry = 0;
    for (int base = 0; base < m; base += IT_THREADS) {
        const int i = base + threadIdx.x;
        int g = 0;
        if (i >= 1 && i < m) {
            const int64_t a = (int64_t)(i - 1) * n;
            g = (int)dky[(int64_t)(i - 1) * n] -
                wrap_cycles(phase_at(psi, valid, a + n) - phase_at(psi, valid, a));
        }
        int tot;
        int ex = block_exclusive_scan(g, &tot);
        if (i < m) K0[i] = carry + ex + g;
        carry += tot;
    }
    // K(ref) = K0[ri] + sum_{j < rj} g_x(ri, j)
    int part = 0;
    for (int j = threadIdx.x; j < rj; j += IT_THREADS) part += gx_at(psi, valid, dkx, n, ri, j);
    int tot;
    (void)block_exclusive_scan(part, &tot);
    __syncthreads();
    if (threadIdx.x == 0) st->kref = K0[ri] + tot;
}

__global__ __launch_bounds__(IT_THREADS) void k_rows(const float *__restrict__ psi,
                                                    const uint8_t *__restrict__ valid,
                                                    const int8_t *__restrict__ dkx, int m, int n,
                                                    const IntegState *__restrict__ st,
                                                    const int *__restrict__ K0, float nodata,
                                                    int32_t *__restrict__ K,
                                                    float *__restrict__ phi) {
    const int i = blockIdx.x;
    const int64_t row = (int64_t)i * n;
    int carry = K0[i] - st->kref;
    for (int base = 0; base < n; base += IT_CHUNK) {
        const int j0 = base + threadIdx.x * IT_PER;
        float ps[IT_PER + 1];
        uint8_t vd[IT_PER + 1];
        int8_t dk[IT_PER];
#pragma unroll
        for (int q = 0; q <= IT_PER; ++q) {
            const int j = j0 + q;
            if (j < n) {
                vd[q] = valid ? valid[row + j] : 1;
                ps[q] = psi[row + j];
            } else {
                vd[q] = 0;
                ps[q] = 0.f;
            }
        }
#pragma unroll
        for (int q = 0; q < IT_PER; ++q) {
            const int j = j0 + q;
            dk[q] = (j < n - 1) ? dkx[(int64_t)i * (n - 1) + j] : (int8_t)0;
        }
        int g[IT_PER];
        int local = 0;
#pragma unroll
        for (int q = 0; q < IT_PER; ++q) {
            const int j = j0 + q;
            int v = 0;
            if (j < n - 1) {
                const double a = vd[q] ? (double)ps[q] : 0.0;
                const double b = vd[q + 1] ? (double)ps[q + 1] : 0.0;
                v = (int)dk[q] - wrap_cycles(b - a);
            }
            g[q] = v;
            local += v;
        }
        int tot;
        int ex = block_exclusive_scan(local, &tot);
        int k = carry + ex;
#pragma unroll
        for (int q = 0; q < IT_PER; ++q) {
            const int j = j0 + q;
            if (j < n) {
                K[row + j] = k;
                phi[row + j] = vd[q] ? (float)((double)ps[q] + TWO_PI_D * (double)k) : nodata;
            }
            k += g[q];
        }
        carry += tot;
    }
}

ww_status integrate_impl(const float *psi, const uint8_t *valid, const int8_t *dkx,
                         const int8_t *dky, int m, int n, const ww_cost_params &cp, int32_t *K,
                         float *phi, hipStream_t stream) {
    char *buf = nullptr;
    const size_t k0_off = 256;
    WW_TRY(scratch(SLOT_INTEG, k0_off + sizeof(int) * (size_t)m, (void **)&buf));
    IntegState *st = (IntegState *)buf;
    int *K0 = (int *)(buf + k0_off);
    const int64_t N = (int64_t)m * n;
    IntegState init;
    init.first_valid = valid ? (long long)N : 0;
    init.kref = 0;
    init.pad = 0;
    WW_HIP(hipMemcpyAsync(st, &init, sizeof(init), hipMemcpyHostToDevice, stream));
    if (valid && cp.ref_i < 0) {
        hipLaunchKernelGGL(k_first_valid, dim3(1), dim3(1024), 0, stream, valid, N, st);
        WW_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_col0, dim3(1), dim3(IT_THREADS), 0, stream, psi, valid, dkx, dky, m, n,
                       cp.ref_i, cp.ref_j, st, K0);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rows, dim3(m), dim3(IT_THREADS), 0, stream, psi, valid, dkx, m, n, st, K0,
                       cp.nodata, K, phi);
    WW_LAUNCH_CHECK();
    // the host-side init struct must outlive the async copy
    WW_HIP(hipStreamSynchronize(stream));
    return WW_OK;
}

}  // namespace ww
