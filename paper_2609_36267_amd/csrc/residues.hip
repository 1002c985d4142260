// Residues of every 2x2 loop (Section II-A, eq. 1) and the one-sided charges
// of the boundary ring.
//
// One thread per loop column j walks a strip of ROWS loop rows.  Pixel row
// i+1 read in one step is row i of the next, so every psi/valid byte is
// fetched once per strip (plus one halo row); the right neighbour (j+1) is a
// second load that hits the same cache line.  Lanes are consecutive in j, so
// every load and the int8 store are coalesced.  Bytes moved per loop:
// 4 (psi) + 1 (valid) + 1 (res) = 6.
#include "ww_internal.h"

namespace ww {

constexpr int RES_ROWS = 32;
constexpr int RES_THREADS = 256;

__global__ __launch_bounds__(RES_THREADS) void k_residues(const float *__restrict__ psi,
                                                          const uint8_t *__restrict__ valid,
                                                          int m, int n, int8_t *__restrict__ res,
                                                          int64_t *__restrict__ ground) {
    const int j = blockIdx.x * RES_THREADS + threadIdx.x;
    const int i0 = blockIdx.y * RES_ROWS;
    const int C = n - 1;
    int sum = 0;
    if (j < C) {
        int64_t a = (int64_t)i0 * n + j;
        double p0 = phase_at(psi, valid, a), p1 = phase_at(psi, valid, a + 1);
        int w_top = wrap_cycles(p1 - p0);  // hx(i0, j)
        const int iend = min(i0 + RES_ROWS, m - 1);
        for (int i = i0; i < iend; ++i) {
            int64_t b = a + n;
            double q0 = phase_at(psi, valid, b), q1 = phase_at(psi, valid, b + 1);
            int w_bot = wrap_cycles(q1 - q0);    // hx(i+1, j)
            int w_left = wrap_cycles(q0 - p0);   // vy(i, j)
            int w_right = wrap_cycles(q1 - p1);  // vy(i, j+1)
            int r = -(w_top + w_right - w_bot - w_left);
            res[(int64_t)i * C + j] = (int8_t)r;
            sum += r;
            w_top = w_bot;
            p0 = q0;
            p1 = q1;
            a = b;
        }
    }
    // block reduction of the charge, one atomic per block
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
    __shared__ int part[RES_THREADS / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < RES_THREADS / 64; ++w) s += part[w];
        if (s) atomicAdd((unsigned long long *)ground, (unsigned long long)(int64_t)(-s));
    }
}

// One-sided ring charges: top x-edges (+w), bottom x-edges (-w), left
// y-edges (-w), right y-edges (+w).
__global__ void k_perimeter(const float *__restrict__ psi, const uint8_t *__restrict__ valid,
                            int m, int n, int8_t *__restrict__ perim) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int C = n - 1, R = m - 1;
    const int64_t total = 2 * (int64_t)C + 2 * (int64_t)R;
    if (k >= total) return;
    int8_t v;
    if (k < C) {
        int64_t a = k;
        v = (int8_t)wrap_cycles(phase_at(psi, valid, a + 1) - phase_at(psi, valid, a));
    } else if (k < 2 * C) {
        int64_t a = (int64_t)(m - 1) * n + (k - C);
        v = (int8_t)-wrap_cycles(phase_at(psi, valid, a + 1) - phase_at(psi, valid, a));
    } else if (k < 2 * C + R) {
        int64_t a = (int64_t)(k - 2 * C) * n;
        v = (int8_t)-wrap_cycles(phase_at(psi, valid, a + n) - phase_at(psi, valid, a));
    } else {
        int64_t a = (int64_t)(k - 2 * C - R) * n + (n - 1);
        v = (int8_t)wrap_cycles(phase_at(psi, valid, a + n) - phase_at(psi, valid, a));
    }
    perim[k] = v;
}

ww_status residues_impl(const float *psi, const uint8_t *valid, int m, int n, int8_t *res,
                        int8_t *perim, int64_t *ground_dev, hipStream_t stream) {
    WW_HIP(hipMemsetAsync(ground_dev, 0, sizeof(int64_t), stream));
    if (m >= 2 && n >= 2) {
        dim3 grid(ceil_div(n - 1, RES_THREADS), ceil_div(m - 1, RES_ROWS));
        hipLaunchKernelGGL(k_residues, grid, dim3(RES_THREADS), 0, stream, psi, valid, m, n, res,
                           ground_dev);
        WW_LAUNCH_CHECK();
    }
    if (perim) {
        int64_t total = 2 * (int64_t)(n - 1) + 2 * (int64_t)(m - 1);
        if (total > 0) {
            hipLaunchKernelGGL(k_perimeter, dim3(ceil_div(total, 256)), dim3(256), 0, stream, psi,
                               valid, m, n, perim);
            WW_LAUNCH_CHECK();
        }
    }
    return WW_OK;
}

}  // namespace ww
