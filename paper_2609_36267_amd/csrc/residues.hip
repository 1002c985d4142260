// Residues of every 2x2 loop (Section II-A, eq. 1) and the one-sided charges
// of the boundary ring.
//
// Each thread owns VEC consecutive loop columns (VEC = 4 with 16-byte phase
// loads when the row length is a multiple of 4, else 1) and walks a strip of
// RES_ROWS loop rows; a wrap count shared by two loops is computed once.  Pixel rows are fetched in batches of RES_BATCH, all
// loads of a batch issued before any arithmetic, so that many rows are in
// flight per thread; pixel row i+1 of one step is row i of the next, so
// every psi/valid byte is read once per strip (plus one halo row and one
// halo column).  Bytes moved per loop: 4 (psi) + 1 (valid) + 1 (res) = 6.
#include <algorithm>

#include "ww_internal.h"

namespace ww {

constexpr int RES_ROWS = 32;
constexpr int RES_BATCH = 8;
constexpr int RES_THREADS = 256;
constexpr int RES_GRID = 1024;  // workgroups resident at once (256 CUs x 4)

template <int VEC>
__device__ __forceinline__ void load_row(const float *__restrict__ psi,
                                         const uint8_t *__restrict__ valid, int a, int ncol,
                                         double *out) {
    // pixel columns a .. a+ncol-1 of one row (ncol <= VEC+1), phase read as
    // 0 at invalid pixels; columns past ncol are not read
    float f[VEC + 1];
    uint8_t v[VEC + 1];
    if (VEC == 4 && ncol == 5) {
        const float4 q = *reinterpret_cast<const float4 *>(psi + a);
        f[0] = q.x; f[1] = q.y; f[2] = q.z; f[3] = q.w;
        f[VEC] = psi[a + 4];
        if (valid) {
            const uchar4 w = *reinterpret_cast<const uchar4 *>(valid + a);
            v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
            v[VEC] = valid[a + 4];
        }
    } else {
#pragma unroll
        for (int k = 0; k <= VEC; ++k) {
            f[k] = k < ncol ? psi[a + k] : 0.f;
            if (valid) v[k] = k < ncol ? valid[a + k] : 0;
        }
    }
#pragma unroll
    for (int k = 0; k <= VEC; ++k) out[k] = (!valid || v[k]) ? (double)f[k] : 0.0;
}

template <int VEC>
__global__ __launch_bounds__(RES_THREADS) void k_residues(const float *__restrict__ psi,
                                                          const uint8_t *__restrict__ valid,
                                                          int m, int n, int8_t *__restrict__ res,
                                                          int64_t *__restrict__ ground, int nbx,
                                                          int nitems) {
    const int C = n - 1;
    int sum = 0;
    // work items: (row strip, column block), strided over a grid sized to
    // the resident capacity
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int bx = item % nbx, by = item / nbx;
        const int j0 = (bx * RES_THREADS + threadIdx.x) * VEC;
        const int i0 = by * RES_ROWS;
        if (j0 >= C) continue;
        const int nl = min(VEC, C - j0);  // loops owned (columns j0 .. j0+nl-1)
        const int ncol = nl + 1;           // pixel columns read
        double p[VEC + 1];
        load_row<VEC>(psi, valid, i0 * n + j0, ncol, p);  // m * n < 2^31
        int wh[VEC];  // wrap counts of the x-edges of the current pixel row
#pragma unroll
        for (int k = 0; k < VEC; ++k) wh[k] = wrap_cycles(p[k + 1] - p[k]);
        const int iend = min(i0 + RES_ROWS, m - 1);
        for (int ib = i0; ib < iend; ib += RES_BATCH) {
            const int nb = min(RES_BATCH, iend - ib);
            double q[RES_BATCH][VEC + 1];
#pragma unroll
            for (int r = 0; r < RES_BATCH; ++r)
                if (r < nb) load_row<VEC>(psi, valid, (ib + r + 1) * n + j0, ncol, q[r]);
#pragma unroll
            for (int r = 0; r < RES_BATCH; ++r) {
                if (r >= nb) break;
                const int i = ib + r;
                int wv[VEC + 1];  // y-edges vy(i, j0 .. j0+VEC)
#pragma unroll
                for (int k = 0; k <= VEC; ++k) wv[k] = wrap_cycles(q[r][k] - p[k]);
                int8_t *dst = res + (i * C + j0);
#pragma unroll
                for (int k = 0; k < VEC; ++k) {
                    const int wb = wrap_cycles(q[r][k + 1] - q[r][k]);  // hx(i+1, j)
                    const int rr = -(wh[k] + wv[k + 1] - wb - wv[k]);
                    if (k < nl) {
                        dst[k] = (int8_t)rr;
                        sum += rr;
                    }
                    wh[k] = wb;
                }
#pragma unroll
                for (int k = 0; k <= VEC; ++k) p[k] = q[r][k];
            }
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
        // 16-byte phase loads need 4-aligned rows and base pointers
        const bool vec = (n % 4 == 0) && ((uintptr_t)psi % 16 == 0) &&
                         (!valid || (uintptr_t)valid % 4 == 0);
        const int nby = ceil_div(m - 1, RES_ROWS);
        if (vec) {
            const int nbx = ceil_div(ceil_div(n - 1, 4), RES_THREADS), nitems = nbx * nby;
            hipLaunchKernelGGL(k_residues<4>, dim3(std::min(nitems, RES_GRID)), dim3(RES_THREADS), 0,
                               stream, psi, valid, m, n, res, ground_dev, nbx, nitems);
        } else {
            const int nbx = ceil_div(n - 1, RES_THREADS), nitems = nbx * nby;
            hipLaunchKernelGGL(k_residues<1>, dim3(std::min(nitems, RES_GRID)), dim3(RES_THREADS), 0,
                               stream, psi, valid, m, n, res, ground_dev, nbx, nitems);
        }
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
