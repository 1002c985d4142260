// Bridging of mask-separated regions (Section II-D post-processing).
//
// Regions are the 4-connected components of valid pixels, numbered in
// row-major order of their first pixel (the component labelling with every
// edge between two valid pixels taken as reliable).  They are ranked by
// decreasing size, ties by number.  Region k >= 1 attaches to the region of
// smaller rank that holds the pixel closest to it: the pair (p in region k,
// q of smaller rank) minimising (|p - q|^2, index p, index q).  The lower
// medians of phi = psi + 2 pi K over the same-region pixels of the
// (2h+1)^2 windows around q and p give the offset
// d = floor((med_q - med_p) / 2 pi + 1/2); a region's shift is its parent's
// plus d, the largest region keeps 0.
//
//   k_br_rankpix   rank of every pixel's region (or none)
//   k_br_blockmin  smallest rank per 16 x 16 block
//   k_br_search    every boundary pixel of a region of rank r >= 1 searches
//                  blocks in rings of growing Chebyshev distance for pixels
//                  of rank < r, skipping blocks whose smallest rank is >= r;
//                  a ring whose lower distance bound exceeds the pixel's own
//                  best, or the best of its region so far, ends the search.
//                  The region keeps min over its pixels of (d^2, p) by a
//                  64-bit atomicMin.  Only boundary pixels (a 4-neighbour
//                  inside the image outside the region) can be closest, so
//                  no other pixel searches.
//   k_br_pair      the winning pixel's partner q (smallest index at the
//                  winning distance), kept per boundary pixel by the search
//   k_br_median    one workgroup per tree edge: both windows' values
//                  gathered into LDS and sorted (bitonic), lower medians, d
//   host           shifts in rank order (each parent ranks before its child)
//   k_br_apply     K_out = K + shift, phi = (float)(psi + 2 pi K_out)
#include <algorithm>
#include <numeric>
#include <vector>

#include "ww_internal.h"

namespace ww {

namespace {

constexpr uint32_t BR_NONE = 0xffffffffu;
constexpr int BR_B = 16;                 // block side of the rank pyramid
constexpr int BR_MED_SLOTS = 8192;       // >= (2 * 32 + 1)^2, power of two
constexpr int BR_MED_THREADS = 256;
constexpr int BR_MAX_HALF = 32;

__global__ void k_br_rankpix(const uint32_t *__restrict__ labels,
                             const uint32_t *__restrict__ rank_of_label, int64_t N,
                             uint32_t *__restrict__ rankpix) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t l = labels[p];
        rankpix[p] = l == 0 ? BR_NONE : rank_of_label[l - 1];
    }
}

__global__ void k_br_blockmin(const uint32_t *__restrict__ rankpix, int m, int n, int nbi, int nbj,
                              uint32_t *__restrict__ blockmin) {
    const int64_t nb = (int64_t)nbi * nbj;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x) {
        const int bi = (int)(b / nbj), bj = (int)(b % nbj);
        uint32_t mn = BR_NONE;
        for (int i = bi * BR_B; i < min(m, bi * BR_B + BR_B); ++i)
            for (int j = bj * BR_B; j < min(n, bj * BR_B + BR_B); ++j)
                mn = min(mn, rankpix[(int64_t)i * n + j]);
        blockmin[b] = mn;
    }
}

// Closest pixel of rank < r to pixel p (row i, column j): (d2, q) minimal
// lexicographically.  `region_best` (nullable) is the region's best key so
// far, (d2 << 32) | pixel, read at every ring to stop early.
__device__ void nearest_lower(const uint32_t *__restrict__ rankpix,
                              const uint32_t *__restrict__ blockmin, int m, int n, int nbi,
                              int nbj, int i, int j, uint32_t r,
                              const unsigned long long *region_best, unsigned long long &best_d2,
                              long long &best_q) {
    best_d2 = ~0ull;
    best_q = -1;
    const int bi = i / BR_B, bj = j / BR_B;
    const int rho_max = max(max(bi, nbi - 1 - bi), max(bj, nbj - 1 - bj));
    unsigned long long rbd2 = ~0ull;  // region's best squared distance so far
    for (int rho = 0; rho <= rho_max; ++rho) {
        if (region_best)
            rbd2 = __hip_atomic_load(region_best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32;
        const unsigned long long bound = best_d2 < rbd2 ? best_d2 : rbd2;
        if (rho >= 1) {
            const unsigned long long lb = (unsigned long long)((rho - 1) * BR_B + 1);
            if (lb * lb > bound) break;
        }
        for (int di = -rho; di <= rho; ++di) {
            const int ci = bi + di;
            if (ci < 0 || ci >= nbi) continue;
            const bool edge_row = di == -rho || di == rho;
            for (int dj = -rho; dj <= rho; dj += edge_row ? 1 : 2 * rho) {
                const int cj = bj + dj;
                if (cj >= 0 && cj < nbj && blockmin[(int64_t)ci * nbj + cj] < r) {
                    // nearest point of the block: skip it when even that is too far
                    const int y0 = ci * BR_B, y1 = min(m, y0 + BR_B) - 1;
                    const int x0 = cj * BR_B, x1 = min(n, x0 + BR_B) - 1;
                    const long long gy = i < y0 ? y0 - i : (i > y1 ? i - y1 : 0);
                    const long long gx = j < x0 ? x0 - j : (j > x1 ? j - x1 : 0);
                    const unsigned long long lbb = (unsigned long long)(gy * gy + gx * gx);
                    const unsigned long long lim = best_d2 < rbd2 ? best_d2 : rbd2;
                    if (lbb > lim) {
                        if (rho == 0) break;
                        continue;
                    }
                    for (int y = y0; y <= y1; ++y) {
                        const long long dy = y - i;
                        if ((unsigned long long)(dy * dy) > best_d2) continue;
                        for (int x = x0; x <= x1; ++x) {
                            const int64_t q = (int64_t)y * n + x;
                            if (rankpix[q] >= r) continue;
                            const long long dx = x - j;
                            const unsigned long long d2 = (unsigned long long)(dy * dy + dx * dx);
                            if (d2 < best_d2 || (d2 == best_d2 && q < best_q)) {
                                best_d2 = d2;
                                best_q = q;
                            }
                        }
                    }
                }
                if (rho == 0) break;  // the one block of ring 0
            }
        }
    }
}

__device__ __forceinline__ bool is_boundary(const uint32_t *rankpix, int m, int n, int i, int j,
                                            int64_t p, uint32_t r) {
    return (j > 0 && rankpix[p - 1] != r) || (j + 1 < n && rankpix[p + 1] != r) ||
           (i > 0 && rankpix[p - n] != r) || (i + 1 < m && rankpix[p + n] != r);
}

__global__ void k_br_search(const uint32_t *__restrict__ rankpix,
                            const uint32_t *__restrict__ blockmin, int m, int n, int nbi, int nbj,
                            unsigned long long *region_best, uint32_t *__restrict__ partner) {
    const int64_t N = (int64_t)m * n;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t r = rankpix[p];
        if (r == BR_NONE || r == 0) continue;
        const int i = (int)(p / n), j = (int)(p % n);
        if (!is_boundary(rankpix, m, n, i, j, p, r)) continue;
        unsigned long long d2;
        long long q;
        nearest_lower(rankpix, blockmin, m, n, nbi, nbj, i, j, r, &region_best[r], d2, q);
        if (q >= 0) {
            // exact for every pixel that can win: a search cut short by the
            // region's best already lost to it
            partner[p] = (uint32_t)q;
            atomicMin(&region_best[r], (d2 << 32) | (unsigned long long)p);
        }
    }
}

struct BrEdge {
    long long p, q;
    unsigned int parent;
    int d;
};

__global__ void k_br_pair(const uint32_t *__restrict__ rankpix,
                          const uint32_t *__restrict__ partner,
                          const unsigned long long *__restrict__ region_best, uint32_t R,
                          BrEdge *__restrict__ edges) {
    for (uint32_t r = 1 + blockIdx.x * blockDim.x + threadIdx.x; r < R;
         r += gridDim.x * blockDim.x) {
        const unsigned long long key = region_best[r];
        edges[r].d = 0;
        if (key == ~0ull) {  // no candidate (cannot happen with more than one region)
            edges[r].p = edges[r].q = -1;
            edges[r].parent = 0;
            continue;
        }
        const long long p = (long long)(key & 0xffffffffull);
        const long long q = (long long)partner[p];
        edges[r].p = p;
        edges[r].q = q;
        edges[r].parent = rankpix[q];
    }
}

// Lower median of phi over the pixels of rank `r` in the window of half-width
// h around pixel c; the whole workgroup takes part, the result is returned to
// every thread.
__device__ double window_median(const float *__restrict__ psi, const int32_t *__restrict__ K,
                                const uint32_t *__restrict__ rankpix, int m, int n, long long c,
                                uint32_t r, int h, double *vals, int *cnt) {
#pragma clang fp contract(off)
    const int ci = (int)(c / n), cj = (int)(c % n);
    const int i0 = max(0, ci - h), i1 = min(m - 1, ci + h);
    const int j0 = max(0, cj - h), j1 = min(n - 1, cj + h);
    const int w = j1 - j0 + 1, cells = (i1 - i0 + 1) * w;
    if (threadIdx.x == 0) *cnt = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < cells; t += blockDim.x) {
        const int64_t q = (int64_t)(i0 + t / w) * n + (j0 + t % w);
        if (rankpix[q] == r) {
            const int slot = atomicAdd(cnt, 1);
            vals[slot] = (double)psi[q] + TWO_PI_D * (double)K[q];
        }
    }
    __syncthreads();
    const int c_n = *cnt;
    int len = 1;
    while (len < c_n) len <<= 1;
    for (int t = c_n + threadIdx.x; t < len; t += blockDim.x) vals[t] = __builtin_huge_val();
    __syncthreads();
    // bitonic sort of vals[0, len)
    for (int k = 2; k <= len; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int t = threadIdx.x; t < len; t += blockDim.x) {
                const int u = t ^ jj;
                if (u > t) {
                    const bool up = (t & k) == 0;
                    const double a = vals[t], b = vals[u];
                    if ((a > b) == up) {
                        vals[t] = b;
                        vals[u] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    const double med = vals[(c_n - 1) / 2];
    __syncthreads();  // vals is reused by the next call
    return med;
}

__global__ __launch_bounds__(BR_MED_THREADS) void k_br_median(
    const float *__restrict__ psi, const int32_t *__restrict__ K,
    const uint32_t *__restrict__ rankpix, int m, int n, int h, BrEdge *__restrict__ edges) {
#pragma clang fp contract(off)
    __shared__ double vals[BR_MED_SLOTS];
    __shared__ int cnt;
    const uint32_t r = 1 + blockIdx.x;
    const BrEdge e = edges[r];
    if (e.p < 0 || e.q < 0) return;  // no partner: offset 0
    const double mq = window_median(psi, K, rankpix, m, n, e.q, e.parent, h, vals, &cnt);
    const double mp = window_median(psi, K, rankpix, m, n, e.p, r, h, vals, &cnt);
    if (threadIdx.x == 0) edges[r].d = (int)floor((mq - mp) / TWO_PI_D + 0.5);
}

__global__ void k_br_apply(const float *__restrict__ psi, const uint32_t *__restrict__ rankpix,
                           const int32_t *__restrict__ shift, const int32_t *K_in, int64_t N,
                           float nodata, int32_t *K_out, float *__restrict__ phi) {
#pragma clang fp contract(off)
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t r = rankpix[p];
        const int32_t k = K_in[p];
        if (r == BR_NONE) {
            K_out[p] = k;
            phi[p] = nodata;
            continue;
        }
        const int32_t kb = k + shift[r];
        K_out[p] = kb;
        phi[p] = (float)((double)psi[p] + TWO_PI_D * (double)kb);
    }
}

__global__ void k_br_fill64(unsigned long long *a, int64_t n, unsigned long long v) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        a[t] = v;
}

}  // namespace

ww_status bridge_impl(const float *psi, const uint8_t *valid, const int32_t *K_in, int m, int n,
                      int h, float nodata, int32_t *K_out, float *phi, uint32_t *regions,
                      int64_t *nregions, hipStream_t st) {
    const int64_t N = (int64_t)m * n;
    if (h < 0 || h > BR_MAX_HALF) return fail(WW_E_INVALID_ARG, "half_window must lie in [0, 32]");
    // squared distances and pixel indices share one 64-bit key
    if (m > 46000 || n > 46000) return fail(WW_E_INVALID_ARG, "bridging needs m, n <= 46000");
    uint32_t *labels = regions, *rankpix = nullptr, *sizes = nullptr;
    if (!labels) WW_TRY(scratch(SLOT_BR_LABEL, sizeof(uint32_t) * (size_t)N, (void **)&labels));
    WW_TRY(scratch(SLOT_BR_RANK, sizeof(uint32_t) * (size_t)N, (void **)&rankpix));
    // at most ceil(N / 2) regions of 4-connected pixels
    const int64_t rmax = N / 2 + 1;
    WW_TRY(scratch(SLOT_BR_SIZES, sizeof(uint32_t) * (size_t)rmax, (void **)&sizes));
    int64_t R = 0;
    WW_TRY(components_impl(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, valid, m, n, 0,
                           0.0, labels, &R, st, 1, sizes));
    *nregions = R;
    const int grid = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (N + 255) / 256));
    // rank by size (descending), ties by region number
    std::vector<uint32_t> hsize((size_t)R), rank_of((size_t)R);
    if (R > 0) {
        WW_HIP(hipMemcpyAsync(hsize.data(), sizes, sizeof(uint32_t) * (size_t)R,
                              hipMemcpyDeviceToHost, st));
        WW_HIP(hipStreamSynchronize(st));
    }
    std::vector<uint32_t> order((size_t)R);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return hsize[a] > hsize[b]; });
    for (int64_t k = 0; k < R; ++k) rank_of[order[(size_t)k]] = (uint32_t)k;
    const int nbi = (m + BR_B - 1) / BR_B, nbj = (n + BR_B - 1) / BR_B;
    const int64_t nb = (int64_t)nbi * nbj;
    char *small = nullptr;
    const size_t off_rank = 0, off_bmin = ((size_t)R * 4 + 255) / 256 * 256;
    const size_t off_best = off_bmin + ((size_t)nb * 4 + 255) / 256 * 256;
    const size_t off_edge = off_best + ((size_t)R * 8 + 255) / 256 * 256;
    const size_t off_shift = off_edge + ((size_t)R * sizeof(BrEdge) + 255) / 256 * 256;
    const size_t small_bytes = off_shift + (size_t)R * 4 + 256;
    WW_TRY(scratch(SLOT_BR_SMALL, small_bytes, (void **)&small));
    uint32_t *d_rank = (uint32_t *)(small + off_rank), *blockmin = (uint32_t *)(small + off_bmin);
    unsigned long long *best = (unsigned long long *)(small + off_best);
    BrEdge *edges = (BrEdge *)(small + off_edge);
    int32_t *d_shift = (int32_t *)(small + off_shift);
    if (R > 0)
        WW_HIP(hipMemcpyAsync(d_rank, rank_of.data(), sizeof(uint32_t) * (size_t)R,
                              hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_br_rankpix, dim3(grid), dim3(256), 0, st, labels, d_rank, N, rankpix);
    WW_LAUNCH_CHECK();
    std::vector<int32_t> shift((size_t)std::max<int64_t>(R, 1), 0);
    if (R > 1) {
        const int bgrid = (int)std::min<int64_t>(8192, (nb + 255) / 256);
        hipLaunchKernelGGL(k_br_blockmin, dim3(bgrid), dim3(256), 0, st, rankpix, m, n, nbi, nbj,
                           blockmin);
        WW_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_br_fill64, dim3((unsigned)std::min<int64_t>(1024, (R + 255) / 256)),
                           dim3(256), 0, st, best, R, ~0ull);
        WW_LAUNCH_CHECK();
        uint32_t *partner = nullptr;
        WW_TRY(scratch(SLOT_BR_Q, sizeof(uint32_t) * (size_t)N, (void **)&partner));
        hipLaunchKernelGGL(k_br_search, dim3(grid), dim3(256), 0, st, rankpix, blockmin, m, n, nbi,
                           nbj, best, partner);
        WW_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_br_pair, dim3((unsigned)std::min<int64_t>(1024, (R + 255) / 256)),
                           dim3(256), 0, st, rankpix, partner, best, (uint32_t)R, edges);
        WW_LAUNCH_CHECK();
        if (R - 1 >= ((int64_t)1 << 31)) return fail(WW_E_INVALID_ARG, "too many regions");
        hipLaunchKernelGGL(k_br_median, dim3((unsigned)(R - 1)), dim3(BR_MED_THREADS), 0, st, psi,
                           K_in, rankpix, m, n, h, edges);
        WW_LAUNCH_CHECK();
        std::vector<BrEdge> he((size_t)R);
        WW_HIP(hipMemcpyAsync(he.data(), edges, sizeof(BrEdge) * (size_t)R, hipMemcpyDeviceToHost,
                              st));
        WW_HIP(hipStreamSynchronize(st));
        for (int64_t k = 1; k < R; ++k) {
            const uint32_t par = he[(size_t)k].parent;
            if (par >= (uint32_t)k) return fail(WW_E_DEVICE, "bridging tree out of order");
            shift[(size_t)k] = shift[par] + he[(size_t)k].d;
        }
    }
    if (R > 0)
        WW_HIP(hipMemcpyAsync(d_shift, shift.data(), sizeof(int32_t) * (size_t)R,
                              hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_br_apply, dim3(grid), dim3(256), 0, st, psi, rankpix, d_shift, K_in, N,
                       nodata, K_out, phi);
    WW_LAUNCH_CHECK();
    // the host vectors must outlive the asynchronous copies
    WW_HIP(hipStreamSynchronize(st));
    return WW_OK;
}

}  // namespace ww
