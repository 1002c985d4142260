// Connected components of reliably unwrapped pixels (Section II-D).
//
// An edge is reliable when both pixels are valid, its cycle difference is 0
// and changing it by +1 or -1 would each raise its cost by more than the
// threshold (c+ > T and c- > T); a corrected edge (dk = +-1) could be
// changed back for a refund, so it is never reliable.  Components over the
// reliable edges are found by union-find on the device:
//
//   k_cc_local        every 32 x 32 tile joins its own pixels in LDS (hooks
//                     and pointer jumping until nothing changes) and points
//                     them at the smallest pixel of their tile-local part;
//   k_cc_hook_border  rounds over the edges that cross tile borders: the
//                     larger root is lowered to the smaller by atomicMin,
//                     then the pixels of those edges are compressed
//                     (k_cc_jump_border);
//   k_cc_jump         full path compression once the rounds are done: every
//                     pixel points at its root.
//
// Pointers only ever decrease, so every root ends as the smallest pixel
// index of its component, whatever the order of the atomics; the border
// rounds repeat until one changes nothing.  Sizes are counted per wave and
// per workgroup before the global atomics; components with at least
// min_size pixels are
// numbered 1, 2, ... in row-major order of their smallest pixel by a
// two-level scan, all others and invalid pixels get 0.
#include <cmath>

#include "ww_internal.h"

namespace ww {

namespace {

constexpr uint32_t CC_NONE = 0xffffffffu;  // invalid pixel
constexpr int CC_THREADS = 256;
constexpr int CC_PER = 16;                 // pixels per thread in the scan kernels
constexpr int CC_CHUNK = CC_THREADS * CC_PER;

struct CcState {
    unsigned int changed;
    unsigned int min_size;  // size threshold, set once the valid pixels are counted
    unsigned long long nvalid;
    unsigned long long ncomp;
};

__device__ __forceinline__ bool cc_reliable(int8_t dk, int16_t cp, int16_t cn, int T) {
    return dk == 0 && cp > T && cn > T;
}

__device__ __forceinline__ uint32_t cc_find(const uint32_t *L, uint32_t x) {
    // pointers decrease along every chain, so the walk ends at a root
    uint32_t y = L[x];
    while (y != x) {
        x = y;
        y = L[x];
    }
    return x;
}

// Reliability of the edge to the right of pixel (i, j) / below it (both
// pixels valid is checked by the caller).
__device__ __forceinline__ bool cc_right_ok(const int8_t *dkx, const int16_t *cxp,
                                            const int16_t *cxn, int n, int i, int j, int T,
                                            int all_edges) {
    if (all_edges) return true;
    const int64_t e = (int64_t)i * (n - 1) + j;
    return cc_reliable(dkx[e], cxp[e], cxn[e], T);
}

__device__ __forceinline__ bool cc_down_ok(const int8_t *dky, const int16_t *cyp,
                                           const int16_t *cyn, int n, int i, int j, int T,
                                           int all_edges) {
    if (all_edges) return true;
    const int64_t e = (int64_t)i * n + j;
    return cc_reliable(dky[e], cyp[e], cyn[e], T);
}

// Components inside one CC_TH x CC_TW tile, by union-find in LDS (hooks by
// atomicMin towards the smaller local index, then pointer jumping, until no
// hook changes anything).  Every pixel's global pointer is set to the
// smallest pixel of its tile-local component: local indices run row-major
// inside the tile like the global ones, so that pixel is the smallest
// global index too, and the global rounds that follow only have to join
// components across tile borders.
constexpr int CC_TH = 32, CC_TW = 32, CC_PX = CC_TH * CC_TW / 256;

__global__ __launch_bounds__(256) void k_cc_local(
    const int8_t *__restrict__ dkx, const int8_t *__restrict__ dky,
    const int16_t *__restrict__ cxp, const int16_t *__restrict__ cxn,
    const int16_t *__restrict__ cyp, const int16_t *__restrict__ cyn,
    const uint8_t *__restrict__ valid, int m, int n, int T, int all_edges, int ntx,
    uint32_t *__restrict__ L) {
    __shared__ int lab[CC_TH * CC_TW];
    __shared__ unsigned char rel[CC_TH * CC_TW];  // bit 0: right edge, bit 1: edge below
    const int ti = blockIdx.x / ntx, tj = blockIdx.x % ntx;
    const int i0 = ti * CC_TH, j0 = tj * CC_TW;
    int whole = 1;  // every in-image pixel valid and every in-tile edge reliable
#pragma unroll
    for (int k = 0; k < CC_PX; ++k) {
        const int t = threadIdx.x + 256 * k;
        const int r = t / CC_TW, c = t % CC_TW, i = i0 + r, j = j0 + c;
        const bool in = i < m && j < n;
        const int64_t p = (int64_t)i * n + j;
        const bool v = in && (!valid || valid[p]);
        lab[t] = v ? t : -1;
        unsigned char b = 0;
        const bool has_r = in && c + 1 < CC_TW && j + 1 < n;
        const bool has_d = in && r + 1 < CC_TH && i + 1 < m;
        if (v && has_r && (!valid || valid[p + 1]) &&
            cc_right_ok(dkx, cxp, cxn, n, i, j, T, all_edges))
            b |= 1;
        if (v && has_d && (!valid || valid[p + n]) &&
            cc_down_ok(dky, cyp, cyn, n, i, j, T, all_edges))
            b |= 2;
        rel[t] = b;
        if ((in && !v) || (has_r && !(b & 1)) || (has_d && !(b & 2))) whole = 0;
    }
    if (__syncthreads_and(whole)) {
        // one component: its smallest pixel is the tile's first
#pragma unroll
        for (int k = 0; k < CC_PX; ++k) {
            const int t = threadIdx.x + 256 * k;
            const int i = i0 + t / CC_TW, j = j0 + t % CC_TW;
            if (i < m && j < n) L[(int64_t)i * n + j] = (uint32_t)((int64_t)i0 * n + j0);
        }
        return;
    }
    auto find = [&](int x) {
        int y = lab[x];
        while (y != x) {
            x = y;
            y = lab[x];
        }
        return x;
    };
    // at most one hook round per pixel pair of the tile can change anything
    for (int round = 0; round < CC_TH * CC_TW; ++round) {
        int changed = 0;
#pragma unroll
        for (int k = 0; k < CC_PX; ++k) {
            const int t = threadIdx.x + 256 * k;
            const unsigned char b = rel[t];
            if (b & 1) {
                const int a = find(t), q = find(t + 1);
                if (a != q) {
                    atomicMin(&lab[a > q ? a : q], a > q ? q : a);
                    changed = 1;
                }
            }
            if (b & 2) {
                const int a = find(t), q = find(t + CC_TW);
                if (a != q) {
                    atomicMin(&lab[a > q ? a : q], a > q ? q : a);
                    changed = 1;
                }
            }
        }
        if (!__syncthreads_or(changed)) break;
#pragma unroll
        for (int k = 0; k < CC_PX; ++k) {
            const int t = threadIdx.x + 256 * k;
            if (lab[t] >= 0) lab[t] = find(t);
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < CC_PX; ++k) {
        const int t = threadIdx.x + 256 * k;
        const int r = t / CC_TW, c = t % CC_TW, i = i0 + r, j = j0 + c;
        if (i >= m || j >= n) continue;
        const int root = lab[t] >= 0 ? find(t) : -1;
        L[(int64_t)i * n + j] =
            root < 0 ? CC_NONE : (uint32_t)((int64_t)(i0 + root / CC_TW) * n + (j0 + root % CC_TW));
    }
}

// Hooks across tile borders only: the right edges of every tile's last
// column and the edges below every tile's last row.
__global__ void k_cc_hook_border(const int8_t *__restrict__ dkx, const int8_t *__restrict__ dky,
                                 const int16_t *__restrict__ cxp, const int16_t *__restrict__ cxn,
                                 const int16_t *__restrict__ cyp, const int16_t *__restrict__ cyn,
                                 int m, int n, int T, int all_edges, int ntx, int nty, uint32_t *L,
                                 CcState *st) {
    const int64_t nvb = (int64_t)m * (ntx - 1), nhb = (int64_t)(nty - 1) * n;
    int changed = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nvb + nhb;
         k += (int64_t)gridDim.x * blockDim.x) {
        int i, j;
        bool ok;
        int64_t p, q;
        if (k < nvb) {  // right edge of column (b + 1) CC_TW - 1
            i = (int)(k / (ntx - 1));
            j = (int)(k % (ntx - 1) + 1) * CC_TW - 1;
            if (j + 1 >= n) continue;
            p = (int64_t)i * n + j;
            q = p + 1;
            if (L[p] == CC_NONE || L[q] == CC_NONE) continue;
            ok = cc_right_ok(dkx, cxp, cxn, n, i, j, T, all_edges);
        } else {  // edge below row (b + 1) CC_TH - 1
            const int64_t k2 = k - nvb;
            i = (int)(k2 / n + 1) * CC_TH - 1;
            j = (int)(k2 % n);
            if (i + 1 >= m) continue;
            p = (int64_t)i * n + j;
            q = p + n;
            if (L[p] == CC_NONE || L[q] == CC_NONE) continue;
            ok = cc_down_ok(dky, cyp, cyn, n, i, j, T, all_edges);
        }
        if (!ok) continue;
        const uint32_t a = cc_find(L, (uint32_t)p), b = cc_find(L, (uint32_t)q);
        if (a != b) {
            atomicMin(&L[a > b ? a : b], a > b ? b : a);
            changed = 1;
        }
    }
    if (__any(changed) && (threadIdx.x & 63) == 0) st->changed = 1;
}

// Path compression for the pixels on both sides of the tile-border edges
// only (between border rounds; the full pass runs once at the end).
__global__ void k_cc_jump_border(int m, int n, int ntx, int nty, uint32_t *L) {
    const int64_t nvb = (int64_t)m * (ntx - 1), nhb = (int64_t)(nty - 1) * n;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nvb + nhb;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t p, q;
        if (k < nvb) {
            const int i = (int)(k / (ntx - 1)), j = (int)(k % (ntx - 1) + 1) * CC_TW - 1;
            if (j + 1 >= n) continue;
            p = (int64_t)i * n + j;
            q = p + 1;
        } else {
            const int64_t k2 = k - nvb;
            const int i = (int)(k2 / n + 1) * CC_TH - 1, j = (int)(k2 % n);
            if (i + 1 >= m) continue;
            p = (int64_t)i * n + j;
            q = p + n;
        }
        const uint32_t lp = L[p], lq = L[q];
        if (lp != CC_NONE && lp != (uint32_t)p) L[p] = cc_find(L, lp);
        if (lq != CC_NONE && lq != (uint32_t)q) L[q] = cc_find(L, lq);
    }
}

// Also counts the valid pixels, one partial sum per workgroup (a single
// global counter would serialise tens of thousands of atomics on one
// address).
__global__ __launch_bounds__(256) void k_cc_jump(int64_t N, uint32_t *L, uint32_t *vpart) {
    __shared__ uint32_t wsum[4];
    uint32_t nv = 0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t l = L[p];
        nv += l != CC_NONE;
        if (l == CC_NONE || l == (uint32_t)p) continue;
        L[p] = cc_find(L, l);
    }
    for (int off = 32; off > 0; off >>= 1) nv += __shfl_down(nv, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = nv;
    __syncthreads();
    if (threadIdx.x == 0) vpart[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Total of the valid pixels and the size threshold ceil(min_size_frac *
// valid pixels), at least 1 (one workgroup).
__global__ __launch_bounds__(256) void k_cc_total(const uint32_t *__restrict__ vpart, int nparts,
                                                  double min_size_frac, CcState *st) {
    __shared__ unsigned long long wsum[4];
    unsigned long long nv = 0;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) nv += vpart[k];
    for (int off = 32; off > 0; off >>= 1) nv += __shfl_down(nv, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = nv;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        const double want = ceil(min_size_frac * (double)tot);
        st->nvalid = tot;
        st->min_size = want < 1.0 ? 1u : (want > 4294967295.0 ? 0xffffffffu : (unsigned)want);
    }
}

// Component sizes at the roots.  Lanes of a wave holding the same root are
// counted together (ballot), the wave's leader adds the count into a small
// per-workgroup table in LDS (open addressing on the root index), and the
// table is flushed to the global counters once at the end; a root that
// finds no free slot is added to its global counter directly.
constexpr int CC_SLOTS = 128;
constexpr int CC_PROBES = 8;

__global__ __launch_bounds__(256) void k_cc_size(const uint32_t *__restrict__ L, int64_t N,
                                                 uint32_t *S) {
    __shared__ uint32_t keys[CC_SLOTS];
    __shared__ uint32_t cnts[CC_SLOTS];
    for (int t = threadIdx.x; t < CC_SLOTS; t += blockDim.x) {
        keys[t] = CC_NONE;
        cnts[t] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < N;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = base + threadIdx.x;
        const uint32_t l = p < N ? L[p] : CC_NONE;
        bool todo = l != CC_NONE;
        for (;;) {
            const unsigned long long pending = __ballot(todo);
            if (!pending) break;
            const int leader = __ffsll((long long)pending) - 1;
            const uint32_t root = __shfl(l, leader, 64);
            const unsigned long long same = __ballot(todo && l == root);
            if (lane == leader) {
                const uint32_t c = (uint32_t)__popcll(same);
                uint32_t slot = (root * 2654435761u) % CC_SLOTS;
                bool done = false;
                for (int probe = 0; probe < CC_PROBES && !done; ++probe) {
                    const uint32_t k = atomicCAS(&keys[slot], CC_NONE, root);
                    if (k == CC_NONE || k == root) {
                        atomicAdd(&cnts[slot], c);
                        done = true;
                    } else {
                        slot = (slot + 1) % CC_SLOTS;
                    }
                }
                if (!done) atomicAdd(&S[root], c);
            }
            if (todo && l == root) todo = false;
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < CC_SLOTS; t += blockDim.x)
        if (keys[t] != CC_NONE) atomicAdd(&S[keys[t]], cnts[t]);
}

// qualifying roots: L[p] == p and size >= min_size
__device__ __forceinline__ int cc_flag(const uint32_t *L, const uint32_t *S, int64_t p, int64_t N,
                                       uint32_t min_size) {
    return p < N && L[p] == (uint32_t)p && S[p] >= min_size;
}

__device__ int cc_block_scan(int v, int *total) {
    __shared__ int wsum[CC_THREADS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < CC_THREADS / 64; ++w) {
        if (w < wid) before += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// per chunk of CC_CHUNK pixels: number of qualifying roots
__global__ __launch_bounds__(CC_THREADS) void k_cc_count(const uint32_t *__restrict__ L,
                                                         const uint32_t *__restrict__ S, int64_t N,
                                                         const CcState *st, uint32_t *chunk_sum) {
    const uint32_t min_size = st->min_size;
    const int64_t p0 = (int64_t)blockIdx.x * CC_CHUNK + (int64_t)threadIdx.x * CC_PER;
    int c = 0;
    for (int k = 0; k < CC_PER; ++k) c += cc_flag(L, S, p0 + k, N, min_size);
    int tot;
    (void)cc_block_scan(c, &tot);
    if (threadIdx.x == 0) chunk_sum[blockIdx.x] = (uint32_t)tot;
}

// exclusive scan of the chunk sums (one workgroup) and the total
__global__ __launch_bounds__(CC_THREADS) void k_cc_scan(uint32_t *chunk_sum, int nchunks,
                                                        CcState *st) {
    unsigned long long carry = 0;
    for (int base = 0; base < nchunks; base += CC_THREADS) {
        const int k = base + threadIdx.x;
        const int v = k < nchunks ? (int)chunk_sum[k] : 0;
        int tot;
        const int ex = cc_block_scan(v, &tot);
        if (k < nchunks) chunk_sum[k] = (uint32_t)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0) st->ncomp = carry;
}

// every root gets its label (rank + 1, or 0 when too small) in S
__global__ __launch_bounds__(CC_THREADS) void k_cc_rank(const uint32_t *__restrict__ L, uint32_t *S,
                                                        int64_t N, const CcState *st,
                                                        const uint32_t *__restrict__ chunk_off,
                                                        uint32_t *__restrict__ sizes_out) {
    const uint32_t min_size = st->min_size;
    const int64_t p0 = (int64_t)blockIdx.x * CC_CHUNK + (int64_t)threadIdx.x * CC_PER;
    int f[CC_PER];
    int c = 0;
    for (int k = 0; k < CC_PER; ++k) {
        f[k] = cc_flag(L, S, p0 + k, N, min_size);
        c += f[k];
    }
    int tot;
    uint32_t r = chunk_off[blockIdx.x] + (uint32_t)cc_block_scan(c, &tot);
    for (int k = 0; k < CC_PER; ++k) {
        const int64_t p = p0 + k;
        if (p < N && L[p] == (uint32_t)p) {
            // roots are written only by the thread that owns them
            if (f[k]) {
                ++r;
                if (sizes_out) sizes_out[r - 1] = S[p];
                S[p] = r;
            } else {
                S[p] = 0u;
            }
        }
    }
}

__global__ void k_cc_label(const uint32_t *__restrict__ L, const uint32_t *__restrict__ S,
                           int64_t N, uint32_t *__restrict__ labels) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t l = L[p];
        labels[p] = l == CC_NONE ? 0u : S[l];
    }
}

}  // namespace

ww_status components_impl(const int8_t *dkx, const int8_t *dky, const int16_t *cxp,
                          const int16_t *cxn, const int16_t *cyp, const int16_t *cyn,
                          const uint8_t *valid, int m, int n, int threshold, double min_size_frac,
                          uint32_t *labels, int64_t *ncomp, hipStream_t st, int all_edges,
                          uint32_t *sizes_out) {
    const int64_t N = (int64_t)m * n;
    uint32_t *L = nullptr, *S = nullptr, *chunk = nullptr;
    CcState *cs = nullptr, *hcs = nullptr;
    const int nchunks = (int)((N + CC_CHUNK - 1) / CC_CHUNK);
    WW_TRY(scratch(SLOT_CC_LABEL, sizeof(uint32_t) * (size_t)N, (void **)&L));
    WW_TRY(scratch(SLOT_CC_SIZE, sizeof(uint32_t) * (size_t)N, (void **)&S));
    char *small = nullptr;
    const int grid = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (N + 255) / 256));
    WW_TRY(scratch(SLOT_CC_SMALL, 256 + sizeof(uint32_t) * ((size_t)nchunks + (size_t)grid),
                   (void **)&small));
    cs = (CcState *)small;
    chunk = (uint32_t *)(small + 256);
    uint32_t *vpart = chunk + nchunks;
    WW_TRY(host_scratch(sizeof(CcState), (void **)&hcs));
    WW_HIP(hipMemsetAsync(cs, 0, sizeof(CcState), st));
    WW_HIP(hipMemsetAsync(S, 0, sizeof(uint32_t) * (size_t)N, st));
    // components inside tiles first, then joins across tile borders
    const int ntx = (n + CC_TW - 1) / CC_TW, nty = (m + CC_TH - 1) / CC_TH;
    if ((int64_t)ntx * nty >= ((int64_t)1 << 31)) return fail(WW_E_INVALID_ARG, "image too large");
    hipLaunchKernelGGL(k_cc_local, dim3((unsigned)(ntx * nty)), dim3(256), 0, st, dkx, dky, cxp,
                       cxn, cyp, cyn, valid, m, n, threshold, all_edges, ntx, L);
    WW_LAUNCH_CHECK();
    const int64_t nborder = (int64_t)m * (ntx - 1) + (int64_t)(nty - 1) * n;
    const int bgrid = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (nborder + 255) / 256));
    // union-find rounds until a hook round changes nothing (each round that
    // changes something merges at least two components, so at most N rounds)
    for (int64_t round = 0;; ++round) {
        if (round > N + 1) return fail(WW_E_DEVICE, "connected components did not converge");
        WW_HIP(hipMemsetAsync(&cs->changed, 0, sizeof(unsigned int), st));
        hipLaunchKernelGGL(k_cc_hook_border, dim3(bgrid), dim3(256), 0, st, dkx, dky, cxp, cxn,
                           cyp, cyn, m, n, threshold, all_edges, ntx, nty, L, cs);
        WW_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cc_jump_border, dim3(bgrid), dim3(256), 0, st, m, n, ntx, nty, L);
        WW_LAUNCH_CHECK();
        WW_HIP(hipMemcpyAsync(hcs, cs, sizeof(CcState), hipMemcpyDeviceToHost, st));
        WW_HIP(hipStreamSynchronize(st));
        if (!hcs->changed) break;
    }
    hipLaunchKernelGGL(k_cc_jump, dim3(grid), dim3(256), 0, st, N, L, vpart);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cc_total, dim3(1), dim3(256), 0, st, vpart, grid, min_size_frac, cs);
    WW_LAUNCH_CHECK();
    // fewer workgroups for the sizes: each flushes its table of roots with
    // global atomics, and a large component's root takes one from every one
    const int sgrid = std::min(grid, 2048);
    hipLaunchKernelGGL(k_cc_size, dim3(sgrid), dim3(256), 0, st, L, N, S);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cc_count, dim3(nchunks), dim3(CC_THREADS), 0, st, L, S, N, cs, chunk);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cc_scan, dim3(1), dim3(CC_THREADS), 0, st, chunk, nchunks, cs);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cc_rank, dim3(nchunks), dim3(CC_THREADS), 0, st, L, S, N, cs, chunk,
                       sizes_out);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cc_label, dim3(grid), dim3(256), 0, st, L, S, N, labels);
    WW_LAUNCH_CHECK();
    WW_HIP(hipMemcpyAsync(hcs, cs, sizeof(CcState), hipMemcpyDeviceToHost, st));
    WW_HIP(hipStreamSynchronize(st));
    *ncomp = (int64_t)hcs->ncomp;
    return WW_OK;
}

}  // namespace ww
