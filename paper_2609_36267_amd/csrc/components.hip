// Connected components of reliably unwrapped pixels (Section II-D).
//
// An edge is reliable when both pixels are valid, its cycle difference is 0
// and changing it by +1 or -1 would each raise its cost by more than the
// threshold (c+ > T and c- > T); a corrected edge (dk = +-1) could be
// changed back for a refund, so it is never reliable.  Components over the
// reliable edges are found by union-find on the device:
//
//   k_cc_local        every 32 x 32 tile joins its own pixels in LDS (runs
//                     along the rows by ballot, then unions over the edges
//                     below) and points them at the smallest pixel of their
//                     tile-local part;
//   k_cc_hook_border  unions over the edges that cross tile borders: the
//                     larger root is hooked under the smaller by
//                     compare-and-swap, retried until the two roots agree;
//                     a union that gives up after a few attempts is finished
//                     by another pass, after the pixels of the border edges
//                     are compressed (k_cc_jump_border);
//   k_cc_jump         full path compression once the rounds are done: every
//                     pixel points at its root.
//
// Pointers only ever decrease and only roots are hooked, so no union is
// ever undone and every root ends as the smallest pixel index of its
// component, whatever the order of the atomics.  Sizes are counted per wave
// and per workgroup before the global atomics; components with at least
// min_size pixels are numbered 1, 2, ... in row-major order of their
// smallest pixel by a two-level scan, all others and invalid pixels get 0.
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

// Root of x with path halving: every visited pixel is pointed at its
// grandparent.  The plain stores only ever replace a non-root's pointer by
// another of its ancestors, and a root's pointer is only changed by
// compare-and-swap, so racing finds and unions leave every pointer valid.
__device__ __forceinline__ uint32_t cc_find_halve(uint32_t *L, uint32_t x) {
    uint32_t y = L[x];
    while (y != x) {
        const uint32_t z = L[y];
        if (z != y) L[x] = z;
        x = y;
        y = z;
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

// Components inside one CC_TH x CC_TW tile: every pixel first points at
// the first pixel of its run of reliable edges along the row (one ballot per
// wave), then the runs are joined by union-find in LDS over the edges below
// (hooks by atomicMin towards the smaller local index, then pointer
// jumping, until no hook changes anything).  Every pixel's global pointer is set to the
// smallest pixel of its tile-local component: local indices run row-major
// inside the tile like the global ones, so that pixel is the smallest
// global index too, and the global rounds that follow only have to join
// components across tile borders.  The reliability of the edges that leave
// the tile to the right and downwards (both pixels valid included) is
// stored as one byte per border edge in bb, so that the border rounds read
// one coalesced byte instead of four strided cost planes:
//   bb[b * m + i]             edge right of (i, (b + 1) CC_TW - 1), b < ntx - 1
//   bb[nvb + b * n + j]       edge below ((b + 1) CC_TH - 1, j),    b < nty - 1
// with nvb = m (ntx - 1).  Every entry is written.
constexpr int CC_TH = 32, CC_TW = 32, CC_PX = CC_TH * CC_TW / 256;
constexpr int CC_TRIES = 16;  // compare-and-swap attempts per union and pass

__global__ __launch_bounds__(256) void k_cc_local(
    const int8_t *__restrict__ dkx, const int8_t *__restrict__ dky,
    const int16_t *__restrict__ cxp, const int16_t *__restrict__ cxn,
    const int16_t *__restrict__ cyp, const int16_t *__restrict__ cyn,
    const uint8_t *__restrict__ valid, int m, int n, int T, int all_edges, int ntx, int64_t nvb,
    uint32_t *__restrict__ L, uint8_t *__restrict__ bb) {
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
        // runs along the row: a wave holds two tile rows (lanes 0-31 and
        // 32-63), a pixel starts a run unless the edge from its left
        // neighbour is reliable (never across the two rows: lane 31 has no
        // right edge), and it points at the first pixel of its run
        const int lane = threadIdx.x & 63;
        const unsigned long long starts = ~(__ballot(b & 1) << 1);
        const int head = 63 - __clzll(starts & (~0ull >> (63 - lane)));
        lab[t] = v ? t - lane + head : -1;
        if ((in && !v) || (has_r && !(b & 1)) || (has_d && !(b & 2))) whole = 0;
        if (in && c == CC_TW - 1 && j + 1 < n)
            bb[(int64_t)tj * m + i] = v && (!valid || valid[p + 1]) &&
                                      cc_right_ok(dkx, cxp, cxn, n, i, j, T, all_edges);
        if (in && r == CC_TH - 1 && i + 1 < m)
            bb[nvb + (int64_t)ti * n + j] = v && (!valid || valid[p + n]) &&
                                            cc_down_ok(dky, cyp, cyn, n, i, j, T, all_edges);
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
    // other lanes hook roots while a union is in progress: read through a
    // volatile view
    volatile int *vlab = lab;
    auto find = [&](int x) {
        int y = vlab[x];
        while (y != x) {
            x = y;
            y = vlab[x];
        }
        return x;
    };
    // The runs are joined over the edges below.  A union hooks the larger
    // root under the smaller by compare-and-swap and retries from fresh
    // roots when another lane hooked one of them first; a union still open
    // after CC_TRIES attempts is left to another pass.  Every failed attempt
    // means another union succeeded, so each pass joins at least two runs.
    const int lane = threadIdx.x & 63;
    for (int pass = 0; pass < CC_TH * CC_TW; ++pass) {
        int open = 0;
#pragma unroll
        for (int k = 0; k < CC_PX; ++k) {
            const int t = threadIdx.x + 256 * k;
            bool act = rel[t] & 2;
            int x = 0, y = 0;
            if (act) {
                x = find(t);
                y = find(t + CC_TW);
                if (x > y) {
                    const int z = x;
                    x = y;
                    y = z;
                }
                act = x != y;
            }
            // a row of edges below mostly joins the same two runs: a lane
            // whose pair equals the previous lane's leaves the union to it
            const int px = __shfl_up(x, 1, 64), py = __shfl_up(y, 1, 64);
            const int pact = __shfl_up((int)act, 1, 64);
            if (act && lane > 0 && pact && px == x && py == y) act = false;
            if (!act) continue;
            for (int tries = 0;; ++tries) {
                const int old = atomicCAS(&lab[y], y, x);
                if (old == y) break;
                if (tries == CC_TRIES) {
                    open = 1;
                    break;
                }
                x = find(x);
                y = find(old);
                if (x == y) break;
                if (x > y) {
                    const int z = x;
                    x = y;
                    y = z;
                }
            }
        }
        if (!__syncthreads_or(open)) break;
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

// Pixels on both sides of border edge k (the numbering of bb above).
__device__ __forceinline__ void cc_border_edge(int64_t k, int m, int n, int64_t nvb, int64_t &p,
                                               int64_t &q) {
    if (k < nvb) {
        const int b = (int)(k / m), i = (int)(k % m);
        p = (int64_t)i * n + (int64_t)b * CC_TW + CC_TW - 1;
        q = p + 1;
    } else {
        const int64_t k2 = k - nvb;
        const int b = (int)(k2 / n), j = (int)(k2 % n);
        p = ((int64_t)b * CC_TH + CC_TH - 1) * n + j;
        q = p + n;
    }
}

// Unions across tile borders, over the edges marked in bb, by the same
// compare-and-swap hooks as inside the tiles.  A failed attempt returns the
// root's current pointer, from which the next attempt continues.  Unions
// still open after CC_TRIES attempts (another union won each time, or this
// XCD's cache still held an older pointer) raise st->changed, and the host
// runs another pass after compressing the border pixels.
__global__ __launch_bounds__(256) void k_cc_hook_border(const uint8_t *__restrict__ bb, int m,
                                                        int n, int64_t nvb, int64_t nb,
                                                        uint32_t *L, CcState *st) {
    const int lane = threadIdx.x & 63;
    int open = 0;
    // the loop bound is the same for the whole workgroup, so that every
    // lane takes part in the shuffle below
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nb;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = base + threadIdx.x;
        bool act = k < nb && bb[k];
        uint32_t x = 0, y = 0;
        if (act) {
            int64_t p, q;
            cc_border_edge(k, m, n, nvb, p, q);
            x = cc_find_halve(L, (uint32_t)p);
            y = cc_find_halve(L, (uint32_t)q);
            if (x > y) {
                const uint32_t z = x;
                x = y;
                y = z;
            }
            act = x != y;
        }
        // neighbouring border edges mostly join the same two roots: a lane
        // whose pair equals the previous lane's leaves the union to it (if
        // that one gives up, the next pass sees this edge again)
        const uint32_t px = __shfl_up(x, 1, 64), py = __shfl_up(y, 1, 64);
        const int pact = __shfl_up((int)act, 1, 64);
        if (act && lane > 0 && pact && px == x && py == y) act = false;
        if (!act) continue;
        for (int tries = 0;; ++tries) {
            const uint32_t old = atomicCAS(&L[y], y, x);
            if (old == y) break;
            if (tries == CC_TRIES) {
                open = 1;
                break;
            }
            x = cc_find_halve(L, x);
            y = cc_find_halve(L, old);
            if (x == y) break;
            if (x > y) {
                const uint32_t z = x;
                x = y;
                y = z;
            }
        }
    }
    if (__any(open) && lane == 0) st->changed = 1;
}

// Path compression for the pixels on both sides of the marked border edges
// only (between border rounds; the full pass runs once at the end).
__global__ void k_cc_jump_border(const uint8_t *__restrict__ bb, int m, int n, int64_t nvb,
                                 int64_t nb, uint32_t *L) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (!bb[k]) continue;
        int64_t p, q;
        cc_border_edge(k, m, n, nvb, p, q);
        const uint32_t lp = L[p], lq = L[q];
        if (lp != (uint32_t)p) L[p] = cc_find(L, lp);
        if (lq != (uint32_t)q) L[q] = cc_find(L, lq);
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
// counted together (ballot); a count of at least CC_TABLE_MIN goes into a
// small per-workgroup table in LDS (open addressing on the root index),
// flushed to the global counters once at the end, so that a large
// component's root takes one global atomic per workgroup rather than one
// per wave.  Smaller counts, and roots that find no free slot, are added to
// their global counters directly: these are spread over many addresses.
constexpr int CC_SLOTS = 128;
constexpr int CC_PROBES = 8;

__device__ __forceinline__ void cc_table_add(uint32_t *keys, uint32_t *cnts, uint32_t *S,
                                             uint32_t root, uint32_t c) {
    uint32_t slot = (root * 2654435761u) % CC_SLOTS;
    for (int probe = 0; probe < CC_PROBES; ++probe) {
        const uint32_t k = atomicCAS(&keys[slot], CC_NONE, root);
        if (k == CC_NONE || k == root) {
            atomicAdd(&cnts[slot], c);
            return;
        }
        slot = (slot + 1) % CC_SLOTS;
    }
    atomicAdd(&S[root], c);
}

// Every thread takes CC_SZV consecutive pixels per step (two 16-byte
// loads); a wave whose 64 x CC_SZV pixels all share one root adds them in
// one go, which is the common case inside large components.
constexpr int CC_SZV = 8;
constexpr uint32_t CC_TABLE_MIN = 16;

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
    const int64_t step = (int64_t)gridDim.x * blockDim.x * CC_SZV;
    for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x * CC_SZV; b0 < N; b0 += step) {
        const int64_t p = b0 + (int64_t)threadIdx.x * CC_SZV;
        uint32_t v[CC_SZV];
        if (p + CC_SZV <= N) {
            const uint4 x = *reinterpret_cast<const uint4 *>(L + p);
            const uint4 y = *reinterpret_cast<const uint4 *>(L + p + 4);
            v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
            v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
        } else {
#pragma unroll
            for (int k = 0; k < CC_SZV; ++k) v[k] = p + k < N ? L[p + k] : CC_NONE;
        }
        bool uni = v[0] != CC_NONE;
#pragma unroll
        for (int k = 1; k < CC_SZV; ++k) uni = uni && v[k] == v[0];
        const uint32_t w0 = __shfl(v[0], 0, 64);
        if (__all(uni && v[0] == w0)) {
            if (lane == 0) cc_table_add(keys, cnts, S, w0, 64u * CC_SZV);
            continue;
        }
#pragma unroll
        for (int k = 0; k < CC_SZV; ++k) {
            const uint32_t l = v[k];
            bool todo = l != CC_NONE;
            for (;;) {
                const unsigned long long pending = __ballot(todo);
                if (!pending) break;
                const int leader = __ffsll((long long)pending) - 1;
                const uint32_t root = __shfl(l, leader, 64);
                const unsigned long long same = __ballot(todo && l == root);
                if (lane == leader) {
                    // small counts (mostly the roots of one-pixel components)
                    // go straight to their own global counters, which keeps
                    // the table for the few large components
                    const uint32_t c = (uint32_t)__popcll(same);
                    if (c >= CC_TABLE_MIN)
                        cc_table_add(keys, cnts, S, root, c);
                    else
                        atomicAdd(&S[root], c);
                }
                if (todo && l == root) todo = false;
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < CC_SLOTS; t += blockDim.x)
        if (keys[t] != CC_NONE) atomicAdd(&S[keys[t]], cnts[t]);
}

// the CC_PER pointers of pixels p0 ... p0 + CC_PER - 1 (CC_NONE past N)
__device__ __forceinline__ void cc_load_run(const uint32_t *__restrict__ L, int64_t p0, int64_t N,
                                            uint32_t v[CC_PER]) {
    if (p0 + CC_PER <= N) {
#pragma unroll
        for (int k = 0; k < CC_PER; k += 4) {
            const uint4 x = *reinterpret_cast<const uint4 *>(L + p0 + k);
            v[k] = x.x;
            v[k + 1] = x.y;
            v[k + 2] = x.z;
            v[k + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < CC_PER; ++k) v[k] = p0 + k < N ? L[p0 + k] : CC_NONE;
    }
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
    uint32_t v[CC_PER];
    cc_load_run(L, p0, N, v);
    int c = 0;
#pragma unroll
    for (int k = 0; k < CC_PER; ++k)
        c += v[k] == (uint32_t)(p0 + k) && S[p0 + k] >= min_size;
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
    uint32_t v[CC_PER];
    cc_load_run(L, p0, N, v);
    int f[CC_PER];
    int c = 0;
#pragma unroll
    for (int k = 0; k < CC_PER; ++k) {
        f[k] = v[k] == (uint32_t)(p0 + k) && S[p0 + k] >= min_size;
        c += f[k];
    }
    int tot;
    uint32_t r = chunk_off[blockIdx.x] + (uint32_t)cc_block_scan(c, &tot);
    for (int k = 0; k < CC_PER; ++k) {
        const int64_t p = p0 + k;
        if (v[k] == (uint32_t)p) {
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
    // components inside tiles first, then joins across tile borders; the
    // border-edge bytes live in the size buffer until the sizes are counted
    // (at most N / 16 bytes)
    const int ntx = (n + CC_TW - 1) / CC_TW, nty = (m + CC_TH - 1) / CC_TH;
    if ((int64_t)ntx * nty >= ((int64_t)1 << 31)) return fail(WW_E_INVALID_ARG, "image too large");
    const int64_t nvb = (int64_t)m * (ntx - 1), nborder = nvb + (int64_t)(nty - 1) * n;
    uint8_t *bb = reinterpret_cast<uint8_t *>(S);
    hipLaunchKernelGGL(k_cc_local, dim3((unsigned)(ntx * nty)), dim3(256), 0, st, dkx, dky, cxp,
                       cxn, cyp, cyn, valid, m, n, threshold, all_edges, ntx, nvb, L, bb);
    WW_LAUNCH_CHECK();
    const int bgrid = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (nborder + 255) / 256));
    // border passes until no union is left open (each pass with open unions
    // completes at least one, so at most N passes)
    for (int64_t pass = 0;; ++pass) {
        if (pass > N + 1) return fail(WW_E_DEVICE, "connected components did not converge");
        if (pass > 0) {
            hipLaunchKernelGGL(k_cc_jump_border, dim3(bgrid), dim3(256), 0, st, bb, m, n, nvb,
                               nborder, L);
            WW_LAUNCH_CHECK();
        }
        WW_HIP(hipMemsetAsync(&cs->changed, 0, sizeof(unsigned int), st));
        hipLaunchKernelGGL(k_cc_hook_border, dim3(bgrid), dim3(256), 0, st, bb, m, n, nvb, nborder,
                           L, cs);
        WW_LAUNCH_CHECK();
        WW_HIP(hipMemcpyAsync(hcs, cs, sizeof(CcState), hipMemcpyDeviceToHost, st));
        WW_HIP(hipStreamSynchronize(st));
        if (!hcs->changed) break;
    }
    hipLaunchKernelGGL(k_cc_jump, dim3(grid), dim3(256), 0, st, N, L, vpart);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cc_total, dim3(1), dim3(256), 0, st, vpart, grid, min_size_frac, cs);
    WW_LAUNCH_CHECK();
    WW_HIP(hipMemsetAsync(S, 0, sizeof(uint32_t) * (size_t)N, st));
    // each workgroup flushes its table of roots with global atomics, and a
    // large component's root takes one from every workgroup: 4096 at most
    const int sgrid = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (N + 2047) / 2048));
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
