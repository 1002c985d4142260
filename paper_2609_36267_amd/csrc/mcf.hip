// Exact minimum-cost flow of eq. 2 by successive shortest paths with node
// potentials (Section II-C), on the loop graph of an m x n image plus one
// ground node G that stands for the outer ring of zero-cost, unbounded arcs.
//
// State: the net flow of every pixel edge is its cycle difference dk in
// {-1,0,1} (the dk_x / dk_y outputs).  A residual move of +1 on an edge with
// dk = 0 costs c+, of -1 costs c-; undoing a correction refunds its cost;
// moving past +-1 is not allowed.  Potentials pot (int32, guarded) keep every
// residual arc's reduced cost c - pot(u) + pot(v) >= 0.
//
// One pass:
//  1. Multi-source shortest paths from every node with positive excess over
//     reduced costs.  Labels are 64-bit (dist:32 | hops:29 | dir:3) and every
//     node keeps the lexicographic minimum over its in-arcs, so the fixpoint
//     is unique (independent of scheduling) and predecessor links form a
//     forest (hops strictly grow along them).  The search is bounded by a
//     distance window B; candidates beyond B are parked and the window grows
//     until enough deficits are reached.
//     Relaxation runs on 32 x 32 node tiles: a workgroup stages the tile's
//     labels and reduced in-arc costs in LDS and iterates to local
//     convergence; tiles whose border labels changed activate their
//     neighbours for the next round (one launch per round).  Round r works
//     through list r % 3 and appends to list (r + 1) % 3; a per-tile round
//     stamp (atomic exchange) keeps a tile from being listed twice, and a
//     visit reserves list slots for all the tiles it activates with one
//     atomic add.  Tiles relaxed in a pass, and tiles holding candidates
//     beyond the current window, are marked with plain-store pass stamps.
//  2. Every reached deficit walks its predecessor chain to its tree root;
//     each root keeps its nearest deficit (64-bit atomicMin on dist|node).
//  3. One unit is augmented along each root's chosen path.  Different trees
//     are vertex-disjoint, so all paths are applied in parallel.  Trees that
//     hang off the ground as a supply are split at the ground's arcs and at
//     most its excess of them augment.
//  4. pot(v) += B - d(v) for every reached node.  Every tree arc is then
//     tight and reversing it keeps all reduced costs >= 0, so the final flow
//     is optimal whatever the window and the number of paths per pass.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <cstring>
#include <atomic>
#include <vector>

#include "ww_internal.h"

namespace ww {

namespace {

constexpr unsigned long long LINF = ~0ull;
constexpr int RC_INF = 0x7fffffff;
constexpr int DIR_NONE = 0, DIR_UP = 1, DIR_DOWN = 2, DIR_LEFT = 3, DIR_RIGHT = 4;
constexpr int POT_LIMIT = 1 << 30;

enum : int { ERR_NEG_RC = 1, ERR_POT = 2, ERR_WALK = 4, ERR_ITERS = 8 };

struct Ctl {
    unsigned long long glab;   // ground label
    long long gex;             // ground excess
    long long gpot;            // ground potential
    unsigned int count[3][32]; // list lengths (one 128-byte line each)
    unsigned int nsrc, ndef;   // node lists
    unsigned int nsrc2, ndef2; // compaction targets
    unsigned int gsub_count;   // ground-rooted subtrees with a deficit
    unsigned int gpred;        // ground predecessor (perimeter arc index)
    unsigned int wsettled[2];  // deficits reached in the window (by window parity)
    unsigned int naug;         // augmentations in this pass
    unsigned long long arcs;   // arcs flipped in this pass
    int error;
    int max_pot;
    long long total_cost;
    long long sum_res;
    unsigned long long wminrej[2];  // smallest candidate beyond the window (by parity)
    unsigned long long iters;   // in-tile relaxation iterations, all visits
    unsigned long long vt_sum;  // visit durations (wall-clock ticks), all visits
    unsigned long long vt_max;  // longest visit
    unsigned long long vt_stage;  // staging part of the visits
    unsigned long long vt_sweep;  // staging and sweeps of the visits
    unsigned int prev_naug;       // naug and arcs of the previous pass, kept by
    unsigned long long prev_arcs;  // the pass set-up when it clears them
};

struct Graph {
    int R, C, n;               // loop rows, loop cols, image cols (= C + 1)
    int th, tw;                // tile shape (rows, cols)
    int TR, TC;                // tile grid
    const int16_t *cxp, *cxn, *cyp, *cyn;
    int8_t *fx, *fy;
    unsigned long long *lab;
    int *pot;
    int8_t *ex;
    unsigned long long *best;
};

__device__ __forceinline__ unsigned int ldist(unsigned long long l) { return (unsigned int)(l >> 32); }
__device__ __forceinline__ unsigned int lhops(unsigned long long l) {
    return (unsigned int)((l >> 3) & 0x1fffffffu);
}

// cost of moving an edge's net flow f by delta, RC_INF if not allowed
__device__ __forceinline__ int move_cost(int f, int delta, int cp, int cn) {
    if (f == 0) return delta > 0 ? cp : cn;
    if (f == -delta) return -(f > 0 ? cp : cn);
    return RC_INF;
}

// Append tile t to the list of round r unless it is already there
// (act[t] == r).  Lists: lists[(r % 3) * NT ...], lengths ctl->count[r % 3].
__device__ __forceinline__ void activate(unsigned int *act, unsigned int *lists, unsigned int NT,
                                         Ctl *ctl, unsigned int t, unsigned int r) {
    if (atomicExch(&act[t], r) != r) {
        const unsigned int pos = atomicAdd(&ctl->count[r % 3][0], 1u);
        lists[(size_t)(r % 3) * NT + pos] = t;
    }
}

// perimeter arc a -> (node row, node col, edge kind, edge index, delta of
// the move node -> ground)
__device__ __forceinline__ void ground_arc(const Graph &g, unsigned int a, int &i, int &j,
                                           int &kind, long long &e, int &delta) {
    const int C = g.C, R = g.R;
    if (a < (unsigned)C) {  // top: up across hx(0, j)
        i = 0; j = a; kind = 0; e = j; delta = -1;
    } else if (a < 2u * C) {  // bottom: down across hx(R, j)
        i = R - 1; j = a - C; kind = 0; e = (long long)R * C + j; delta = +1;
    } else if (a < 2u * C + R) {  // left: left across vy(i, 0)
        i = a - 2 * C; j = 0; kind = 1; e = (long long)i * g.n; delta = +1;
    } else {  // right: right across vy(i, C)
        i = a - 2 * C - R; j = C - 1; kind = 1; e = (long long)i * g.n + C; delta = -1;
    }
}

}  // namespace

// ------------------------------------------------------------ set-up ------

// Set-up in three launches with no contended atomics: every block of
// INIT_CHUNK nodes initialises its state and counts its supplies / demands;
// one block scans the counts; every block then writes its supplies and
// demands in node order.
constexpr int INIT_THREADS = 256;
constexpr int INIT_PER = 16;
constexpr int INIT_CHUNK = INIT_THREADS * INIT_PER;
static_assert(INIT_CHUNK < (1 << 16), "packed per-block counts of the list writer");

__device__ __forceinline__ int block_sum_int(int v, int *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    __syncthreads();
    return t;
}

// exclusive block scan (blockDim.x <= 1024), returns the prefix, *total = sum
__device__ __forceinline__ int block_scan_int(int v, int *red, int *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        int o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) red[wid] = inc;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        if (w < wid) before += red[w];
        tot += red[w];
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// The residues of loop nodes v0 .. v0 + INIT_PER - 1 (zero beyond N): one
// 16-byte load where the plane is 16-byte aligned and the group is whole.
static_assert(INIT_PER == 16, "residue groups are 16-byte loads");
__device__ __forceinline__ bool load_res16(const int8_t *res, long long v0, long long N, int8_t r[16]) {
    const bool whole = v0 + 16 <= N;
    if (whole && ((uintptr_t)res & 15u) == 0) {
        const uint4 x = *reinterpret_cast<const uint4 *>(res + v0);
        const unsigned int w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int q = 0; q < 16; ++q) r[q] = (int8_t)(w[q >> 2] >> (8 * (q & 3)));
    } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) r[q] = v0 + q < N ? res[v0 + q] : (int8_t)0;
    }
    return whole;
}

// Node state of a block's chunk of INIT_CHUNK nodes, each thread taking
// INIT_PER consecutive nodes: the excess is a copy of the residues, the
// potentials zero, the labels infinite, all in 16-byte stores.
__global__ __launch_bounds__(INIT_THREADS) void k_mcf_init_count(Graph g, const int8_t *__restrict__ res,
                                                                int *__restrict__ bc,
                                                                unsigned int *__restrict__ flip) {
    __shared__ int red[INIT_THREADS / 64];
    const long long N = (long long)g.R * g.C;
    const long long c0 = (long long)blockIdx.x * INIT_CHUNK;
    const long long v0 = c0 + (long long)threadIdx.x * INIT_PER;
    int8_t r[INIT_PER];
    const bool whole = load_res16(res, v0, N, r);
    int np = 0, nn = 0, sum = 0;
    unsigned int w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < INIT_PER; ++q) {
        np += r[q] > 0;
        nn += r[q] < 0;
        sum += r[q];
        w[q >> 2] |= (unsigned int)(uint8_t)r[q] << (8 * (q & 3));
        // best (a root's chosen deficit) is only kept at roots: supplies,
        // which are residues in one frame or the other, and perimeter nodes
        // (ground-rooted subtrees); other nodes' entries are never read
        if (r[q] != 0) g.best[v0 + q] = LINF;
    }
    if (whole) {
        *reinterpret_cast<uint4 *>(g.ex + v0) = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
        for (int q = 0; q < INIT_PER; ++q)
            if (v0 + q < N) g.ex[v0 + q] = r[q];
    }
    if (c0 + INIT_CHUNK <= N) {
        uint4 *pot = reinterpret_cast<uint4 *>(g.pot + c0);
        uint4 *fl = reinterpret_cast<uint4 *>(flip + c0);
        uint4 *lab = reinterpret_cast<uint4 *>(g.lab + c0);
        const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
        const uint4 inf = make_uint4((unsigned int)LINF, (unsigned int)(LINF >> 32), (unsigned int)LINF,
                                     (unsigned int)(LINF >> 32));
#pragma unroll
        for (int k = 0; k < INIT_CHUNK / 4 / INIT_THREADS; ++k) {
            pot[k * INIT_THREADS + threadIdx.x] = zero;
            fl[k * INIT_THREADS + threadIdx.x] = zero;
        }
#pragma unroll
        for (int k = 0; k < INIT_CHUNK / 2 / INIT_THREADS; ++k) lab[k * INIT_THREADS + threadIdx.x] = inf;
    } else {
        for (long long v = c0 + threadIdx.x; v < N; v += INIT_THREADS) {
            g.pot[v] = 0;
            flip[v] = 0;
            g.lab[v] = LINF;
        }
    }
    for (unsigned int a = blockIdx.x * blockDim.x + threadIdx.x; a < 2u * g.C + 2u * g.R;
         a += gridDim.x * blockDim.x) {
        int i, j, kind, delta;
        long long e;
        ground_arc(g, a, i, j, kind, e, delta);
        g.best[(long long)i * g.C + j] = LINF;
    }
    np = block_sum_int(np, red);
    nn = block_sum_int(nn, red);
    sum = block_sum_int(sum, red);
    if (threadIdx.x == 0) {
        bc[3 * blockIdx.x + 0] = np;
        bc[3 * blockIdx.x + 1] = nn;
        bc[3 * blockIdx.x + 2] = sum;
    }
}

// one block: exclusive scans of the per-block counts, totals into ctl; each
// thread sums a run of consecutive blocks, one block scan joins the runs
__global__ __launch_bounds__(1024) void k_mcf_init_scan(int nb, int *__restrict__ bc, Ctl *ctl) {
    __shared__ int red[16];
    const int per = (nb + (int)blockDim.x - 1) / (int)blockDim.x;
    const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
    int p = 0, q = 0, s = 0;
    // unrolled so that the loads of several blocks' counts are in flight at once
#pragma unroll 8
    for (int b = b0; b < b1; ++b) {
        p += bc[3 * b];
        q += bc[3 * b + 1];
        s += bc[3 * b + 2];
    }
    int tp, tq;
    int ep = block_scan_int(p, red, &tp);
    int eq = block_scan_int(q, red, &tq);
    const int ts = block_sum_int(s, red);
#pragma unroll 8
    for (int b = b0; b < b1; ++b) {
        const int bp = bc[3 * b], bq = bc[3 * b + 1];
        bc[3 * b] = ep;
        bc[3 * b + 1] = eq;
        ep += bp;
        eq += bq;
    }
    if (threadIdx.x == 0) {
        ctl->nsrc = tp;
        ctl->ndef = tq;
        ctl->sum_res = ts;
        ctl->gex = -(long long)ts;
        ctl->gpot = 0;
        ctl->glab = LINF;
        ctl->wminrej[0] = ctl->wminrej[1] = LINF;
    }
}

__global__ __launch_bounds__(INIT_THREADS) void k_mcf_init_write(Graph g, const int8_t *__restrict__ res,
                                                                const int *__restrict__ bc,
                                                                unsigned int *__restrict__ src,
                                                                unsigned int *__restrict__ def) {
    // each thread takes INIT_PER consecutive nodes of the block's chunk, so
    // one scan of the packed (supplies, demands) counts places them all in
    // node order (a thread's counts are at most INIT_PER and a block's at
    // most INIT_CHUNK < 2^16, so the two halves never carry into each other)
    __shared__ int red[INIT_THREADS / 64];
    const long long N = (long long)g.R * g.C;
    const long long v0 = (long long)blockIdx.x * INIT_CHUNK + (long long)threadIdx.x * INIT_PER;
    int8_t r[INIT_PER];
    load_res16(res, v0, N, r);
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < INIT_PER; ++q) cnt += (r[q] > 0) + ((r[q] < 0) << 16);
    int tot;
    const int ex = block_scan_int(cnt, red, &tot);
    int op = bc[3 * blockIdx.x] + (ex & 0xffff), on = bc[3 * blockIdx.x + 1] + (ex >> 16);
#pragma unroll
    for (int q = 0; q < INIT_PER; ++q) {
        if (r[q] > 0) src[op++] = (unsigned int)(v0 + q);
        if (r[q] < 0) def[on++] = (unsigned int)(v0 + q);
    }
}

// Pass start: sources get label 0 and their tiles are activated for round rr.
// The ground is a source while it holds surplus; that is read here rather
// than passed in, so that a pass can be queued before the host has seen how
// the previous one ended.
__global__ void k_pass_init(Graph g, Ctl *ctl, const unsigned int *src, unsigned int *act,
                            unsigned int *lists, unsigned int NT, unsigned int rr,
                            const unsigned int *perim_tiles, int nperim) {
    const unsigned int ns = ctl->nsrc;
    const int ground_source = ctl->gex > 0;
    for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k < ns; k += gridDim.x * blockDim.x) {
        const unsigned int v = src[k];
        g.lab[v] = 0ull;
        const int i = v / g.C, j = v % g.C;
        const int ti = i / g.th, tj = j / g.tw, li = i % g.th, lj = j % g.tw;
        const unsigned int t = ti * g.TC + tj;
        activate(act, lists, NT, ctl, t, rr);
        // a supply on a tile border also feeds the tile across that border,
        // whose relaxation must run although this label never "changes"
        if (li == 0 && ti > 0) activate(act, lists, NT, ctl, t - g.TC, rr);
        if (li == g.th - 1 && ti < g.TR - 1) activate(act, lists, NT, ctl, t + g.TC, rr);
        if (lj == 0 && tj > 0) activate(act, lists, NT, ctl, t - 1, rr);
        if (lj == g.tw - 1 && tj < g.TC - 1) activate(act, lists, NT, ctl, t + 1, rr);
    }
    if (ground_source) {
        for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nperim; k += gridDim.x * blockDim.x)
            activate(act, lists, NT, ctl, perim_tiles[k], rr);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->glab = ground_source ? 0ull : LINF;
        // per-pass counters back to zero (none of them is read by this kernel)
        ctl->prev_naug = ctl->naug;
        ctl->prev_arcs = ctl->arcs;
        ctl->naug = 0;
        ctl->gsub_count = 0;
        ctl->gpred = 0xffffffffu;
        ctl->arcs = 0;
        ctl->nsrc2 = 0;
        ctl->ndef2 = 0;
    }
}

// ------------------------------------------------------ relaxation round ---

struct RoundArgs {
    unsigned int *act;          // round stamp: the tile is in that round's list
    unsigned int *lists;        // 3 x NT tile lists
    unsigned int *pstamp;       // pass stamp: the tile parked a candidate
    unsigned int *tstamp;       // pass stamp: the tile was relaxed
    unsigned long long *tile_rej;  // smallest parked candidate of each tile
    unsigned long long *vpart;  // striped visit counters (64 x 16)
    const unsigned int *perim_tiles;
    int nperim;
    unsigned int NT;
};

// 32 x 32 loop tiles, 256 threads, 4 nodes per thread.
constexpr int TJ = 32;

// Reduced costs of the in-arcs are staged as unsigned words, RC_NONE where
// there is no arc (a valid reduced cost is below 2^31).
constexpr unsigned int RC_NONE = 0xffffffffu;

// Candidate label of a node reached from neighbour label u over an arc of
// reduced cost rc (direction code dir): the distance in the high word, hops
// + 1 and the direction in the low word.  A distance sum that carries out
// of 32 bits (no arc, a neighbour without a label, or a distance of 2^32
// or more) becomes 0xffffffff, above the distance of every window bound, so
// such a candidate is never taken inside a window.
__device__ __forceinline__ unsigned long long cand_of(unsigned long long u, unsigned int rc,
                                                      unsigned int dir) {
    unsigned int d;
    const bool carry = __builtin_add_overflow((unsigned int)(u >> 32), rc, &d);
    const unsigned int lo = (((unsigned int)u | 7u) + 1u) | dir;
    return ((unsigned long long)(carry ? 0xffffffffu : d) << 32) | lo;
}

__device__ __forceinline__ unsigned long long umin64(unsigned long long a, unsigned long long b) {
    return a < b ? a : b;
}

// A candidate beyond the window for a node without a label, kept in rej
// (the smallest such over the tile parks the tile for a later window).
// Every label lies inside the window, so a beyond-window candidate can
// only ever matter to a node without one.
__device__ __forceinline__ void rej_one(unsigned long long &rej, unsigned long long u,
                                        unsigned int rc, unsigned int dir, unsigned long long lb) {
    unsigned int d;
    const bool carry = __builtin_add_overflow((unsigned int)(u >> 32), rc, &d);
    const bool ok = rc != RC_NONE && u != LINF && !carry;
    const unsigned long long cand = ((unsigned long long)d << 32) | ((((unsigned int)u | 7u) + 1u) | dir);
    rej = (ok && cand > lb && cand < rej) ? cand : rej;
}

// Sweeps per tile visit at most (a speed knob: the labels are the same for
// any value).
#ifndef WW_VISIT_ITERS
#define WW_VISIT_ITERS 8
#endif
constexpr int VISIT_ITERS = WW_VISIT_ITERS;  // sweeps per tile visit at most

__global__ __launch_bounds__(256) void k_sssp_round(Graph g, Ctl *ctl, RoundArgs ra,
                                                   unsigned int round, unsigned int pass_stamp,
                                                   unsigned long long lb, int stats) {
    __shared__ unsigned long long L[TJ + 2][TJ + 3];
    __shared__ int P[TJ + 2][TJ + 2];
    __shared__ int4 RC4[TJ][TJ];  // reduced costs of the in-arcs: from above, below, left, right
    __shared__ int wchg[3][4];    // per-iteration "a label changed" flag of each wave's band
    __shared__ int flags[4];  // changed border: top, bottom, left, right
    __shared__ int sh_any;
    __shared__ unsigned long long sh_gcand, sh_rej;

    const unsigned int NT = ra.NT;
    const unsigned int cnt = ctl->count[round % 3][0];
    const unsigned int *list = ra.lists + (size_t)(round % 3) * NT;
    // list (round + 2) % 3 was consumed by the previous round
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->count[(round + 2) % 3][0] = 0;
    const unsigned long long glab = ctl->glab;
    const int gpot = (int)ctl->gpot;
    const int R = g.R, C = g.C;
    unsigned int my_visits = 0;

    for (unsigned int idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
        const unsigned int tile = list[idx];
        ++my_visits;
        const unsigned long long t_start = stats ? wall_clock64() : 0ull;
        const int ti = tile / g.TC, tj = tile % g.TC;
        const int i0 = ti * TJ, j0 = tj * TJ;
        const int rows = min(TJ, R - i0), cols = min(TJ, C - j0);
        if (threadIdx.x < 4) flags[threadIdx.x] = 0;
        if (threadIdx.x == 0) {
            sh_rej = LINF;
            sh_gcand = LINF;
        }
        // stage labels and potentials with a one-node halo; outside = ground.
        // All loads of a thread (labels, potentials, arc costs and flows) are
        // issued before any LDS store, so that their latencies overlap.
        constexpr int NSTAGE = ((TJ + 2) * (TJ + 2) + 255) / 256;
        constexpr int NRC = TJ * TJ / 256;
        int cst[NRC][4];
        {
            unsigned long long lv[NSTAGE];
            int pv[NSTAGE];
#pragma unroll
            for (int s = 0; s < NSTAGE; ++s) {
                const int t = threadIdx.x + 256 * s;
                const int r = t / (TJ + 2), c = t % (TJ + 2);
                const int i = i0 - 1 + r, j = j0 - 1 + c;
                lv[s] = LINF;
                pv[s] = 0;
                if (t < (TJ + 2) * (TJ + 2) && r <= rows + 1 && c <= cols + 1) {
                    if (i >= 0 && i < R && j >= 0 && j < C) {
                        const long long v = (long long)i * C + j;
                        lv[s] = g.lab[v];
                        pv[s] = g.pot[v];
                    } else {
                        lv[s] = glab;
                        pv[s] = gpot;
                    }
                }
            }
            // arc costs and flows of the four in-arcs of every node, issued
            // with the label and potential loads (one memory latency for all)
#pragma unroll
            for (int s = 0; s < NRC; ++s) {
                const int t = threadIdx.x + 256 * s;
                const int li = t / TJ, lj = t % TJ;
                cst[s][0] = cst[s][1] = cst[s][2] = cst[s][3] = RC_INF;
                if (li < rows && lj < cols) {
                    const int i = i0 + li, j = j0 + lj;
                    long long e;
                    e = (long long)i * C + j;  // hx(i,j): from above, +1
                    cst[s][0] = move_cost(g.fx[e], +1, g.cxp[e], g.cxn[e]);
                    e = (long long)(i + 1) * C + j;  // hx(i+1,j): from below, -1
                    cst[s][1] = move_cost(g.fx[e], -1, g.cxp[e], g.cxn[e]);
                    e = (long long)i * g.n + j;  // vy(i,j): from the left, -1
                    cst[s][2] = move_cost(g.fy[e], -1, g.cyp[e], g.cyn[e]);
                    e = (long long)i * g.n + j + 1;  // vy(i,j+1): from the right, +1
                    cst[s][3] = move_cost(g.fy[e], +1, g.cyp[e], g.cyn[e]);
                }
            }
#pragma unroll
            for (int s = 0; s < NSTAGE; ++s) {
                const int t = threadIdx.x + 256 * s;
                if (t < (TJ + 2) * (TJ + 2)) {
                    L[t / (TJ + 2)][t % (TJ + 2)] = lv[s];
                    P[t / (TJ + 2)][t % (TJ + 2)] = pv[s];
                }
            }
        }
        __syncthreads();
        // reduced costs of the four in-arcs of every node
#pragma unroll
        for (int s = 0; s < NRC; ++s) {
            const int t = threadIdx.x + 256 * s;
            const int li = t / TJ, lj = t % TJ;
            int ru = RC_INF, rd = RC_INF, rl = RC_INF, rr = RC_INF;
            if (li < rows && lj < cols) {
                const int pv = P[li + 1][lj + 1];
                if (cst[s][0] != RC_INF) ru = cst[s][0] - P[li][lj + 1] + pv;
                if (cst[s][1] != RC_INF) rd = cst[s][1] - P[li + 2][lj + 1] + pv;
                if (cst[s][2] != RC_INF) rl = cst[s][2] - P[li + 1][lj] + pv;
                if (cst[s][3] != RC_INF) rr = cst[s][3] - P[li + 1][lj + 2] + pv;
                if (ru < 0 || rd < 0 || rl < 0 || rr < 0) {
                    atomicOr(&ctl->error, ERR_NEG_RC);
                    ru = max(ru, 0); rd = max(rd, 0); rl = max(rl, 0); rr = max(rr, 0);
                }
            }
            RC4[li][lj] = make_int4(ru == RC_INF ? (int)RC_NONE : ru, rd == RC_INF ? (int)RC_NONE : rd,
                                    rl == RC_INF ? (int)RC_NONE : rl, rr == RC_INF ? (int)RC_NONE : rr);
        }
        __syncthreads();
        const unsigned long long t_staged = stats ? wall_clock64() : 0ull;
        // Each thread owns a column segment of 4 nodes (column lj, rows
        // 4q..4q+3): their labels and in-arc reduced costs stay in registers,
        // and every iteration sweeps down the segment and back up.  The left,
        // right and end neighbours are re-read from LDS at every step, so a
        // label written by the neighbouring lane of the same wave one step
        // earlier is already seen (labels only decrease, so any value read is
        // a valid label).  Wave w owns rows 8w..8w+7; it skips an iteration
        // when no label changed in its band or the two adjacent bands during
        // the previous one.
        const int lj = threadIdx.x % TJ, q = threadIdx.x / TJ, wv = threadIdx.x >> 6;
        const int r0 = q * 4;
        unsigned long long init[4], y[4];
        int4 rc[4];
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            init[k] = L[r0 + k + 1][lj + 1];
            y[k] = init[k];
            rc[k] = RC4[r0 + k][lj];
            ok[k] = r0 + k < rows && lj < cols;
        }
        if (threadIdx.x < 12) wchg[threadIdx.x / 4][threadIdx.x % 4] = threadIdx.x < 8 ? 0 : 1;
        __syncthreads();
        unsigned long long rej = LINF;  // smallest useful candidate beyond the window
        const unsigned long long lb1 = lb + 1ull;  // lb < LINF: its hop field is at most HMAX
        // A visit stops after VISIT_ITERS sweeps even when labels still
        // change: it writes back what it has (labels only decrease, so every
        // label is valid) and lists the tile again for the next round, so
        // that one slow tile does not hold up the whole round.
        bool unconverged = true;
        for (int it = 0; it < VISIT_ITERS; ++it) {
            const int rd = (it + 2) % 3, wr = it % 3;
            const bool live = wchg[rd][wv] || (wv > 0 && wchg[rd][wv - 1]) || (wv < 3 && wchg[rd][wv + 1]);
            int changed = 0;
            if (live) {
// the smallest of the four candidates is taken when it is inside the window
// and below the node's label: one comparison with min(label, lb + 1)
#define WW_RELAX_NODE(k, PREV, NEXT)                                                  \
    if (ok[k]) {                                                                      \
        const unsigned long long c = umin64(                                          \
            umin64(cand_of(PREV, (unsigned)rc[k].x, 1u), cand_of(NEXT, (unsigned)rc[k].y, 2u)), \
            umin64(cand_of(L[r0 + k + 1][lj], (unsigned)rc[k].z, 3u),                  \
                   cand_of(L[r0 + k + 1][lj + 2], (unsigned)rc[k].w, 4u)));            \
        if (c < umin64(y[k], lb1)) {                                                  \
            y[k] = c;                                                                 \
            L[r0 + k + 1][lj + 1] = c;                                                \
            changed = 1;                                                              \
        }                                                                             \
    }
                WW_RELAX_NODE(0, L[r0][lj + 1], y[1])
                WW_RELAX_NODE(1, y[0], y[2])
                WW_RELAX_NODE(2, y[1], y[3])
                WW_RELAX_NODE(3, y[2], L[r0 + 5][lj + 1])
                WW_RELAX_NODE(2, y[1], y[3])
                WW_RELAX_NODE(1, y[0], y[2])
                WW_RELAX_NODE(0, L[r0][lj + 1], y[1])
#undef WW_RELAX_NODE
                if (changed) wchg[wr][wv] = 1;
            }
            if (threadIdx.x < 4) wchg[(it + 1) % 3][threadIdx.x] = 0;
            // the waves' change flags of this sweep decide for the whole
            // workgroup after one barrier (slot wr is next cleared two sweeps
            // later, after another barrier)
            __syncthreads();
            if (!(wchg[wr][0] | wchg[wr][1] | wchg[wr][2] | wchg[wr][3])) {
                if (stats && threadIdx.x == 0) atomicAdd(&ctl->iters, (unsigned long long)(it + 1));
                unconverged = false;
                break;
            }
        }
        if (unconverged && stats && threadIdx.x == 0)
            atomicAdd(&ctl->iters, (unsigned long long)VISIT_ITERS);
        // beyond-window candidates of the nodes still without a label, from
        // the final labels of the visit (all LDS writes are done: the loop
        // above ends on a barrier)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!ok[k] || y[k] != LINF) continue;
            const unsigned long long up = k == 0 ? L[r0][lj + 1] : y[k > 0 ? k - 1 : 0];
            const unsigned long long dn = k == 3 ? L[r0 + 5][lj + 1] : y[k < 3 ? k + 1 : 3];
            rej_one(rej, up, (unsigned)rc[k].x, 1u, lb);
            rej_one(rej, dn, (unsigned)rc[k].y, 2u, lb);
            rej_one(rej, L[r0 + k + 1][lj], (unsigned)rc[k].z, 3u, lb);
            rej_one(rej, L[r0 + k + 1][lj + 2], (unsigned)rc[k].w, 4u, lb);
        }
        const unsigned long long t_swept = stats ? wall_clock64() : 0ull;
        // write back, note changed borders
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int li = q * 4 + k;
            if (li >= rows || lj >= cols) continue;
            const unsigned long long l = L[li + 1][lj + 1];
            if (l != init[k]) {
                g.lab[(long long)(i0 + li) * C + (j0 + lj)] = l;
                if (li == 0) flags[0] = 1;
                if (li == rows - 1) flags[1] = 1;
                if (lj == 0) flags[2] = 1;
                if (lj == cols - 1) flags[3] = 1;
            }
        }
        // candidate labels for the ground from perimeter nodes of this tile
        unsigned long long gc = LINF;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int li = q * 4 + k;
            if (li >= rows || lj >= cols) continue;
            const int i = i0 + li, j = j0 + lj;
            const unsigned long long l = L[li + 1][lj + 1];
            if (l == LINF) continue;
            const int pv = P[li + 1][lj + 1];
            for (int side = 0; side < 4; ++side) {
                long long e;
                int c;
                if (side == 0) {
                    if (i != 0) continue;
                    e = j;
                    c = move_cost(g.fx[e], -1, g.cxp[e], g.cxn[e]);
                } else if (side == 1) {
                    if (i != R - 1) continue;
                    e = (long long)R * C + j;
                    c = move_cost(g.fx[e], +1, g.cxp[e], g.cxn[e]);
                } else if (side == 2) {
                    if (j != 0) continue;
                    e = (long long)i * g.n;
                    c = move_cost(g.fy[e], +1, g.cyp[e], g.cyn[e]);
                } else {
                    if (j != C - 1) continue;
                    e = (long long)i * g.n + C;
                    c = move_cost(g.fy[e], -1, g.cyp[e], g.cyn[e]);
                }
                if (c == RC_INF) continue;
                int rc = c - pv + gpot;
                if (rc < 0) {
                    atomicOr(&ctl->error, ERR_NEG_RC);
                    rc = 0;
                }
                const unsigned long long nd = (unsigned long long)ldist(l) + (unsigned)rc;
                if (nd > 0xffffffffull) continue;
                const unsigned long long cand = (nd << 32) | ((unsigned long long)(lhops(l) + 1) << 3);
                if (cand > lb) {
                    if (glab == LINF && cand < rej) rej = cand;
                    continue;
                }
                if (cand < gc) gc = cand;
            }
        }
        if (gc != LINF) atomicMin(&sh_gcand, gc);
        if (rej != LINF) atomicMin(&sh_rej, rej & ~7ull);
        __syncthreads();
        // activations for the next round (lanes 0-3, one neighbour each, so
        // that the atomics' round trips overlap), stamps for this pass
        // (lane 4) and the ground label (lane 5), all in wave 0
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            const unsigned int nr = round + 1;
            unsigned int nb = 0;
            bool want = false;
            if (lane == 0) { want = flags[0] && ti > 0; nb = tile - g.TC; }
            if (lane == 1) { want = flags[1] && ti < g.TR - 1; nb = tile + g.TC; }
            if (lane == 2) { want = flags[2] && tj > 0; nb = tile - 1; }
            if (lane == 3) { want = flags[3] && tj < g.TC - 1; nb = tile + 1; }
            if (lane == 7) { want = unconverged; nb = tile; }
            const bool fresh = want && atomicExch(&ra.act[nb], nr) != nr;
            const unsigned long long fm = __ballot(fresh);
            if (fm) {
                const int leader = __ffsll((long long)fm) - 1;
                unsigned int pos = 0;
                if (lane == leader) pos = atomicAdd(&ctl->count[nr % 3][0], (unsigned int)__popcll(fm));
                pos = __shfl(pos, leader, 64);
                if (fresh) {
                    const unsigned int rank = (unsigned int)__popcll(fm & ((1ull << lane) - 1ull));
                    ra.lists[(size_t)(nr % 3) * NT + pos + rank] = nb;
                }
            }
            if (lane == 4) {
                // the tile's parked candidates (recomputed in full at every visit)
                ra.tile_rej[tile] = sh_rej;
                if (sh_rej != LINF) ra.pstamp[tile] = pass_stamp;
                ra.tstamp[tile] = pass_stamp;
            }
            if (lane == 5) {
                int any = 0;
                if (sh_gcand != LINF && sh_gcand < ctl->glab) {
                    unsigned long long old = atomicMin(&ctl->glab, sh_gcand);
                    if (sh_gcand < old) any = 1;
                }
                sh_any = any;
            }
            if (stats && lane == 6) {
                const unsigned long long t_end = wall_clock64();
                atomicAdd(&ctl->vt_sum, t_end - t_start);
                atomicAdd(&ctl->vt_stage, t_staged - t_start);
                atomicAdd(&ctl->vt_sweep, t_swept - t_start);
                atomicMax(&ctl->vt_max, t_end - t_start);
            }
        }
        __syncthreads();
        if (sh_any) {
            for (int k = threadIdx.x; k < ra.nperim; k += 256)
                activate(ra.act, ra.lists, NT, ctl, ra.perim_tiles[k], round + 1);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && my_visits)
        atomicAdd(&ra.vpart[(blockIdx.x % 64) * 16], (unsigned long long)my_visits);
}

__global__ void k_requeue_pending(Ctl *ctl, const unsigned int *pstamp, unsigned int pass,
                                  const unsigned long long *tile_rej, unsigned long long lb,
                                  unsigned int *act, unsigned int *lists, unsigned int NT,
                                  unsigned int rr) {
    for (unsigned int t = blockIdx.x * blockDim.x + threadIdx.x; t < NT; t += gridDim.x * blockDim.x)
        if (pstamp[t] == pass && tile_rej[t] <= lb) activate(act, lists, NT, ctl, t, rr);
}

// End of a window, in one launch: the deficits settled in it (a settled
// ground absorbs all of its deficit units) and the smallest candidate parked
// by a tile in this pass, in the counters of slot w; the other slot's
// counters are cleared for the next launch.  The host launches it after
// every batch of rounds; it counts only when the list of round rr is empty,
// i.e. when the batch ended the window.
__global__ void k_window_end(Graph g, Ctl *ctl, const unsigned int *def, unsigned long long lb,
                             const unsigned int *pstamp, unsigned int pass,
                             const unsigned long long *tile_rej, unsigned int NT, int w,
                             unsigned int rr) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->wsettled[w ^ 1] = 0;
        ctl->wminrej[w ^ 1] = LINF;
    }
    if (ctl->count[rr % 3][0] != 0) return;
    const unsigned int nd = ctl->ndef;
    unsigned int c = 0;
    for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k < nd; k += gridDim.x * blockDim.x) {
        const unsigned long long l = g.lab[def[k]];
        if (l <= lb) ++c;
    }
    unsigned long long mn = LINF;
    for (unsigned int t = blockIdx.x * blockDim.x + threadIdx.x; t < NT; t += gridDim.x * blockDim.x)
        if (pstamp[t] == pass) {
            const unsigned long long r = tile_rej[t];
            mn = r < mn ? r : mn;
        }
    for (int off = 32; off > 0; off >>= 1) {
        c += __shfl_down(c, off, 64);
        const unsigned long long o = __shfl_down(mn, off, 64);
        mn = o < mn ? o : mn;
    }
    // one counter atomic per workgroup (thousands on one address cost more
    // than the count itself)
    __shared__ unsigned int wc[4];
    if ((threadIdx.x & 63) == 0) {
        wc[threadIdx.x >> 6] = c;
        // only a wave that may lower the minimum takes the atomic
        if (mn != LINF && mn < *(volatile unsigned long long *)&ctl->wminrej[w])
            atomicMin(&ctl->wminrej[w], mn);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int t = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += wc[k];
        if (t) atomicAdd(&ctl->wsettled[w], t);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long gl = ctl->glab;
        if (ctl->gex < 0 && gl <= lb) atomicAdd(&ctl->wsettled[w], (unsigned int)(-ctl->gex));
    }
}

// ---------------------------------------------------------- augmentation ---

// The ground's predecessor: the smallest perimeter arc index whose label
// candidate equals the ground label.
__global__ void k_ground_pred(Graph g, Ctl *ctl, unsigned long long lb) {
    const unsigned long long gl = ctl->glab;
    if (gl > lb || ctl->gex > 0) return;
    const unsigned int na = 2u * g.C + 2u * g.R;
    const int gpot = (int)ctl->gpot;
    for (unsigned int a = blockIdx.x * blockDim.x + threadIdx.x; a < na; a += gridDim.x * blockDim.x) {
        int i, j, kind, delta;
        long long e;
        ground_arc(g, a, i, j, kind, e, delta);
        const long long v = (long long)i * g.C + j;
        const unsigned long long l = g.lab[v];
        if (l == LINF) continue;
        const int c = kind == 0 ? move_cost(g.fx[e], delta, g.cxp[e], g.cxn[e])
                                : move_cost(g.fy[e], delta, g.cyp[e], g.cyn[e]);
        if (c == RC_INF) continue;
        const long long rc = (long long)c - g.pot[v] + gpot;
        const unsigned long long nd = (unsigned long long)ldist(l) + (unsigned long long)max(rc, 0ll);
        const unsigned long long cand = (nd << 32) | ((unsigned long long)(lhops(l) + 1) << 3);
        if (cand == gl) atomicMin(&ctl->gpred, a);
    }
}

// row and column of loop node v (v < 2^29, so 32-bit arithmetic suffices:
// the walks below take one step per memory round trip, and a 64-bit
// division would add to every step)
__device__ __forceinline__ void node_rc(const Graph &g, long long v, int &i, int &j) {
    const unsigned int u = (unsigned int)v, C = (unsigned int)g.C;
    const unsigned int q = u / C;
    i = (int)q;
    j = (int)(u - q * C);
}

// predecessor of loop node v (i,j) along direction dir; -1 = ground
__device__ __forceinline__ long long pred_node(const Graph &g, int i, int j, int dir) {
    switch (dir) {
        case DIR_UP: return i > 0 ? (long long)(i - 1) * g.C + j : -1;
        case DIR_DOWN: return i < g.R - 1 ? (long long)(i + 1) * g.C + j : -1;
        case DIR_LEFT: return j > 0 ? (long long)i * g.C + j - 1 : -1;
        default: return j < g.C - 1 ? (long long)i * g.C + j + 1 : -1;
    }
}

// Walk from v to its root.  Returns the root node; *gsub = 1 when the root
// is a child of the ground acting as a supply.
__device__ long long walk_root(const Graph &g, Ctl *ctl, long long v, int gsrc, int *gsub) {
    *gsub = 0;
    const long long N = (long long)g.R * g.C;
    for (long long steps = 0; steps <= N + 2; ++steps) {
        const unsigned long long l = g.lab[v];
        const int dir = (int)(l & 7);
        if (dir == DIR_NONE) return v;
        int i, j;
        node_rc(g, v, i, j);
        long long u = pred_node(g, i, j, dir);
        if (u < 0) {
            if (gsrc) {
                *gsub = 1;
                return v;
            }
            const unsigned int a = ctl->gpred;
            if (a >= 2u * g.C + 2u * g.R) break;  // no ground predecessor: report below
            int pi, pj, kind, delta;
            long long e;
            ground_arc(g, a, pi, pj, kind, e, delta);
            u = (long long)pi * g.C + pj;
        }
        v = u;
    }
    atomicOr(&ctl->error, ERR_WALK);
    return -1;
}

__global__ void k_roots(Graph g, Ctl *ctl, const unsigned int *def, unsigned long long lb,
                        unsigned int *gsub_list) {
    const unsigned int nd = ctl->ndef;
    const int gsrc = ctl->gex > 0;
    const long long N = (long long)g.R * g.C;
    for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k <= nd; k += gridDim.x * blockDim.x) {
        long long start;
        unsigned long long key;
        if (k < nd) {
            const unsigned int t = def[k];
            const unsigned long long l = g.lab[t];
            if (l > lb) continue;
            start = t;
            key = ((unsigned long long)ldist(l) << 32) | t;
        } else {
            // the ground as a demand: its path enters through gpred
            const unsigned long long gl = ctl->glab;
            if (!(ctl->gex < 0 && gl <= lb)) continue;
            if (ctl->gpred >= 2u * g.C + 2u * g.R) {
                atomicOr(&ctl->error, ERR_WALK);
                continue;
            }
            int pi, pj, kind, delta;
            long long e;
            ground_arc(g, ctl->gpred, pi, pj, kind, e, delta);
            start = (long long)pi * g.C + pj;
            key = ((unsigned long long)ldist(gl) << 32) | (unsigned long long)N;
        }
        int gsub = 0;
        const long long root = walk_root(g, ctl, start, gsrc, &gsub);
        if (root < 0) continue;
        const unsigned long long old = atomicMin(&g.best[root], key);
        if (gsub && old == LINF) gsub_list[atomicAdd(&ctl->gsub_count, 1u)] = (unsigned int)root;
    }
}

// Keep at most gex ground-rooted subtrees: those with the smallest
// (best key, root id).  O(k^2), k <= perimeter length.
__global__ void k_gsub_select(Graph g, Ctl *ctl, const unsigned int *gsub_list,
                              unsigned char *drop) {
    const unsigned int k = ctl->gsub_count;
    const long long allow = ctl->gex;
    for (unsigned int a = blockIdx.x * blockDim.x + threadIdx.x; a < k; a += gridDim.x * blockDim.x) {
        drop[a] = 0;
        if ((long long)k <= allow) continue;
        const unsigned int ra = gsub_list[a];
        const unsigned long long ka = g.best[ra];
        long long rank = 0;
        for (unsigned int b = 0; b < k; ++b) {
            const unsigned int rb = gsub_list[b];
            const unsigned long long kb = g.best[rb];
            if (kb < ka || (kb == ka && rb < ra)) ++rank;
        }
        if (rank >= allow) drop[a] = 1;
    }
}

__device__ __forceinline__ void flip_into(Graph &g, long long v, int dir) {
    int i, j;
    node_rc(g, v, i, j);
    switch (dir) {
        case DIR_UP: g.fx[(long long)i * g.C + j] += 1; break;
        case DIR_DOWN: g.fx[(long long)(i + 1) * g.C + j] -= 1; break;
        case DIR_LEFT: g.fy[(long long)i * g.n + j] -= 1; break;
        default: g.fy[(long long)i * g.n + j + 1] += 1; break;
    }
}

__device__ __forceinline__ void flip_ground_arc(Graph &g, unsigned int a) {
    int i, j, kind, delta;
    long long e;
    ground_arc(g, a, i, j, kind, e, delta);
    if (kind == 0) g.fx[e] += (int8_t)delta;
    else g.fy[e] += (int8_t)delta;
}

// Apply one unit along root r's chosen path: from the deficit back to r.
// The in-grid arcs of a path are not flipped here: the walk stores
// (pass, direction) at the node each arc enters, and k_potentials, which
// visits every node of the tiles relaxed in the pass (path nodes are
// settled, so their tiles were relaxed), applies the flip.  A step of the
// walk is then one dependent label load and one store.  Paths from
// different roots are vertex-disjoint, so a node holds one arc per pass;
// no kernel reads the flows between the two.
__global__ void k_augment(Graph g, Ctl *ctl, const unsigned int *src, const unsigned int *gsub_list,
                          const unsigned char *drop, unsigned int *flip, unsigned int pass) {
    const unsigned int ns = ctl->nsrc, ng = ctl->gsub_count;
    const long long N = (long long)g.R * g.C;
    for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k < ns + ng;
         k += gridDim.x * blockDim.x) {
        const bool is_g = k >= ns;
        const unsigned int r = is_g ? gsub_list[k - ns] : src[k];
        const unsigned long long b = g.best[r];
        if (b == LINF) continue;
        g.best[r] = LINF;
        if (is_g && drop[k - ns]) continue;
        const long long t = (long long)(b & 0xffffffffull);
        long long v;
        unsigned long long flips = 0;
        // A path through the ground needs the ground's predecessor arc, which
        // exists whenever the ground is settled, and only then can a path
        // cross it (labels grow along paths).  Its absence is checked where
        // the arc is used: the walk stops with ERR_WALK, which fails the
        // solve, before any index is formed from it.
        const unsigned int na = 2u * g.C + 2u * g.R;
        if (t == N) {  // into the ground through its predecessor arc
            const unsigned int a = ctl->gpred;
            if (a >= na) {
                atomicOr(&ctl->error, ERR_WALK);
                continue;
            }
            flip_ground_arc(g, a);
            int pi, pj, kind, delta;
            long long e;
            ground_arc(g, a, pi, pj, kind, e, delta);
            v = (long long)pi * g.C + pj;
            ++flips;
        } else {
            v = t;
        }
        unsigned long long l = g.lab[v];
        for (long long steps = 0; steps <= N + 2; ++steps) {
            const int dir = (int)(l & 7);
            if (dir == DIR_NONE) break;  // reached the supply r
            int i, j;
            node_rc(g, v, i, j);
            long long u = pred_node(g, i, j, dir);
            flip[v] = (pass << 3) | (unsigned int)dir;
            ++flips;
            if (u < 0) {
                if (is_g) break;  // the ground is the supply
                const unsigned int a = ctl->gpred;
                if (a >= na) {
                    atomicOr(&ctl->error, ERR_WALK);
                    break;
                }
                flip_ground_arc(g, a);
                ++flips;
                int pi, pj, kind, delta;
                long long e;
                ground_arc(g, a, pi, pj, kind, e, delta);
                u = (long long)pi * g.C + pj;
            }
            l = g.lab[u];
            v = u;
        }
        if (is_g) atomicAdd((unsigned long long *)&ctl->gex, (unsigned long long)-1ll);
        else g.ex[r] -= 1;
        if (t == N) atomicAdd((unsigned long long *)&ctl->gex, 1ull);
        else g.ex[t] += 1;
        atomicAdd(&ctl->naug, 1u);
        atomicAdd(&ctl->arcs, flips);
    }
}

// pot(v) += B - d(v) on every reached node, labels back to infinity.  Each
// workgroup checks the stamps of POT_CHUNK tiles at once and then updates
// only the tiles relaxed in this pass, so that a pass that reached a few
// tiles costs little more than one read of the stamps.  The relaxed tiles
// of a pass lie close together, so chunks are kept small: a workgroup
// updates at most POT_CHUNK tiles one after another.
constexpr int POT_CHUNK = 8;

__global__ __launch_bounds__(256) void k_potentials(Graph g, Ctl *ctl, const unsigned int *tstamp,
                                                    unsigned int pass, unsigned int NT,
                                                    unsigned long long lb, const unsigned int *flip) {
    __shared__ unsigned int todo[POT_CHUNK];
    __shared__ int ntodo;
    const unsigned int bound = ldist(lb);
    int mx = 0;
    for (unsigned int base = blockIdx.x * POT_CHUNK; base < NT; base += gridDim.x * POT_CHUNK) {
        if (threadIdx.x == 0) ntodo = 0;
        __syncthreads();
        if (threadIdx.x < POT_CHUNK) {
            const unsigned int tile = base + threadIdx.x;
            if (tile < NT && tstamp[tile] == pass) todo[atomicAdd(&ntodo, 1)] = tile;
        }
        __syncthreads();
        const int nt = ntodo;
        for (int k = 0; k < nt; ++k) {
            const unsigned int tile = todo[k];
            const int i0 = (int)(tile / g.TC) * TJ, j0 = (int)(tile % g.TC) * TJ;
            long long v[TJ * TJ / 256];
            unsigned long long l[TJ * TJ / 256];
            unsigned int fr[TJ * TJ / 256];
#pragma unroll
            for (int s = 0; s < TJ * TJ / 256; ++s) {
                const int t = threadIdx.x + 256 * s;
                const int i = i0 + t / TJ, j = j0 + t % TJ;
                v[s] = (i < g.R && j < g.C) ? (long long)i * g.C + j : -1;
                l[s] = v[s] >= 0 ? g.lab[v[s]] : LINF;
                fr[s] = v[s] >= 0 ? flip[v[s]] : 0u;
            }
#pragma unroll
            for (int s = 0; s < TJ * TJ / 256; ++s) {
                if (l[s] == LINF) continue;
                // the arc into this node on a path augmented in this pass
                if ((fr[s] >> 3) == pass) flip_into(g, v[s], (int)(fr[s] & 7u));
                g.lab[v[s]] = LINF;
                if (l[s] > lb) continue;
                const unsigned int d = ldist(l[s]);
                const long long np = (long long)g.pot[v[s]] + (bound - d);
                if (np > POT_LIMIT) atomicOr(&ctl->error, ERR_POT);
                g.pot[v[s]] = (int)min(np, (long long)POT_LIMIT);
                mx = max(mx, (int)min(np, (long long)POT_LIMIT));
            }
        }
        __syncthreads();
    }
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_down(mx, off, 64));
    // only a wave that may raise the maximum takes the atomic: thousands of
    // atomics on one address from every wave cost more than the updates
    if ((threadIdx.x & 63) == 0 && mx > 0 && mx > *(volatile int *)&ctl->max_pot)
        atomicMax(&ctl->max_pot, mx);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned long long gl = ctl->glab;
        if (gl <= lb) {
            ctl->gpot += bound - ldist(gl);
            if (ctl->gpot > POT_LIMIT) atomicOr(&ctl->error, ERR_POT);
        }
        ctl->glab = LINF;
    }
}

// Debug check (WW_MCF_CHECK=1): every residual arc must have a non-negative
// reduced cost after a pass.  Records the first offending arc.
struct CheckRec {
    int found;
    int kind;          // in-arc direction at v (1..4) or 8+side for an arc into the ground
    long long u, v;    // tail, head (-1 = ground)
    long long rc;
    long long pu, pv;
    unsigned long long lu, lv;  // labels before the potential update
    int f, cp, cn;
};

__global__ void k_check_rc(Graph g, const Ctl *ctl, const unsigned long long *lab_before,
                           CheckRec *rec) {
    const long long N = (long long)g.R * g.C;
    const long long gpot = ctl->gpot;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < N;
         v += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(v / g.C), j = (int)(v % g.C);
        for (int dir = 1; dir <= 4; ++dir) {
            long long e;
            int kind, delta;
            if (dir == DIR_UP) { e = (long long)i * g.C + j; kind = 0; delta = +1; }
            else if (dir == DIR_DOWN) { e = (long long)(i + 1) * g.C + j; kind = 0; delta = -1; }
            else if (dir == DIR_LEFT) { e = (long long)i * g.n + j; kind = 1; delta = -1; }
            else { e = (long long)i * g.n + j + 1; kind = 1; delta = +1; }
            const int f = kind == 0 ? g.fx[e] : g.fy[e];
            const int cp = kind == 0 ? g.cxp[e] : g.cyp[e];
            const int cn = kind == 0 ? g.cxn[e] : g.cyn[e];
            const int c = move_cost(f, delta, cp, cn);
            if (c == RC_INF) continue;
            const long long u = pred_node(g, i, j, dir);
            const long long pu = u < 0 ? gpot : g.pot[u];
            const long long rc = (long long)c - pu + g.pot[v];
            if (rc < 0 && atomicCAS(&rec->found, 0, 1) == 0) {
                rec->kind = dir; rec->u = u; rec->v = v; rec->rc = rc; rec->pu = pu; rec->pv = g.pot[v];
                rec->lu = u < 0 ? 0 : lab_before[u]; rec->lv = lab_before[v];
                rec->f = f; rec->cp = cp; rec->cn = cn;
            }
            // the reverse move (v -> u) of the same edge
            const int c2 = move_cost(f, -delta, cp, cn);
            if (c2 == RC_INF) continue;
            const long long rc2 = (long long)c2 - g.pot[v] + pu;
            if (rc2 < 0 && atomicCAS(&rec->found, 0, 1) == 0) {
                rec->kind = 8 + dir; rec->u = v; rec->v = u; rec->rc = rc2; rec->pu = g.pot[v]; rec->pv = pu;
                rec->lu = lab_before[v]; rec->lv = u < 0 ? 0 : lab_before[u];
                rec->f = f; rec->cp = cp; rec->cn = cn;
            }
        }
    }
}

// Debug check (WW_MCF_CHECK=1) of the tile-list protocol after a batch of
// rounds: the list of the next round rr holds count <= NT entries, every
// entry is a tile index below NT whose round stamp is rr, and exactly count
// tiles carry that stamp (so no tile is listed twice).  bad[0]: an entry out
// of range; bad[1]: an entry without the stamp; bad[2]: tiles with the stamp.
__global__ void k_check_lists(const Ctl *ctl, const unsigned int *act, const unsigned int *lists,
                              unsigned int NT, unsigned int rr, unsigned int *bad) {
    const unsigned int cnt = ctl->count[rr % 3][0];
    const unsigned int *list = lists + (size_t)(rr % 3) * NT;
    const unsigned int lim = cnt < NT ? cnt : NT;
    for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k < NT; k += gridDim.x * blockDim.x) {
        if (k < lim) {
            const unsigned int t = list[k];
            if (t >= NT) atomicOr(&bad[0], 1u);
            else if (act[t] != rr) atomicOr(&bad[1], 1u);
        }
        if (act[k] == rr) atomicAdd(&bad[2], 1u);
    }
}

// keep supplies / demands that still carry excess; one counter atomic per
// wave and list (the lanes' slots follow from a ballot)
__global__ void k_compact(Graph g, Ctl *ctl, const unsigned int *src, const unsigned int *def,
                          unsigned int *src2, unsigned int *def2) {
    const unsigned int ns = ctl->nsrc, nd = ctl->ndef;
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    // the loop bound is the same for every lane of a wave (blockDim is a
    // multiple of 64), so that all lanes take part in the ballots
    for (unsigned int base = blockIdx.x * blockDim.x; base < ns + nd; base += gridDim.x * blockDim.x) {
        const unsigned int k = base + threadIdx.x;
        const bool in = k < ns + nd;
        const bool is_src = in && k < ns;
        const unsigned int v = !in ? 0u : (is_src ? src[k] : def[k - ns]);
        const bool keep_s = is_src && g.ex[v] > 0;
        const bool keep_d = in && !is_src && g.ex[v] < 0;
        const unsigned long long ms = __ballot(keep_s), md = __ballot(keep_d);
        unsigned int bs = 0, bd = 0;
        if (lane == 0) {
            if (ms) bs = atomicAdd(&ctl->nsrc2, (unsigned int)__popcll(ms));
            if (md) bd = atomicAdd(&ctl->ndef2, (unsigned int)__popcll(md));
        }
        bs = __shfl(bs, 0, 64);
        bd = __shfl(bd, 0, 64);
        if (keep_s) src2[bs + __popcll(ms & below)] = v;
        if (keep_d) def2[bd + __popcll(md & below)] = v;
    }
}

__global__ void k_swap_lists(Ctl *ctl) {
    ctl->nsrc = ctl->nsrc2;
    ctl->ndef = ctl->ndef2;
}

// a[k] = -a[k] for k < n, 16 bytes per thread and step (SWAR negation of
// the bytes, or of the words), with scalar head and tail where a is not
// 16-byte aligned
__device__ __forceinline__ unsigned int neg_bytes(unsigned int w) {
    const unsigned int y = ~w;  // -x = ~x + 1 in every byte, no carry across bytes
    return ((y & 0x7f7f7f7fu) + 0x01010101u) ^ (y & 0x80808080u);
}

template <typename T>
__device__ __forceinline__ void negate_span(T *a, long long n, long long tid, long long stride) {
    constexpr int V = 16 / (int)sizeof(T);
    const long long head =
        min(n, (long long)(((16u - ((unsigned int)(uintptr_t)a & 15u)) & 15u) / sizeof(T)));
    for (long long k = tid; k < head; k += stride) a[k] = (T)-a[k];
    const long long nvec = (n - head) / V;
    uint4 *v = reinterpret_cast<uint4 *>(a + head);
    for (long long k = tid; k < nvec; k += stride) {
        uint4 x = v[k];
        if (sizeof(T) == 1) {
            x.x = neg_bytes(x.x); x.y = neg_bytes(x.y); x.z = neg_bytes(x.z); x.w = neg_bytes(x.w);
        } else {
            x.x = 0u - x.x; x.y = 0u - x.y; x.z = 0u - x.z; x.w = 0u - x.w;
        }
        v[k] = x;
    }
    for (long long k = head + nvec * V + tid; k < n; k += stride) a[k] = (T)-a[k];
}

// The reversed problem: every arc turned round, supplies and demands
// exchanged.  Its residual arc v -> u across an edge has the cost of the
// original residual arc u -> v when the net flows are negated and the two
// cost planes of every edge exchanged (the host swaps the plane pointers);
// with potentials negated its reduced costs equal the original ones, so a
// forward search in the reversed frame is a search towards the demands in
// the original one.  Applying the map twice restores the original state.
__global__ void k_reverse_frame(Graph g, Ctl *ctl, long long nx, long long ny, long long N) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    negate_span(g.fx, nx, tid, stride);
    negate_span(g.fy, ny, tid, stride);
    negate_span(g.ex, N, tid, stride);
    negate_span(g.pot, N, tid, stride);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const unsigned int ns = ctl->nsrc;
        ctl->nsrc = ctl->ndef;
        ctl->ndef = ns;
        ctl->gex = -ctl->gex;
        ctl->gpot = -ctl->gpot;
    }
}

// sum of the costs of the corrected edges of one plane: the flows are read
// 16 bytes at a time (scalar head and tail where f is not 16-byte aligned)
// and a cost is read only where the flow is not zero
__device__ __forceinline__ long long cost_span(const int8_t *f, const int16_t *cp, const int16_t *cn,
                                               long long n, long long tid, long long stride) {
    long long s = 0;
    auto one = [&](long long e, int v) { s += v > 0 ? cp[e] : (v < 0 ? cn[e] : 0); };
    const long long head = min(n, (long long)((16u - ((unsigned int)(uintptr_t)f & 15u)) & 15u));
    for (long long k = tid; k < head; k += stride) one(k, f[k]);
    const long long nvec = (n - head) / 16;
    const uint4 *v = reinterpret_cast<const uint4 *>(f + head);
    for (long long k = tid; k < nvec; k += stride) {
        const uint4 x = v[k];
        if ((x.x | x.y | x.z | x.w) == 0u) continue;
        const unsigned int w[4] = {x.x, x.y, x.z, x.w};
        const long long e0 = head + 16 * k;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!w[q]) continue;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int fv = (int)(signed char)(w[q] >> (8 * b));
                if (fv) one(e0 + 4 * q + b, fv);
            }
        }
    }
    for (long long k = head + nvec * 16 + tid; k < n; k += stride) one(k, f[k]);
    return s;
}

__global__ __launch_bounds__(256) void k_total_cost(const int8_t *fx, const int8_t *fy,
                                                   const int16_t *cxp, const int16_t *cxn,
                                                   const int16_t *cyp, const int16_t *cyn,
                                                   long long nx, long long ny,
                                                   long long *__restrict__ part) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long s = cost_span(fx, cxp, cxn, nx, tid, stride) + cost_span(fy, cyp, cyn, ny, tid, stride);
    __shared__ long long red[4];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_total_finish(int nb, const long long *part, Ctl *ctl) {
    __shared__ long long red[4];
    long long s = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) ctl->total_cost = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_export_pot(const int *pot, const Ctl *ctl, long long N, int64_t *out) {
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v <= N;
         v += (long long)gridDim.x * blockDim.x)
        out[v] = v < N ? (int64_t)pot[v] : (int64_t)ctl->gpot;
}

// ------------------------------------------------------------------ host ---

constexpr unsigned int HMAX = 0x1fffffffu;

// window schedule (ww_set_mcf_params), read once per solve
std::atomic<int> g_first_hops{64};
std::atomic<int> g_first_dstep{256};
std::atomic<int> g_full_passes{0};
std::atomic<int> g_first_deficit{0};
std::atomic<int> g_reverse_below{0};
std::atomic<int> g_hop_growth{2};

static unsigned long long mk_label(unsigned int d, unsigned int h) {
    return ((unsigned long long)d << 32) | ((unsigned long long)h << 3) | 7ull;
}

static ww_status decode_error(int e) {
    if (e & ERR_NEG_RC) return fail(WW_E_DEVICE, "min-cost flow: negative reduced cost (invariant broken)");
    if (e & ERR_POT) return fail(WW_E_OVERFLOW, "min-cost flow: node potential above 2^30");
    if (e & ERR_WALK) return fail(WW_E_DEVICE, "min-cost flow: predecessor walk did not end");
    if (e & ERR_ITERS) return fail(WW_E_DEVICE, "min-cost flow: tile relaxation did not converge");
    return fail(WW_E_DEVICE, "min-cost flow: error flags 0x%x", e);
}

ww_status mcf_impl(const int8_t *res, int m, int n, const int16_t *cxp, const int16_t *cxn,
                   const int16_t *cyp, const int16_t *cyn, int8_t *dkx, int8_t *dky,
                   int64_t *pot_out, int64_t *total, ww_mcf_stats *stats, hipStream_t st) {
    const long long nx = (long long)m * (n - 1), ny = (long long)(m - 1) * n;
    if (nx > 0) WW_HIP(hipMemsetAsync(dkx, 0, nx, st));
    if (ny > 0) WW_HIP(hipMemsetAsync(dky, 0, ny, st));
    ww_mcf_stats S;
    memset(&S, 0, sizeof(S));
    last_mcf_stats() = S;
    const auto t_start = std::chrono::steady_clock::now();
    const int R = m - 1, C = n - 1;
    if (R < 1 || C < 1) {
        if (pot_out) WW_HIP(hipMemsetAsync(pot_out, 0, sizeof(int64_t), st));
        WW_HIP(hipStreamSynchronize(st));
        *total = 0;
        if (stats) *stats = S;
        return WW_OK;
    }
    hipEvent_t ev[2];
    WW_TRY(workspace_events(&ev[0], &ev[1]));
    const long long N = (long long)R * C;
    if (N >= (1ll << 29)) return fail(WW_E_INVALID_ARG, "more than 2^29 loops");
    Graph g;
    g.R = R; g.C = C; g.n = n;
    g.th = TJ;
    g.tw = TJ;
    g.TR = ceil_div(R, g.th); g.TC = ceil_div(C, g.tw);
    g.cxp = cxp; g.cxn = cxn; g.cyp = cyp; g.cyn = cyn;
    g.fx = dkx; g.fy = dky;
    const unsigned int NT = (unsigned)g.TR * g.TC;
    const int nperim_arcs = 2 * C + 2 * R;
    WW_TRY(scratch(SLOT_MCF_LAB, sizeof(unsigned long long) * N, (void **)&g.lab));
    WW_TRY(scratch(SLOT_MCF_BEST, sizeof(unsigned long long) * N, (void **)&g.best));
    WW_TRY(scratch(SLOT_MCF_POT, sizeof(int) * N, (void **)&g.pot));
    WW_TRY(scratch(SLOT_MCF_EX, N, (void **)&g.ex));
    // per-tile state: act, pstamp, tstamp (NT each, cleared per call),
    // lists (3 NT), perim_tiles (NT), tile_rej (NT x 8 B), vpart (64 x 16 x 8 B)
    unsigned int *tiles = nullptr;
    const size_t tiles_words = 8 * (size_t)NT + 2;
    WW_TRY(scratch(SLOT_MCF_TILES, sizeof(unsigned int) * (tiles_words + 2 * (size_t)NT) + 8192 + 256,
                   (void **)&tiles));
    RoundArgs ra;
    ra.NT = NT;
    ra.act = tiles;
    ra.pstamp = tiles + (size_t)NT;
    ra.tstamp = tiles + 2 * (size_t)NT;
    ra.lists = tiles + 3 * (size_t)NT;
    ra.perim_tiles = tiles + 6 * (size_t)NT;
    ra.tile_rej = (unsigned long long *)(tiles + 7 * (size_t)NT + ((7 * (size_t)NT) & 1));
    ra.vpart = (unsigned long long *)(tiles + tiles_words + 2 * (size_t)NT);
    char *nodes = nullptr;
    const size_t nl_bytes = sizeof(unsigned int) * (size_t)N;
    const size_t gs_bytes = sizeof(unsigned int) * (size_t)nperim_arcs + 256;
    WW_TRY(scratch(SLOT_MCF_NODES, 4 * nl_bytes + gs_bytes + nperim_arcs + 1024, (void **)&nodes));
    unsigned int *src = (unsigned int *)nodes, *def = src + N, *src2 = def + N, *def2 = src2 + N;
    unsigned int *gsub_list = def2 + N;
    unsigned char *drop = (unsigned char *)(nodes + 4 * nl_bytes + gs_bytes);
    Ctl *ctl = nullptr;
    WW_TRY(scratch(SLOT_MCF_LISTS, sizeof(Ctl), (void **)&ctl));
    Ctl *h = nullptr;
    WW_TRY(host_scratch(sizeof(Ctl), (void **)&h));

    std::vector<unsigned int> ptiles;
    for (int ti = 0; ti < g.TR; ++ti)
        for (int tj = 0; tj < g.TC; ++tj)
            if (ti == 0 || tj == 0 || ti == g.TR - 1 || tj == g.TC - 1)
                ptiles.push_back((unsigned)(ti * g.TC + tj));
    ra.nperim = (int)ptiles.size();
    WW_HIP(hipMemcpyAsync((void *)ra.perim_tiles, ptiles.data(), sizeof(unsigned int) * ptiles.size(),
                          hipMemcpyHostToDevice, st));
    // stamps start at zero on every call: rounds and passes count from 1
    WW_HIP(hipMemsetAsync(ra.act, 0, sizeof(unsigned int) * 3 * (size_t)NT, st));
    WW_HIP(hipMemsetAsync(ra.vpart, 0, 8192, st));
    WW_HIP(hipMemsetAsync(ctl, 0, sizeof(Ctl), st));
    const int IB = (int)std::min<long long>(8192, std::max<long long>(1, ceil_div(N, 256)));
    const int nib = ceil_div(N, INIT_CHUNK);
    int *bc = nullptr;
    WW_TRY(scratch(SLOT_MCF_PART, sizeof(long long) * (size_t)std::max(3 * nib, 8192) + 256, (void **)&bc));
    unsigned int *flip = nullptr;  // deferred path flips: (pass, direction) per node
    WW_TRY(scratch(SLOT_MCF_FLIP, sizeof(unsigned int) * (size_t)N, (void **)&flip));
    hipLaunchKernelGGL(k_mcf_init_count, dim3(nib), dim3(INIT_THREADS), 0, st, g, res, bc, flip);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mcf_init_scan, dim3(1), dim3(1024), 0, st, nib, bc, ctl);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mcf_init_write, dim3(nib), dim3(INIT_THREADS), 0, st, g, res, bc, src, def);
    WW_LAUNCH_CHECK();
    auto sync_ctl = [&]() -> ww_status {
        WW_HIP(hipMemcpyAsync(h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        WW_TRY(wait_stream(st));
        if (h->error) return decode_error(h->error);
        return WW_OK;
    };
    WW_TRY(sync_ctl());
    S.supplies = (long long)h->nsrc + std::max<long long>(h->gex, 0);

    const char *trace_env = getenv("WW_MCF_TRACE");
    const bool trace = trace_env && (trace_env[0] == '1' || trace_env[0] == '2');
    const char *check_env = getenv("WW_MCF_CHECK");
    const bool check = check_env && check_env[0] == '1';
    // debug-check buffers, released on every way out of the solve (the
    // release waits for the device, so queued kernels never outlive them)
    struct CheckBufs {
        unsigned long long *lab = nullptr;
        CheckRec *rec = nullptr, *hrec = nullptr;
        unsigned int *bad = nullptr;
        ~CheckBufs() {
            if (lab || rec || bad) (void)hipDeviceSynchronize();
            if (lab) (void)hipFree(lab);
            if (rec) (void)hipFree(rec);
            if (bad) (void)hipFree(bad);
            if (hrec) (void)hipHostFree(hrec);
        }
    } cb;
    unsigned long long *&lab_copy = cb.lab;
    CheckRec *&crec = cb.rec, *&hcrec = cb.hrec;
    if (check) {
        WW_HIP(hipMalloc(&lab_copy, sizeof(unsigned long long) * N));
        WW_HIP(hipMalloc(&crec, sizeof(CheckRec)));
        WW_HIP(hipHostMalloc(&hcrec, sizeof(CheckRec)));
        WW_HIP(hipMalloc(&cb.bad, 4 * sizeof(unsigned int)));
    }
#ifndef WW_ROUNDS_PER_SYNC
#define WW_ROUNDS_PER_SYNC 12
#endif
    // relaxation rounds launched between two host checks of the list
    // lengths (a round whose list is empty returns at once)
    const int rounds_per_sync = WW_ROUNDS_PER_SYNC;
    const unsigned int h0 = (unsigned int)g_first_hops.load(), dstep0 = (unsigned int)g_first_dstep.load();
    const unsigned int full_passes = (unsigned int)g_full_passes.load();
    const bool first_deficit = g_first_deficit.load() != 0;
    const long long reverse_below = g_reverse_below.load();
    const unsigned long long hop_growth = (unsigned long long)g_hop_growth.load();
    bool reversed = false;
    const int rev_grid = (int)std::min<long long>(8192, std::max<long long>(1, ceil_div(std::max(nx + ny, N), 256 * 16)));
    auto flip_frame = [&]() -> ww_status {
        hipLaunchKernelGGL(k_reverse_frame, dim3(rev_grid), dim3(256), 0, st, g, ctl, nx, ny, N);
        WW_LAUNCH_CHECK();
        std::swap(g.cxp, g.cxn);
        std::swap(g.cyp, g.cyn);
        std::swap(src, def);
        std::swap(src2, def2);
        reversed = !reversed;
        // the host's copy of the counters follows the kernel's own exchange
        // (no round trip: the next read of the block checks the error flags)
        std::swap(h->nsrc, h->ndef);
        h->gex = -h->gex;
        h->gpot = -h->gpot;
        return WW_OK;
    };
    const bool trace_windows = trace_env && trace_env[0] == '2';
    // one wave of resident workgroups: more would only add workgroups that
    // find the round's list exhausted, which an empty round pays for too
    int dev = 0, ncu = 256, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sssp_round, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 4;
    (void)hipGetLastError();
    const int round_grid = (int)std::min<long long>(NT, (long long)ncu * per_cu);
    const int pot_grid = (int)std::min<unsigned int>((NT + POT_CHUNK - 1) / POT_CHUNK, 16384u);
    unsigned long long nbatch = 0;  // round batches so far (their parity picks the window-end slot)
    int wslot = 0;
    const unsigned int bound_cap = 0xffff0000u;
    unsigned int rr = 1, pass = 0;  // next round, current pass
    const int SB = 256;
    // Kernels over the node lists are grid-stride loops sized from the list
    // lengths the host last read: the lists only shrink between two reads
    // (a frame reversal swaps them and is read at once), and a grid that
    // matches the list spares late passes thousands of idle workgroups.
    auto lgrid = [&](long long items) {
        return (int)std::min<long long>(4096, std::max<long long>(1, ceil_div(items, SB)));
    };
    std::vector<unsigned long long> hv(64 * 16);
    auto host_visits = [&]() -> unsigned long long {
        if (hipMemcpy(hv.data(), ra.vpart, 8192, hipMemcpyDeviceToHost) != hipSuccess) return 0;
        unsigned long long s = 0;
        for (int k = 0; k < 64; ++k) s += hv[k * 16];
        return s;
    };
    // Once no frame reversal can follow, a pass is queued right behind the
    // previous one's augmentation: the host reads how the previous pass ended
    // (its counters kept by the pass set-up) together with the new pass's
    // first batch of rounds, one round trip instead of two.  When no units
    // were left, that queued pass had no sources: its rounds found empty
    // lists and it changed no flow or potential.
    bool prev_unread = false;  // the previous pass ended without a host check
    for (;;) {
        if (!prev_unread) {
            if (h->nsrc == 0 && h->gex <= 0) break;
            // few units left: search from the demands instead (in the
            // reversed frame), where the plateaus that earlier passes made
            // tight around the supplies do not lie
            if (!reversed && reverse_below > 0 &&
                (long long)h->nsrc + std::max<long long>(h->gex, 0) <= reverse_below)
                WW_TRY(flip_frame());
        }
        const auto tp0 = std::chrono::steady_clock::now();
        const long long r0 = S.rounds, w0 = S.windows;
        const unsigned long long v0 = trace ? host_visits() : 0, it0 = h->iters, vs0 = h->vt_sum,
                                 vst0 = h->vt_stage, vsw0 = h->vt_sweep;
        const unsigned int nsrc0 = h->nsrc;
        const long long gex0 = h->gex;
        ++pass;
        const long long ns_h = h->nsrc, nd_h = h->ndef;  // list lengths, upper bounds
        hipLaunchKernelGGL(k_pass_init, dim3(lgrid(std::max<long long>(ns_h, ra.nperim))), dim3(SB), 0, st,
                           g, ctl, src, ra.act,
                           ra.lists, NT, rr, ra.perim_tiles, ra.nperim);
        WW_LAUNCH_CHECK();
        // Windows in lexicographic (distance, hops) order: every label <= lb
        // is exact at the end of a window.  The first window admits only
        // zero-distance labels within h0 hops; later windows jump to the
        // smallest rejected candidate and grow the hop or distance limit.
        unsigned long long lb = mk_label(0, h0);
        unsigned int settled = 0;  // deficits settled by the last window
        unsigned int dstep = dstep0;
        bool finished = false;  // the previous pass left no units: this one is void
        for (;;) {  // windows
            ++S.windows;
            const long long rw0 = S.rounds;
            for (;;) {  // rounds
                WW_HIP(hipEventRecord(ev[0], st));
                for (int k = 0; k < rounds_per_sync; ++k) {
                    hipLaunchKernelGGL(k_sssp_round, dim3(round_grid), dim3(256), 0, st, g, ctl, ra,
                                       rr, pass, lb, trace ? 1 : 0);
                    WW_LAUNCH_CHECK();
                    ++rr;
                }
                WW_HIP(hipEventRecord(ev[1], st));
                // the window-end counts after every batch, so that the batch
                // that ends the window needs no further round trip (each run
                // writes the slot of its batch parity and clears the other)
                wslot = (int)(nbatch++ & 1);
                hipLaunchKernelGGL(k_window_end, dim3(lgrid(std::max<long long>(nd_h, NT))), dim3(SB), 0,
                                   st, g, ctl, def, lb,
                                   ra.pstamp, pass, ra.tile_rej, NT, wslot, rr);
                WW_LAUNCH_CHECK();
                S.rounds += rounds_per_sync;
                if (S.rounds > 50000000)
                    return fail(WW_E_DEVICE, "min-cost flow: relaxation rounds exceeded the limit");
                WW_TRY(sync_ctl());
                if (check) {
                    for (int q = 0; q < 3; ++q)
                        if (h->count[q][0] > NT)
                            return fail(WW_E_DEVICE, "min-cost flow check: list %d holds %u > %u tiles", q,
                                        h->count[q][0], NT);
                    unsigned int hb[4] = {0u, 0u, 0u, 0u};
                    WW_HIP(hipMemsetAsync(cb.bad, 0, sizeof(hb), st));
                    hipLaunchKernelGGL(k_check_lists, dim3(std::min<unsigned int>(1024u, (NT + 255) / 256)),
                                       dim3(256), 0, st, ctl, ra.act, ra.lists, NT, rr, cb.bad);
                    WW_LAUNCH_CHECK();
                    WW_HIP(hipMemcpyAsync(hb, cb.bad, sizeof(hb), hipMemcpyDeviceToHost, st));
                    WW_HIP(hipStreamSynchronize(st));
                    if (hb[0] || hb[1] || hb[2] != h->count[rr % 3][0])
                        return fail(WW_E_DEVICE,
                                    "min-cost flow check: round %u list: out of range %u, unstamped %u, "
                                    "stamped %u, count %u",
                                    rr, hb[0], hb[1], hb[2], h->count[rr % 3][0]);
                }
                float ms = 0.f;
                WW_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
                S.relax_ms += ms;
                if (prev_unread) {  // the previous pass's end
                    prev_unread = false;
                    ++S.passes;
                    S.augmentations += h->prev_naug;
                    S.path_arcs += (long long)h->prev_arcs;
                    if (h->prev_naug == 0)
                        return fail(WW_E_INFEASIBLE, "min-cost flow: a pass augmented no path");
                    if (h->nsrc == 0 && h->gex <= 0) {
                        finished = true;
                        break;
                    }
                }
                if (h->count[rr % 3][0] == 0) break;
            }
            if (finished) break;
            // settled deficits and the smallest parked candidate (the latter
            // is only read when the window does not end the pass)
            const int tg = (int)std::min<unsigned int>(1024u, (NT + SB - 1) / SB);
            settled = h->wsettled[wslot];
            if (trace_windows)
                fprintf(stderr, "[ww-mcf]   window %u/%u rounds %lld settled %u\n",
                        (unsigned)(lb >> 32), (unsigned)((lb >> 3) & 0x1fffffffu), S.rounds - rw0,
                        settled);
            // stop rule: all units in a full pass, else the first deficit or
            // half of the units
            const long long units = (long long)h->nsrc + std::max<long long>(h->gex, 0);
            const long long need = pass <= full_passes ? std::max<long long>(1, units)
                                   : first_deficit    ? 1
                                                      : std::max<long long>(1, (units + 1) / 2);
            if ((long long)settled >= need) break;
            const unsigned long long mr = h->wminrej[wslot];
            if (mr == LINF) break;  // every reachable node is settled
            const unsigned int d = (unsigned int)(lb >> 32), hcur = (unsigned int)((lb >> 3) & 0x1fffffffu);
            if ((unsigned int)(mr >> 32) == d && d == 0) {
                // the zero-distance plateau: widen the hop limit
                unsigned long long hn = std::max<unsigned long long>((mr >> 3) & 0x1fffffffu, hop_growth * hcur);
                lb = mk_label(0, (unsigned int)std::min<unsigned long long>(hn, HMAX));
            } else {
                unsigned long long dn = std::max<unsigned long long>(mr >> 32, (unsigned long long)d + dstep);
                if (dn > bound_cap)
                    return fail(WW_E_OVERFLOW, "min-cost flow: shortest-path distance above 2^32");
                dstep = dstep > (1u << 30) ? dstep : dstep * 2;
                lb = mk_label((unsigned int)dn, HMAX);
            }
            hipLaunchKernelGGL(k_requeue_pending, dim3(tg), dim3(SB), 0, st, ctl, ra.pstamp, pass,
                               ra.tile_rej, lb, ra.act, ra.lists, NT, rr);
            WW_LAUNCH_CHECK();
        }
        if (finished) {  // not a pass: leave the counts as if it never ran
            --S.windows;
            S.rounds -= rounds_per_sync;
            break;
        }
        if (settled == 0)
            return fail(WW_E_INFEASIBLE, "min-cost flow: %u supplies reach no demand", h->nsrc);
        // The host's last read followed the pass's last round, so it holds
        // the pass's final ground label and excess: the ground's predecessor
        // is only needed when the ground is a settled deficit, and subtrees
        // hang off the ground only while it is a source.
        const int pg = (int)std::min<long long>(1024, ceil_div(nperim_arcs, SB));
        if (h->glab <= lb && h->gex <= 0) {
            hipLaunchKernelGGL(k_ground_pred, dim3(pg), dim3(SB), 0, st, g, ctl, lb);
            WW_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_roots, dim3(lgrid(nd_h + 1)), dim3(SB), 0, st, g, ctl, def, lb, gsub_list);
        WW_LAUNCH_CHECK();
        if (h->gex > 0) {
            hipLaunchKernelGGL(k_gsub_select, dim3(pg), dim3(SB), 0, st, g, ctl, gsub_list, drop);
            WW_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_augment, dim3(lgrid(ns_h + nperim_arcs)), dim3(SB), 0, st, g, ctl, src,
                           gsub_list, drop, flip, pass);
        WW_LAUNCH_CHECK();
        if (check)
            WW_HIP(hipMemcpyAsync(lab_copy, g.lab, sizeof(unsigned long long) * N,
                                  hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_potentials, dim3(pot_grid), dim3(SB), 0, st, g, ctl, ra.tstamp, pass,
                           NT, lb, flip);
        WW_LAUNCH_CHECK();
        if (check) {
            WW_HIP(hipMemsetAsync(crec, 0, sizeof(CheckRec), st));
            hipLaunchKernelGGL(k_check_rc, dim3(IB), dim3(256), 0, st, g, ctl, lab_copy, crec);
            WW_LAUNCH_CHECK();
            WW_HIP(hipMemcpyAsync(hcrec, crec, sizeof(CheckRec), hipMemcpyDeviceToHost, st));
            WW_HIP(hipStreamSynchronize(st));
            if (hcrec->found) {
                auto pl = [](unsigned long long l) {
                    return l == LINF ? std::string("inf") :
                        std::to_string(l >> 32) + "/" + std::to_string((l >> 3) & 0x1fffffff) + "/" + std::to_string(l & 7);
                };
                fprintf(stderr,
                        "[ww-mcf-check] pass %lld lb %u/%u: arc kind %d u %lld v %lld rc %lld pot %lld %lld "
                        "labels %s %s flow %d c+ %d c- %d gex %lld\n",
                        (long long)S.passes + 1, (unsigned)(lb >> 32), (unsigned)((lb >> 3) & 0x1fffffff),
                        hcrec->kind, hcrec->u, hcrec->v, hcrec->rc, hcrec->pu, hcrec->pv,
                        pl(hcrec->lu).c_str(), pl(hcrec->lv).c_str(), hcrec->f, hcrec->cp, hcrec->cn,
                        (long long)h->gex);
                return fail(WW_E_DEVICE, "min-cost flow check failed (details on stderr)");
            }
        }
        hipLaunchKernelGGL(k_compact, dim3(lgrid(ns_h + nd_h)), dim3(SB), 0, st, g, ctl, src, def, src2,
                           def2);
        WW_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_swap_lists, dim3(1), dim3(1), 0, st, ctl);
        WW_LAUNCH_CHECK();
        std::swap(src, src2);
        std::swap(def, def2);
        if ((reversed || reverse_below <= 0) && !trace && !check) {
            prev_unread = true;
            continue;
        }
        WW_TRY(sync_ctl());
        ++S.passes;
        S.augmentations += h->naug;
        S.path_arcs += (long long)h->arcs;
        if (trace) {
            const unsigned long long v1 = host_visits();
            fprintf(stderr,
                    "[ww-mcf] pass %lld src %u gex %lld bound %u/%u windows %lld rounds %lld "
                    "tile_visits %llu iters %llu visit_us %.2f stage_us %.2f swept_us %.2f maxvisit_us %.1f aug %u arcs %llu ms %.3f\n",
                    (long long)S.passes, nsrc0, gex0, (unsigned)(lb >> 32),
                    (unsigned)((lb >> 3) & 0x1fffffffu), S.windows - w0, S.rounds - r0,
                    v1 - v0, h->iters - it0,
                    (h->vt_sum - vs0) * 0.01 / std::max<double>(1.0, (double)(v1 - v0)),
                    (h->vt_stage - vst0) * 0.01 / std::max<double>(1.0, (double)(v1 - v0)),
                    (h->vt_sweep - vsw0) * 0.01 / std::max<double>(1.0, (double)(v1 - v0)),
                    h->vt_max * 0.01, h->naug, (unsigned long long)h->arcs,
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp0).count());
        }
        if (h->naug == 0)
            return fail(WW_E_INFEASIBLE, "min-cost flow: a pass augmented no path");
    }
    if (reversed) WW_TRY(flip_frame());
    const int cg = (int)std::min<long long>(8192, std::max<long long>(1, ceil_div(nx + ny, 256 * 8)));
    long long *part = (long long *)bc;
    hipLaunchKernelGGL(k_total_cost, dim3(cg), dim3(256), 0, st, dkx, dky, cxp, cxn, cyp, cyn, nx,
                       ny, part);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_total_finish, dim3(1), dim3(256), 0, st, cg, part, ctl);
    WW_LAUNCH_CHECK();
    if (pot_out) {
        hipLaunchKernelGGL(k_export_pot, dim3(IB), dim3(256), 0, st, g.pot, ctl, N, pot_out);
        WW_LAUNCH_CHECK();
    }
    WW_TRY(sync_ctl());
    *total = h->total_cost;
    S.tile_visits = (long long)host_visits();
    S.max_potential = std::max<long long>(h->max_pot, h->gpot);
    S.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    last_mcf_stats() = S;
    if (stats) *stats = S;
    return WW_OK;
}

}  // namespace ww

extern "C" {

void ww_default_mcf_params(ww_mcf_params *p) {
    if (!p) return;
    p->first_hop_window = 64;
    p->first_distance_step = 256;
    p->full_passes = 0;
    p->first_deficit_after = 0;
    p->reverse_below = 0;
    p->hop_growth = 2;
}

ww_status ww_set_mcf_params(const ww_mcf_params *p) {
    ww::clear_error();
    if (!p || p->first_hop_window < 1 || p->first_hop_window > (int32_t)ww::HMAX - 1 ||
        p->first_distance_step < 1 || p->first_distance_step > (1 << 30))
        return ww::fail(WW_E_INVALID_ARG, "window schedule out of range");
    if (p->full_passes < 0 || p->full_passes > (1 << 20) ||
        (p->first_deficit_after != 0 && p->first_deficit_after != 1) || p->reverse_below < 0 ||
        p->hop_growth < 2 || p->hop_growth > (1 << 20))
        return ww::fail(WW_E_INVALID_ARG, "pass schedule out of range");
    ww::g_first_hops.store(p->first_hop_window);
    ww::g_first_dstep.store(p->first_distance_step);
    ww::g_full_passes.store(p->full_passes);
    ww::g_first_deficit.store(p->first_deficit_after);
    ww::g_reverse_below.store(p->reverse_below);
    ww::g_hop_growth.store(p->hop_growth);
    return WW_OK;
}

void ww_get_mcf_params(ww_mcf_params *p) {
    if (!p) return;
    p->first_hop_window = ww::g_first_hops.load();
    p->first_distance_step = ww::g_first_dstep.load();
    p->full_passes = ww::g_full_passes.load();
    p->first_deficit_after = ww::g_first_deficit.load();
    p->reverse_below = ww::g_reverse_below.load();
    p->hop_growth = ww::g_hop_growth.load();
}

}  // extern "C"
