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
// One solve may hold several images ("jobs") at once: their loop graphs,
// each with its own ground node, form one disjoint graph, and the flow
// problem on it is the sum of the jobs' problems.  Successive shortest paths
// on that union are exact for every job, so the jobs share every pass, every
// window and every relaxation round (one launch relaxes the listed tiles of
// all jobs).  Node and tile indices are global: job k owns nodes
// [noff_k, noff_k + R_k C_k) and tiles [toff_k, toff_k + TR_k TC_k); a tile
// list entry is (job << 24) | tile-within-job.
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
//     each root keeps its nearest deficit (64-bit atomicMin on dist|node),
//     and every node on the way keeps the smallest such key through it.
//  3. One unit is augmented along each root's chosen path.  Different trees
//     are vertex-disjoint, so all paths are applied in parallel: a path
//     node's arc flips when its kept key names a chosen deficit (the key
//     through a node of the chosen path is the root's own).  Trees that
//     hang off a ground as a supply are split at the ground's arcs and at
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
constexpr int DIR_NONE = 0, DIR_UP = 1, DIR_DOWN = 2, DIR_LEFT = 3;
constexpr int POT_LIMIT = 1 << 30;

enum : int { ERR_NEG_RC = 1, ERR_POT = 2, ERR_WALK = 4, ERR_ITERS = 8 };

struct Ctl {
    unsigned int count[3][32]; // list lengths (one 128-byte line each)
    unsigned int nsrc, ndef;   // node lists
    unsigned int nsrc2, ndef2; // compaction targets
    unsigned int wsettled[2];  // deficits reached in the window (by window parity)
    unsigned int naug;         // augmentations in this pass
    unsigned long long arcs;   // arcs flipped in this pass
    int error;
    int max_pot;
    long long sum_res;
    unsigned long long wminrej[2];  // smallest candidate beyond the window (by parity)
    unsigned long long iters;   // in-tile relaxation iterations, all visits
    unsigned long long vt_sum;  // visit durations (wall-clock ticks), all visits
    unsigned long long vt_max;  // longest visit
    unsigned long long vt_stage;  // staging part of the visits
    unsigned long long vt_sweep;  // staging and sweeps of the visits
    unsigned int prev_naug;       // naug and arcs of the previous pass, kept by
    unsigned long long prev_arcs;  // the pass set-up when it clears them
    unsigned long long settled;   // work counters (counting solves only): nodes
    unsigned long long scanned;   // settled and their residual out-arcs
    unsigned int nlong;           // long walks left to the wave walk (this pass)
    unsigned long long t_batch;   // device clock at the start of the current batch of rounds
    unsigned long long relax_ticks;  // device clock ticks spent in batches of rounds
    unsigned int compact_done;    // workgroups of the list compaction that have finished
};
constexpr size_t CTL_BYTES = (sizeof(Ctl) + 63) / 64 * 64;

// State of one job's ground node.
struct GState {
    unsigned long long glab;   // label
    long long gex;             // excess
    long long gpot;            // potential
    unsigned int gpred;        // predecessor (perimeter arc index)
    unsigned int gsub_count;   // ground-rooted subtrees with a deficit
    long long total_cost;      // the job's flow cost at the end of the solve
    unsigned int gchosen;      // pass in which a path into the ground was chosen
    unsigned int gpad;
    long long pad[2];
};
static_assert(sizeof(GState) == 64, "one 64-byte record per ground");

// One job's loop grid inside the solve.
struct Job {
    int R, C, n;               // loop rows, loop cols, image cols (= C + 1)
    int TR, TC;                // tile grid
    unsigned int toff;         // first global tile
    unsigned int poff;         // first entry of its perimeter tiles
    unsigned int nptiles;      // perimeter tiles
    unsigned int aoff;         // first slot of its ground-subtree list (perimeter arcs before it)
    long long noff;            // first global node
    const int16_t *cxp, *cxn, *cyp, *cyn;
    int8_t *fx, *fy;
};

// Node state of all jobs, and the jobs.  A single-job solve reads its job
// from the kernel argument j0; a multi-job solve reads jobs[k].
struct Graph {
    unsigned long long *lab;
    int *pot;
    int8_t *ex;
    unsigned long long *best;
    GState *gs;
    const Job *jobs;
    int njobs;
    long long N;               // nodes of all jobs
    Job j0;
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

template <bool MULTI>
__device__ __forceinline__ Job job_at(const Graph &g, int k) {
    return MULTI ? g.jobs[k] : g.j0;
}

// The job holding global node v, tile t, or ground-subtree slot q: the last
// job whose offset is at most the index (binary search; one job: 0).
__device__ __forceinline__ int job_of_node(const Graph &g, long long v) {
    int lo = 0, hi = g.njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.jobs[mid].noff <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int job_of_tile(const Graph &g, unsigned int t) {
    int lo = 0, hi = g.njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.jobs[mid].toff <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int job_of_slot(const Graph &g, unsigned int q) {
    int lo = 0, hi = g.njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.jobs[mid].aoff <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Append a tile to the list of round r unless it is already there
// (act[gt] == r).  gt: global tile; entry: its list entry.
// Lists: lists[(r % 3) * list_stride(NT) ...], lengths ctl->count[r % 3].
// A tile enters a list only when its round stamp changes, so a list holds
// at most NT entries.
__host__ __device__ __forceinline__ size_t list_stride(unsigned int NT) { return (size_t)NT; }

__device__ __forceinline__ void activate(unsigned int *act, unsigned int *lists, unsigned int NT,
                                         Ctl *ctl, unsigned int gt, unsigned int entry,
                                         unsigned int r) {
    if (atomicExch(&act[gt], r) != r) {
        const unsigned int pos = atomicAdd(&ctl->count[r % 3][0], 1u);
        lists[(size_t)(r % 3) * list_stride(NT) + pos] = entry;
    }
}

constexpr int TILE_NODES = 1024;  // loop nodes per tile (256 threads x 4)

__device__ __forceinline__ unsigned int entry_of(int job, unsigned int lt) {
    return ((unsigned int)job << 24) | lt;
}

// perimeter arc a of job J -> (node row, node col, edge kind, edge index,
// delta of the move node -> ground)
__device__ __forceinline__ void ground_arc(const Job &J, unsigned int a, int &i, int &j, int &kind,
                                           long long &e, int &delta) {
    const int C = J.C, R = J.R;
    if (a < (unsigned)C) {  // top: up across hx(0, j)
        i = 0; j = a; kind = 0; e = j; delta = -1;
    } else if (a < 2u * C) {  // bottom: down across hx(R, j)
        i = R - 1; j = a - C; kind = 0; e = (long long)R * C + j; delta = +1;
    } else if (a < 2u * C + R) {  // left: left across vy(i, 0)
        i = a - 2 * C; j = 0; kind = 1; e = (long long)i * J.n; delta = +1;
    } else {  // right: right across vy(i, C)
        i = a - 2 * C - R; j = C - 1; kind = 1; e = (long long)i * J.n + C; delta = -1;
    }
}

}  // namespace

// ------------------------------------------------------------ set-up ------

// Set-up in three launches with no contended atomics: every block of
// INIT_CHUNK nodes initialises its state and counts its supplies / demands;
// one block scans the counts; every block then writes its supplies and
// demands in node order.  The residues of all jobs are one array in global
// node order.
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

// The residues of nodes v0 .. v0 + INIT_PER - 1 (zero beyond N): one
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
// potentials zero, and (keys != 0) the labels and path keys infinite, all
// in 16-byte stores.  A deficit's flip word needs no clearing: each pass
// writes it (k_roots) before anything reads it.
__global__ __launch_bounds__(INIT_THREADS) void k_mcf_init_count(Graph g, const int8_t *__restrict__ res,
                                                                int *__restrict__ bc, int keys) {
    __shared__ int red[INIT_THREADS / 64];
    const long long N = g.N;
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
    }
    if (whole) {
        *reinterpret_cast<uint4 *>(g.ex + v0) = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
        for (int q = 0; q < INIT_PER; ++q)
            if (v0 + q < N) g.ex[v0 + q] = r[q];
    }
    if (c0 + INIT_CHUNK <= N) {
        uint4 *pot = reinterpret_cast<uint4 *>(g.pot + c0);
        uint4 *lab = reinterpret_cast<uint4 *>(g.lab + c0);
        uint4 *best = reinterpret_cast<uint4 *>(g.best + c0);
        const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
        const uint4 inf = make_uint4((unsigned int)LINF, (unsigned int)(LINF >> 32), (unsigned int)LINF,
                                     (unsigned int)(LINF >> 32));
#pragma unroll
        for (int k = 0; k < INIT_CHUNK / 4 / INIT_THREADS; ++k) pot[k * INIT_THREADS + threadIdx.x] = zero;
        if (keys) {
#pragma unroll
            for (int k = 0; k < INIT_CHUNK / 2 / INIT_THREADS; ++k) {
                lab[k * INIT_THREADS + threadIdx.x] = inf;
                best[k * INIT_THREADS + threadIdx.x] = inf;
            }
        }
    } else {
        for (long long v = c0 + threadIdx.x; v < N; v += INIT_THREADS) {
            g.pot[v] = 0;
            if (keys) {
                g.lab[v] = LINF;
                g.best[v] = LINF;
            }
        }
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

// Ground state of every job (blockIdx.y = job): best entries of its
// perimeter nodes; with several jobs also its charge, minus the sum of its
// residues (a single job's comes from the set-up scan).
__global__ __launch_bounds__(256) void k_init_ground(Graph g, const int8_t *__restrict__ res) {
    __shared__ int red[4];
    const int k = blockIdx.y;
    const Job J = g.njobs > 1 ? g.jobs[k] : g.j0;
    for (unsigned int a = blockIdx.x * blockDim.x + threadIdx.x; a < 2u * J.C + 2u * J.R;
         a += gridDim.x * blockDim.x) {
        int i, j, kind, delta;
        long long e;
        ground_arc(J, a, i, j, kind, e, delta);
        g.best[J.noff + (long long)i * J.C + j] = LINF;
    }
    if (g.njobs > 1) {
        const long long Nk = (long long)J.R * J.C;
        int s = 0;
        for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < Nk;
             v += (long long)gridDim.x * blockDim.x)
            s += res[J.noff + v];
        s = block_sum_int(s, red);
        if (threadIdx.x == 0 && s != 0)
            atomicAdd((unsigned long long *)&g.gs[k].gex, (unsigned long long)(-(long long)s));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        g.gs[k].glab = LINF;
        g.gs[k].gpred = 0xffffffffu;
    }
}

// one block: exclusive scans of the per-block counts, totals into ctl; each
// thread sums a run of consecutive blocks, one block scan joins the runs
__global__ __launch_bounds__(1024) void k_mcf_init_scan(int nb, int *__restrict__ bc, Ctl *ctl,
                                                       GState *gs, int njobs) {
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
        if (njobs == 1) gs[0].gex = -(long long)ts;
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
    const long long N = g.N;
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
// A ground is a source while it holds surplus; that is read here rather
// than passed in, so that a pass can be queued before the host has seen how
// the previous one ended.
template <bool MULTI, int TW>
__global__ void k_pass_init(Graph g, Ctl *ctl, const unsigned int *src, unsigned int *act,
                            unsigned int *lists, unsigned int NT, unsigned int rr,
                            const unsigned int *perim_tiles, int nperim) {
    const unsigned int ns = ctl->nsrc;
    for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k < ns; k += gridDim.x * blockDim.x) {
        const unsigned int v = src[k];
        g.lab[v] = 0ull;
        const int job = MULTI ? job_of_node(g, v) : 0;
        const Job J = job_at<MULTI>(g, job);
        const unsigned int lv = (unsigned int)(v - J.noff);
        const int i = lv / J.C, j = lv % J.C;
        constexpr int TH = TILE_NODES / TW;
        const int ti = i / TH, tj = j / TW, li = i % TH, lj = j % TW;
        const unsigned int lt = ti * J.TC + tj;
        activate(act, lists, NT, ctl, J.toff + lt, entry_of(job, lt), rr);
        // a supply on a tile border also feeds the tile across that border,
        // whose relaxation must run although this label never "changes"
        if (li == 0 && ti > 0) activate(act, lists, NT, ctl, J.toff + lt - J.TC, entry_of(job, lt - J.TC), rr);
        if (li == TH - 1 && ti < J.TR - 1)
            activate(act, lists, NT, ctl, J.toff + lt + J.TC, entry_of(job, lt + J.TC), rr);
        if (lj == 0 && tj > 0) activate(act, lists, NT, ctl, J.toff + lt - 1, entry_of(job, lt - 1), rr);
        if (lj == TW - 1 && tj < J.TC - 1)
            activate(act, lists, NT, ctl, J.toff + lt + 1, entry_of(job, lt + 1), rr);
    }
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nperim; k += gridDim.x * blockDim.x) {
        const unsigned int e = perim_tiles[k];
        const int job = (int)(e >> 24);
        if (g.gs[job].gex > 0) {
            const unsigned int toff = MULTI ? g.jobs[job].toff : g.j0.toff;
            activate(act, lists, NT, ctl, toff + (e & 0xffffffu), e, rr);
        }
    }
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < g.njobs; k += gridDim.x * blockDim.x) {
        GState &G = g.gs[k];
        G.glab = G.gex > 0 ? 0ull : LINF;
        G.gpred = 0xffffffffu;
        G.gsub_count = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // per-pass counters back to zero (none of them is read by this kernel)
        ctl->prev_naug = ctl->naug;
        ctl->prev_arcs = ctl->arcs;
        ctl->naug = 0;
        ctl->arcs = 0;
        ctl->nsrc2 = 0;
        ctl->ndef2 = 0;
        ctl->nlong = 0;
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
    const unsigned int *perim_tiles;  // list entries of every job's perimeter tiles
    int nperim;
    unsigned int NT;
};

// Loop tiles of TILE_NODES nodes, TW columns by TILE_NODES / TW rows (TW =
// 16, 32 or 64: a solve parameter), 256 threads, 4 nodes per thread.

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

// Element idx of an array whose bytes all lie below 2^32 from base (a job's
// node and arc arrays: fewer than 2^29 loops): a 32-bit byte offset from a
// workgroup-uniform base, which the loads and stores take as is.
template <typename T>
__device__ __forceinline__ T &at32(T *base, unsigned int idx) {
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (idx * (unsigned int)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T &at32(const T *base, unsigned int idx) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (idx * (unsigned int)sizeof(T)));
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
#define WW_VISIT_ITERS 12
#endif
constexpr int VISIT_ITERS = WW_VISIT_ITERS;  // sweeps per tile visit at most

template <bool MULTI, int TW>
__global__ __launch_bounds__(256) void k_sssp_round(Graph g, Ctl *ctl, RoundArgs ra,
                                                   unsigned int round, unsigned int pass_stamp,
                                                   unsigned long long lb, int stats, int batch_start) {
    constexpr int TH = TILE_NODES / TW;  // tile rows
    __shared__ unsigned long long L[TH + 2][TW + 3];
    __shared__ int P[TH + 2][TW + 2];
    __shared__ int4 RC4[TH][TW];  // reduced costs of the in-arcs: from above, below, left, right
    __shared__ int GA[TH][TW];    // cheapest move to the ground of a perimeter node (RC_INF: none)
    __shared__ __align__(16) int wchg[3][4];  // per-iteration "a label changed" flag of each wave's band
    __shared__ int flags[4];  // changed border: top, bottom, left, right
    __shared__ int sh_any;
    __shared__ unsigned long long sh_gcand, sh_rej;

    // the first round of a batch stamps its start on the device clock (the
    // window-end count that follows the batch adds up the span)
    if (batch_start && blockIdx.x == 0 && threadIdx.x == 0) ctl->t_batch = (unsigned long long)wall_clock64();
    const unsigned int NT = ra.NT;
    const unsigned int *list = ra.lists + (size_t)(round % 3) * list_stride(NT);
    // the first entry is read together with the length (the slot lies inside
    // the list's storage, whatever the length): one memory round trip less
    const unsigned int first = blockIdx.x < list_stride(NT) ? list[blockIdx.x] : 0u;
    const unsigned int cnt = ctl->count[round % 3][0];
    // list (round + 2) % 3 was consumed by the previous round
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->count[(round + 2) % 3][0] = 0;
    // one job: its ground's label and potential once per launch
    const unsigned long long glab0 = MULTI ? 0ull : g.gs[0].glab;
    const int gpot0 = MULTI ? 0 : (int)g.gs[0].gpot;
    unsigned int my_visits = 0;

    for (unsigned int idx = blockIdx.x; idx < cnt; idx += gridDim.x) {
        const unsigned int entry = idx == blockIdx.x ? first : list[idx];
        const int job = MULTI ? (int)(entry >> 24) : 0;
        const unsigned int lt = entry & 0xffffffu;
        const Job J = job_at<MULTI>(g, job);
        const unsigned int tile = J.toff + lt;  // global tile
        const unsigned long long glab = MULTI ? g.gs[job].glab : glab0;
        const int gpot = MULTI ? (int)g.gs[job].gpot : gpot0;
        const int R = J.R, C = J.C;
        const long long noff = J.noff;
        unsigned long long *const labJ = g.lab + noff;  // the job's labels and potentials
        const int *const potJ = g.pot + noff;
        ++my_visits;
        const unsigned long long t_start = stats ? wall_clock64() : 0ull;
        const int ti = lt / J.TC, tj = lt % J.TC;
        const int i0 = ti * TH, j0 = tj * TW;
        const int rows = min(TH, R - i0), cols = min(TW, C - j0);
        if (threadIdx.x < 4) flags[threadIdx.x] = 0;
        if (threadIdx.x == 0) {
            sh_rej = LINF;
            sh_gcand = LINF;
        }
        // stage labels and potentials with a one-node halo; outside = ground.
        // Every load of a thread (labels, potentials, arc costs and flows)
        // is issued unconditionally, from an address clamped into the tile,
        // before any of them is used: one memory latency for all of them.
        // Values of positions outside the tile are replaced afterwards.
        constexpr int NSTAGE = ((TH + 2) * (TW + 2) + 255) / 256;
        constexpr int NRC = TILE_NODES / 256;
        int cst[NRC][4];
        {
            unsigned long long lv[NSTAGE];
            int pv[NSTAGE];
            bool inside[NSTAGE], halo[NSTAGE];
#pragma unroll
            for (int s = 0; s < NSTAGE; ++s) {
                const int t = threadIdx.x + 256 * s;
                const int r = t / (TW + 2), c = t % (TW + 2);
                const int i = i0 - 1 + r, j = j0 - 1 + c;
                halo[s] = t < (TH + 2) * (TW + 2) && r <= rows + 1 && c <= cols + 1;
                inside[s] = halo[s] && i >= 0 && i < R && j >= 0 && j < C;
                const unsigned int v = (unsigned int)((inside[s] ? i : i0) * C + (inside[s] ? j : j0));
                lv[s] = at32(labJ, v);
                pv[s] = at32(potJ, v);
            }
            // arc flows and both costs of the four in-arcs of every node
            int8_t af[NRC][4];
            int16_t ap[NRC][4], an[NRC][4];
            bool own[NRC];
#pragma unroll
            for (int s = 0; s < NRC; ++s) {
                const int t = threadIdx.x + 256 * s;
                const int li = t / TW, lj = t % TW;
                own[s] = li < rows && lj < cols;
                const int i = i0 + (own[s] ? li : 0), j = j0 + (own[s] ? lj : 0);
                const unsigned int ex0 = (unsigned int)(i * C + j);      // hx(i,j): from above, +1
                const unsigned int ex1 = ex0 + (unsigned int)C;           // hx(i+1,j): from below, -1
                const unsigned int ey0 = (unsigned int)(i * J.n + j);    // vy(i,j): from the left, -1
                const unsigned int ey1 = ey0 + 1u;                        // vy(i,j+1): from the right, +1
                af[s][0] = at32(J.fx, ex0); ap[s][0] = at32(J.cxp, ex0); an[s][0] = at32(J.cxn, ex0);
                af[s][1] = at32(J.fx, ex1); ap[s][1] = at32(J.cxp, ex1); an[s][1] = at32(J.cxn, ex1);
                af[s][2] = at32(J.fy, ey0); ap[s][2] = at32(J.cyp, ey0); an[s][2] = at32(J.cyn, ey0);
                af[s][3] = at32(J.fy, ey1); ap[s][3] = at32(J.cyp, ey1); an[s][3] = at32(J.cyn, ey1);
            }
            // (the empty asm statements use every loaded value here, so that
            // no load is moved into the conditional code below and waited
            // for on its own)
#pragma unroll
            for (int s = 0; s < NRC; ++s)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    int a = af[s][k], b = ap[s][k], c = an[s][k];
                    asm volatile("" : "+v"(a), "+v"(b), "+v"(c));
                    af[s][k] = (int8_t)a;
                    ap[s][k] = (int16_t)b;
                    an[s][k] = (int16_t)c;
                }
            // a node on the image's perimeter reaches the ground across the
            // same edge its in-arc from outside crosses, in the other
            // direction: the cheapest such move, from the values just loaded
#pragma unroll
            for (int s = 0; s < NRC; ++s) {
                const int t = threadIdx.x + 256 * s;
                const int li = t / TW, lj = t % TW;
                const int i = i0 + li, j = j0 + lj;
                int ga = RC_INF;
                if (own[s]) {
                    if (i == 0) ga = min(ga, move_cost(af[s][0], -1, ap[s][0], an[s][0]));
                    if (i == R - 1) ga = min(ga, move_cost(af[s][1], +1, ap[s][1], an[s][1]));
                    if (j == 0) ga = min(ga, move_cost(af[s][2], +1, ap[s][2], an[s][2]));
                    if (j == C - 1) ga = min(ga, move_cost(af[s][3], -1, ap[s][3], an[s][3]));
                }
                GA[li][lj] = ga;
            }
#pragma unroll
            for (int s = 0; s < NRC; ++s) {
                cst[s][0] = own[s] ? move_cost(af[s][0], +1, ap[s][0], an[s][0]) : RC_INF;
                cst[s][1] = own[s] ? move_cost(af[s][1], -1, ap[s][1], an[s][1]) : RC_INF;
                cst[s][2] = own[s] ? move_cost(af[s][2], -1, ap[s][2], an[s][2]) : RC_INF;
                cst[s][3] = own[s] ? move_cost(af[s][3], +1, ap[s][3], an[s][3]) : RC_INF;
            }
#pragma unroll
            for (int s = 0; s < NSTAGE; ++s) {
                const int t = threadIdx.x + 256 * s;
                if (t < (TH + 2) * (TW + 2)) {
                    L[t / (TW + 2)][t % (TW + 2)] = inside[s] ? lv[s] : (halo[s] ? glab : LINF);
                    P[t / (TW + 2)][t % (TW + 2)] = inside[s] ? pv[s] : (halo[s] ? gpot : 0);
                }
            }
        }
        __syncthreads();
        // reduced costs of the four in-arcs of every node (an arc exists
        // only at an owned node, cst != RC_INF; the potentials are read for
        // every position, all inside the staged array, so that the reads go
        // out in one batch)
        bool neg = false;
#pragma unroll
        for (int s = 0; s < NRC; ++s) {
            const int t = threadIdx.x + 256 * s;
            const int li = t / TW, lj = t % TW;
            const int pv = P[li + 1][lj + 1];
            const int pu = P[li][lj + 1], pd = P[li + 2][lj + 1], pl = P[li + 1][lj], pr = P[li + 1][lj + 2];
            int ru = cst[s][0] != RC_INF ? cst[s][0] - pu + pv : RC_INF;
            int rd = cst[s][1] != RC_INF ? cst[s][1] - pd + pv : RC_INF;
            int rl = cst[s][2] != RC_INF ? cst[s][2] - pl + pv : RC_INF;
            int rr = cst[s][3] != RC_INF ? cst[s][3] - pr + pv : RC_INF;
            neg |= (ru < 0) | (rd < 0) | (rl < 0) | (rr < 0);
            ru = max(ru, 0); rd = max(rd, 0); rl = max(rl, 0); rr = max(rr, 0);
            RC4[li][lj] = make_int4(ru == RC_INF ? (int)RC_NONE : ru, rd == RC_INF ? (int)RC_NONE : rd,
                                    rl == RC_INF ? (int)RC_NONE : rl, rr == RC_INF ? (int)RC_NONE : rr);
        }
        if (neg) atomicOr(&ctl->error, ERR_NEG_RC);
        __syncthreads();
        const unsigned long long t_staged = stats ? wall_clock64() : 0ull;
        // Each thread owns a column segment of 4 nodes (column lj, rows
        // 4q..4q+3): their labels and in-arc reduced costs stay in registers,
        // and every iteration sweeps down the segment and back up.  The
        // labels of the side neighbours (lanes lj - 1 and lj + 1 of the same
        // wave) and of the segments above and below are read from LDS in
        // batches, each timed so that it sees what the neighbouring lanes of
        // the same wave wrote in the steps before it: the side labels of all
        // four rows and the label above at the start of the down pass, the
        // label below after the first step (the segment below has just
        // written its top node), the side labels of rows 2..0 and the label
        // above after the down pass.  Labels only decrease, so any value read
        // is a valid label.  Every step stores its node's label, changed or
        // not (the owner is the only writer of a cell).  A node outside the
        // image has no in-arc (all four reduced costs RC_NONE), so no
        // candidate ever passes for it.  Wave w owns the TH / 4 rows of band
        // w (its segments are consecutive); it skips an iteration when no
        // label changed in its band or the two adjacent bands during the
        // previous one.
        const int lj = threadIdx.x % TW, q = threadIdx.x / TW, wv = threadIdx.x >> 6;
        const int r0 = q * 4;
        const int near_bands = ((7 << wv) >> 1) & 15;  // bits of bands wv - 1, wv, wv + 1
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
        int rd = 2, wr = 0, cl = 1;  // flag slots: read, written, cleared in this sweep
        for (int it = 0; it < VISIT_ITERS; ++it) {
            const int4 f = *reinterpret_cast<const int4 *>(&wchg[rd][0]);
            const int fm = __builtin_amdgcn_readfirstlane((f.x ? 1 : 0) | (f.y ? 2 : 0) | (f.z ? 4 : 0) |
                                                          (f.w ? 8 : 0));
            if (fm & near_bands) {
                bool changed = false;
// the smallest of the four candidates is taken when it is inside the window
// and below the node's label: one comparison with min(label, lb + 1)
#define WW_RELAX_NODE(k, PREV, NEXT, LEFT, RIGHT)                                          \
    {                                                                                      \
        const unsigned long long c = umin64(                                               \
            umin64(cand_of(PREV, (unsigned)rc[k].x, 1u), cand_of(NEXT, (unsigned)rc[k].y, 2u)), \
            umin64(cand_of(LEFT, (unsigned)rc[k].z, 3u), cand_of(RIGHT, (unsigned)rc[k].w, 4u))); \
        const bool upd = c < umin64(y[k], lb1);                                            \
        y[k] = upd ? c : y[k];                                                             \
        changed |= upd;                                                                    \
        L[r0 + k + 1][lj + 1] = y[k];                                                      \
    }
                unsigned long long sl[4], sr[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    sl[k] = L[r0 + k + 1][lj];
                    sr[k] = L[r0 + k + 1][lj + 2];
                }
                unsigned long long above = L[r0][lj + 1];
                WW_RELAX_NODE(0, above, y[1], sl[0], sr[0])
                // (the empty asm statements keep the LDS accesses in program
                // order: each store stays, and each read follows the stores
                // before it)
                asm volatile("" ::: "memory");
                const unsigned long long below = L[r0 + 5][lj + 1];
                WW_RELAX_NODE(1, y[0], y[2], sl[1], sr[1])
                WW_RELAX_NODE(2, y[1], y[3], sl[2], sr[2])
                WW_RELAX_NODE(3, y[2], below, sl[3], sr[3])
                asm volatile("" ::: "memory");
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    sl[k] = L[r0 + k + 1][lj];
                    sr[k] = L[r0 + k + 1][lj + 2];
                }
                above = L[r0][lj + 1];
                WW_RELAX_NODE(2, y[1], y[3], sl[2], sr[2])
                WW_RELAX_NODE(1, y[0], y[2], sl[1], sr[1])
                WW_RELAX_NODE(0, above, y[1], sl[0], sr[0])
#undef WW_RELAX_NODE
                if (changed) wchg[wr][wv] = 1;
            }
            if (threadIdx.x < 4) wchg[cl][threadIdx.x] = 0;
            // the waves' change flags of this sweep decide for the whole
            // workgroup after one barrier (slot wr is next cleared two sweeps
            // later, after another barrier)
            __syncthreads();
            const int4 w = *reinterpret_cast<const int4 *>(&wchg[wr][0]);
            if (!__builtin_amdgcn_readfirstlane(w.x | w.y | w.z | w.w)) {
                if (stats && threadIdx.x == 0) atomicAdd(&ctl->iters, (unsigned long long)(it + 1));
                unconverged = false;
                break;
            }
            const int t = rd;
            rd = wr;
            wr = cl;
            cl = t;
        }
        if (unconverged && stats && threadIdx.x == 0)
            atomicAdd(&ctl->iters, (unsigned long long)VISIT_ITERS);
        // The rest of the visit needs the labels around each segment, the
        // ground moves and the potentials of its own nodes: read from LDS in
        // one batch (the loop above ended on a barrier, so every LDS write
        // is done).  A node's own label is y[k], equal to its LDS cell.
        unsigned long long sl[4], sr[4];
        int gak[4], pk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sl[k] = L[r0 + k + 1][lj];
            sr[k] = L[r0 + k + 1][lj + 2];
            gak[k] = GA[r0 + k][lj];
            pk[k] = P[r0 + k + 1][lj + 1];
        }
        const unsigned long long above = L[r0][lj + 1], below = L[r0 + 5][lj + 1];
        // beyond-window candidates of the nodes still without a label
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!ok[k] || y[k] != LINF) continue;
            rej_one(rej, k == 0 ? above : y[k > 0 ? k - 1 : 0], (unsigned)rc[k].x, 1u, lb);
            rej_one(rej, k == 3 ? below : y[k < 3 ? k + 1 : 3], (unsigned)rc[k].y, 2u, lb);
            rej_one(rej, sl[k], (unsigned)rc[k].z, 3u, lb);
            rej_one(rej, sr[k], (unsigned)rc[k].w, 4u, lb);
        }
        const unsigned long long t_swept = stats ? wall_clock64() : 0ull;
        // write back, note changed borders
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!ok[k] || y[k] == init[k]) continue;
            const int li = r0 + k;
            at32(labJ, (unsigned int)((i0 + li) * C + (j0 + lj))) = y[k];
            if (li == 0) flags[0] = 1;
            if (li == rows - 1) flags[1] = 1;
            if (lj == 0) flags[2] = 1;
            if (lj == cols - 1) flags[3] = 1;
        }
        // candidate labels for the ground from perimeter nodes of this tile
        // (the cheapest of a corner's two moves gives its smallest candidate)
        unsigned long long gc = LINF;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned long long l = y[k];
            if (!ok[k] || gak[k] == RC_INF || l == LINF) continue;
            int rc = gak[k] - pk[k] + gpot;
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
            if (lane == 0) { want = flags[0] && ti > 0; nb = lt - J.TC; }
            if (lane == 1) { want = flags[1] && ti < J.TR - 1; nb = lt + J.TC; }
            if (lane == 2) { want = flags[2] && tj > 0; nb = lt - 1; }
            if (lane == 3) { want = flags[3] && tj < J.TC - 1; nb = lt + 1; }
            if (lane == 7) { want = unconverged; nb = lt; }
            const bool fresh = want && atomicExch(&ra.act[J.toff + nb], nr) != nr;
            const unsigned long long fm = __ballot(fresh);
            if (fm) {
                const int leader = __ffsll((long long)fm) - 1;
                unsigned int pos = 0;
                if (lane == leader) pos = atomicAdd(&ctl->count[nr % 3][0], (unsigned int)__popcll(fm));
                pos = __shfl(pos, leader, 64);
                if (fresh) {
                    const unsigned int rank = (unsigned int)__popcll(fm & ((1ull << lane) - 1ull));
                    ra.lists[(size_t)(nr % 3) * list_stride(NT) + pos + rank] = entry_of(job, nb);
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
                unsigned long long *gl = &g.gs[job].glab;
                // the label read at the visit's start is an upper bound of
                // the current one: no second read before the atomic
                if (sh_gcand != LINF && sh_gcand < glab) {
                    unsigned long long old = atomicMin(gl, sh_gcand);
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
            for (unsigned int k = threadIdx.x; k < J.nptiles; k += 256) {
                const unsigned int e = ra.perim_tiles[J.poff + k];
                activate(ra.act, ra.lists, NT, ctl, J.toff + (e & 0xffffffu), e, round + 1);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && my_visits)
        atomicAdd(&ra.vpart[(blockIdx.x % 64) * 16], (unsigned long long)my_visits);
}

template <bool MULTI>
__global__ void k_requeue_pending(Graph g, Ctl *ctl, const unsigned int *pstamp, unsigned int pass,
                                  const unsigned long long *tile_rej, unsigned long long lb,
                                  unsigned int *act, unsigned int *lists, unsigned int NT,
                                  unsigned int rr) {
    for (unsigned int t = blockIdx.x * blockDim.x + threadIdx.x; t < NT; t += gridDim.x * blockDim.x)
        if (pstamp[t] == pass && tile_rej[t] <= lb) {
            const int job = MULTI ? job_of_tile(g, t) : 0;
            const unsigned int toff = MULTI ? g.jobs[job].toff : 0u;
            activate(act, lists, NT, ctl, t, entry_of(job, t - toff), rr);
        }
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
        ctl->relax_ticks += (unsigned long long)wall_clock64() - ctl->t_batch;
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
    // settled grounds with a deficit absorb all of it
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < g.njobs; k += gridDim.x * blockDim.x) {
        const long long gx = g.gs[k].gex;
        if (gx < 0 && g.gs[k].glab <= lb) c += (unsigned int)(-gx);
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
}

// ---------------------------------------------------------- augmentation ---

// A ground's predecessor (blockIdx.y = job): the smallest perimeter arc
// index whose label candidate equals the ground label.
__global__ void k_ground_pred(Graph g, unsigned long long lb) {
    const int k = blockIdx.y;
    GState &G = g.gs[k];
    const unsigned long long gl = G.glab;
    if (gl > lb || G.gex > 0) return;
    const Job J = g.njobs > 1 ? g.jobs[k] : g.j0;
    const unsigned int na = 2u * J.C + 2u * J.R;
    const int gpot = (int)G.gpot;
    for (unsigned int a = blockIdx.x * blockDim.x + threadIdx.x; a < na; a += gridDim.x * blockDim.x) {
        int i, j, kind, delta;
        long long e;
        ground_arc(J, a, i, j, kind, e, delta);
        const long long v = J.noff + (long long)i * J.C + j;
        const unsigned long long l = g.lab[v];
        if (l == LINF) continue;
        const int c = kind == 0 ? move_cost(J.fx[e], delta, J.cxp[e], J.cxn[e])
                                : move_cost(J.fy[e], delta, J.cyp[e], J.cyn[e]);
        if (c == RC_INF) continue;
        const long long rc = (long long)c - g.pot[v] + gpot;
        const unsigned long long nd = (unsigned long long)ldist(l) + (unsigned long long)max(rc, 0ll);
        const unsigned long long cand = (nd << 32) | ((unsigned long long)(lhops(l) + 1) << 3);
        if (cand == gl) atomicMin(&G.gpred, a);
    }
}

// row and column of global node v of job J (v - noff < 2^29, so 32-bit
// arithmetic suffices: the walks below take one step per memory round trip,
// and a 64-bit division would add to every step)
__device__ __forceinline__ void node_rc(const Job &J, long long v, int &i, int &j) {
    const unsigned int u = (unsigned int)(v - J.noff), C = (unsigned int)J.C;
    const unsigned int q = u / C;
    i = (int)q;
    j = (int)(u - q * C);
}

// predecessor of node (i,j) of job J along direction dir; -1 = its ground
__device__ __forceinline__ long long pred_node(const Job &J, int i, int j, int dir) {
    switch (dir) {
        case DIR_UP: return i > 0 ? J.noff + (long long)(i - 1) * J.C + j : -1;
        case DIR_DOWN: return i < J.R - 1 ? J.noff + (long long)(i + 1) * J.C + j : -1;
        case DIR_LEFT: return j > 0 ? J.noff + (long long)i * J.C + j - 1 : -1;
        default: return j < J.C - 1 ? J.noff + (long long)i * J.C + j + 1 : -1;
    }
}

// Walk from v to its root within job J.  Returns the root node; *gsub = 1
// when the root is a child of the job's ground acting as a supply.
// Walks from v along the predecessor arcs to the tree's root and returns it
// (-1 on a broken walk).  Every node before the root gets the walk's key as
// a candidate path tag (best[u] = the smallest key of the walks through u)
// and the pass's stamp in its tag byte; *crossed is set when the walk
// passes through the ground.
__device__ long long walk_root(const Graph &g, const Job &J, const GState &G, Ctl *ctl, long long v,
                               int gsrc, int *gsub, unsigned long long key, int *crossed,
                               uint8_t *tag, uint8_t stamp) {
    *gsub = 0;
    *crossed = 0;
    const long long Nk = (long long)J.R * J.C;
    unsigned long long l = g.lab[v];
    // the first label is waited for here, so that the loop's head waits for
    // nothing (the latch waits for the next label alone)
    asm volatile("" ::"v"(l));
    for (long long steps = 0; steps <= Nk + 2; ++steps) {
        const int dir = (int)(l & 7);
        if (dir == DIR_NONE) return v;
        int i, j;
        node_rc(J, v, i, j);
        long long u = pred_node(J, i, j, dir);
        if (u < 0) {
            if (gsrc) {
                *gsub = 1;
                return v;
            }
            const unsigned int a = G.gpred;
            if (a >= 2u * J.C + 2u * J.R) break;  // no ground predecessor: report below
            int pi, pj, kind, delta;
            long long e;
            ground_arc(J, a, pi, pj, kind, e, delta);
            u = J.noff + (long long)pi * J.C + pj;
            *crossed = 1;
        }
        // the next label is requested before the tag is offered, so that
        // the walk waits for the load alone, not for the atomic behind it
        const unsigned long long ln = g.lab[u];
        atomicMin(&g.best[v], key);
        tag[v] = stamp;
        v = u;
        l = ln;
    }
    atomicOr(&ctl->error, ERR_WALK);
    return -1;
}

// Every settled deficit (and every job's ground as a settled demand) walks
// to its tree's root and offers its key (distance, deficit) there; the
// walks also tag their nodes (walk_root).  A deficit's own flip word
// records the pass, and whether its walk crossed the ground (bit 2).
// A deficit whose label is more than defer_hops arcs from its root (when
// defer_hops > 0) is left to the wave walk instead: its index goes to longw.
template <bool MULTI>
__global__ void k_roots(Graph g, Ctl *ctl, const unsigned int *def, unsigned long long lb,
                        unsigned int *gsub_list, unsigned int *flip, uint8_t *tag,
                        unsigned int pass, unsigned int *longw, unsigned int defer_hops) {
    const unsigned int nd = ctl->ndef;
    for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k < nd + (unsigned)g.njobs;
         k += gridDim.x * blockDim.x) {
        long long start;
        unsigned long long key;
        int job;
        if (k < nd) {
            const unsigned int t = def[k];
            const unsigned long long l = g.lab[t];
            if (l > lb) continue;
            if (defer_hops && lhops(l) > defer_hops) {
                longw[atomicAdd(&ctl->nlong, 1u)] = k;
                continue;
            }
            start = t;
            key = ((unsigned long long)ldist(l) << 32) | t;
            job = MULTI ? job_of_node(g, t) : 0;
        } else {
            // a ground as a demand: its path enters through gpred
            job = (int)(k - nd);
            const GState &G = g.gs[job];
            const unsigned long long gl = G.glab;
            if (!(G.gex < 0 && gl <= lb)) continue;
            const Job J = job_at<MULTI>(g, job);
            if (G.gpred >= 2u * J.C + 2u * J.R) {
                atomicOr(&ctl->error, ERR_WALK);
                continue;
            }
            int pi, pj, kind, delta;
            long long e;
            ground_arc(J, G.gpred, pi, pj, kind, e, delta);
            start = J.noff + (long long)pi * J.C + pj;
            key = ((unsigned long long)ldist(gl) << 32) | (unsigned long long)(g.N + job);
        }
        const Job J = job_at<MULTI>(g, job);
        GState &G = g.gs[job];
        int gsub = 0, crossed = 0;
        const long long root =
            walk_root(g, J, G, ctl, start, G.gex > 0, &gsub, key, &crossed, tag, (uint8_t)pass);
        if (k < nd) flip[start] = (pass << 3) | (crossed ? 4u : 0u);
        if (root < 0) continue;
        tag[root] = (uint8_t)pass;
        const unsigned long long old = atomicMin(&g.best[root], key);
        if (gsub && old == LINF) gsub_list[J.aoff + atomicAdd(&G.gsub_count, 1u)] = (unsigned int)root;
    }
}

// The same walks with one workgroup per walk, for the long walks: a walk of
// one thread waits a memory round trip per step.  The workgroup stages an
// RW_H x RW_W region of the walk's job in LDS around the current node (at
// the start centred on it, later with the node near the edge the walk came
// in through; clamped to the job), from one coalesced read of the labels' low words
// shared by its four waves: per node the region index of its predecessor,
// or RW_OUT with the predecessor's direction when the predecessor lies
// outside the region or the job (or the node is a root).  A step inside the
// region is one LDS read.  All four waves take every step (the same values,
// so that they meet at the barriers around each staging); wave 0 keeps the
// nodes passed one per lane (their region index) and offers them their key
// and tag 64 at a time and before the next region.
constexpr int RW_H = 64, RW_W = 64;
constexpr int RW_WAVES = 4;            // waves per walk (rows staged: RW_H / RW_WAVES each)
constexpr unsigned int RW_OUT = 0x8000u;
constexpr int ROOTS_WAVE_MAX = 1024;   // walks (deficits + grounds) that all take this kernel
constexpr unsigned int RW_SHORT = 16;  // walks of at most this many arcs take one thread
constexpr unsigned int RW_LONG = 32;   // in larger passes, walks of more arcs take a workgroup
constexpr int ROOTS_WAVE_GRID = 1024;  // workgroups of the walk over the long walks

__device__ __forceinline__ void stage_region(const Graph &g, const Job &J, int ri0, int rj0, uint16_t *sd) {
    constexpr int RPW = RW_H / RW_WAVES;
    const int lane = threadIdx.x & 63, r0 = (int)(threadIdx.x >> 6) * RPW;
    const unsigned int *lo = reinterpret_cast<const unsigned int *>(g.lab);
    // rows and columns past the job's edge read its last row or column (in
    // bounds; a walk never steps there)
    const long long col = J.noff + min(rj0 + lane, J.C - 1);
    unsigned int w[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) w[r] = lo[2 * (col + (long long)min(ri0 + r0 + r, J.R - 1) * J.C)];
    // a node's code: RW_OUT | dir when it is a root (dir 0) or its
    // predecessor lies past the region's or the job's edge (bit dir of the
    // exit mask), else its predecessor's region index (index + the offset
    // for dir, one signed byte per direction in RW_STEP)
    const int rmax = min(RW_H, J.R - ri0), cmax = min(RW_W, J.C - rj0);
    const unsigned int lane_exit = 1u | (lane == 0 ? 1u << DIR_LEFT : 0u) | (lane == cmax - 1 ? 0xf0u : 0u);
    constexpr unsigned long long RW_STEP = 0x01010101ff40c000ull;  // 0, -64, +64, -1, +1, +1, +1, +1
    static_assert(RW_W == 64, "RW_STEP holds the row offset of 64-column regions");
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int rr = r0 + r;
        const unsigned int dir = w[r] & 7u;
        const unsigned int ex = lane_exit | (rr == 0 ? 1u << DIR_UP : 0u) | (rr == rmax - 1 ? 1u << DIR_DOWN : 0u);
        const int off = (int)(signed char)(unsigned char)(RW_STEP >> (8u * dir));
        const unsigned int e = (ex >> dir) & 1u, in = (unsigned int)(rr * RW_W + lane + off);
        sd[rr * RW_W + lane] = (uint16_t)(in + e * ((RW_OUT | dir) - in));  // a select without a branch
    }
}

__device__ long long walk_root_wave(const Graph &g, const Job &J, const GState &G, Ctl *ctl, long long v,
                                    int gsrc, int *gsub, unsigned long long key, int *crossed, uint8_t *tag,
                                    uint8_t stamp, uint16_t *sd) {
    const int lane = threadIdx.x & 63;
    const bool w0 = threadIdx.x < 64;  // the wave that offers
    *gsub = 0;
    *crossed = 0;
    const long long limit = (long long)J.R * J.C + 2;
    int i, j;
    node_rc(J, v, i, j);
    int mine = 0;  // region index of a node passed, one per lane of wave 0
    int np = 0;
    long long steps = 0, res = -1;
    bool broken = false;
    // where the current node sits in the next region: centred at the start
    // and after the ground; else near the edge the walk came in through
    int at_r = RW_H / 2, at_c = RW_W / 2;
    for (;;) {
        const int ri0 = max(0, min(i - at_r, J.R - RW_H)), rj0 = max(0, min(j - at_c, J.C - RW_W));
        // key and tag to the np nodes passed in this region
        auto offer = [&]() {
            if (w0 && lane < np) {
                const long long u = J.noff + (long long)(ri0 + mine / RW_W) * J.C + rj0 + mine % RW_W;
                atomicMin(&g.best[u], key);
                tag[u] = stamp;
            }
            steps += np;
            np = 0;
            broken = broken || steps > limit;
        };
        __syncthreads();  // every wave is done with the previous region
        stage_region(g, J, ri0, rj0, sd);
        __syncthreads();
        int li = (i - ri0) * RW_W + (j - rj0);
        unsigned int code;
        for (;;) {
            const int raw = sd[li];
            // kept while the read is in flight; counted once the node is
            // known to be passed
            mine = lane == np ? li : mine;
            code = (unsigned int)__builtin_amdgcn_readfirstlane(raw);
            if (code & RW_OUT) break;
            if (++np == 64) {
                offer();
                if (broken) break;
            }
            li = (int)code;
        }
        if (broken) break;
        const int dir = (int)(code & 7u);
        i = ri0 + li / RW_W;
        j = rj0 + li % RW_W;
        v = J.noff + (long long)i * J.C + j;
        if (dir == DIR_NONE) {
            offer();
            res = v;
            break;
        }
        int ui = i, uj = j;
        bool ground;
        at_r = RW_H / 2;
        at_c = RW_W / 2;
        switch (dir) {
            case DIR_UP: ui = i - 1; ground = i == 0; at_r = RW_H - 8; break;
            case DIR_DOWN: ui = i + 1; ground = i == J.R - 1; at_r = 7; break;
            case DIR_LEFT: uj = j - 1; ground = j == 0; at_c = RW_W - 8; break;
            default: uj = j + 1; ground = j == J.C - 1; at_c = 7; break;
        }
        if (ground) {
            at_r = RW_H / 2;
            at_c = RW_W / 2;
            if (gsrc) {
                offer();
                *gsub = 1;
                res = v;
                break;
            }
            const unsigned int a = G.gpred;
            if (a >= 2u * J.C + 2u * J.R) {  // no ground predecessor: reported below
                offer();
                break;
            }
            int kind, delta;
            long long e;
            ground_arc(J, a, ui, uj, kind, e, delta);
            *crossed = 1;
        }
        mine = lane == np ? li : mine;
        ++np;
        offer();
        if (broken) break;
        i = ui;
        j = uj;
    }
    if (res < 0 && threadIdx.x == 0) atomicOr(&ctl->error, ERR_WALK);
    return res;
}

template <bool MULTI>
__global__ __launch_bounds__(64 * RW_WAVES) void k_roots_wave(Graph g, Ctl *ctl, const unsigned int *def,
                                                              unsigned long long lb, unsigned int *gsub_list,
                                                              unsigned int *flip, uint8_t *tag, unsigned int pass,
                                                              const unsigned int *longw, unsigned int short_hops) {
    __shared__ uint16_t sdir[RW_H * RW_W];
    const unsigned int nd = ctl->ndef;
    // every walk of the pass, or (longw) the long walks k_roots left
    const unsigned int items = longw ? ctl->nlong : nd + (unsigned)g.njobs;
    for (unsigned int q = blockIdx.x; q < items; q += gridDim.x) {
        const unsigned int k = longw ? longw[q] : q;
        long long start;
        unsigned long long key;
        unsigned int hops;  // arcs from the root
        int job;
        if (k < nd) {
            const unsigned int t = def[k];
            const unsigned long long l = g.lab[t];
            if (l > lb) continue;
            hops = lhops(l);
            start = t;
            key = ((unsigned long long)ldist(l) << 32) | t;
            job = MULTI ? job_of_node(g, t) : 0;
        } else {
            job = (int)(k - nd);
            const GState &G = g.gs[job];
            const unsigned long long gl = G.glab;
            if (!(G.gex < 0 && gl <= lb)) continue;
            const Job J = job_at<MULTI>(g, job);
            if (G.gpred >= 2u * J.C + 2u * J.R) {
                if (threadIdx.x == 0) atomicOr(&ctl->error, ERR_WALK);
                continue;
            }
            int pi, pj, kind, delta;
            long long e;
            ground_arc(J, G.gpred, pi, pj, kind, e, delta);
            start = J.noff + (long long)pi * J.C + pj;
            key = ((unsigned long long)ldist(gl) << 32) | (unsigned long long)(g.N + job);
            hops = lhops(gl);
        }
        const Job J = job_at<MULTI>(g, job);
        GState &G = g.gs[job];
        int gsub = 0, crossed = 0;
        long long root = -1;
        if (hops > short_hops) {
            root = walk_root_wave(g, J, G, ctl, start, G.gex > 0, &gsub, key, &crossed, tag, (uint8_t)pass, sdir);
        } else if (threadIdx.x == 0) {
            // a short walk: fewer memory round trips than staging a region takes
            root = walk_root(g, J, G, ctl, start, G.gex > 0, &gsub, key, &crossed, tag, (uint8_t)pass);
        }
        if (threadIdx.x == 0) {
            if (k < nd) flip[start] = (pass << 3) | (crossed ? 4u : 0u);
            if (root >= 0) {
                tag[root] = (uint8_t)pass;
                const unsigned long long old = atomicMin(&g.best[root], key);
                if (gsub && old == LINF) gsub_list[J.aoff + atomicAdd(&G.gsub_count, 1u)] = (unsigned int)root;
            }
        }
    }
}

// Keep at most gex of a ground's subtrees (blockIdx.y = job): those with
// the smallest (best key, root id).  O(k^2), k <= the job's perimeter.
__global__ void k_gsub_select(Graph g, const unsigned int *gsub_list, unsigned char *drop) {
    const int job = blockIdx.y;
    const Job J = g.njobs > 1 ? g.jobs[job] : g.j0;
    const unsigned int k = g.gs[job].gsub_count;
    const long long allow = g.gs[job].gex;
    const unsigned int *list = gsub_list + J.aoff;
    for (unsigned int a = blockIdx.x * blockDim.x + threadIdx.x; a < k; a += gridDim.x * blockDim.x) {
        drop[J.aoff + a] = 0;
        if ((long long)k <= allow) continue;
        const unsigned int ra = list[a];
        const unsigned long long ka = g.best[ra];
        long long rank = 0;
        for (unsigned int b = 0; b < k; ++b) {
            const unsigned int rb = list[b];
            const unsigned long long kb = g.best[rb];
            if (kb < ka || (kb == ka && rb < ra)) ++rank;
        }
        if (rank >= allow) drop[J.aoff + a] = 1;
    }
}

__device__ __forceinline__ void flip_into(const Job &J, long long v, int dir) {
    int i, j;
    node_rc(J, v, i, j);
    switch (dir) {
        case DIR_UP: J.fx[(long long)i * J.C + j] += 1; break;
        case DIR_DOWN: J.fx[(long long)(i + 1) * J.C + j] -= 1; break;
        case DIR_LEFT: J.fy[(long long)i * J.n + j] -= 1; break;
        default: J.fy[(long long)i * J.n + j + 1] += 1; break;
    }
}

__device__ __forceinline__ void flip_ground_arc(const Job &J, unsigned int a) {
    int i, j, kind, delta;
    long long e;
    ground_arc(J, a, i, j, kind, e, delta);
    if (kind == 0) J.fx[e] += (int8_t)delta;
    else J.fy[e] += (int8_t)delta;
}

// Choose the paths that augment: every root takes the deficit with its
// smallest key (distance, deficit id), the flip word of that deficit gets
// bit 0 (a ground demand: its gchosen field the pass), and the excesses
// move by one unit.  The arcs of a chosen path are not walked here: the
// walks of k_roots tagged each path node with the smallest key through it,
// which on the chosen path is the root's own key (every walk through a
// node ends at the same root), so k_potentials, which visits every settled
// node, flips the arc into each node whose tag names a chosen deficit.
// Only the arcs into and through the ground are flipped here.  Work items:
// the supplies, then every job's ground-subtree slots (nslots in all).
template <bool MULTI>
__global__ void k_augment(Graph g, Ctl *ctl, const unsigned int *src, const unsigned int *gsub_list,
                          const unsigned char *drop, unsigned int *flip, unsigned int pass,
                          unsigned int nslots) {
    const unsigned int ns = ctl->nsrc;
    for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k < ns + nslots;
         k += gridDim.x * blockDim.x) {
        const bool is_g = k >= ns;
        int job;
        unsigned int r;
        if (is_g) {
            const unsigned int qs = k - ns;
            job = MULTI ? job_of_slot(g, qs) : 0;
            const unsigned int aoff = MULTI ? g.jobs[job].aoff : 0u;
            if (qs - aoff >= g.gs[job].gsub_count) continue;
            r = gsub_list[qs];
        } else {
            r = src[k];
            job = MULTI ? job_of_node(g, r) : 0;
        }
        const unsigned long long b = g.best[r];  // reset by k_potentials
        if (b == LINF) continue;
        if (is_g && drop[k - ns]) continue;
        const Job J = job_at<MULTI>(g, job);
        GState &G = g.gs[job];
        const long long t = (long long)(b & 0xffffffffull);
        const bool into_ground = t >= g.N;
        unsigned long long flips = 0;
        const unsigned int na = 2u * J.C + 2u * J.R;
        bool through_ground = into_ground;
        if (into_ground) {
            G.gchosen = pass;
        } else {
            const unsigned int f = flip[t];
            flip[t] = f | 1u;
            through_ground = (f & 4u) != 0;
        }
        // a path into or through the ground uses the ground's predecessor
        // arc, which exists whenever the ground is settled; its absence
        // fails the solve
        if (through_ground) {
            const unsigned int a = G.gpred;
            if (a >= na) {
                atomicOr(&ctl->error, ERR_WALK);
                continue;
            }
            flip_ground_arc(J, a);
            ++flips;
        }
        if (is_g) atomicAdd((unsigned long long *)&G.gex, (unsigned long long)-1ll);
        else g.ex[r] -= 1;
        if (into_ground) atomicAdd((unsigned long long *)&G.gex, 1ull);
        else g.ex[t] += 1;
        atomicAdd(&ctl->naug, 1u);
        if (flips) atomicAdd(&ctl->arcs, flips);
    }
}

// pot(v) += B - d(v) on every reached node, labels and path tags back to
// infinity, and the arc into every node of a chosen path flipped.  A grid
// of at most POT_GRID workgroups reads every tile's stamp once (workgroup w
// owns the tiles w, w + G, w + 2G, ... of a grid of G, all read in one
// batch while there are at most 256 of them) and updates only the tiles
// relaxed in this pass, so that a pass that reached a few tiles costs one
// small launch and one read of the stamps.  The relaxed tiles of a pass lie
// close together, and the stride spreads neighbouring tiles over different
// workgroups.  A counting solve also adds up the settled nodes and their
// residual out-arcs (the work of a textbook search that settles the same
// nodes).
constexpr int POT_GRID = 1024;

template <bool MULTI, int TW>
__global__ __launch_bounds__(256) void k_potentials(Graph g, Ctl *ctl, const unsigned int *tstamp,
                                                    unsigned int pass, unsigned int NT,
                                                    unsigned long long lb, const unsigned int *flip,
                                                    const uint8_t *tag, int count, int pot_limit) {
    __shared__ unsigned int todo[256];
    __shared__ int ntodo;
    const unsigned int bound = ldist(lb);
    int mx = 0;
    unsigned long long n_set = 0, n_arc = 0, n_flip = 0;
    for (unsigned long long base = blockIdx.x; base < NT; base += 256ull * gridDim.x) {
        if (threadIdx.x == 0) ntodo = 0;
        __syncthreads();
        const unsigned long long tile = base + (unsigned long long)threadIdx.x * gridDim.x;
        if (tile < NT && tstamp[tile] == pass) todo[atomicAdd(&ntodo, 1)] = (unsigned int)tile;
        __syncthreads();
        const int nt = ntodo;
        for (int k = 0; k < nt; ++k) {
            const unsigned int tile = todo[k];
            const int job = MULTI ? job_of_tile(g, tile) : 0;
            const Job J = job_at<MULTI>(g, job);
            const unsigned int lt = tile - J.toff;
            constexpr int TH = TILE_NODES / TW;
            const int i0 = (int)(lt / J.TC) * TH, j0 = (int)(lt % J.TC) * TW;
            long long v[TILE_NODES / 256];
            unsigned long long l[TILE_NODES / 256];
            uint8_t tb[TILE_NODES / 256];
#pragma unroll
            for (int s = 0; s < TILE_NODES / 256; ++s) {
                const int t = threadIdx.x + 256 * s;
                const int i = i0 + t / TW, j = j0 + t % TW;
                v[s] = (i < J.R && j < J.C) ? J.noff + (long long)i * J.C + j : -1;
                l[s] = v[s] >= 0 ? g.lab[v[s]] : LINF;
                tb[s] = v[s] >= 0 ? tag[v[s]] : (uint8_t)0;
            }
#pragma unroll
            for (int s = 0; s < TILE_NODES / 256; ++s) {
                if (l[s] == LINF) continue;
                // a walk of this pass passed here (a stale byte of a pass 256
                // earlier finds the key cleared: no effect)
                const unsigned long long tgk = tb[s] == (uint8_t)pass ? g.best[v[s]] : LINF;
                if (tgk != LINF) {
                    // a path node (only settled nodes are tagged): the arc
                    // into it flips when its key names a chosen deficit
                    g.best[v[s]] = LINF;
                    const int dir = (int)(l[s] & 7u);
                    const long long t = (long long)(tgk & 0xffffffffull);
                    const bool chosen = t < g.N ? flip[t] == ((pass << 3) | 1u) || flip[t] == ((pass << 3) | 5u)
                                                : g.gs[t - g.N].gchosen == pass;
                    if (dir != DIR_NONE && chosen) {
                        flip_into(J, v[s], dir);
                        ++n_flip;
                    }
                }
                g.lab[v[s]] = LINF;
                if (l[s] > lb) continue;
                if (count) {
                    int i, j;
                    node_rc(J, v[s], i, j);
                    long long e;
                    ++n_set;
                    e = (long long)i * J.C + j;  // up across hx(i,j): -1
                    n_arc += move_cost(J.fx[e], -1, J.cxp[e], J.cxn[e]) != RC_INF;
                    e = (long long)(i + 1) * J.C + j;  // down across hx(i+1,j): +1
                    n_arc += move_cost(J.fx[e], +1, J.cxp[e], J.cxn[e]) != RC_INF;
                    e = (long long)i * J.n + j;  // left across vy(i,j): +1
                    n_arc += move_cost(J.fy[e], +1, J.cyp[e], J.cyn[e]) != RC_INF;
                    e = (long long)i * J.n + j + 1;  // right across vy(i,j+1): -1
                    n_arc += move_cost(J.fy[e], -1, J.cyp[e], J.cyn[e]) != RC_INF;
                }
                const unsigned int d = ldist(l[s]);
                const long long np = (long long)g.pot[v[s]] + (bound - d);
                if (np > pot_limit) atomicOr(&ctl->error, ERR_POT);
                g.pot[v[s]] = (int)min(np, (long long)pot_limit);
                mx = max(mx, (int)min(np, (long long)pot_limit));
            }
        }
        __syncthreads();
    }
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_down(mx, off, 64));
    // only a wave that may raise the maximum takes the atomic: thousands of
    // atomics on one address from every wave cost more than the updates
    if ((threadIdx.x & 63) == 0 && mx > 0 && mx > *(volatile int *)&ctl->max_pot)
        atomicMax(&ctl->max_pot, mx);
    for (int off = 32; off > 0; off >>= 1) n_flip += __shfl_down(n_flip, off, 64);
    if ((threadIdx.x & 63) == 0 && n_flip) atomicAdd(&ctl->arcs, n_flip);
    if (count) {
        for (int off = 32; off > 0; off >>= 1) {
            n_set += __shfl_down(n_set, off, 64);
            n_arc += __shfl_down(n_arc, off, 64);
        }
        if ((threadIdx.x & 63) == 0 && n_set) {
            atomicAdd(&ctl->settled, n_set);
            atomicAdd(&ctl->scanned, n_arc);
        }
    }
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < g.njobs; k += gridDim.x * blockDim.x) {
        GState &G = g.gs[k];
        const unsigned long long gl = G.glab;
        if (gl <= lb) {
            G.gpot += bound - ldist(gl);
            if (G.gpot > pot_limit) atomicOr(&ctl->error, ERR_POT);
            if (count) atomicAdd(&ctl->settled, 1ull);
        }
        G.glab = LINF;
    }
}

// Debug check (WW_MCF_CHECK=1): every residual arc must have a non-negative
// reduced cost after a pass (blockIdx.y = job).  Records the first
// offending arc.
struct CheckRec {
    int found;
    int kind;          // in-arc direction at v (1..4) or 8+side for an arc into the ground
    long long u, v;    // tail, head (-1 = ground)
    long long rc;
    long long pu, pv;
    unsigned long long lu, lv;  // labels before the potential update
    int f, cp, cn;
};

__global__ void k_check_rc(Graph g, const unsigned long long *lab_before, CheckRec *rec) {
    const int job = blockIdx.y;
    const Job J = g.njobs > 1 ? g.jobs[job] : g.j0;
    const long long Nk = (long long)J.R * J.C;
    const long long gpot = g.gs[job].gpot;
    for (long long lv = (long long)blockIdx.x * blockDim.x + threadIdx.x; lv < Nk;
         lv += (long long)gridDim.x * blockDim.x) {
        const long long v = J.noff + lv;
        const int i = (int)(lv / J.C), j = (int)(lv % J.C);
        for (int dir = 1; dir <= 4; ++dir) {
            long long e;
            int kind, delta;
            if (dir == DIR_UP) { e = (long long)i * J.C + j; kind = 0; delta = +1; }
            else if (dir == DIR_DOWN) { e = (long long)(i + 1) * J.C + j; kind = 0; delta = -1; }
            else if (dir == DIR_LEFT) { e = (long long)i * J.n + j; kind = 1; delta = -1; }
            else { e = (long long)i * J.n + j + 1; kind = 1; delta = +1; }
            const int f = kind == 0 ? J.fx[e] : J.fy[e];
            const int cp = kind == 0 ? J.cxp[e] : J.cyp[e];
            const int cn = kind == 0 ? J.cxn[e] : J.cyn[e];
            const int c = move_cost(f, delta, cp, cn);
            if (c == RC_INF) continue;
            const long long u = pred_node(J, i, j, dir);
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
// entry names a tile below NT whose round stamp is rr, and exactly count
// tiles carry that stamp (so no tile is listed twice).  bad[0]: an entry out
// of range; bad[1]: an entry without the stamp; bad[2]: tiles with the
// stamp; bad[3]: entries read.
template <bool MULTI>
__global__ void k_check_lists(Graph g, const Ctl *ctl, const unsigned int *act,
                              const unsigned int *lists, unsigned int NT, unsigned int rr,
                              unsigned int *bad) {
    const unsigned int cnt = ctl->count[rr % 3][0];
    const size_t ls = list_stride(NT);
    const unsigned int *list = lists + (size_t)(rr % 3) * ls;
    const unsigned int lim = cnt < ls ? cnt : (unsigned int)ls;
    for (unsigned int k = blockIdx.x * blockDim.x + threadIdx.x; k < (unsigned int)ls;
         k += gridDim.x * blockDim.x) {
        if (k < lim) {
            atomicAdd(&bad[3], 1u);
            const unsigned int e = list[k];
            const unsigned int job = e >> 24, lt = e & 0xffffffu;
            if ((int)job >= g.njobs) {
                atomicOr(&bad[0], 1u);
            } else {
                const Job J = job_at<MULTI>(g, (int)job);
                if (lt >= (unsigned)(J.TR * J.TC) || J.toff + lt >= NT) atomicOr(&bad[0], 1u);
                else if (act[J.toff + lt] != rr) atomicOr(&bad[1], 1u);
            }
        }
        if (k < NT && act[k] == rr) atomicAdd(&bad[2], 1u);
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
    // the last workgroup to finish makes the compacted lists current (their
    // lengths; the host swaps the pointers): no launch of its own per pass
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(&ctl->compact_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        ctl->nsrc = atomicAdd(&ctl->nsrc2, 0u);  // read at the device's coherence point
        ctl->ndef = atomicAdd(&ctl->ndef2, 0u);
        ctl->compact_done = 0;
    }
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
// The flow planes of all jobs are two contiguous arrays (fx: nx entries,
// fy: ny).  nodes = 0 leaves the node excesses and potentials as they are:
// the way back after the last pass, when only the flows, the grounds and
// (negated on export) the potentials are read any more.
__global__ void k_reverse_frame(Graph g, Ctl *ctl, int8_t *fx, long long nx, int8_t *fy,
                                long long ny, int nodes) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    negate_span(fx, nx, tid, stride);
    negate_span(fy, ny, tid, stride);
    if (nodes) {
        negate_span(g.ex, g.N, tid, stride);
        negate_span(g.pot, g.N, tid, stride);
    }
    for (long long k = tid; k < g.njobs; k += stride) {
        g.gs[k].gex = -g.gs[k].gex;
        g.gs[k].gpot = -g.gs[k].gpot;
    }
    if (tid == 0) {
        const unsigned int ns = ctl->nsrc;
        ctl->nsrc = ctl->ndef;
        ctl->ndef = ns;
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

// Each job's flow cost (blockIdx.y = job), one atomic per workgroup into
// its ground record (zeroed at set-up).
__global__ __launch_bounds__(256) void k_total_cost(Graph g) {
    const int job = blockIdx.y;
    const Job J = g.njobs > 1 ? g.jobs[job] : g.j0;
    const long long nx = (long long)(J.R + 1) * J.C, ny = (long long)J.R * J.n;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long s = cost_span(J.fx, J.cxp, J.cxn, nx, tid, stride) +
                  cost_span(J.fy, J.cyp, J.cyn, ny, tid, stride);
    __shared__ long long red[4];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = red[0] + red[1] + red[2] + red[3];
        if (t) atomicAdd((unsigned long long *)&g.gs[job].total_cost, (unsigned long long)t);
    }
}

// (sign -1: the node potentials were left in the reversed frame)
// The solver's counters and ground records (bytes, a multiple of 16)
// copied into coherent pinned host memory, then the sequence word seq after
// a system-scope fence: a host that sees seq there reads counters that are
// complete, and knows that all work queued before this kernel is done.
__global__ void k_mirror(const uint4 *__restrict__ src, uint4 *dst, size_t bytes, unsigned int *flag,
                         unsigned int seq) {
    for (size_t k = threadIdx.x; k < bytes / 16; k += blockDim.x) dst[k] = src[k];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        __threadfence_system();
    }
}

__global__ void k_export_pot(const int *pot, const GState *gs, long long N, int64_t *out, int sign) {
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v <= N;
         v += (long long)gridDim.x * blockDim.x)
        out[v] = v < N ? (int64_t)sign * pot[v] : (int64_t)gs[0].gpot;
}

// ------------------------------------------------------------------ host ---

constexpr unsigned int HMAX = 0x1fffffffu;

// process-wide window schedule (ww_set_mcf_params), read once per solve by
// the calls that take no schedule of their own
std::atomic<int> g_first_hops{64};
std::atomic<int> g_first_dstep{256};
std::atomic<int> g_full_passes{0};
std::atomic<int> g_first_deficit{0};
std::atomic<int> g_reverse_below{0};
std::atomic<int> g_hop_growth{2};
std::atomic<int> g_tile_cols{32};

ww_mcf_params process_mcf_params() {
    ww_mcf_params p;
    p.first_hop_window = g_first_hops.load();
    p.first_distance_step = g_first_dstep.load();
    p.full_passes = g_full_passes.load();
    p.first_deficit_after = g_first_deficit.load();
    p.reverse_below = g_reverse_below.load();
    p.hop_growth = g_hop_growth.load();
    p.tile_cols = g_tile_cols.load();
    return p;
}

ww_status check_mcf_params(const ww_mcf_params &p) {
    if (p.first_hop_window < 1 || p.first_hop_window > (int32_t)HMAX - 1 || p.first_distance_step < 1 ||
        p.first_distance_step > (1 << 30))
        return fail(WW_E_INVALID_ARG, "window schedule out of range");
    if (p.full_passes < 0 || p.full_passes > (1 << 20) ||
        (p.first_deficit_after != 0 && p.first_deficit_after != 1) || p.reverse_below < 0 ||
        p.hop_growth < 2 || p.hop_growth > (1 << 20))
        return fail(WW_E_INVALID_ARG, "pass schedule out of range");
    if (p.tile_cols != 16 && p.tile_cols != 32 && p.tile_cols != 64)
        return fail(WW_E_INVALID_ARG, "tile_cols must be 16, 32 or 64");
    return WW_OK;
}

static unsigned long long mk_label(unsigned int d, unsigned int h) {
    return ((unsigned long long)d << 32) | ((unsigned long long)h << 3) | 7ull;
}

static ww_status decode_error(int e) {
    // a potential clamped at the limit breaks the reduced costs of later
    // passes: the overflow is the cause to report
    if (e & ERR_POT) return fail(WW_E_OVERFLOW, "min-cost flow: node potential above its limit (2^30)");
    if (e & ERR_NEG_RC) return fail(WW_E_DEVICE, "min-cost flow: negative reduced cost (invariant broken)");
    if (e & ERR_WALK) return fail(WW_E_DEVICE, "min-cost flow: predecessor walk did not end");
    if (e & ERR_ITERS) return fail(WW_E_DEVICE, "min-cost flow: tile relaxation did not converge");
    return fail(WW_E_DEVICE, "min-cost flow: error flags 0x%x", e);
}

// The solve of one job (mj.size() == 1, MULTI = false) or of several at
// once.  The jobs' residues, x-flow planes and y-flow planes each lie in one
// contiguous array, job after job (res_all, fx_all, fy_all, flows zeroed by
// the caller); each job's total goes to *mj[k].total.
template <bool MULTI, int TW>
static ww_status solve(const std::vector<McfJob> &mj, const int8_t *res_all, int8_t *fx_all,
                       int8_t *fy_all, int64_t *pot_out, ww_mcf_stats *stats,
                       const ww_mcf_params &sp, hipStream_t st) {
    ww_mcf_stats S;
    memset(&S, 0, sizeof(S));
    last_mcf_stats() = S;
    const auto t_start = std::chrono::steady_clock::now();
    const int nj = (int)mj.size();
    // job layout: nodes, tiles, perimeter tiles and ground-subtree slots
    std::vector<Job> jobs(nj);
    std::vector<unsigned int> ptiles;
    long long N = 0, nx_all = 0, ny_all = 0;
    unsigned int NT = 0, nslots = 0;
    int max_arcs = 0;
    for (int k = 0; k < nj; ++k) {
        const McfJob &q = mj[k];
        Job &J = jobs[k];
        J.R = q.m - 1;
        J.C = q.n - 1;
        J.n = q.n;
        J.TR = ceil_div(J.R, TILE_NODES / TW);
        J.TC = ceil_div(J.C, TW);
        J.noff = N;
        J.toff = NT;
        J.aoff = nslots;
        J.cxp = q.cxp; J.cxn = q.cxn; J.cyp = q.cyp; J.cyn = q.cyn;
        J.fx = fx_all + nx_all;
        J.fy = fy_all + ny_all;
        if (q.dkx != J.fx || q.dky != J.fy || q.res != res_all + N)
            return fail(WW_E_INVALID_ARG, "min-cost flow: job %d planes are not contiguous", k);
        J.poff = (unsigned int)ptiles.size();
        for (int ti = 0; ti < J.TR; ++ti)
            for (int tj = 0; tj < J.TC; ++tj)
                if (ti == 0 || tj == 0 || ti == J.TR - 1 || tj == J.TC - 1)
                    ptiles.push_back(((unsigned int)k << 24) | (unsigned)(ti * J.TC + tj));
        J.nptiles = (unsigned int)ptiles.size() - J.poff;
        N += (long long)J.R * J.C;
        NT += (unsigned int)(J.TR * J.TC);
        nslots += 2u * J.C + 2u * J.R;
        max_arcs = std::max(max_arcs, 2 * J.C + 2 * J.R);
        nx_all += (long long)q.m * (q.n - 1);
        ny_all += (long long)(q.m - 1) * q.n;
    }
    if (N >= (1ll << 31) - 512) return fail(WW_E_INVALID_ARG, "more than 2^31 loops in one solve");
    Graph g;
    g.N = N;
    g.njobs = nj;
    g.j0 = jobs[0];
    WW_TRY(scratch(SLOT_MCF_LAB, sizeof(unsigned long long) * N, (void **)&g.lab));
    WW_TRY(scratch(SLOT_MCF_BEST, sizeof(unsigned long long) * N, (void **)&g.best));
    WW_TRY(scratch(SLOT_MCF_POT, sizeof(int) * N, (void **)&g.pot));
    WW_TRY(scratch(SLOT_MCF_EX, N, (void **)&g.ex));
    // per-tile state: act, pstamp, tstamp (NT each, cleared per call),
    // lists (3 x list_stride(NT)), perim_tiles (NT), tile_rej (NT x 8 B,
    // 8-byte aligned), vpart (64 x 16 x 8 B)
    unsigned int *tiles = nullptr;
    const size_t lists_end = 3 * (size_t)NT + 3 * list_stride(NT);  // perim_tiles start
    const size_t rej_at = lists_end + (size_t)NT + ((lists_end + (size_t)NT) & 1);  // 8-byte aligned
    const size_t tiles_words = rej_at + 2 * (size_t)NT;
    WW_TRY(scratch(SLOT_MCF_TILES, sizeof(unsigned int) * tiles_words + 8192 + 256, (void **)&tiles));
    RoundArgs ra;
    ra.NT = NT;
    ra.act = tiles;
    ra.pstamp = tiles + (size_t)NT;
    ra.tstamp = tiles + 2 * (size_t)NT;
    ra.lists = tiles + 3 * (size_t)NT;
    ra.perim_tiles = tiles + lists_end;
    ra.tile_rej = (unsigned long long *)(tiles + rej_at);
    ra.vpart = (unsigned long long *)(tiles + tiles_words + ((tiles_words) & 1));
    char *nodes = nullptr;
    const size_t nl_bytes = sizeof(unsigned int) * (size_t)N;
    const size_t gs_bytes = sizeof(unsigned int) * (size_t)nslots + 256;
    WW_TRY(scratch(SLOT_MCF_NODES, 4 * nl_bytes + gs_bytes + nslots + 1024, (void **)&nodes));
    unsigned int *src = (unsigned int *)nodes, *def = src + N, *src2 = def + N, *def2 = src2 + N;
    unsigned int *gsub_list = def2 + N;
    unsigned char *drop = (unsigned char *)(nodes + 4 * nl_bytes + gs_bytes);
    // counters, ground records and (several jobs) the two frames' job tables
    const size_t jobs_bytes = MULTI ? (sizeof(Job) * (size_t)nj + 255) / 256 * 256 : 0;
    const size_t cg_bytes = CTL_BYTES + sizeof(GState) * (size_t)nj;
    const size_t cg_round = (cg_bytes + 255) / 256 * 256;
    char *cg = nullptr;
    WW_TRY(scratch(SLOT_MCF_LISTS, cg_round + 2 * jobs_bytes, (void **)&cg));
    Ctl *ctl = (Ctl *)cg;
    g.gs = (GState *)(cg + CTL_BYTES);
    Job *jobs_dev[2] = {nullptr, nullptr};
    char *hc = nullptr;
    WW_TRY(host_scratch(cg_round + 2 * jobs_bytes, (void **)&hc));
    // the host's copy of the counters and ground records, in a coherent
    // pinned block that k_mirror writes after each batch of rounds, with
    // the sequence word behind it
    char *hm = nullptr;
    WW_TRY(host_mirror(cg_round + 64, (void **)&hm));
    unsigned int *const hflag = reinterpret_cast<unsigned int *>(hm + cg_round);
    __atomic_store_n(hflag, 0u, __ATOMIC_RELEASE);  // no mirror kernel is in flight here
    unsigned int mseq = 0;
    Ctl *h = (Ctl *)hm;
    GState *hg = (GState *)(hm + CTL_BYTES);
    g.jobs = nullptr;
    if (MULTI) {
        // the job tables of both frames, uploaded once (a frame reversal
        // exchanges each job's two cost planes)
        jobs_dev[0] = (Job *)(cg + cg_round);
        jobs_dev[1] = (Job *)(cg + cg_round + jobs_bytes);
        Job *hj0 = (Job *)(hc + cg_round), *hj1 = (Job *)(hc + cg_round + jobs_bytes);
        for (int k = 0; k < nj; ++k) {
            hj0[k] = jobs[k];
            hj1[k] = jobs[k];
            std::swap(hj1[k].cxp, hj1[k].cxn);
            std::swap(hj1[k].cyp, hj1[k].cyn);
        }
        WW_HIP(hipMemcpyAsync(jobs_dev[0], hc + cg_round, 2 * jobs_bytes, hipMemcpyHostToDevice, st));
        g.jobs = jobs_dev[0];
    }
    WW_HIP(hipMemcpyAsync((void *)ra.perim_tiles, ptiles.data(), sizeof(unsigned int) * ptiles.size(),
                          hipMemcpyHostToDevice, st));
    ra.nperim = (int)ptiles.size();
    // stamps start at zero on every call: rounds and passes count from 1
    WW_HIP(hipMemsetAsync(ra.act, 0, sizeof(unsigned int) * 3 * (size_t)NT, st));
    WW_HIP(hipMemsetAsync(ra.vpart, 0, 8192, st));
    WW_HIP(hipMemsetAsync(ctl, 0, cg_bytes, st));
    const int IB = (int)std::min<long long>(8192, std::max<long long>(1, ceil_div(N, 256)));
    const int nib = ceil_div(N, INIT_CHUNK);
    int *bc = nullptr;
    WW_TRY(scratch(SLOT_MCF_PART, sizeof(long long) * (size_t)std::max(3 * nib, 8192) + 256, (void **)&bc));
    // per node: the flip word of a deficit ((pass << 3) | crossed the ground
    // << 2 | chosen), and one byte with the pass of the last walk through it
    unsigned int *flip = nullptr;
    WW_TRY(scratch(SLOT_MCF_FLIP, (sizeof(unsigned int) + 1) * (size_t)N + 256, (void **)&flip));
    uint8_t *tag = reinterpret_cast<uint8_t *>(flip + N);
    // Every solve that ends well leaves all labels and path keys at
    // infinity again (each pass's potential update resets those of the
    // nodes it reached, and only those carry any), so a solve whose buffers
    // are known to be in that state does not write them.  The marks stay
    // cleared until this solve ends well.
    size_t *const clean_lab = scratch_clean(SLOT_MCF_LAB), *const clean_best = scratch_clean(SLOT_MCF_BEST);
    const size_t key_bytes = sizeof(unsigned long long) * (size_t)N;
    const size_t was_clean = std::min(*clean_lab, *clean_best);
    *clean_lab = *clean_best = 0;
    hipLaunchKernelGGL(k_mcf_init_count, dim3(nib), dim3(INIT_THREADS), 0, st, g, res_all, bc,
                       was_clean >= key_bytes ? 0 : 1);
    WW_LAUNCH_CHECK();
    const int gx = MULTI ? (int)std::min<long long>(64, std::max<long long>(1, ceil_div(N / nj, 4096)))
                         : std::max(1, ceil_div(max_arcs, 256));
    hipLaunchKernelGGL(k_init_ground, dim3(gx, nj), dim3(256), 0, st, g, res_all);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mcf_init_scan, dim3(1), dim3(1024), 0, st, nib, bc, ctl, g.gs, nj);
    WW_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mcf_init_write, dim3(nib), dim3(INIT_THREADS), 0, st, g, res_all, bc, src, def);
    WW_LAUNCH_CHECK();
    auto sync_ctl = [&]() -> ww_status {
        WW_HIP(hipMemcpyAsync(h, ctl, cg_bytes, hipMemcpyDeviceToHost, st));
        WW_TRY(wait_stream(st));
        if (h->error) return decode_error(h->error);
        return WW_OK;
    };
    // The same after a batch of rounds, without a copy or an event: the
    // device writes the counters into the host's block and then a sequence
    // word, which the host polls (about 8 us sooner than a copy and an event
    // poll).  A wait longer than 2 ms (a failed kernel among them) goes
    // through the stream wait, which reports errors.
    auto mirror_ctl = [&]() -> ww_status {
        const unsigned int seq = ++mseq;
        hipLaunchKernelGGL(k_mirror, dim3(1), dim3(256), 0, st, reinterpret_cast<const uint4 *>(ctl),
                           reinterpret_cast<uint4 *>(hm), cg_bytes, hflag, seq);
        WW_LAUNCH_CHECK();
        const auto t0 = std::chrono::steady_clock::now();
        while (__atomic_load_n(hflag, __ATOMIC_ACQUIRE) != seq) {
            if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
                WW_TRY(wait_stream(st));
                if (__atomic_load_n(hflag, __ATOMIC_ACQUIRE) != seq)
                    return fail(WW_E_DEVICE, "min-cost flow: counters did not arrive");
                break;
            }
        }
        if (h->error) return decode_error(h->error);
        return WW_OK;
    };
    // units still to route: supplies plus the grounds' surplus
    auto ground_surplus = [&]() {
        long long s = 0;
        for (int k = 0; k < nj; ++k) s += std::max<long long>(hg[k].gex, 0);
        return s;
    };
    WW_TRY(sync_ctl());
    S.supplies = (long long)h->nsrc + ground_surplus();

    const char *trace_env = getenv("WW_MCF_TRACE");
    const bool trace = trace_env && (trace_env[0] == '1' || trace_env[0] == '2');
    const char *check_env = getenv("WW_MCF_CHECK");
    const bool check = check_env && check_env[0] == '1';
    const char *count_env = getenv("WW_MCF_COUNT");
    const int count = (count_env && count_env[0] == '1') ? 1 : 0;
    // how the root walks are taken (the results do not depend on it; tests
    // compare the ways): by size (default), every walk by one thread
    // (WW_MCF_ROOTS=t), or every walk by a workgroup (WW_MCF_ROOTS=w)
    const char *roots_env = getenv("WW_MCF_ROOTS");
    const char roots_mode = roots_env ? roots_env[0] : 'a';
    const long long wave_max = roots_mode == 't' ? -1 : roots_mode == 'w' ? (1ll << 40) : ROOTS_WAVE_MAX;
    const unsigned int short_hops = roots_mode == 'w' ? 0u : RW_SHORT;
    const unsigned int defer_hops = roots_mode == 't' ? 0u : RW_LONG;
    // range guards (lowered only by tests of the error path): the largest
    // potential, and the largest distance bound of a window
    int pot_limit = POT_LIMIT;
    unsigned int bound_cap = 0xffff0000u;
    if (const char *e = getenv("WW_MCF_POT_LIMIT")) pot_limit = (int)std::min<long long>(POT_LIMIT, std::max(0ll, atoll(e)));
    if (const char *e = getenv("WW_MCF_DIST_CAP"))
        bound_cap = (unsigned int)std::min<long long>(0xffff0000ll, std::max(0ll, atoll(e)));
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
    if (check) {
        WW_HIP(hipMalloc(&cb.lab, sizeof(unsigned long long) * N));
        WW_HIP(hipMalloc(&cb.rec, sizeof(CheckRec)));
        WW_HIP(hipHostMalloc(&cb.hrec, sizeof(CheckRec)));
        WW_HIP(hipMalloc(&cb.bad, 4 * sizeof(unsigned int)));
    }
#ifndef WW_ROUNDS_PER_SYNC
#define WW_ROUNDS_PER_SYNC 12
#endif
    // relaxation rounds launched between two host checks of the list
    // lengths (a round whose list is empty returns at once)
    const int rounds_per_sync = WW_ROUNDS_PER_SYNC;
    const unsigned int h0 = (unsigned int)sp.first_hop_window, dstep0 = (unsigned int)sp.first_distance_step;
    const unsigned int full_passes = (unsigned int)sp.full_passes;
    const bool first_deficit = sp.first_deficit_after != 0;
    const long long reverse_below = sp.reverse_below;
    const unsigned long long hop_growth = (unsigned long long)sp.hop_growth;
    bool reversed = false;
    const int rev_grid =
        (int)std::min<long long>(8192, std::max<long long>(1, ceil_div(std::max(nx_all + ny_all, N), 256 * 16)));
    int pot_sign = 1;  // -1: node potentials left in the reversed frame
    auto flip_frame = [&](int nodes) -> ww_status {
        hipLaunchKernelGGL(k_reverse_frame, dim3(rev_grid), dim3(256), 0, st, g, ctl, fx_all, nx_all,
                           fy_all, ny_all, nodes);
        if (!nodes) pot_sign = -pot_sign;
        WW_LAUNCH_CHECK();
        reversed = !reversed;
        if (MULTI) g.jobs = jobs_dev[reversed ? 1 : 0];
        std::swap(g.j0.cxp, g.j0.cxn);
        std::swap(g.j0.cyp, g.j0.cyn);
        std::swap(src, def);
        std::swap(src2, def2);
        // the host's copy of the counters follows the kernel's own exchange
        // (no round trip: the next read of the block checks the error flags)
        std::swap(h->nsrc, h->ndef);
        for (int k = 0; k < nj; ++k) {
            hg[k].gex = -hg[k].gex;
            hg[k].gpot = -hg[k].gpot;
        }
        return WW_OK;
    };
    const bool trace_windows = trace_env && trace_env[0] == '2';
    // one wave of resident workgroups: more would only add workgroups that
    // find the round's list exhausted, which an empty round pays for too
    int dev = 0, ncu = 256, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sssp_round<MULTI, TW>, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 4;
    int clock_khz = 0;  // rate of the device clock that times the rounds
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || clock_khz < 1)
        clock_khz = 100000;
    (void)hipGetLastError();
    const int round_grid = (int)std::min<long long>(NT, (long long)ncu * per_cu);
    const int pot_grid = (int)std::min<unsigned int>(NT, (unsigned int)POT_GRID);
    unsigned long long nbatch = 0;  // round batches so far (their parity picks the window-end slot)
    int wslot = 0;
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
            if (h->nsrc == 0 && ground_surplus() == 0) break;
            // few units left: search from the demands instead (in the
            // reversed frame), where the plateaus that earlier passes made
            // tight around the supplies do not lie
            if (!reversed && reverse_below > 0 && (long long)h->nsrc + ground_surplus() <= reverse_below)
                WW_TRY(flip_frame(1));
        }
        const auto tp0 = std::chrono::steady_clock::now();
        const long long r0 = S.rounds, w0 = S.windows;
        const unsigned long long v0 = trace ? host_visits() : 0, it0 = h->iters, vs0 = h->vt_sum,
                                 vst0 = h->vt_stage, vsw0 = h->vt_sweep;
        const unsigned int nsrc0 = h->nsrc;
        const long long gex0 = ground_surplus();
        ++pass;
        const long long ns_h = h->nsrc, nd_h = h->ndef;  // list lengths, upper bounds
        hipLaunchKernelGGL((k_pass_init<MULTI, TW>), dim3(lgrid(std::max<long long>(ns_h, ra.nperim))), dim3(SB), 0,
                           st, g, ctl, src, ra.act, ra.lists, NT, rr, ra.perim_tiles, ra.nperim);
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
                for (int k = 0; k < rounds_per_sync; ++k) {
                    hipLaunchKernelGGL((k_sssp_round<MULTI, TW>), dim3(round_grid), dim3(256), 0, st, g, ctl, ra,
                                       rr, pass, lb, trace ? 1 : 0, k == 0 ? 1 : 0);
                    WW_LAUNCH_CHECK();
                    ++rr;
                }
                // the window-end counts after every batch, so that the batch
                // that ends the window needs no further round trip (each run
                // writes the slot of its batch parity and clears the other)
                wslot = (int)(nbatch++ & 1);
                hipLaunchKernelGGL(k_window_end, dim3(lgrid(std::max<long long>(nd_h, NT))), dim3(SB), 0,
                                   st, g, ctl, def, lb, ra.pstamp, pass, ra.tile_rej, NT, wslot, rr);
                WW_LAUNCH_CHECK();
                S.rounds += rounds_per_sync;
                if (S.rounds > 50000000)
                    return fail(WW_E_DEVICE, "min-cost flow: relaxation rounds exceeded the limit");
                WW_TRY(mirror_ctl());
                if (check) {
                    for (int q = 0; q < 3; ++q)
                        if (h->count[q][0] > list_stride(NT))
                            return fail(WW_E_DEVICE, "min-cost flow check: list %d holds %u > %zu slots", q,
                                        h->count[q][0], list_stride(NT));
                    unsigned int hb[4] = {0u, 0u, 0u, 0u};
                    WW_HIP(hipMemsetAsync(cb.bad, 0, sizeof(hb), st));
                    hipLaunchKernelGGL(k_check_lists<MULTI>,
                                       dim3((unsigned)std::min<size_t>(1024u, (list_stride(NT) + 255) / 256)),
                                       dim3(256), 0, st, g, ctl, ra.act, ra.lists, NT, rr, cb.bad);
                    WW_LAUNCH_CHECK();
                    WW_HIP(hipMemcpyAsync(hb, cb.bad, sizeof(hb), hipMemcpyDeviceToHost, st));
                    WW_HIP(hipStreamSynchronize(st));
                    if (hb[0] || hb[1] || hb[2] != h->count[rr % 3][0] || hb[3] != h->count[rr % 3][0])
                        return fail(WW_E_DEVICE,
                                    "min-cost flow check: round %u list: out of range %u, unstamped %u, "
                                    "stamped %u, read %u, count %u",
                                    rr, hb[0], hb[1], hb[2], hb[3], h->count[rr % 3][0]);
                }
                if (prev_unread) {  // the previous pass's end
                    prev_unread = false;
                    ++S.passes;
                    S.augmentations += h->prev_naug;
                    S.path_arcs += (long long)h->prev_arcs;
                    if (h->prev_naug == 0)
                        return fail(WW_E_INFEASIBLE, "min-cost flow: a pass augmented no path");
                    if (h->nsrc == 0 && ground_surplus() == 0) {
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
            const long long units = (long long)h->nsrc + ground_surplus();
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
            hipLaunchKernelGGL(k_requeue_pending<MULTI>, dim3(tg), dim3(SB), 0, st, g, ctl, ra.pstamp, pass,
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
        // the pass's final ground labels and excesses: a ground's predecessor
        // is only needed when it is a settled deficit, and subtrees hang off
        // a ground only while it is a source.
        bool ground_deficit = false, ground_source = false;
        for (int k = 0; k < nj; ++k) {
            ground_deficit |= hg[k].glab <= lb && hg[k].gex <= 0;
            ground_source |= hg[k].gex > 0;
        }
        const int pg = (int)std::min<long long>(1024, ceil_div(max_arcs, SB));
        if (ground_deficit) {
            hipLaunchKernelGGL(k_ground_pred, dim3(pg, nj), dim3(SB), 0, st, g, lb);
            WW_LAUNCH_CHECK();
        }
        // few walks: one workgroup each; more: one thread each, the long
        // ones (listed in def2, free until the compaction) one workgroup each
        if (nd_h + nj <= wave_max) {
            hipLaunchKernelGGL(k_roots_wave<MULTI>, dim3((unsigned)std::min<long long>(nd_h + nj, 1ll << 30)),
                               dim3(64 * RW_WAVES), 0, st, g, ctl, def, lb, gsub_list, flip, tag, pass,
                               (const unsigned int *)nullptr, short_hops);
        } else {
            hipLaunchKernelGGL(k_roots<MULTI>, dim3(lgrid(nd_h + nj)), dim3(SB), 0, st, g, ctl, def, lb,
                               gsub_list, flip, tag, pass, def2, defer_hops);
            WW_LAUNCH_CHECK();
            if (defer_hops)
                hipLaunchKernelGGL(k_roots_wave<MULTI>, dim3((unsigned)std::min<long long>(ROOTS_WAVE_GRID, nd_h)),
                                   dim3(64 * RW_WAVES), 0, st, g, ctl, def, lb, gsub_list, flip, tag, pass,
                                   (const unsigned int *)def2, short_hops);
        }
        WW_LAUNCH_CHECK();
        if (ground_source) {
            hipLaunchKernelGGL(k_gsub_select, dim3(pg, nj), dim3(SB), 0, st, g, gsub_list, drop);
            WW_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_augment<MULTI>, dim3(lgrid(ns_h + nslots)), dim3(SB), 0, st, g, ctl, src,
                           gsub_list, drop, flip, pass, nslots);
        WW_LAUNCH_CHECK();
        if (check)
            WW_HIP(hipMemcpyAsync(cb.lab, g.lab, sizeof(unsigned long long) * N, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL((k_potentials<MULTI, TW>), dim3(pot_grid), dim3(SB), 0, st, g, ctl, ra.tstamp, pass, NT,
                           lb, flip, tag, count, pot_limit);
        WW_LAUNCH_CHECK();
        if (check) {
            WW_HIP(hipMemsetAsync(cb.rec, 0, sizeof(CheckRec), st));
            hipLaunchKernelGGL(k_check_rc, dim3(std::min(IB, 2048), nj), dim3(256), 0, st, g, cb.lab, cb.rec);
            WW_LAUNCH_CHECK();
            WW_HIP(hipMemcpyAsync(cb.hrec, cb.rec, sizeof(CheckRec), hipMemcpyDeviceToHost, st));
            WW_HIP(hipStreamSynchronize(st));
            if (cb.hrec->found) {
                auto pl = [](unsigned long long l) {
                    return l == LINF ? std::string("inf") :
                        std::to_string(l >> 32) + "/" + std::to_string((l >> 3) & 0x1fffffff) + "/" + std::to_string(l & 7);
                };
                const CheckRec &c = *cb.hrec;
                fprintf(stderr,
                        "[ww-mcf-check] pass %lld lb %u/%u: arc kind %d u %lld v %lld rc %lld pot %lld %lld "
                        "labels %s %s flow %d c+ %d c- %d\n",
                        (long long)S.passes + 1, (unsigned)(lb >> 32), (unsigned)((lb >> 3) & 0x1fffffff),
                        c.kind, c.u, c.v, c.rc, c.pu, c.pv, pl(c.lu).c_str(), pl(c.lv).c_str(), c.f, c.cp, c.cn);
                return fail(WW_E_DEVICE, "min-cost flow check failed (details on stderr)");
            }
        }
        hipLaunchKernelGGL(k_compact, dim3(lgrid(ns_h + nd_h)), dim3(SB), 0, st, g, ctl, src, def, src2, def2);
        WW_LAUNCH_CHECK();
        std::swap(src, src2);
        std::swap(def, def2);
        if ((reversed || reverse_below <= 0) && !trace && !check) {
            prev_unread = true;
            continue;
        }
        WW_TRY(mirror_ctl());
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
    if (reversed) WW_TRY(flip_frame(0));
    {
        // each job's cost from its flows (original frame)
        long long mx_e = 0;
        for (int k = 0; k < nj; ++k)
            mx_e = std::max<long long>(mx_e, (long long)jobs[k].R * jobs[k].n + (long long)(jobs[k].R + 1) * jobs[k].C);
        const int tcg = (int)std::min<long long>(MULTI ? 256 : 8192, std::max<long long>(1, ceil_div(mx_e, 256 * 8)));
        hipLaunchKernelGGL(k_total_cost, dim3(tcg, nj), dim3(256), 0, st, g);
        WW_LAUNCH_CHECK();
    }
    if (pot_out && !MULTI) {
        hipLaunchKernelGGL(k_export_pot, dim3(IB), dim3(256), 0, st, g.pot, g.gs, N, pot_out, pot_sign);
        WW_LAUNCH_CHECK();
    }
    WW_TRY(sync_ctl());
    // the rounds' time: batches timed on the device clock (timing events
    // between the launches delayed the next kernel by several microseconds)
    S.relax_ms = (double)h->relax_ticks / (double)clock_khz;
    for (int k = 0; k < nj; ++k) *mj[k].total = hg[k].total_cost;
    S.tile_visits = (long long)host_visits();
    long long mxp = h->max_pot;
    for (int k = 0; k < nj; ++k) mxp = std::max<long long>(mxp, hg[k].gpot);
    S.max_potential = mxp;
    S.settled_nodes = count ? (long long)h->settled : -1;
    S.arcs_scanned = count ? (long long)h->scanned : -1;
    S.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    last_mcf_stats() = S;
    if (stats) *stats = S;
    *clean_lab = *clean_best = std::max(was_clean, key_bytes);
    return WW_OK;
}

// The solve for the schedule's tile shape (checked by check_mcf_params).
template <bool MULTI>
static ww_status solve_shape(const std::vector<McfJob> &mj, const int8_t *res_all, int8_t *fx_all,
                             int8_t *fy_all, int64_t *pot_out, ww_mcf_stats *stats,
                             const ww_mcf_params &sp, hipStream_t st) {
    switch (sp.tile_cols) {
        case 16: return solve<MULTI, 16>(mj, res_all, fx_all, fy_all, pot_out, stats, sp, st);
        case 32: return solve<MULTI, 32>(mj, res_all, fx_all, fy_all, pot_out, stats, sp, st);
        case 64: return solve<MULTI, 64>(mj, res_all, fx_all, fy_all, pot_out, stats, sp, st);
        default: return fail(WW_E_INVALID_ARG, "tile_cols must be 16, 32 or 64");
    }
}

ww_status mcf_impl(const int8_t *res, int m, int n, const int16_t *cxp, const int16_t *cxn,
                   const int16_t *cyp, const int16_t *cyn, int8_t *dkx, int8_t *dky,
                   int64_t *pot_out, int64_t *total, ww_mcf_stats *stats, hipStream_t st,
                   const ww_mcf_params *sched) {
    const long long nx = (long long)m * (n - 1), ny = (long long)(m - 1) * n;
    if (nx > 0) WW_HIP(hipMemsetAsync(dkx, 0, nx, st));
    if (ny > 0) WW_HIP(hipMemsetAsync(dky, 0, ny, st));
    const int R = m - 1, C = n - 1;
    if (R < 1 || C < 1) {
        ww_mcf_stats S;
        memset(&S, 0, sizeof(S));
        last_mcf_stats() = S;
        if (pot_out) WW_HIP(hipMemsetAsync(pot_out, 0, sizeof(int64_t), st));
        WW_HIP(hipStreamSynchronize(st));
        *total = 0;
        if (stats) *stats = S;
        return WW_OK;
    }
    if ((long long)R * C >= (1ll << 29)) return fail(WW_E_INVALID_ARG, "more than 2^29 loops");
    const ww_mcf_params sp = sched ? *sched : process_mcf_params();
    std::vector<McfJob> one(1);
    one[0] = McfJob{m, n, res, cxp, cxn, cyp, cyn, dkx, dky, total};
    return solve_shape<false>(one, res, dkx, dky, pot_out, stats, sp, st);
}

ww_status mcf_multi_impl(const std::vector<McfJob> &jobs, const int8_t *res_all, int8_t *fx_all,
                         int8_t *fy_all, ww_mcf_stats *stats, const ww_mcf_params &sp, hipStream_t st) {
    if (jobs.empty()) return WW_OK;
    if (jobs.size() > 256) return fail(WW_E_INVALID_ARG, "more than 256 jobs in one solve");
    long long nx = 0, ny = 0;
    for (const McfJob &q : jobs) {
        if (q.m < 2 || q.n < 2) return fail(WW_E_INVALID_ARG, "multi-job solve: every job needs loops");
        if ((long long)(q.m - 1) * (q.n - 1) >= (1ll << 29)) return fail(WW_E_INVALID_ARG, "more than 2^29 loops");
        const int tw = sp.tile_cols, th = 1024 / std::max(1, tw);
        if ((long long)ceil_div(q.m - 1, th) * ceil_div(q.n - 1, std::max(1, tw)) >= (1ll << 24))
            return fail(WW_E_INVALID_ARG, "more than 2^24 tiles in one job");
        nx += (long long)q.m * (q.n - 1);
        ny += (long long)(q.m - 1) * q.n;
    }
    WW_HIP(hipMemsetAsync(fx_all, 0, nx, st));
    WW_HIP(hipMemsetAsync(fy_all, 0, ny, st));
    if (jobs.size() == 1) return solve_shape<false>(jobs, res_all, fx_all, fy_all, nullptr, stats, sp, st);
    return solve_shape<true>(jobs, res_all, fx_all, fy_all, nullptr, stats, sp, st);
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
    p->tile_cols = 32;
}

ww_status ww_set_mcf_params(const ww_mcf_params *p) {
    ww::clear_error();
    if (!p) return ww::fail(WW_E_INVALID_ARG, "window schedule out of range");
    WW_TRY(ww::check_mcf_params(*p));
    ww::g_first_hops.store(p->first_hop_window);
    ww::g_first_dstep.store(p->first_distance_step);
    ww::g_full_passes.store(p->full_passes);
    ww::g_first_deficit.store(p->first_deficit_after);
    ww::g_reverse_below.store(p->reverse_below);
    ww::g_hop_growth.store(p->hop_growth);
    ww::g_tile_cols.store(p->tile_cols);
    return WW_OK;
}

void ww_get_mcf_params(ww_mcf_params *p) {
    if (!p) return;
    *p = ww::process_mcf_params();
}

}  // extern "C"
