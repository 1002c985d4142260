// Per-edge integer arc costs (Section II-B).
//
// k_edge_costs_stream (box half-width h <= 4, table of at most 8192
// entries): waves stream down column strips (described at the kernel).
// k_edge_costs (any h up to 8, any table): one workgroup per 16 x 64 pixel
// tile.  The tile's wrapped
// phase and mask, plus a halo of h+1, are staged in LDS; each x- and y-edge
// sample gets its wrapped gradient in 2^-20 rad fixed point; separable
// integer box sums give the clipped (2h+1)^2 mean slope of every output edge,
// which selects the slope bin; min(coh_u, coh_v) selects the coherence bin;
// the table gather gives c+ and its mirror c-.  Masked edges cost 0.  Edges
// steeper than the threshold are appended (wave-aggregated) to a candidate
// list with the key (|d| as IEEE bits, edge id) for the steep rule.
//
// Steep rule: at most floor(pct * valid_edges / 100) candidates get cost 0,
// the largest |d| first and ties by the smaller edge id (x-edges row-major,
// then y-edges row-major).  The selection is an exact 96-bit radix select
// over (|d| bits, ~id) decided on the device, so the zeroed set does not
// depend on the order in which candidates were appended.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ww_internal.h"

namespace ww {

constexpr int CT_H = 16;   // tile rows
constexpr int CT_W = 64;   // tile cols
constexpr int CT_THREADS = 256;


// Steep-rule selection.  A pre-pass counts the valid edges and histograms
// the candidates (|d| > threshold) into SC_BINS coarse bins of their key,
// bin = (bits(|d|) - bits(threshold) - 1) >> shift (the bits of non-negative
// doubles order like their values, and every candidate key exceeds
// bits(threshold)).  The bins above the boundary bin bstar hold fewer than
// cap candidates: the cost kernels zero those edges themselves and append
// only the boundary bin's candidates, whose remaining places an exact radix
// select over (|d| bits, ~edge id) then fills.
constexpr int SC_BINS = 4096;
constexpr int SC_THREADS = 1024;
constexpr int SC_SMALL = 65536;  // boundary sets up to this size: one-workgroup select

struct SteepState {
    unsigned long long nvalid, ncand, cap, remaining;
    unsigned long long prefix_hi, mask_hi;
    unsigned int prefix_lo, mask_lo;
    unsigned int done;  // the threshold is known before the last digit
    unsigned int hist[256];
    unsigned long long base;   // bits of the threshold
    int shift;                 // coarse bin width 2^shift key units
    int bstar;                 // boundary bin; -1: every candidate is selected, SC_BINS: none
    unsigned long long above;  // candidates in bins above bstar
    unsigned long long ncand_all;
    // keys >= kzero lie above the boundary bin (selected: cost zeroed in
    // place); keys in [kbound, kzero) lie in it (appended for the select)
    unsigned long long kzero, kbound;
    unsigned int chist[SC_BINS];
};

__device__ __forceinline__ int steep_coarse_bin(unsigned long long kb, unsigned long long base, int shift) {
    const unsigned long long b = (kb - base - 1ull) >> shift;
    return b > (unsigned long long)(SC_BINS - 1) ? SC_BINS - 1 : (int)b;
}

__device__ __forceinline__ int coh_bin(float c, int NG) {
    double g = (double)c;
    if (!(g > 0.0)) g = 0.0;  // NaN and negatives read as 0
    if (g > 1.0) g = 1.0;
    int b = (int)floor(g * NG);
    return b > NG - 1 ? NG - 1 : b;
}

// Interpolated lookup (Section II-B, the table read between its entries):
// positions relative to the bin centres in 2^-16 bin units, a cell index and
// a 16-bit fraction per axis, clamped to the outermost centres, and the
// bilinear blend of the four surrounding entries rounded down.
__device__ __forceinline__ int64_t coh_pos16(float c, int NG) {
    double g = (double)c;
    if (!(g > 0.0)) g = 0.0;
    if (g > 1.0) g = 1.0;
    return (int64_t)floor(g * (double)NG * 65536.0) - 32768;
}

template <typename TP>
__device__ __forceinline__ int16_t lut_blend(TP T, int NA, int NG, int64_t t16, int64_t u16) {
    int64_t ia = t16 >> 16, ig = u16 >> 16;
    int64_t fa = t16 - (ia << 16), fg = u16 - (ig << 16);
    if (ia < 0) { ia = 0; fa = 0; }
    if (ia >= NA - 1) { ia = NA - 1; fa = 0; }
    if (ig < 0) { ig = 0; fg = 0; }
    if (ig >= NG - 1) { ig = NG - 1; fg = 0; }
    const int a0 = (int)ia, a1 = a0 + 1 < NA ? a0 + 1 : a0;
    const int g0 = (int)ig * NA, g1 = ((int)ig + 1 < NG ? (int)ig + 1 : (int)ig) * NA;
    const int64_t r0 = (int64_t)T[g0 + a0] * (65536 - fa) + (int64_t)T[g0 + a1] * fa;
    const int64_t r1 = (int64_t)T[g1 + a0] * (65536 - fa) + (int64_t)T[g1 + a1] * fa;
    return (int16_t)((r0 * (65536 - fg) + r1 * fg) >> 32);
}

// Table lookup of the tile kernel: num / den is the slope position
// (S + K P) NA / (2 K P) with num >= 0 for phases in [-pi, pi].
__device__ __forceinline__ void tile_lookup(const int16_t *__restrict__ lut, int NA, int NG,
                                            int64_t num, int64_t den, float g, int interp,
                                            int16_t &cp, int16_t &cn) {
    if (interp) {
        const int64_t t16 = (num * 65536) / den - 32768;
        const int64_t u16 = coh_pos16(g, NG);
        cp = lut_blend(lut, NA, NG, t16, u16);
        cn = lut_blend(lut, NA, NG, (int64_t)(NA - 1) * 65536 - t16, u16);
        return;
    }
    int ba = (int)floor((double)num / (double)den);
    ba = ba < 0 ? 0 : (ba > NA - 1 ? NA - 1 : ba);
    const int bg = coh_bin(g, NG);
    cp = lut[bg * NA + ba];
    cn = lut[bg * NA + (NA - 1 - ba)];
}

__global__ __launch_bounds__(CT_THREADS) void k_edge_costs(
    const float *__restrict__ psi, const float *__restrict__ coh, const uint8_t *__restrict__ valid,
    int m, int n, const int16_t *__restrict__ lut, int NA, int NG, int h, double steep_thresh,
    int steep_on, int interp, int16_t *__restrict__ cxp, int16_t *__restrict__ cxn, int16_t *__restrict__ cyp,
    int16_t *__restrict__ cyn, unsigned long long *__restrict__ cand_key,
    unsigned int *__restrict__ cand_id, SteepState *__restrict__ st) {
    extern __shared__ unsigned char smem[];
    const int i0 = blockIdx.y * CT_H, j0 = blockIdx.x * CT_W;
    const int PR = CT_H + 2 * h + 1, PC = CT_W + 2 * h + 1;  // pixel tile
    const int ER = CT_H + 2 * h, EC = CT_W + 2 * h;          // edge samples
    float *ph = (float *)smem;                               // PR x PC
    int *qx = (int *)(ph + PR * PC);                         // ER x EC
    int *qy = qx + ER * EC;                                  // ER x EC
    int *sx = qy + ER * EC;                                  // ER x CT_W row sums
    int *sy = sx + ER * CT_W;
    unsigned short *kx = (unsigned short *)(sy + ER * CT_W); // ER x CT_W row counts
    unsigned short *ky = kx + ER * CT_W;
    unsigned char *vd = (unsigned char *)(ky + ER * CT_W);   // PR x PC pixel validity
    unsigned char *ex = vd + PR * PC;                        // ER x EC x-sample validity
    unsigned char *ey = ex + ER * EC;
    const int tid = threadIdx.x;

    // 1. stage phase (0 at invalid pixels) and validity; outside = invalid
    for (int t = tid; t < PR * PC; t += CT_THREADS) {
        const int r = t / PC, c = t % PC;
        const int i = i0 - h + r, j = j0 - h + c;
        float v = 0.f;
        unsigned char ok = 0;
        if (i >= 0 && i < m && j >= 0 && j < n) {
            const int64_t a = (int64_t)i * n + j;
            ok = valid ? (valid[a] != 0) : 1;
            v = ok ? psi[a] : 0.f;
        }
        ph[t] = v;
        vd[t] = ok;
    }
    __syncthreads();
    // 2. fixed-point wrapped gradients of every sample in the window
    for (int t = tid; t < ER * EC; t += CT_THREADS) {
        const int r = t / EC, c = t % EC;
        const int p = r * PC + c;
        // x-sample (r, c): pixel (r,c) -> (r,c+1)
        {
            const unsigned char ok = vd[p] & vd[p + 1];
            int q = 0;
            if (ok) {
                double diff = (double)ph[p + 1] - (double)ph[p];
                double d = diff - TWO_PI_D * wrap_cycles(diff);
                q = (int)floor(d * 1048576.0);
            }
            qx[t] = q;
            ex[t] = ok;
        }
        // y-sample (r, c): pixel (r,c) -> (r+1,c)
        {
            const unsigned char ok = vd[p] & vd[p + PC];
            int q = 0;
            if (ok) {
                double diff = (double)ph[p + PC] - (double)ph[p];
                double d = diff - TWO_PI_D * wrap_cycles(diff);
                q = (int)floor(d * 1048576.0);
            }
            qy[t] = q;
            ey[t] = ok;
        }
    }
    __syncthreads();
    // 3. horizontal window sums for the output columns
    const int W = 2 * h + 1;
    for (int t = tid; t < ER * CT_W; t += CT_THREADS) {
        const int r = t / CT_W, c = t % CT_W;
        int s1 = 0, s2 = 0, k1 = 0, k2 = 0;
        const int base = r * EC + c;  // sample columns c .. c+2h
        for (int d = 0; d < W; ++d) {
            s1 += qx[base + d];
            k1 += ex[base + d];
            s2 += qy[base + d];
            k2 += ey[base + d];
        }
        sx[t] = s1;
        kx[t] = (unsigned short)k1;
        sy[t] = s2;
        ky[t] = (unsigned short)k2;
    }
    __syncthreads();
    // 4. vertical window sums, bins, table gather, steep candidates
    const unsigned long long kzero = st->kzero, kbound = st->kbound;
    const int nx_cols = n - 1;
    const int64_t nx_total = (int64_t)m * (n - 1);
    int nvalid = 0;
    const int c = tid % CT_W;
    const int rstart = tid / CT_W;
    constexpr int ITERS = CT_H / (CT_THREADS / CT_W);
    unsigned long long ckey[2 * ITERS];
    unsigned int cid[2 * ITERS];
    unsigned int cmask = 0;  // fixed slots 2*it (x-edge) and 2*it+1 (y-edge)
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const int r = rstart + it * (CT_THREADS / CT_W);
        const int i = i0 + r, j = j0 + c;
        int64_t S1 = 0, S2 = 0;
        int K1 = 0, K2 = 0;
        for (int d = 0; d < W; ++d) {
            S1 += sx[(r + d) * CT_W + c];
            K1 += kx[(r + d) * CT_W + c];
            S2 += sy[(r + d) * CT_W + c];
            K2 += ky[(r + d) * CT_W + c];
        }
        const int sc = (r + h) * EC + (c + h);  // own sample
        // ---- x-edge hx(i, j)
        if (i < m && j < n - 1) {
            const int64_t idx_x = (int64_t)i * nx_cols + j;
            int16_t cp = 0, cn = 0;
            if (ex[sc]) {
                ++nvalid;
                const int64_t num = (S1 + (int64_t)K1 * PI_FIX) * NA;
                const int64_t den = 2 * (int64_t)K1 * PI_FIX;
                const int64_t a = (int64_t)i * n + j;
                float c0 = coh[a], c1 = coh[a + 1];
                c0 = (c0 != c0) ? 0.f : c0;  // NaN reads as 0 (fminf would drop it)
                c1 = (c1 != c1) ? 0.f : c1;
                tile_lookup(lut, NA, NG, num, den, fminf(c0, c1), interp, cp, cn);
                const int p = (r + h) * PC + (c + h);
                double diff = (double)ph[p + 1] - (double)ph[p];
                double dd = fabs(diff - TWO_PI_D * wrap_cycles(diff));
                if (steep_on && dd > steep_thresh) {
                    const unsigned long long kb = (unsigned long long)__double_as_longlong(dd);
                    if (kb >= kzero) {
                        cp = 0;
                        cn = 0;
                    } else if (kb >= kbound) {
                        ckey[2 * it] = kb;
                        cid[2 * it] = (unsigned int)idx_x;
                        cmask |= 1u << (2 * it);
                    }
                }
            }
            cxp[idx_x] = cp;
            cxn[idx_x] = cn;
        }
        // ---- y-edge vy(i, j)
        if (i < m - 1 && j < n) {
            const int64_t idx_y = (int64_t)i * n + j;
            int16_t cp = 0, cn = 0;
            if (ey[sc]) {
                ++nvalid;
                const int64_t num = (S2 + (int64_t)K2 * PI_FIX) * NA;
                const int64_t den = 2 * (int64_t)K2 * PI_FIX;
                const int64_t a = (int64_t)i * n + j;
                float c0 = coh[a], c1 = coh[a + n];
                c0 = (c0 != c0) ? 0.f : c0;
                c1 = (c1 != c1) ? 0.f : c1;
                tile_lookup(lut, NA, NG, num, den, fminf(c0, c1), interp, cp, cn);
                const int p = (r + h) * PC + (c + h);
                double diff = (double)ph[p + PC] - (double)ph[p];
                double dd = fabs(diff - TWO_PI_D * wrap_cycles(diff));
                if (steep_on && dd > steep_thresh) {
                    const unsigned long long kb = (unsigned long long)__double_as_longlong(dd);
                    if (kb >= kzero) {
                        cp = 0;
                        cn = 0;
                    } else if (kb >= kbound) {
                        ckey[2 * it + 1] = kb;
                        cid[2 * it + 1] = (unsigned int)(nx_total + idx_y);
                        cmask |= 1u << (2 * it + 1);
                    }
                }
            }
            cyp[idx_y] = cp;
            cyn[idx_y] = cn;
        }
    }
    // one reservation per block for the boundary candidates
    __shared__ int red_cand[CT_THREADS / 64];
    __shared__ unsigned long long cand_base;
    const int lane = tid & 63, wid = tid >> 6;
    const int ncand = __popc(cmask);
    (void)nvalid;
    int incl = ncand;
    for (int off = 1; off < 64; off <<= 1) {
        int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) red_cand[wid] = incl;
    __syncthreads();
    if (tid == 0) {
        int tc = 0;
        for (int w = 0; w < CT_THREADS / 64; ++w) tc += red_cand[w];
        cand_base = tc ? atomicAdd(&st->ncand, (unsigned long long)tc) : 0ull;
    }
    __syncthreads();
    if (ncand) {
        unsigned long long pos = cand_base + (unsigned long long)(incl - ncand);
        for (int w = 0; w < wid; ++w) pos += red_cand[w];
#pragma unroll
        for (int k = 0; k < 2 * ITERS; ++k) {
            if (cmask & (1u << k)) {
                cand_key[pos] = ckey[k];
                cand_id[pos] = cid[k];
                ++pos;
            }
        }
    }
}

// ------------------------------------------------ streaming variant (h <= 4)
//
// One wave per strip of OW = 63 - 2H output columns, walking down a segment
// of CS_ROWS output rows.  Lane l holds sample column c = js - H + l; every
// pixel row is loaded once (coalesced, W = 2H + 1 rows ahead), the
// horizontal window sums come from wave shuffles and the vertical ones from
// the last W rows' sums, so the only re-read data are the 2H halo columns of
// a strip and the 2H halo rows of a segment.  The row loop is unrolled by W,
// so that every per-row register history (loads in flight, window rows,
// delayed samples) rotates at compile time instead of by register moves;
// rows are addressed through a wave-uniform row base plus the lane's fixed
// column offset.  Steep candidates are buffered per wave in LDS and
// appended with one atomic reservation per CS_CB entries.  Same arithmetic
// as k_edge_costs, so the outputs are identical.
#ifndef WW_CS_ROWS
#define WW_CS_ROWS 64
#endif
constexpr int CS_ROWS = WW_CS_ROWS;  // output rows per wave
constexpr int CS_CB = 256;
constexpr int CS_WAVES = 4;
constexpr int CS_LUT_MAX = 8192;  // table entries staged in LDS (16 KB)

struct CandBuf {
    unsigned long long key[CS_CB];
    unsigned int id[CS_CB];
};

__device__ __forceinline__ void cand_flush(CandBuf &b, int &cnt, int lane,
                                           unsigned long long *__restrict__ cand_key,
                                           unsigned int *__restrict__ cand_id, SteepState *st) {
    __builtin_amdgcn_wave_barrier();
    unsigned long long base = 0;
    if (lane == 0 && cnt) base = atomicAdd(&st->ncand, (unsigned long long)cnt);
    base = __shfl(base, 0, 64);
    for (int k = lane; k < cnt; k += 64) {
        cand_key[base + k] = b.key[k];
        cand_id[base + k] = b.id[k];
    }
    __builtin_amdgcn_wave_barrier();
    cnt = 0;
}

__device__ __forceinline__ void cand_push(CandBuf &b, int &cnt, int lane, bool has,
                                          unsigned long long key, unsigned int id,
                                          unsigned long long *__restrict__ cand_key,
                                          unsigned int *__restrict__ cand_id, SteepState *st) {
    const unsigned long long bal = __ballot(has);
    if (!bal) return;
    if (cnt + 64 > CS_CB) cand_flush(b, cnt, lane, cand_key, cand_id, st);
    if (has) {
        const int off = __popcll(bal & ((1ull << lane) - 1ull));
        b.key[cnt + off] = key;
        b.id[cnt + off] = id;
    }
    cnt += __popcll(bal);
}

// Slope bin floor((S + K P) NA / (2 K P)) clamped to [0, NA-1], P = PI_FIX,
// for 1 <= K <= 81 samples of sum S (every sample lies in [-P, P), so
// 0 <= u = S + K P < 2 K P < 2^30): a float estimate of u NA / (2 K P) from
// the hardware reciprocal (relative error near 2^-22, far below one unit of
// a quotient under 4096) and one exact correction step.  The remainder
// e = u NA - t 2 K P of an estimate t within one of the quotient lies in
// [-2KP, 4KP), well inside 32 bits, so it is formed in wrapping 32-bit
// arithmetic: equal to the true remainder.
__device__ __forceinline__ int slope_bin(int S, int K, int NA) {
    const int u = S + K * (int)PI_FIX;
    const int den = 2 * K * (int)PI_FIX;
    const float est = (float)u * ((float)NA * __builtin_amdgcn_rcpf((float)den));
    int t = (int)floorf(est);
    const int e = (int)((unsigned int)u * (unsigned int)NA - (unsigned int)t * (unsigned int)den);
    t += (e >= den) - (e < 0);
    return t < 0 ? 0 : (t > NA - 1 ? NA - 1 : t);
}

// Slope position of the interpolated lookup, floor((S + K P) NA 2^16 /
// (2 K P)) - 2^15: the quotient q and remainder e of u NA / (2 K P) as in
// slope_bin (unclamped), then floor(e 2^16 / (2 K P)) < 2^16 by the same
// float estimate and exact correction (remainders again within 32 bits).
__device__ __forceinline__ int64_t slope_pos16(int S, int K, int NA) {
    const int u = S + K * (int)PI_FIX;
    const int den = 2 * K * (int)PI_FIX;
    const float rden = __builtin_amdgcn_rcpf((float)den);
    int q = (int)floorf((float)u * ((float)NA * rden));
    int e = (int)((unsigned int)u * (unsigned int)NA - (unsigned int)q * (unsigned int)den);
    const int c = (e >= den) - (e < 0);
    q += c;
    e -= c * den;
    int f = (int)floorf((float)e * (65536.f * rden));
    const int e2 = (int)((unsigned int)e * 65536u - (unsigned int)f * (unsigned int)den);
    f += (e2 >= den) - (e2 < 0);
    return (int64_t)q * 65536 + f - 32768;
}

// Coherence clamped to [0, 1], NaN read as 0.
__device__ __forceinline__ float coh_clamp(float c) {
    return (c > 0.f) ? (c < 1.f ? c : 1.f) : 0.f;  // NaN fails c > 0
}

// Coherence bin and interpolation position.  With NG a power of two the
// product g NG (and g NG 2^16) is exact in float, so float floors equal the
// double ones of coh_bin / coh_pos16.
template <bool NGP2>
__device__ __forceinline__ int coh_bin_s(float g, int NG) {
    if constexpr (NGP2) {
        const int b = (int)floorf(coh_clamp(g) * (float)NG);
        return b > NG - 1 ? NG - 1 : b;
    } else {
        return coh_bin(g, NG);
    }
}
template <bool NGP2>
__device__ __forceinline__ int64_t coh_pos16_s(float g, int NG) {
    if constexpr (NGP2) return (int64_t)floorf(coh_clamp(g) * ((float)NG * 65536.f)) - 32768;
    else return coh_pos16(g, NG);
}

template <bool INTERP, bool NGP2>
__device__ __forceinline__ void stream_lookup(const int16_t *slut, int NA, int NG, int S, int K,
                                              float g, int16_t &cp, int16_t &cn) {
    if constexpr (INTERP) {
        const int64_t t16 = slope_pos16(S, K, NA);
        const int64_t u16 = coh_pos16_s<NGP2>(g, NG);
        cp = lut_blend(slut, NA, NG, t16, u16);
        cn = lut_blend(slut, NA, NG, (int64_t)(NA - 1) * 65536 - t16, u16);
    } else {
        const int ba = slope_bin(S, K, NA);
        const int bg = coh_bin_s<NGP2>(g, NG);
        cp = slut[bg * NA + ba];
        cn = slut[bg * NA + (NA - 1 - ba)];
    }
}

template <int H, bool INTERP, bool NGP2>
__global__ __launch_bounds__(64 * CS_WAVES) void k_edge_costs_stream(
    const float *__restrict__ psi, const float *__restrict__ coh, const uint8_t *__restrict__ valid,
    int m, int n, const int16_t *__restrict__ lut, int NA, int NG, double steep_thresh,
    int16_t *__restrict__ cxp, int16_t *__restrict__ cxn, int16_t *__restrict__ cyp,
    int16_t *__restrict__ cyn, unsigned long long *__restrict__ cand_key,
    unsigned int *__restrict__ cand_id, SteepState *__restrict__ st, int nstrips, int nwaves) {
    constexpr int OW = 63 - 2 * H;
    constexpr int W = 2 * H + 1;  // window rows
    // history depth = loads in flight = unroll factor: the window, and at
    // least the H + 2 rows of coherence a y-edge looks back over
    constexpr int U = W > H + 2 ? W : H + 2;
    __shared__ CandBuf cbuf[CS_WAVES];
    __shared__ int16_t slut[CS_LUT_MAX];
    for (int t = threadIdx.x; t < NA * NG; t += 64 * CS_WAVES) slut[t] = lut[t];
    __syncthreads();
    // the wave index is the same in every lane: made explicit, so that the
    // wave's strip, segment and row bases live in scalar registers
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = blockIdx.x * CS_WAVES + wv;
    if (gw >= nwaves) return;  // whole waves only: no workgroup barrier below
    CandBuf &cb = cbuf[wv];
    int ccnt = 0;
    const int strip = gw % nstrips, seg = gw / nstrips;
    const int js = strip * OW;
    const int r0 = seg * CS_ROWS, r1 = min(r0 + CS_ROWS, m);
    const int c = js - H + lane;  // sample / pixel column of this lane
    const bool col_in = c >= 0 && c < n;
    const unsigned int cc_off = col_in ? (unsigned int)c : 0u;  // in-range column for the loads
    const int j = c;                    // output column of an output lane
    const bool out_lane = lane >= H && lane < H + OW;
    const int nx_cols = n - 1;
    const unsigned int nx_total = (unsigned int)m * (unsigned int)(n - 1);
    const unsigned long long kzero = st->kzero, kbound = st->kbound;

    // per-row histories, slot (row index mod U); with the loop unrolled by U
    // every slot index below is a compile-time constant
    int hx[U], hy[U];            // packed horizontal window sums 16 S + K
    double dx[U], dy[U];         // wrapped gradients of the samples
    bool okx_r[U], oky_r[U];     // sample validity
    float ch[U];                 // coherence of the pixel row
    float p_q[U], c_q[U];        // loads in flight
    uint8_t v_q[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        hx[k] = hy[k] = 0;
        dx[k] = dy[k] = 0.0;
        okx_r[k] = oky_r[k] = false;
        ch[k] = 0.f;
    }
    double ph_prev = 0.0;
    bool vd_prev = false;
    int nvalid = 0;
    int RSx = 0, RKx = 0, RSy = 0, RKy = 0;  // vertical sums of the last W rows

    const int i_start = max(0, r0 - H);
    const int i_last = r1 + H;  // inclusive; rows >= m are absent (zero samples)
    // Loads of row i, issued unconditionally from a row inside the image
    // (the last one for rows past it) and zeroed afterwards, so that the
    // histories stay straight-line code.
    auto fetch = [&](int i, float &p, uint8_t &v, float &cc) {
        const bool use = i < m && i <= i_last;
        const size_t row = (size_t)min(i, m - 1) * (size_t)n;  // wave-uniform row base
        const uint8_t vv = valid ? (valid + row)[cc_off] : (uint8_t)1;
        const float pp = (psi + row)[cc_off];
        const float c2 = (coh + row)[cc_off];
        v = use ? vv : (uint8_t)0;
        p = use ? pp : 0.f;
        cc = use ? c2 : 0.f;
    };
#pragma unroll
    for (int k = 0; k < U; ++k) fetch(i_start + k, p_q[k], v_q[k], c_q[k]);
    for (int ib = i_start; ib <= i_last; ib += U) {
#pragma unroll
        for (int t = 0; t < U; ++t) {
            const int i = ib + t;
            if (i > i_last) continue;  // (so do the later slots: the trip count stays U)
            const bool row_in = i < m;
            const float p = p_q[t], cc = c_q[t];
            const uint8_t v = v_q[t];
            fetch(i + U, p_q[t], v_q[t], c_q[t]);
            const bool vd = row_in && col_in && v != 0;
            const float pf = vd ? p : 0.f;
            const double ph = (double)pf;
            // x-sample (i, c): pixels c and c+1 (lane 63's right neighbour lies
            // outside every output window)
            const double ph_r = (double)__shfl_down(pf, 1, 64);
            const int vd_r = __shfl_down((int)vd, 1, 64);
            const bool okx = vd && vd_r && (c + 1 < n);
            int qx = 0;
            double dxv = 0.0;
            if (okx) {
                const double diff = ph_r - ph;
                dxv = diff - TWO_PI_D * wrap_cycles(diff);
                qx = (int)floor(dxv * 1048576.0);
            }
            // y-sample (i-1, c): pixels (i-1, c) and (i, c)
            const bool oky = vd && vd_prev;
            int qy = 0;
            double dyv = 0.0;
            if (oky) {
                const double diff = ph - ph_prev;
                dyv = diff - TWO_PI_D * wrap_cycles(diff);
                qy = (int)floor(dyv * 1048576.0);
            }
            // horizontal window sums (meaningful on output lanes), packed as
            // 16 q + ok: at most 2H+1 <= 9 samples, |q| <= P + 1, so the count
            // stays in the low 4 bits and the packed sum within 31 bits
            const int px = qx * 16 + (int)okx, py = qy * 16 + (int)oky;
            int spx = px, spy = py;
#pragma unroll
            for (int d = 1; d <= H; ++d) {
                spx += __shfl(px, lane - d, 64) + __shfl(px, lane + d, 64);
                spy += __shfl(py, lane - d, 64) + __shfl(py, lane + d, 64);
            }
            // vertical sums: add this row, drop the row W back
            const int tW = (t + U - W) % U;
            RSx += (spx >> 4) - (hx[tW] >> 4);
            RKx += (spx & 15) - (hx[tW] & 15);
            RSy += (spy >> 4) - (hy[tW] >> 4);
            RKy += (spy & 15) - (hy[tW] & 15);
            hx[t] = spx;
            hy[t] = spy;
            dx[t] = dxv;
            dy[t] = dyv;
            okx_r[t] = okx;
            oky_r[t] = oky;
            ch[t] = (row_in && col_in) ? cc : 0.f;
            ph_prev = ph;
            vd_prev = vd;
            // slots of the rows H and H + 1 back
            const int tH = (t + U - H) % U, tH1 = (t + U - H - 1) % U;

            // ---- x-edges of row r = i - H
            {
                const int r = i - H;
                const float c_right = __shfl_down(ch[tH], 1, 64);  // coh(r, j+1)
                bool has = false;
                unsigned long long key = 0;
                unsigned int id = 0;
                if (r >= r0 && r < r1 && out_lane && j < n - 1) {
                    int16_t cpv = 0, cnv = 0;
                    if (okx_r[tH]) {
                        ++nvalid;
                        float c0 = ch[tH], c1 = c_right;
                        c0 = (c0 != c0) ? 0.f : c0;  // NaN reads as 0 (fminf would drop it)
                        c1 = (c1 != c1) ? 0.f : c1;
                        stream_lookup<INTERP, NGP2>(slut, NA, NG, RSx, RKx, fminf(c0, c1), cpv, cnv);
                        const double dd = fabs(dx[tH]);
                        const unsigned long long kb = (unsigned long long)__double_as_longlong(dd);
                        const bool cand = dd > steep_thresh;
                        const bool sel = cand && kb >= kzero;
                        has = cand && !sel && kb >= kbound;
                        cpv = sel ? (int16_t)0 : cpv;
                        cnv = sel ? (int16_t)0 : cnv;
                        key = kb;
                        id = (unsigned int)r * (unsigned int)nx_cols + (unsigned int)j;
                    }
                    const size_t xrow = (size_t)r * (size_t)nx_cols;  // wave-uniform row base
                    (cxp + xrow)[(unsigned int)j] = cpv;
                    (cxn + xrow)[(unsigned int)j] = cnv;
                }
                cand_push(cb, ccnt, lane, has, key, id, cand_key, cand_id, st);
            }
            // ---- y-edges of row r = i - 1 - H
            {
                const int r = i - 1 - H;
                bool has = false;
                unsigned long long key = 0;
                unsigned int id = 0;
                if (r >= r0 && r < r1 && r < m - 1 && out_lane && j < n) {
                    int16_t cpv = 0, cnv = 0;
                    if (oky_r[tH]) {
                        ++nvalid;
                        float c0 = ch[tH1], c1 = ch[tH];  // coh(r, j), coh(r+1, j)
                        c0 = (c0 != c0) ? 0.f : c0;
                        c1 = (c1 != c1) ? 0.f : c1;
                        stream_lookup<INTERP, NGP2>(slut, NA, NG, RSy, RKy, fminf(c0, c1), cpv, cnv);
                        const double dd = fabs(dy[tH]);
                        const unsigned long long kb = (unsigned long long)__double_as_longlong(dd);
                        const bool cand = dd > steep_thresh;
                        const bool sel = cand && kb >= kzero;
                        has = cand && !sel && kb >= kbound;
                        cpv = sel ? (int16_t)0 : cpv;
                        cnv = sel ? (int16_t)0 : cnv;
                        key = kb;
                        id = nx_total + (unsigned int)r * (unsigned int)n + (unsigned int)j;
                    }
                    const size_t yrow = (size_t)r * (size_t)n;
                    (cyp + yrow)[(unsigned int)j] = cpv;
                    (cyn + yrow)[(unsigned int)j] = cnv;
                }
                cand_push(cb, ccnt, lane, has, key, id, cand_key, cand_id, st);
            }
        }
    }
    if (ccnt) cand_flush(cb, ccnt, lane, cand_key, cand_id, st);
    (void)nvalid;
}

// Pre-pass of the steep rule: counts the valid edges (both pixels valid)
// and histograms the candidates (|d| > threshold, d the wrapped gradient
// exactly as the cost kernels compute it) into the coarse bins.  Each
// thread owns VEC consecutive pixel columns and walks a strip of SC_ROWS
// pixel rows (their x-edges to the right and y-edges downwards), fetching
// SC_BATCH rows at a time before any arithmetic; a pixel row is read once
// per strip plus one halo row.  Every workgroup writes its own partial
// histogram and valid count (no global atomics); k_steep_reduce sums them.
constexpr int SC_ROWS = 32;
constexpr int SC_BATCH = 4;    // divides SC_ROWS
constexpr int SC_W = 256;      // threads across a work item (its columns)
constexpr int SC_PT = 1024;    // pre-pass workgroup: four items at a time, one histogram
constexpr int SC_GRID = 256;   // pre-pass workgroups at most (one per CU; partial histograms)
constexpr int SC_RED = 64;     // partial histograms summed per reduce workgroup

// Pixel columns a .. a+ncol-1 of one row (ncol <= VEC+1): phases, and the
// validity as a bit mask (bit k: column a+k); absent columns read invalid.
template <int VEC>
__device__ __forceinline__ unsigned int sc_load_row(const float *__restrict__ psi,
                                                    const uint8_t *__restrict__ valid, size_t a,
                                                    int ncol, float *f) {
    unsigned int vm;
    if (VEC == 4 && ncol == 5) {
        const float4 q = *reinterpret_cast<const float4 *>(psi + a);
        f[0] = q.x; f[1] = q.y; f[2] = q.z; f[3] = q.w;
        f[4] = psi[a + 4];
        if (valid) {
            const unsigned int w4 = *reinterpret_cast<const unsigned int *>(valid + a);
            // byte k != 0 -> bit k
            vm = (w4 & 0xffu ? 1u : 0u) | (w4 & 0xff00u ? 2u : 0u) | (w4 & 0xff0000u ? 4u : 0u) |
                 (w4 & 0xff000000u ? 8u : 0u) | (valid[a + 4] ? 16u : 0u);
        } else {
            vm = 31u;
        }
    } else {
        vm = 0;
#pragma unroll
        for (int k = 0; k <= VEC; ++k) {
            f[k] = k < ncol ? psi[a + k] : 0.f;
            if (k < ncol && (!valid || valid[a + k])) vm |= 1u << k;
        }
    }
    return vm;
}

// |wrapped gradient| of the edge a -> b, in the cost kernels' arithmetic
__device__ __forceinline__ double sc_absgrad(float a, float b) {
    const double diff = (double)b - (double)a;
    return fabs(diff - TWO_PI_D * wrap_cycles(diff));
}

template <int VEC>
__global__ __launch_bounds__(SC_PT) void k_steep_coarse(const float *__restrict__ psi,
                                                       const uint8_t *__restrict__ valid, int m,
                                                       int n, double thr, unsigned long long base,
                                                       int shift, int nbx, int nitems,
                                                       unsigned int *__restrict__ parts,
                                                       unsigned long long *__restrict__ vparts) {
    __shared__ unsigned int h[SC_BINS];
    __shared__ unsigned long long vsum[SC_PT / 64];
    for (int t = threadIdx.x; t < SC_BINS; t += SC_PT) h[t] = 0;
    __syncthreads();
    unsigned int nv = 0;
    const int sub = threadIdx.x / SC_W, lt = threadIdx.x % SC_W;
    for (int item = blockIdx.x * (SC_PT / SC_W) + sub; item < nitems; item += gridDim.x * (SC_PT / SC_W)) {
        const int bx = item % nbx, by = item / nbx;
        const int j0 = (bx * SC_W + lt) * VEC;
        const int i0 = by * SC_ROWS;
        if (j0 >= n) continue;
        const int ncol = min(VEC + 1, n - j0);             // pixel columns read
        const unsigned int own = (1u << min(VEC, n - j0)) - 1u;  // pixel columns owned
        float p[VEC + 1];
        unsigned int pv = sc_load_row<VEC>(psi, valid, (size_t)i0 * n + j0, ncol, p);
        // every strip row is visited; rows past the image read as invalid
        // and contribute no edge
        for (int ib = i0; ib < i0 + SC_ROWS && ib < m; ib += SC_BATCH) {
            float q[SC_BATCH][VEC + 1];
            unsigned int qv[SC_BATCH];
#pragma unroll
            for (int r = 0; r < SC_BATCH; ++r) {
                if (ib + r + 1 < m) {
                    qv[r] = sc_load_row<VEC>(psi, valid, (size_t)(ib + r + 1) * n + j0, ncol, q[r]);
                } else {
                    qv[r] = 0;
#pragma unroll
                    for (int k = 0; k <= VEC; ++k) q[r][k] = 0.f;
                }
            }
#pragma unroll
            for (int r = 0; r < SC_BATCH; ++r) {
                // x-edges (i, j0+k): both ends valid; y-edges (i, j0+k): with row i+1
                const unsigned int okx = pv & (pv >> 1) & own;
                const unsigned int oky = pv & qv[r] & own;
                nv += __popc(okx) + __popc(oky);
#pragma unroll
                for (int k = 0; k < VEC; ++k) {
                    const double dx = sc_absgrad(p[k], p[k + 1]);
                    const double dy = sc_absgrad(p[k], q[r][k]);
                    if (((okx >> k) & 1u) && dx > thr)
                        atomicAdd(&h[steep_coarse_bin((unsigned long long)__double_as_longlong(dx), base,
                                                      shift)], 1u);
                    if (((oky >> k) & 1u) && dy > thr)
                        atomicAdd(&h[steep_coarse_bin((unsigned long long)__double_as_longlong(dy), base,
                                                      shift)], 1u);
                }
#pragma unroll
                for (int k = 0; k <= VEC; ++k) p[k] = q[r][k];
                pv = qv[r];
            }
        }
    }
    unsigned long long v = nv;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) vsum[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned int *dst = parts + (size_t)blockIdx.x * SC_BINS;
    for (int t = threadIdx.x; t < SC_BINS; t += SC_PT) dst[t] = h[t];
    if (threadIdx.x == 0) {
        unsigned long long s2 = 0;
        for (int w = 0; w < SC_PT / 64; ++w) s2 += vsum[w];
        vparts[blockIdx.x] = s2;
    }
}

// Sums of the pre-pass partials into the (zeroed) state: workgroup
// (x, y) adds partials y SC_RED .. y SC_RED + SC_RED - 1 of bins
// x 256 .. x 256 + 255, one atomic per bin, and their valid counts.
__global__ __launch_bounds__(256) void k_steep_reduce(const unsigned int *__restrict__ parts,
                                                      const unsigned long long *__restrict__ vparts,
                                                      int nparts, SteepState *st) {
    const int bin = blockIdx.x * 256 + threadIdx.x;
    const int g0 = blockIdx.y * SC_RED, g1 = min(nparts, g0 + SC_RED);
    unsigned int s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int g = g0;
    for (; g + 4 <= g1; g += 4) {
        s0 += parts[(size_t)g * SC_BINS + bin];
        s1 += parts[(size_t)(g + 1) * SC_BINS + bin];
        s2 += parts[(size_t)(g + 2) * SC_BINS + bin];
        s3 += parts[(size_t)(g + 3) * SC_BINS + bin];
    }
    for (; g < g1; ++g) s0 += parts[(size_t)g * SC_BINS + bin];
    const unsigned int tot = s0 + s1 + s2 + s3;
    if (tot) atomicAdd(&st->chist[bin], tot);
    if (blockIdx.x == 0) {
        unsigned long long v = (g0 + (int)threadIdx.x < g1) ? vparts[g0 + threadIdx.x] : 0ull;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(&st->nvalid, v);
    }
}

// cap = floor(pct * valid / 100) and the boundary bin: the largest bin b
// whose candidates in bins >= b number at least cap.  Everything above it
// is selected, and cap - above places remain for the boundary bin's
// candidates.  Fewer candidates than cap: every one is selected
// (bstar = -1); cap = 0: none (bstar = SC_BINS).  One workgroup.
__global__ __launch_bounds__(SC_THREADS) void k_steep_bstar(int pct, unsigned long long base,
                                                           int shift, SteepState *st) {
    constexpr int PER = SC_BINS / SC_THREADS;
    __shared__ unsigned long long wsum[SC_THREADS / 64];
    __shared__ int best;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    unsigned long long c[PER];
    unsigned long long own = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        c[q] = st->chist[t * PER + q];
        own += c[q];
    }
    if (t == 0) best = -1;
    // thread t holds bins t PER .. t PER + PER - 1; inc = sum of own over the
    // lanes >= this one in the wave (a reversed scan)
    unsigned long long inc = own;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long o = __shfl_down(inc, off, 64);
        if (lane + off < 64) inc += o;
    }
    if (lane == 0) wsum[wid] = inc;
    __syncthreads();
    unsigned long long after = 0, total_cand = 0;
    for (int w = 0; w < SC_THREADS / 64; ++w) {
        total_cand += wsum[w];
        if (w > wid) after += wsum[w];
    }
    const unsigned long long cap = st->nvalid * (unsigned long long)pct / 100ull;
    // suf[q] = candidates in bins >= t PER + q
    unsigned long long suf[PER];
    {
        unsigned long long run = after + (inc - own);
#pragma unroll
        for (int q = PER - 1; q >= 0; --q) {
            run += c[q];
            suf[q] = run;
        }
    }
    const bool boundary = cap > 0 && total_cand > cap;
    if (boundary) {
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (suf[q] >= cap) atomicMax(&best, t * PER + q);
    }
    __syncthreads();
    if (boundary) {
        const int bs = best;  // >= 0: suf of bin 0 is total_cand > cap
        if (bs / PER == t) {
            const int q = bs % PER;
            const unsigned long long above = suf[q] - c[q];
            st->bstar = bs;
            st->above = above;
            st->remaining = cap - above;
        }
    } else if (t == 0) {
        st->bstar = cap == 0 ? SC_BINS : -1;
        st->above = cap == 0 ? 0ull : total_cand;
        st->remaining = 0;
    }
    if (t == 0) {
        st->ncand_all = total_cand;
        st->cap = cap;
        st->base = base;
        st->shift = shift;
        // bin(k) > b  <=>  k >= base + 1 + ((b + 1) << shift) for b < SC_BINS - 1
        // (the last bin also holds every larger key); no overflow: the bins
        // span at most twice (PI_D bits - base)
        const int bs = boundary ? best : (cap == 0 ? SC_BINS : -1);
        const unsigned long long NONE = ~0ull;  // above every key of a non-negative double
        st->kzero = bs < 0 ? base + 1ull
                           : (bs >= SC_BINS - 1 ? NONE : base + 1ull + ((unsigned long long)(bs + 1) << shift));
        st->kbound = (bs < 0 || bs >= SC_BINS) ? NONE : base + 1ull + ((unsigned long long)bs << shift);
    }
}

// The boundary bin needs a select: it holds more candidates than places.
__device__ __forceinline__ bool steep_selecting(const SteepState *st) {
    return st->bstar >= 0 && st->bstar < SC_BINS && st->remaining > 0 && st->ncand > st->remaining;
}

// The exact select of the boundary bin when it holds at most SC_SMALL
// candidates, in one workgroup: the twelve 8-bit digits of (key, ~id) from
// the top, each pass histogramming the candidates that match the digits
// chosen so far (they stay in L2 between passes).  Larger sets go through
// the multi-workgroup passes below.
constexpr int SS_THREADS = 1024;
__global__ __launch_bounds__(SS_THREADS) void k_steep_select_small(
    const unsigned long long *__restrict__ key, const unsigned int *__restrict__ id, SteepState *st) {
    if (!steep_selecting(st) || st->ncand > (unsigned long long)SC_SMALL) return;
    __shared__ unsigned int h[256];
    __shared__ unsigned int suf[257];       // suf[d]: candidates with digit >= d (suf[256] = 0)
    __shared__ unsigned int wtot[4];
    __shared__ int best;
    const int d = threadIdx.x, lane = d & 63, w = d >> 6;
    const int nc = (int)st->ncand;
    unsigned int remaining = (unsigned int)st->remaining;  // <= nc <= SC_SMALL
    unsigned long long ph = 0, mh = 0;
    unsigned int pl = 0, ml = 0;
    if (d < 256) h[d] = 0;
    if (d == 0) {
        best = -1;
        suf[256] = 0;
    }
    __syncthreads();
    for (int pass = 0; pass < 12; ++pass) {
        for (int k = d; k < nc; k += SS_THREADS) {
            const unsigned long long hi = key[k];
            const unsigned int lo = ~id[k];
            if ((hi & mh) != ph || (lo & ml) != pl) continue;
            const unsigned int digit = pass < 8 ? (unsigned int)((hi >> (8 * (7 - pass))) & 0xff)
                                                : ((lo >> (8 * (11 - pass))) & 0xffu);
            atomicAdd(&h[digit], 1u);
        }
        __syncthreads();
        // suffix sums over the 256 digits: within each of the four waves
        // that hold them, then across the waves
        unsigned int v = 0;
        if (d < 256) {
            v = h[d];
            for (int off = 1; off < 64; off <<= 1) {
                const unsigned int o = __shfl_down(v, off, 64);
                if (lane + off < 64) v += o;
            }
            if (lane == 0) wtot[w] = v;
        }
        __syncthreads();
        if (d < 256) {
            for (int w2 = w + 1; w2 < 4; ++w2) v += wtot[w2];
            suf[d] = v;
            if (v >= remaining) atomicMax(&best, d);  // suf is non-increasing in d
        }
        __syncthreads();
        const int digit = best < 0 ? 0 : best;
        const unsigned int take = remaining - suf[digit + 1];
        const bool whole = take == h[digit];
        remaining = take;
        if (pass < 8) {
            const int sh = 8 * (7 - pass);
            ph |= (unsigned long long)digit << sh;
            mh |= 0xffull << sh;
        } else {
            const int sh = 8 * (11 - pass);
            pl |= (unsigned int)digit << sh;
            ml |= 0xffu << sh;
        }
        __syncthreads();  // every thread has read h, suf and best
        if (whole) break;
        if (d < 256) h[d] = 0;
        if (d == 0) best = -1;
        __syncthreads();
    }
    if (d == 0) {
        st->remaining = remaining;
        st->prefix_hi = ph;
        st->mask_hi = mh;
        st->prefix_lo = pl;
        st->mask_lo = ml;
        st->done = 1;
    }
}

__global__ void k_steep_hist(const unsigned long long *key, const unsigned int *id, SteepState *st,
                             int pass) {
    if (!steep_selecting(st) || st->done) return;
    __shared__ unsigned int h[256];
    for (int t = threadIdx.x; t < 256; t += blockDim.x) h[t] = 0;
    __syncthreads();
    const unsigned long long nc = st->ncand;
    const unsigned long long ph = st->prefix_hi, mh = st->mask_hi;
    const unsigned int pl = st->prefix_lo, ml = st->mask_lo;
    for (unsigned long long k = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; k < nc;
         k += (unsigned long long)gridDim.x * blockDim.x) {
        const unsigned long long hi = key[k];
        const unsigned int lo = ~id[k];
        if ((hi & mh) != ph || (lo & ml) != pl) continue;
        unsigned int digit = pass < 8 ? (unsigned int)((hi >> (8 * (7 - pass))) & 0xff)
                                      : ((lo >> (8 * (11 - pass))) & 0xffu);
        atomicAdd(&h[digit], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 256; t += blockDim.x)
        if (h[t]) atomicAdd(&st->hist[t], h[t]);
}

// The digit of this pass: the largest d whose candidates with digits >= d
// (among those matching the prefix so far) number at least `remaining`,
// from suffix sums of the histogram (256 threads, one bin each).  When
// that bucket is taken whole, the digits below it are left at zero: the
// threshold is then the smallest key of the bucket and selects the same
// candidates, so the remaining passes are skipped.
__global__ __launch_bounds__(256) void k_steep_pick(SteepState *st, int pass) {
    __shared__ unsigned long long suf[256];
    __shared__ int best;
    const int d = threadIdx.x;
    const bool active = steep_selecting(st) && !st->done;
    const unsigned int hd = st->hist[d];
    suf[d] = hd;
    if (d == 0) best = -1;
    __syncthreads();
    // inclusive suffix sums: suf[d] = sum of hist[d'] for d' >= d
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned long long add = d + off < 256 ? suf[d + off] : 0ull;
        __syncthreads();
        suf[d] += add;
        __syncthreads();
    }
    if (active && suf[d] >= st->remaining) atomicMax(&best, d);
    __syncthreads();
    if (active && d == 0) {
        const int digit = best < 0 ? 0 : best;
        const unsigned long long above = digit < 255 ? suf[digit + 1] : 0ull;
        const unsigned long long take = st->remaining - above;
        st->remaining = take;
        if (pass < 8) {
            const int sh = 8 * (7 - pass);
            st->prefix_hi |= (unsigned long long)digit << sh;
            st->mask_hi |= 0xffull << sh;
        } else {
            const int sh = 8 * (11 - pass);
            st->prefix_lo |= (unsigned int)digit << sh;
            st->mask_lo |= 0xffu << sh;
        }
        if (take == (unsigned long long)st->hist[digit]) st->done = 1;
    }
    __syncthreads();
    st->hist[d] = 0;
}

// Zero the selected candidates: all of them when they fit under the cap,
// otherwise those whose (|d| bits, ~id) is at least the selected threshold.
__global__ void k_steep_zero(const unsigned long long *key, const unsigned int *id,
                             const SteepState *st, long long nx_total, int16_t *cxp, int16_t *cxn,
                             int16_t *cyp, int16_t *cyn) {
    const unsigned long long nc = st->ncand;  // the boundary bin's candidates
    if (st->remaining == 0) return;
    const bool all = nc <= st->remaining;
    const unsigned long long th = st->prefix_hi;
    const unsigned int tl = st->prefix_lo;
    for (unsigned long long k = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; k < nc;
         k += (unsigned long long)gridDim.x * blockDim.x) {
        const unsigned long long hi = key[k];
        const unsigned int e = id[k];
        const unsigned int lo = ~e;
        if (!all && !(hi > th || (hi == th && lo >= tl))) continue;
        if ((long long)e < nx_total) {
            cxp[e] = 0;
            cxn[e] = 0;
        } else {
            cyp[e - nx_total] = 0;
            cyn[e - nx_total] = 0;
        }
    }
}

ww_status edge_costs_impl(const float *psi, const float *coh, const uint8_t *valid, int m, int n,
                          const int16_t *lut, int NA, int NG, const ww_cost_params &cp,
                          int16_t *cxp, int16_t *cxn, int16_t *cyp, int16_t *cyn,
                          hipStream_t stream) {
    const int64_t nx = (int64_t)m * (n - 1), ny = (int64_t)(m - 1) * n;
    if (nx + ny == 0) return WW_OK;
    if (nx + ny >= ((int64_t)1 << 32)) return fail(WW_E_INVALID_ARG, "too many edges");
    SteepState *st = nullptr;
    unsigned long long *keys = nullptr;
    unsigned int *ids = nullptr;
    WW_TRY(scratch(SLOT_STEEP, sizeof(SteepState), (void **)&st));
    const int steep_on = cp.steep_rule != 0;
    const int64_t capn = steep_on ? (nx + ny) : 1;
    char *kbuf = nullptr;
    WW_TRY(scratch(SLOT_STEEP_KEYS, (size_t)capn * 12 + 512, (void **)&kbuf));
    keys = (unsigned long long *)kbuf;
    ids = (unsigned int *)(kbuf + ((size_t)capn * 8 + 255) / 256 * 256);
    WW_HIP(hipMemsetAsync(st, 0, sizeof(SteepState), stream));
    if (steep_on) {
        // coarse bins over the candidate keys (threshold, bits(PI_D)]: wider
        // gradients (inputs outside one cycle) share the last bin
        const double thr = cp.steep_thresh_rad + 0.0;  // -0 as +0: its bits order below every key
        unsigned long long base;
        std::memcpy(&base, &thr, sizeof base);
        unsigned long long top;
        const double pid = PI_D;
        std::memcpy(&top, &pid, sizeof top);
        int shift = 0;
        if (top > base) {
            const unsigned long long span = top - base;  // keys base+1 .. top
            int bits = 0;
            while (bits < 64 && (span >> bits) != 0) ++bits;
            shift = bits > 12 ? bits - 12 : 0;
        }
        const bool vec = (n % 4 == 0) && ((uintptr_t)psi % 16 == 0) &&
                         (!valid || (uintptr_t)valid % 4 == 0);
        const int V = vec ? 4 : 1;
        const int nbx = ceil_div(ceil_div(n, V), SC_W), nby = ceil_div(m, SC_ROWS);
        const int64_t items = (int64_t)nbx * nby;
        if (items >= ((int64_t)1 << 31)) return fail(WW_E_INVALID_ARG, "image too large");
        const int grid = (int)std::min<int64_t>(ceil_div(items, SC_PT / SC_W), SC_GRID);
        char *pb = nullptr;
        WW_TRY(scratch(SLOT_STEEP_PARTS, (size_t)grid * (SC_BINS * 4 + 8), (void **)&pb));
        unsigned int *parts = (unsigned int *)pb;
        unsigned long long *vparts = (unsigned long long *)(pb + (size_t)grid * SC_BINS * 4);
        if (vec)
            hipLaunchKernelGGL(k_steep_coarse<4>, dim3(grid), dim3(SC_PT), 0, stream, psi, valid, m, n,
                               thr, base, shift, nbx, (int)items, parts, vparts);
        else
            hipLaunchKernelGGL(k_steep_coarse<1>, dim3(grid), dim3(SC_PT), 0, stream, psi, valid, m, n,
                               thr, base, shift, nbx, (int)items, parts, vparts);
        WW_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_steep_reduce, dim3(SC_BINS / 256, ceil_div(grid, SC_RED)), dim3(256), 0,
                           stream, parts, vparts, grid, st);
        WW_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_steep_bstar, dim3(1), dim3(SC_THREADS), 0, stream, cp.steep_cap_pct,
                           base, shift, st);
        WW_LAUNCH_CHECK();
    }
    const int h = cp.box_half;
    // no candidates at all without the rule (nothing, NaN included, exceeds +inf)
    const double cand_thresh = steep_on ? cp.steep_thresh_rad : HUGE_VAL;
    if (h <= 4 && NA * NG <= CS_LUT_MAX) {
        const int OW = 63 - 2 * h;
        const int nstrips = ceil_div(n, OW), nsegs = ceil_div(m, CS_ROWS);
        const int nwaves = nstrips * nsegs;
        // a power-of-two coherence bin count (at most 2^16) makes the bin
        // products exact in float
        const bool ngp2 = NG > 0 && NG <= (1 << 16) && (NG & (NG - 1)) == 0;
        const dim3 grid(ceil_div(nwaves, CS_WAVES));
#define WW_STREAM(HH, IP)                                                                         \
    if (ngp2)                                                                                      \
        hipLaunchKernelGGL((k_edge_costs_stream<HH, IP, true>), grid, dim3(64 * CS_WAVES), 0, stream, \
                           psi, coh, valid, m, n, lut, NA, NG, cand_thresh, cxp,                \
                           cxn, cyp, cyn, keys, ids, st, nstrips, nwaves);                           \
    else                                                                                           \
        hipLaunchKernelGGL((k_edge_costs_stream<HH, IP, false>), grid, dim3(64 * CS_WAVES), 0, stream, \
                           psi, coh, valid, m, n, lut, NA, NG, cand_thresh, cxp,                 \
                           cxn, cyp, cyn, keys, ids, st, nstrips, nwaves)
#define WW_STREAM_H(IP)                   \
    switch (h) {                          \
        case 0: WW_STREAM(0, IP); break;  \
        case 1: WW_STREAM(1, IP); break;  \
        case 2: WW_STREAM(2, IP); break;  \
        case 3: WW_STREAM(3, IP); break;  \
        default: WW_STREAM(4, IP); break; \
    }
        if (cp.lut_interp) {
            WW_STREAM_H(true)
        } else {
            WW_STREAM_H(false)
        }
#undef WW_STREAM_H
#undef WW_STREAM
        WW_LAUNCH_CHECK();
    } else {
        const int PR = CT_H + 2 * h + 1, PC = CT_W + 2 * h + 1, ER = CT_H + 2 * h, EC = CT_W + 2 * h;
        const size_t lds = (size_t)PR * PC * 4 + 2 * (size_t)ER * EC * 4 + 2 * (size_t)ER * CT_W * 4 +
                           2 * (size_t)ER * CT_W * 2 + (size_t)PR * PC + 2 * (size_t)ER * EC;
        if (lds > 64 * 1024)
            return fail(WW_E_INVALID_ARG, "box_half %d too large for the tile (max 8)", h);
        dim3 grid(ceil_div(n, CT_W), ceil_div(m, CT_H));
        hipLaunchKernelGGL(k_edge_costs, grid, dim3(CT_THREADS), lds, stream, psi, coh, valid, m,
                           n, lut, NA, NG, h, cp.steep_thresh_rad, steep_on, cp.lut_interp, cxp,
                           cxn, cyp, cyn,
                           keys, ids, st);
        WW_LAUNCH_CHECK();
    }
    if (steep_on) {
        // the boundary bin's candidate count decides the select (none, one
        // workgroup, or the multi-workgroup passes) and sizes its grids
        unsigned long long *hs = nullptr;
        WW_TRY(host_scratch(4 * sizeof(unsigned long long), (void **)&hs));
        WW_HIP(hipMemcpyAsync(hs, st, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
        WW_TRY(wait_stream(stream));
        const unsigned long long nc = hs[1], remaining = hs[3];  // ncand, remaining
        if (remaining > 0 && nc > 0) {
            if (nc > remaining) {
                if (nc <= (unsigned long long)SC_SMALL) {
                    hipLaunchKernelGGL(k_steep_select_small, dim3(1), dim3(SS_THREADS), 0, stream, keys,
                                       ids, st);
                    WW_LAUNCH_CHECK();
                } else {
                    const int hb = (int)std::min<unsigned long long>(2048, (nc + 1023) / 1024);
                    for (int pass = 0; pass < 12; ++pass) {
                        hipLaunchKernelGGL(k_steep_hist, dim3(hb), dim3(256), 0, stream, keys, ids, st,
                                           pass);
                        WW_LAUNCH_CHECK();
                        hipLaunchKernelGGL(k_steep_pick, dim3(1), dim3(256), 0, stream, st, pass);
                        WW_LAUNCH_CHECK();
                    }
                }
            }
            const int zb = (int)std::min<unsigned long long>(2048, (nc + 255) / 256);
            hipLaunchKernelGGL(k_steep_zero, dim3(zb), dim3(256), 0, stream, keys, ids, st,
                               (long long)nx, cxp, cxn, cyp, cyn);
            WW_LAUNCH_CHECK();
        }
    }
    return WW_OK;
}

}  // namespace ww
