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
#include <cmath>

#include "ww_internal.h"

namespace ww {

constexpr int CT_H = 16;   // tile rows
constexpr int CT_W = 64;   // tile cols
constexpr int CT_THREADS = 256;

constexpr int STRIPES = 256;

struct SteepState {
    unsigned long long nvalid_part[STRIPES];  // per-stripe valid-edge counts
    unsigned long long nvalid, ncand, cap, remaining;
    unsigned long long prefix_hi, mask_hi;
    unsigned int prefix_lo, mask_lo;
    unsigned int done;  // the threshold is known before the last digit
    unsigned int hist[256];
};

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
                    ckey[2 * it] = (unsigned long long)__double_as_longlong(dd);
                    cid[2 * it] = (unsigned int)idx_x;
                    cmask |= 1u << (2 * it);
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
                    ckey[2 * it + 1] = (unsigned long long)__double_as_longlong(dd);
                    cid[2 * it + 1] = (unsigned int)(nx_total + idx_y);
                    cmask |= 1u << (2 * it + 1);
                }
            }
            cyp[idx_y] = cp;
            cyn[idx_y] = cn;
        }
    }
    // block totals: one striped atomic for the valid count, one reservation
    // for the candidates
    __shared__ int red_valid[CT_THREADS / 64], red_cand[CT_THREADS / 64];
    __shared__ unsigned long long cand_base;
    const int lane = tid & 63, wid = tid >> 6;
    const int ncand = __popc(cmask);
    int v = nvalid, incl = ncand;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    for (int off = 1; off < 64; off <<= 1) {
        int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 0) red_valid[wid] = v;
    if (lane == 63) red_cand[wid] = incl;
    __syncthreads();
    if (tid == 0) {
        int tv = 0, tc = 0;
        for (int w = 0; w < CT_THREADS / 64; ++w) {
            tv += red_valid[w];
            tc += red_cand[w];
        }
        const int blk = blockIdx.y * gridDim.x + blockIdx.x;
        if (tv) atomicAdd(&st->nvalid_part[blk % STRIPES], (unsigned long long)tv);
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
// One wave per strip of CS_OW = 63 - 2H output columns, walking down a
// segment of CS_ROWS output rows.  Lane l holds sample column
// c = js - H + l; every pixel row is loaded once (coalesced, the next row
// prefetched), the horizontal window sums come from wave shuffles and the
// vertical ones from shift registers of the last 2H+1 sample rows, so the
// only re-read data are the 2H halo columns of a strip and the 2H halo rows
// of a segment.  Steep candidates are buffered per wave in LDS and appended
// with one atomic reservation per CS_CB entries.  Same arithmetic as
// k_edge_costs, so the outputs are identical.
#ifndef WW_CS_ROWS
#define WW_CS_ROWS 64
#endif
#ifndef WW_CS_PF
#define WW_CS_PF 4
#endif
constexpr int CS_ROWS = WW_CS_ROWS;  // output rows per wave
constexpr int CS_PF = WW_CS_PF;      // pixel rows loaded ahead
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
// a quotient under 4096) and one exact integer correction step.
__device__ __forceinline__ int slope_bin(int S, int K, int NA) {
    const int u = S + K * (int)PI_FIX;
    const int den = 2 * K * (int)PI_FIX;
    const float est = (float)u * ((float)NA * __builtin_amdgcn_rcpf((float)den));
    int t = (int)floorf(est);
    const int64_t e = (int64_t)u * NA - (int64_t)t * den;
    t += (e >= den) - (e < 0);
    return t < 0 ? 0 : (t > NA - 1 ? NA - 1 : t);
}

// Slope position of the interpolated lookup, floor((S + K P) NA 2^16 /
// (2 K P)) - 2^15: the quotient q and remainder e of u NA / (2 K P) as in
// slope_bin (unclamped), then floor(e 2^16 / (2 K P)) < 2^16 by the same
// float estimate and exact correction.
__device__ __forceinline__ int64_t slope_pos16(int S, int K, int NA) {
    const int u = S + K * (int)PI_FIX;
    const int den = 2 * K * (int)PI_FIX;
    const float rden = __builtin_amdgcn_rcpf((float)den);
    int q = (int)floorf((float)u * ((float)NA * rden));
    int64_t e = (int64_t)u * NA - (int64_t)q * den;
    const int c = (e >= den) - (e < 0);
    q += c;
    e -= (int64_t)c * den;
    int f = (int)floorf((float)e * (65536.f * rden));
    const int64_t e2 = e * 65536 - (int64_t)f * den;
    f += (e2 >= den) - (e2 < 0);
    return (int64_t)q * 65536 + f - 32768;
}

template <bool INTERP>
__device__ __forceinline__ void stream_lookup(const int16_t *slut, int NA, int NG, int S, int K,
                                              float g, int16_t &cp, int16_t &cn) {
    if constexpr (INTERP) {
        const int64_t t16 = slope_pos16(S, K, NA);
        const int64_t u16 = coh_pos16(g, NG);
        cp = lut_blend(slut, NA, NG, t16, u16);
        cn = lut_blend(slut, NA, NG, (int64_t)(NA - 1) * 65536 - t16, u16);
    } else {
        const int ba = slope_bin(S, K, NA);
        const int bg = coh_bin(g, NG);
        cp = slut[bg * NA + ba];
        cn = slut[bg * NA + (NA - 1 - ba)];
    }
}

template <int H, bool INTERP>
__global__ __launch_bounds__(64 * CS_WAVES) void k_edge_costs_stream(
    const float *__restrict__ psi, const float *__restrict__ coh, const uint8_t *__restrict__ valid,
    int m, int n, const int16_t *__restrict__ lut, int NA, int NG, double steep_thresh,
    int steep_on, int16_t *__restrict__ cxp, int16_t *__restrict__ cxn, int16_t *__restrict__ cyp,
    int16_t *__restrict__ cyn, unsigned long long *__restrict__ cand_key,
    unsigned int *__restrict__ cand_id, SteepState *__restrict__ st, int nstrips, int nwaves) {
    constexpr int OW = 63 - 2 * H;
    __shared__ CandBuf cbuf[CS_WAVES];
    __shared__ int16_t slut[CS_LUT_MAX];
    for (int t = threadIdx.x; t < NA * NG; t += 64 * CS_WAVES) slut[t] = lut[t];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gw = blockIdx.x * CS_WAVES + wv;
    if (gw >= nwaves) return;  // whole waves only: no workgroup barrier below
    CandBuf &cb = cbuf[wv];
    int ccnt = 0;
    const int strip = gw % nstrips, seg = gw / nstrips;
    const int js = strip * OW;
    const int r0 = seg * CS_ROWS, r1 = min(r0 + CS_ROWS, m);
    const int c = js - H + lane;  // sample / pixel column of this lane
    const bool col_in = c >= 0 && c < n;
    const int j = c;              // output column of an output lane
    const bool out_lane = lane >= H && lane < H + OW;
    const int nx_cols = n - 1;
    const int64_t nx_total = (int64_t)m * (n - 1);

    constexpr int W = 2 * H + 1;
    int hxs[W], hxk[W], hys[W], hyk[W];  // index 0: newest sample row
    double dx[H + 1], dy[H + 1];
    bool okx_r[H + 1], oky_r[H + 1];
    float ch[H + 2];
#pragma unroll
    for (int k = 0; k < W; ++k) hxs[k] = hxk[k] = hys[k] = hyk[k] = 0;
#pragma unroll
    for (int k = 0; k <= H; ++k) {
        dx[k] = dy[k] = 0.0;
        okx_r[k] = oky_r[k] = false;
    }
#pragma unroll
    for (int k = 0; k < H + 2; ++k) ch[k] = 0.f;
    double ph_prev = 0.0;
    bool vd_prev = false;
    int nvalid = 0;

    const int i_start = max(0, r0 - H);
    const int i_last = r1 + H;  // inclusive; rows >= m are absent (zero samples)
    // CS_PF rows of loads in flight ahead of the row being processed
    auto fetch = [&](int i, float &p, uint8_t &v, float &cc) {
        if (i < m && i <= i_last && col_in) {
            const int a = i * n + c;  // m * n < 2^31
            v = valid ? valid[a] : 1;
            p = psi[a];
            cc = coh[a];
        } else {
            v = 0;
            p = 0.f;
            cc = 0.f;
        }
    };
    float p_q[CS_PF], c_q[CS_PF];
    uint8_t v_q[CS_PF];
#pragma unroll
    for (int k = 0; k < CS_PF; ++k) fetch(i_start + k, p_q[k], v_q[k], c_q[k]);
    for (int i = i_start; i <= i_last; ++i) {
        const bool row_in = i < m;
        const float p = p_q[0], cc = c_q[0];
        const uint8_t v = v_q[0];
#pragma unroll
        for (int k = 0; k + 1 < CS_PF; ++k) {
            p_q[k] = p_q[k + 1];
            c_q[k] = c_q[k + 1];
            v_q[k] = v_q[k + 1];
        }
        fetch(i + CS_PF, p_q[CS_PF - 1], v_q[CS_PF - 1], c_q[CS_PF - 1]);
        const bool vd = row_in && col_in && v != 0;
        const double ph = vd ? (double)p : 0.0;
        // x-sample (i, c): pixels c and c+1 (lane 63's right neighbour lies
        // outside every output window)
        const double ph_r = __shfl_down(ph, 1, 64);
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
#pragma unroll
        for (int k = W - 1; k > 0; --k) {
            hxs[k] = hxs[k - 1];
            hxk[k] = hxk[k - 1];
            hys[k] = hys[k - 1];
            hyk[k] = hyk[k - 1];
        }
        hxs[0] = spx >> 4;
        hxk[0] = spx & 15;
        hys[0] = spy >> 4;
        hyk[0] = spy & 15;
#pragma unroll
        for (int k = H; k > 0; --k) {
            dx[k] = dx[k - 1];
            dy[k] = dy[k - 1];
            okx_r[k] = okx_r[k - 1];
            oky_r[k] = oky_r[k - 1];
        }
        dx[0] = dxv;
        dy[0] = dyv;
        okx_r[0] = okx;
        oky_r[0] = oky;
#pragma unroll
        for (int k = H + 1; k > 0; --k) ch[k] = ch[k - 1];
        ch[0] = (row_in && col_in) ? cc : 0.f;
        ph_prev = ph;
        vd_prev = vd;

        // ---- x-edges of row r = i - H
        {
            const int r = i - H;
            const float c_right = __shfl_down(ch[H], 1, 64);  // coh(r, j+1)
            bool has = false;
            unsigned long long key = 0;
            unsigned int id = 0;
            if (r >= r0 && r < r1 && out_lane && j < n - 1) {
                const int idx_x = r * nx_cols + j;
                int16_t cp = 0, cn = 0;
                if (okx_r[H]) {
                    ++nvalid;
                    int S = 0, K = 0;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        S += hxs[k];
                        K += hxk[k];
                    }
                    float c0 = ch[H], c1 = c_right;
                    c0 = (c0 != c0) ? 0.f : c0;  // NaN reads as 0 (fminf would drop it)
                    c1 = (c1 != c1) ? 0.f : c1;
                    stream_lookup<INTERP>(slut, NA, NG, S, K, fminf(c0, c1), cp, cn);
                    const double dd = fabs(dx[H]);
                    if (steep_on && dd > steep_thresh) {
                        has = true;
                        key = (unsigned long long)__double_as_longlong(dd);
                        id = (unsigned int)idx_x;
                    }
                }
                cxp[idx_x] = cp;
                cxn[idx_x] = cn;
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
                const int idx_y = r * n + j;
                int16_t cp = 0, cn = 0;
                if (oky_r[H]) {
                    ++nvalid;
                    int S = 0, K = 0;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        S += hys[k];
                        K += hyk[k];
                    }
                    float c0 = ch[H + 1], c1 = ch[H];  // coh(r, j), coh(r+1, j)
                    c0 = (c0 != c0) ? 0.f : c0;
                    c1 = (c1 != c1) ? 0.f : c1;
                    stream_lookup<INTERP>(slut, NA, NG, S, K, fminf(c0, c1), cp, cn);
                    const double dd = fabs(dy[H]);
                    if (steep_on && dd > steep_thresh) {
                        has = true;
                        key = (unsigned long long)__double_as_longlong(dd);
                        id = (unsigned int)nx_total + (unsigned int)idx_y;
                    }
                }
                cyp[idx_y] = cp;
                cyn[idx_y] = cn;
            }
            cand_push(cb, ccnt, lane, has, key, id, cand_key, cand_id, st);
        }
    }
    if (ccnt) cand_flush(cb, ccnt, lane, cand_key, cand_id, st);
    for (int off = 32; off > 0; off >>= 1) nvalid += __shfl_down(nvalid, off, 64);
    if (lane == 0 && nvalid)
        atomicAdd(&st->nvalid_part[gw % STRIPES], (unsigned long long)nvalid);
}

// cap = floor(pct * valid / 100); remaining = cap
__global__ void k_steep_init(SteepState *st, int pct) {
    unsigned long long nv = 0;
    for (int k = 0; k < STRIPES; ++k) nv += st->nvalid_part[k];
    st->nvalid = nv;
    st->cap = nv * (unsigned long long)pct / 100ull;
    st->remaining = st->cap;
    st->prefix_hi = 0;
    st->mask_hi = 0;
    st->prefix_lo = 0;
    st->mask_lo = 0;
    st->done = 0;
}

__device__ __forceinline__ bool steep_selecting(const SteepState *st) {
    return st->ncand > st->cap && st->cap > 0;
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
    const unsigned long long nc = st->ncand;
    if (st->cap == 0) return;
    const bool all = nc <= st->cap;
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
    const int h = cp.box_half;
    if (h <= 4 && NA * NG <= CS_LUT_MAX) {
        const int OW = 63 - 2 * h;
        const int nstrips = ceil_div(n, OW), nsegs = ceil_div(m, CS_ROWS);
        const int nwaves = nstrips * nsegs;
        const dim3 grid(ceil_div(nwaves, CS_WAVES));
#define WW_STREAM(HH, IP)                                                                   \
    hipLaunchKernelGGL((k_edge_costs_stream<HH, IP>), grid, dim3(64 * CS_WAVES), 0, stream, psi, \
                       coh, valid, m, n, lut, NA, NG, cp.steep_thresh_rad, steep_on, cxp, cxn,   \
                       cyp, cyn, keys, ids, st, nstrips, nwaves)
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
        hipLaunchKernelGGL(k_steep_init, dim3(1), dim3(1), 0, stream, st, cp.steep_cap_pct);
        WW_LAUNCH_CHECK();
        const int hb = (int)std::min<int64_t>(2048, std::max<int64_t>(1, ceil_div(nx + ny, 1024)));
        for (int pass = 0; pass < 12; ++pass) {
            hipLaunchKernelGGL(k_steep_hist, dim3(hb), dim3(256), 0, stream, keys, ids, st, pass);
            WW_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_steep_pick, dim3(1), dim3(256), 0, stream, st, pass);
            WW_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(k_steep_zero, dim3(hb), dim3(256), 0, stream, keys, ids, st,
                           (long long)nx, cxp, cxn, cyp, cyn);
        WW_LAUNCH_CHECK();
    }
    return WW_OK;
}

}  // namespace ww
