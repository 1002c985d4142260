// Integration of the corrected gradients into the integer cycle field K and
// the unwrapped phase (Sections II-A and II-C).
//
// Along every edge K_v - K_u = dk_e - w_e (w_e = wrap count of psi), exact
// in integers, so any integration order gives the same K when the corrected
// gradients are curl-free.  K is fixed by K(ref) = 0.
//
//   k_col0        : one workgroup of 1024: the reference pixel (first valid
//                   pixel, row-major, unless given), column-0 prefix sums
//                   K0[i] and K(ref)
//   k_rows        : one workgroup per row; chunked workgroup scan of the
//                   row's x-edge increments (8 pixels per thread, 16-byte
//                   accesses where rows are 4-aligned, next chunk prefetched),
//                   then K and phi = (float)((double)psi + 2 pi K) (nodata
//                   if invalid).
// Bytes per pixel: psi 4 + valid 1 + dk_x 1 read, K 4 + phi 4 written.
#pragma clang fp contract(off)

#include "ww_internal.h"

namespace ww {

constexpr int IT_THREADS = 256;

struct IntegState {
    long long first_valid;
    int kref;
    int pad;
};

// Block-wide exclusive scan of one int per thread (THREADS a multiple of
// 64, at most 1024); returns the exclusive prefix and writes the block
// total to *total.
template <int THREADS>
__device__ int block_exclusive_scan(int v, int *total) {
    __shared__ int wsum[THREADS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        int o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < THREADS / 64; ++w) {
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

// Everything before the rows, in one workgroup of COL_THREADS:
//  1. the reference pixel: ref_i/ref_j, or the first valid pixel in
//     row-major order (chunks scanned from the start, stopping at the first
//     chunk holding one: typical masks end the search in the first chunk);
//  2. column 0: K0[i] = sum over 1 <= i' <= i of g(i') = dk_y(i'-1, 0) -
//     w_y(i'-1, 0), in chunks of COL_THREADS x COL_PER rows (each thread's
//     COL_PER loads issued together; 8192 rows per chunk);
//  3. K(ref) = K0[ref_i] + the x-edge increments along the reference row
//     before ref_j.
constexpr int COL_THREADS = 1024;
constexpr int COL_PER = 8;

__global__ __launch_bounds__(COL_THREADS) void k_col0(const float *__restrict__ psi,
                                                     const uint8_t *__restrict__ valid,
                                                     const int8_t *__restrict__ dkx,
                                                     const int8_t *__restrict__ dky, int m, int n,
                                                     int ref_i, int ref_j, IntegState *st,
                                                     int *__restrict__ K0) {
    __shared__ unsigned long long best;
    __shared__ int kref_row;
    const int64_t N = (int64_t)m * n;
    if (threadIdx.x == 0) best = (unsigned long long)N;
    __syncthreads();
    if (valid && ref_i < 0) {
        for (int64_t base = 0; base < N; base += COL_THREADS * 16) {
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
    }
    __syncthreads();
    int ri = ref_i, rj = ref_j;
    if (ri < 0) {
        long long fv = valid ? (long long)best : 0ll;
        if (threadIdx.x == 0) st->first_valid = valid ? fv : 0ll;
        if (fv >= N) fv = 0;
        ri = (int)(fv / n);
        rj = (int)(fv % n);
    } else if (threadIdx.x == 0) {
        st->first_valid = valid ? (long long)N : 0ll;
    }
    auto g_col = [&](int i) -> int {  // increment from row i-1 to row i, i >= 1
        const int64_t a = (int64_t)(i - 1) * n;
        return (int)dky[a] - wrap_cycles(phase_at(psi, valid, a + n) - phase_at(psi, valid, a));
    };
    int carry = 0;
    for (int base = 0; base < m; base += COL_THREADS * COL_PER) {
        const int lo = base + threadIdx.x * COL_PER;
        int g[COL_PER];
        int local = 0;
#pragma unroll
        for (int q = 0; q < COL_PER; ++q) {
            const int i = lo + q;
            g[q] = (i >= 1 && i < m) ? g_col(i) : 0;
            local += g[q];
        }
        int tot;
        int run = carry + block_exclusive_scan<COL_THREADS>(local, &tot);
#pragma unroll
        for (int q = 0; q < COL_PER; ++q) {
            run += g[q];
            if (lo + q < m) K0[lo + q] = run;
            if (lo + q == ri) kref_row = run;
        }
        carry += tot;
    }
    __syncthreads();
    int part = 0, tot;
    for (int j = threadIdx.x; j < rj; j += COL_THREADS) part += gx_at(psi, valid, dkx, n, ri, j);
    (void)block_exclusive_scan<COL_THREADS>(part, &tot);
    if (threadIdx.x == 0) {
        st->kref = kref_row + tot;
        st->pad = 0;
    }
}

// Loads of one chunk of a row: elements j0 .. j0+RP-1 of psi/valid/dk_x and
// the pixel after them (psi/valid), for a thread of k_rows.
template <int VEC>
struct RowChunk {
    static constexpr int RP = 8;
    float ps[RP + 1];
    uint8_t vd[RP + 1];
    int8_t dk[RP];

    __device__ __forceinline__ void load(const float *__restrict__ psi,
                                         const uint8_t *__restrict__ valid,
                                         const int8_t *__restrict__ dkx, int n, int64_t row,
                                         int64_t drow, int j0) {
        if (VEC == 4 && j0 + RP < n) {
            // 16-byte loads; rows are 4-aligned when VEC == 4
            const float4 a = *reinterpret_cast<const float4 *>(psi + row + j0);
            const float4 b = *reinterpret_cast<const float4 *>(psi + row + j0 + 4);
            ps[0] = a.x; ps[1] = a.y; ps[2] = a.z; ps[3] = a.w;
            ps[4] = b.x; ps[5] = b.y; ps[6] = b.z; ps[7] = b.w;
            ps[RP] = psi[row + j0 + RP];
            if (valid) {
                const uchar4 u = *reinterpret_cast<const uchar4 *>(valid + row + j0);
                const uchar4 w = *reinterpret_cast<const uchar4 *>(valid + row + j0 + 4);
                vd[0] = u.x; vd[1] = u.y; vd[2] = u.z; vd[3] = u.w;
                vd[4] = w.x; vd[5] = w.y; vd[6] = w.z; vd[7] = w.w;
                vd[RP] = valid[row + j0 + RP];
            } else {
#pragma unroll
                for (int q = 0; q <= RP; ++q) vd[q] = 1;
            }
#pragma unroll
            for (int q = 0; q < RP; ++q) dk[q] = dkx[drow + j0 + q];
        } else {
#pragma unroll
            for (int q = 0; q <= RP; ++q) {
                const int j = j0 + q;
                ps[q] = j < n ? psi[row + j] : 0.f;
                vd[q] = j < n ? (valid ? valid[row + j] : 1) : 0;
            }
#pragma unroll
            for (int q = 0; q < RP; ++q) dk[q] = (j0 + q < n - 1) ? dkx[drow + j0 + q] : (int8_t)0;
        }
    }
};

// One workgroup per row: K along the row is the carried value plus the
// exclusive scan of the x-edge increments g = dk - w.  Chunks of
// IT_THREADS * 8 pixels; the next chunk's loads are issued before the
// current chunk is scanned.
template <int VEC>
__global__ __launch_bounds__(IT_THREADS) void k_rows(const float *__restrict__ psi,
                                                    const uint8_t *__restrict__ valid,
                                                    const int8_t *__restrict__ dkx, int m, int n,
                                                    const IntegState *__restrict__ st,
                                                    const int *__restrict__ K0, float nodata,
                                                    int32_t *__restrict__ K,
                                                    float *__restrict__ phi) {
    constexpr int RP = RowChunk<VEC>::RP;
    constexpr int CH = IT_THREADS * RP;
    const int i = blockIdx.x;
    const int64_t row = (int64_t)i * n, drow = (int64_t)i * (n - 1);
    int carry = K0[i] - st->kref;
    RowChunk<VEC> cur, nxt;
    cur.load(psi, valid, dkx, n, row, drow, threadIdx.x * RP);
    for (int base = 0; base < n; base += CH) {
        const int j0 = base + threadIdx.x * RP;
        if (base + CH < n) nxt.load(psi, valid, dkx, n, row, drow, j0 + CH);
        int g[RP];
        int local = 0;
#pragma unroll
        for (int q = 0; q < RP; ++q) {
            const int j = j0 + q;
            int v = 0;
            if (j < n - 1) {
                const double a = cur.vd[q] ? (double)cur.ps[q] : 0.0;
                const double b = cur.vd[q + 1] ? (double)cur.ps[q + 1] : 0.0;
                v = (int)cur.dk[q] - wrap_cycles(b - a);
            }
            g[q] = v;
            local += v;
        }
        int tot;
        const int ex = block_exclusive_scan<IT_THREADS>(local, &tot);
        int k = carry + ex;
        int kk[RP];
        float ph[RP];
#pragma unroll
        for (int q = 0; q < RP; ++q) {
            kk[q] = k;
            ph[q] = cur.vd[q] ? (float)((double)cur.ps[q] + TWO_PI_D * (double)k) : nodata;
            k += g[q];
        }
        if (VEC == 4 && j0 + RP <= n) {
            *reinterpret_cast<int4 *>(K + row + j0) = make_int4(kk[0], kk[1], kk[2], kk[3]);
            *reinterpret_cast<int4 *>(K + row + j0 + 4) = make_int4(kk[4], kk[5], kk[6], kk[7]);
            *reinterpret_cast<float4 *>(phi + row + j0) = make_float4(ph[0], ph[1], ph[2], ph[3]);
            *reinterpret_cast<float4 *>(phi + row + j0 + 4) = make_float4(ph[4], ph[5], ph[6], ph[7]);
        } else {
#pragma unroll
            for (int q = 0; q < RP; ++q)
                if (j0 + q < n) {
                    K[row + j0 + q] = kk[q];
                    phi[row + j0 + q] = ph[q];
                }
        }
        carry += tot;
        cur = nxt;
    }
}

// The integration proper, on caller-provided state: st (an IntegState) and
// K0 (m ints of column-0 prefix sums).
static ww_status integrate_run(const float *psi, const uint8_t *valid, const int8_t *dkx,
                               const int8_t *dky, int m, int n, const ww_cost_params &cp,
                               int32_t *K, float *phi, IntegState *st, int *K0,
                               hipStream_t stream) {
    hipLaunchKernelGGL(k_col0, dim3(1), dim3(COL_THREADS), 0, stream, psi, valid, dkx, dky, m, n,
                       cp.ref_i, cp.ref_j, st, K0);
    WW_LAUNCH_CHECK();
    // 16-byte accesses need 4-aligned rows and base pointers
    const bool vec = (n % 4 == 0) && (uintptr_t)psi % 16 == 0 && (uintptr_t)K % 16 == 0 &&
                     (uintptr_t)phi % 16 == 0 && (!valid || (uintptr_t)valid % 4 == 0);
    if (vec)
        hipLaunchKernelGGL(k_rows<4>, dim3(m), dim3(IT_THREADS), 0, stream, psi, valid, dkx, m, n,
                           st, K0, cp.nodata, K, phi);
    else
        hipLaunchKernelGGL(k_rows<1>, dim3(m), dim3(IT_THREADS), 0, stream, psi, valid, dkx, m, n,
                           st, K0, cp.nodata, K, phi);
    WW_LAUNCH_CHECK();
    return WW_OK;
}

constexpr size_t K0_OFF = 256;  // K0 follows the state, 256-byte aligned

ww_status integrate_impl(const float *psi, const uint8_t *valid, const int8_t *dkx,
                         const int8_t *dky, int m, int n, const ww_cost_params &cp, int32_t *K,
                         float *phi, hipStream_t stream) {
    char *buf = nullptr;
    WW_TRY(scratch(SLOT_INTEG, K0_OFF + sizeof(int) * (size_t)m, (void **)&buf));
    return integrate_run(psi, valid, dkx, dky, m, n, cp, K, phi, (IntegState *)buf,
                         (int *)(buf + K0_OFF), stream);
}

const long long *integrate_ref_index() {
    char *buf = nullptr;
    if (scratch(SLOT_INTEG, sizeof(IntegState), (void **)&buf) != WW_OK) return nullptr;
    return &((IntegState *)buf)->first_valid;
}

}  // namespace ww

// ------------------------------------------------------ allocation-free ---

// Scratch of ww_integrate_noalloc: the integration state and the column-0
// prefix sums of up to NOALLOC_MAX_ROWS rows.  Every device the library runs
// on holds its own copy until the process ends.  In host code the name is
// not a device address: host code only ever uses the address that
// hipGetSymbolAddress returns for the current device.
constexpr int NOALLOC_MAX_ROWS = 1 << 16;
static __device__ __align__(256) char scratch[ww::K0_OFF + sizeof(int) * NOALLOC_MAX_ROWS];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

extern "C" ww_status ww_integrate_noalloc(const float *psi, const uint8_t *valid,
                                          const int8_t *dk_x, const int8_t *dk_y, int32_t m,
                                          int32_t n, const ww_cost_params *cpin, int32_t *K,
                                          float *phi, void *stream) {
    ww::clear_error();
    if (m < 1 || n < 1 || (int64_t)m * n >= ((int64_t)1 << 31))
        return ww::fail(WW_E_INVALID_ARG, "image shape %d x %d outside 1 <= m,n, m*n < 2^31", m, n);
    if (m > NOALLOC_MAX_ROWS)
        return ww::fail(WW_E_INVALID_ARG, "ww_integrate_noalloc: %d rows above its limit of %d", m,
                    NOALLOC_MAX_ROWS);
    ww_cost_params cp;
    if (cpin) cp = *cpin;
    else ww_default_cost_params(&cp);
    if (cp.ref_i >= 0 && (cp.ref_i >= m || cp.ref_j < 0 || cp.ref_j >= n))
        return ww::fail(WW_E_INVALID_ARG, "reference pixel outside the image");
    if (!psi || !K || !phi || (n > 1 && !dk_x) || (m > 1 && !dk_y))
        return ww::fail(WW_E_INVALID_ARG, "input or output array is NULL");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ww::fail(WW_E_DEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return ww::fail(WW_E_INVALID_ARG, "device %d above the supported %d", dev, NOALLOC_MAX_DEVICES);
    void *base = nullptr;
    {
        // the device address of this device's copy, looked up once per device
        // (with that device current: each device has its own address)
        std::lock_guard<std::mutex> g(g_noalloc_mu);
        if (!g_noalloc_ptr[dev]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess)
                return ww::fail(WW_E_DEVICE, "hipGetSymbolAddress failed: %s", hipGetErrorString(e));
            if (!p) return ww::fail(WW_E_DEVICE, "hipGetSymbolAddress returned NULL");
            g_noalloc_ptr[dev] = p;
        }
        base = g_noalloc_ptr[dev];
    }
    char *buf = (char *)base;
    return ww::integrate_run(psi, valid, dk_x, dk_y, m, n, cp, K, phi, (ww::IntegState *)buf,
                             (int *)(buf + ww::K0_OFF), (hipStream_t)stream);
}
