// C ABI entry points: argument checks, workspace, error reporting.  Every
// numeric step runs in the HIP kernels of the sibling sources.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "ww_internal.h"

namespace ww {

static thread_local std::string g_error;

ww_status fail(ww_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

void clear_error() { g_error.clear(); }

std::mutex &lock() {
    static std::mutex mu;
    return mu;
}

int current_device() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return 0;
    return d;
}

struct Workspace {
    int device = 0;
    Buffer slot[SLOT_COUNT];
    void *host = nullptr;
    size_t host_bytes = 0;
    void *mirror = nullptr;  // coherent pinned block the device writes counters into
    size_t mirror_bytes = 0;
    hipEvent_t wait_ev = nullptr;  // marks the point a host wait returns at
    ww_mcf_stats stats{};
};

static thread_local Workspace *t_ws = nullptr;

void set_thread_workspace(Workspace *ws) { t_ws = ws; }

Workspace *workspace_create(int device) {
    Workspace *ws = new Workspace();
    ws->device = device;
    return ws;
}

void workspace_destroy(Workspace *ws) {
    if (!ws) return;
    for (auto &b : ws->slot)
        if (b.ptr) (void)hipFree(b.ptr);
    if (ws->host) (void)hipHostFree(ws->host);
    if (ws->mirror) (void)hipHostFree(ws->mirror);
    if (ws->wait_ev) (void)hipEventDestroy(ws->wait_ev);
    delete ws;
}

size_t workspace_bytes(const Workspace *ws) {
    size_t s = 0;
    for (auto &b : ws->slot) s += b.bytes;
    return s;
}

Workspace *current_workspace() {
    if (t_ws) return t_ws;
    static std::map<int, Workspace *> per_device;
    static std::mutex mu;
    std::lock_guard<std::mutex> g(mu);
    const int d = current_device();
    Workspace *&w = per_device[d];
    if (!w) w = workspace_create(d);
    return w;
}

std::mutex &lut_lock() {
    static std::mutex mu;
    return mu;
}

ww_mcf_stats &last_mcf_stats() { return current_workspace()->stats; }

ww_status scratch(int slot, size_t bytes, void **out) {
    if (bytes == 0) bytes = 256;
    Workspace *ws = current_workspace();
    Buffer &b = ws->slot[slot];
    if (b.bytes < bytes) {
        if (b.ptr) {
            // the buffer may still be read by work queued on any stream
            WW_HIP(hipDeviceSynchronize());
            WW_HIP(hipFree(b.ptr));
            b.ptr = nullptr;
            b.bytes = 0;
            b.clean = 0;
        }
        size_t want = bytes + bytes / 8;
        void *p = nullptr;
        // WW_SCRATCH_LIMIT (bytes): a test of the out-of-memory path makes
        // any larger buffer fail as a failed allocation would
        const char *lim = getenv("WW_SCRATCH_LIMIT");
        if (lim && want > (size_t)std::max(0ll, atoll(lim)))
            return fail(WW_E_OOM, "device allocation of %zu bytes refused (WW_SCRATCH_LIMIT)", want);
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(WW_E_OOM, "device allocation of %zu bytes failed", want);
        }
        b.ptr = p;
        b.bytes = want;
        b.clean = 0;
    }
    *out = b.ptr;
    return WW_OK;
}

size_t *scratch_clean(int slot) { return &current_workspace()->slot[slot].clean; }

ww_status host_scratch(size_t bytes, void **out) {
    Workspace *ws = current_workspace();
    if (ws->host_bytes < bytes) {
        if (ws->host) WW_HIP(hipHostFree(ws->host));
        ws->host = nullptr;
        ws->host_bytes = 0;
        if (hipHostMalloc(&ws->host, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(WW_E_OOM, "pinned host allocation of %zu bytes failed", bytes);
        }
        ws->host_bytes = bytes;
    }
    *out = ws->host;
    return WW_OK;
}

ww_status host_mirror(size_t bytes, void **out) {
    Workspace *ws = current_workspace();
    if (ws->mirror_bytes < bytes) {
        if (ws->mirror) WW_HIP(hipHostFree(ws->mirror));
        ws->mirror = nullptr;
        ws->mirror_bytes = 0;
        if (hipHostMalloc(&ws->mirror, bytes, hipHostMallocCoherent) != hipSuccess) {
            (void)hipGetLastError();
            return fail(WW_E_OOM, "pinned host allocation of %zu bytes failed", bytes);
        }
        ws->mirror_bytes = bytes;
    }
    *out = ws->mirror;
    return WW_OK;
}

ww_status wait_stream(hipStream_t st) {
    Workspace *ws = current_workspace();
    if (!ws->wait_ev) WW_HIP(hipEventCreateWithFlags(&ws->wait_ev, hipEventDisableTiming));
    WW_HIP(hipEventRecord(ws->wait_ev, st));
    // Poll first: a blocking wait sleeps until an interrupt, which costs
    // tens of microseconds per return and the solver loop returns to the
    // host after every batch of rounds.  Long waits block after 2 ms.
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipEventQuery(ws->wait_ev);
        if (e == hipSuccess) return WW_OK;
        if (e != hipErrorNotReady) WW_HIP(e);
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) break;
    }
    WW_HIP(hipEventSynchronize(ws->wait_ev));
    return WW_OK;
}

ww_status check_lut_params(const ww_lut_params &p) {
    if (p.n_alpha < 2 || p.n_alpha > 4096 || p.n_gamma < 1 || p.n_gamma > 4096 ||
        p.n_eta < 8 || p.n_eta > 16384 || (p.n_eta & 1) || p.n_gpanel < 1 || p.n_gnode < 1 ||
        p.n_gnode > 64 || (int64_t)p.n_gpanel * p.n_gnode > 65536 || p.n_aquad < 2 ||
        p.n_aquad > 65536 || !(p.sigma_span > 0.0) || !(p.sigma_span < 64.0))
        return fail(WW_E_INVALID_ARG, "cost-table parameters out of range");
    return WW_OK;
}

ww_status check_cost_params(const ww_cost_params &p) {
    if (p.box_half < 0 || p.box_half > 16)
        return fail(WW_E_INVALID_ARG, "box_half must lie in [0, 16]");
    if (p.steep_cap_pct < 0 || p.steep_cap_pct > 100 || !(p.steep_thresh_rad >= 0.0))
        return fail(WW_E_INVALID_ARG, "steep-rule parameters out of range");
    if (p.lut_interp != 0 && p.lut_interp != 1)
        return fail(WW_E_INVALID_ARG, "lut_interp must be 0 or 1");
    if (p.looks_frac16 < 0 || p.looks_frac16 > 65535)
        return fail(WW_E_INVALID_ARG, "looks_frac16 must lie in [0, 65535]");
    return WW_OK;
}

static ww_status check_shape(int32_t m, int32_t n) {
    if (m < 1 || n < 1 || (int64_t)m * n >= ((int64_t)1 << 31))
        return fail(WW_E_INVALID_ARG, "image shape %d x %d outside 1 <= m,n, m*n < 2^31", m, n);
    return WW_OK;
}

// Device-resident cost tables, one per (device, looks in 2^-16 fixed point,
// parameters).
struct LutKey {
    int dev, looks_q16;
    ww_lut_params p;
    bool operator<(const LutKey &o) const {
        if (dev != o.dev) return dev < o.dev;
        if (looks_q16 != o.looks_q16) return looks_q16 < o.looks_q16;
        return memcmp(&p, &o.p, sizeof(p)) < 0;
    }
};

// lut_lock() held.  A non-integer number of looks blends the cached tables
// of its two integer neighbours (each built on first use).
static ww_status lut_device_locked(int looks_q16, const ww_lut_params &p, hipStream_t stream,
                                   const int16_t **out) {
    static std::map<LutKey, int16_t *> cache;
    LutKey key;
    memset(&key, 0, sizeof(key));
    key.dev = current_device();
    key.looks_q16 = looks_q16;
    key.p = p;
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return WW_OK;
    }
    const int l0 = looks_q16 >> 16, f = looks_q16 & 0xffff;
    const int16_t *t0 = nullptr, *t1 = nullptr;
    if (f) {
        WW_TRY(lut_device_locked(l0 << 16, p, stream, &t0));
        WW_TRY(lut_device_locked((l0 + 1) << 16, p, stream, &t1));
    }
    int16_t *d = nullptr;
    const size_t n = (size_t)p.n_alpha * p.n_gamma;
    if (hipMalloc(&d, sizeof(int16_t) * n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(WW_E_OOM, "cost-table allocation failed");
    }
    ww_status s = f ? blend_lut_looks(t0, t1, (int64_t)n, f, d, stream) : build_lut_impl(l0, p, d, stream);
    // other streams may use the table as soon as it is in the cache
    if (s == WW_OK && hipStreamSynchronize(stream) != hipSuccess)
        s = fail(WW_E_DEVICE, "cost-table build failed: %s", hipGetErrorString(hipGetLastError()));
    if (s != WW_OK) {
        (void)hipFree(d);
        return s;
    }
    cache[key] = d;
    *out = d;
    return WW_OK;
}

ww_status lut_device(int looks_q16, const ww_lut_params &p, hipStream_t stream, const int16_t **out) {
    std::lock_guard<std::mutex> g(lut_lock());
    return lut_device_locked(looks_q16, p, stream, out);
}

ww_status check_unwrap_args(const float *psi, const float *coh, int m, int n, int looks,
                            const int32_t *K, const float *phi, const ww_cost_params &cp) {
    WW_TRY(check_shape(m, n));
    if (looks < 2 || looks > 64) return fail(WW_E_INVALID_ARG, "looks must lie in [2, 64]");
    if (!psi || !coh || !K || !phi) return fail(WW_E_INVALID_ARG, "input or output array is NULL");
    WW_TRY(check_cost_params(cp));
    if (looks == 64 && cp.looks_frac16) return fail(WW_E_INVALID_ARG, "looks must lie in [2, 64]");
    if (cp.ref_i >= 0 && (cp.ref_i >= m || cp.ref_j < 0 || cp.ref_j >= n))
        return fail(WW_E_INVALID_ARG, "reference pixel outside the image");
    return WW_OK;
}

int64_t unwrap_workspace_bytes(int m, int n) {
    const int64_t N = (int64_t)(m - 1) * (n - 1), nx = (int64_t)m * (n - 1), ny = (int64_t)(m - 1) * n;
    const int64_t NT = (int64_t)ceil_div(m - 1, 32) * ceil_div(n - 1, 32);
    int64_t b = 0;
    b += N + 2 * (2 * nx + 2 * ny) + nx + ny + 64;          // residues, costs, flows, counters
    b += 12 * (nx + ny) + 512 + 4096;                       // steep-rule keys and state
    b += (8 + 8 + 4 + 1 + 16 + 5) * N + 2 * (2 * n + 2 * m) + 4096;  // solver node state and lists
    b += 256 * (4096 * 4 + 8) + 4096;                       // steep pre-pass partial histograms
    b += 40 * NT + 8192 + 8 * std::max<int64_t>(3 * ceil_div(N, 4096), 8192) + 4096;  // tiles, parts
    b += 256 + 4 * (int64_t)m;                              // integration
    return b + b / 8;                                       // the workspace's growth margin
}

ww_status unwrap_impl(const float *psi, const float *coh, const uint8_t *valid, int m, int n,
                      int looks, const ww_cost_params &cp, int32_t *K, float *phi,
                      int64_t *total_out, hipStream_t st, const ww_mcf_params *sched) {
    ww_lut_params lp;
    ww_default_lut_params(&lp);
    const int16_t *lut = nullptr;
    WW_TRY(lut_device((looks << 16) | cp.looks_frac16, lp, st, &lut));
    int64_t nl = (int64_t)(m - 1) * (n - 1), nx = (int64_t)m * (n - 1), ny = (int64_t)(m - 1) * n;
    int8_t *res, *dkx, *dky;
    int16_t *cxp, *cxn, *cyp, *cyn;
    int64_t *gdev;
    WW_TRY(scratch(SLOT_RES, nl, (void **)&res));
    WW_TRY(scratch(SLOT_CXP, 2 * nx, (void **)&cxp));
    WW_TRY(scratch(SLOT_CXN, 2 * nx, (void **)&cxn));
    WW_TRY(scratch(SLOT_CYP, 2 * ny, (void **)&cyp));
    WW_TRY(scratch(SLOT_CYN, 2 * ny, (void **)&cyn));
    WW_TRY(scratch(SLOT_DKX, nx, (void **)&dkx));
    WW_TRY(scratch(SLOT_DKY, ny, (void **)&dky));
    WW_TRY(scratch(SLOT_COUNTERS, 64, (void **)&gdev));
    WW_TRY(residues_impl(psi, valid, m, n, res, nullptr, gdev, st));
    WW_TRY(edge_costs_impl(psi, coh, valid, m, n, lut, lp.n_alpha, lp.n_gamma, cp, cxp, cxn, cyp,
                           cyn, st));
    int64_t total = 0;
    WW_TRY(mcf_impl(res, m, n, cxp, cxn, cyp, cyn, dkx, dky, nullptr, &total, nullptr, st, sched));
    WW_TRY(integrate_impl(psi, valid, dkx, dky, m, n, cp, K, phi, st));
    WW_HIP(hipStreamSynchronize(st));
    *total_out = total;
    return WW_OK;
}

}  // namespace ww

using namespace ww;

extern "C" {

const char *ww_last_error(void) { return g_error.c_str(); }

const char *ww_version(void) { return "ww-gfx950 0.1"; }

void ww_last_mcf_stats(ww_mcf_stats *out) {
    if (!out) return;
    std::lock_guard<std::mutex> g(lock());
    *out = last_mcf_stats();
}

void ww_default_lut_params(ww_lut_params *p) {
    if (!p) return;
    p->n_alpha = 128;
    p->n_gamma = 64;
    p->n_eta = 2048;
    p->n_gpanel = 64;
    p->n_gnode = 16;
    p->n_aquad = 513;
    p->sigma_span = 8.0;
}

void ww_default_cost_params(ww_cost_params *p) {
    if (!p) return;
    p->box_half = 2;
    p->steep_rule = 1;
    p->steep_thresh_rad = 1.0;
    p->steep_cap_pct = 3;
    p->ref_i = -1;
    p->ref_j = -1;
    p->nodata = std::nanf("");
    p->lut_interp = 0;
    p->looks_frac16 = 0;
}

ww_status ww_residues(const float *psi, const uint8_t *valid, int32_t m, int32_t n, int8_t *res,
                      int8_t *perim, int64_t *ground_charge_host, void *stream) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    WW_TRY(check_shape(m, n));
    if (!psi || (!res && (int64_t)(m - 1) * (n - 1) > 0))
        return fail(WW_E_INVALID_ARG, "psi and res must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    int64_t *gdev = nullptr;
    WW_TRY(scratch(SLOT_COUNTERS, 64, (void **)&gdev));
    WW_TRY(residues_impl(psi, valid, m, n, res, perim, gdev, st));
    if (ground_charge_host) {
        WW_HIP(hipMemcpyAsync(ground_charge_host, gdev, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        WW_HIP(hipStreamSynchronize(st));
    }
    return WW_OK;
}

ww_status ww_build_cost_lut(int32_t looks, const ww_lut_params *pin, int16_t *lut_host) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    ww_lut_params p;
    if (pin) p = *pin;
    else ww_default_lut_params(&p);
    WW_TRY(check_lut_params(p));
    if (looks < 2 || looks > 64) return fail(WW_E_INVALID_ARG, "looks must lie in [2, 64]");
    if (!lut_host) return fail(WW_E_INVALID_ARG, "lut_host must be non-NULL");
    const int16_t *d = nullptr;
    WW_TRY(lut_device(looks << 16, p, nullptr, &d));
    WW_HIP(hipMemcpy(lut_host, d, sizeof(int16_t) * (size_t)p.n_alpha * p.n_gamma,
                     hipMemcpyDeviceToHost));
    return WW_OK;
}

ww_status ww_build_cost_lut_q16(int32_t looks_q16, const ww_lut_params *pin, int16_t *lut_host) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    ww_lut_params p;
    if (pin) p = *pin;
    else ww_default_lut_params(&p);
    WW_TRY(check_lut_params(p));
    if (looks_q16 < (2 << 16) || looks_q16 > (64 << 16))
        return fail(WW_E_INVALID_ARG, "looks must lie in [2, 64]");
    if (!lut_host) return fail(WW_E_INVALID_ARG, "lut_host must be non-NULL");
    const int16_t *d = nullptr;
    WW_TRY(lut_device(looks_q16, p, nullptr, &d));
    WW_HIP(hipMemcpy(lut_host, d, sizeof(int16_t) * (size_t)p.n_alpha * p.n_gamma,
                     hipMemcpyDeviceToHost));
    return WW_OK;
}

ww_status ww_edge_costs(const float *psi, const float *coh, const uint8_t *valid, int32_t m,
                        int32_t n, const int16_t *lut, const ww_lut_params *lp,
                        const ww_cost_params *cpin, int16_t *cx_pos, int16_t *cx_neg,
                        int16_t *cy_pos, int16_t *cy_neg, void *stream) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    WW_TRY(check_shape(m, n));
    ww_lut_params p;
    if (lp) p = *lp;
    else ww_default_lut_params(&p);
    ww_cost_params cp;
    if (cpin) cp = *cpin;
    else ww_default_cost_params(&cp);
    WW_TRY(check_cost_params(cp));
    if (p.n_alpha < 2 || p.n_gamma < 1 || p.n_alpha > 4096 || p.n_gamma > 4096)
        return fail(WW_E_INVALID_ARG, "table shape out of range");
    if (!psi || !coh || !lut) return fail(WW_E_INVALID_ARG, "psi, coh and lut must be non-NULL");
    if ((n > 1 && (!cx_pos || !cx_neg)) || (m > 1 && (!cy_pos || !cy_neg)))
        return fail(WW_E_INVALID_ARG, "cost planes must be non-NULL");
    return edge_costs_impl(psi, coh, valid, m, n, lut, p.n_alpha, p.n_gamma, cp, cx_pos, cx_neg,
                           cy_pos, cy_neg, (hipStream_t)stream);
}

ww_status ww_mcf_solve(const int8_t *res, int32_t m, int32_t n, const int16_t *cx_pos,
                       const int16_t *cx_neg, const int16_t *cy_pos, const int16_t *cy_neg,
                       int8_t *dk_x, int8_t *dk_y, int64_t *potentials, int64_t *total_cost_host,
                       ww_mcf_stats *stats_host, void *stream) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    WW_TRY(check_shape(m, n));
    if (!total_cost_host) return fail(WW_E_INVALID_ARG, "total_cost_host must be non-NULL");
    if ((m > 1 && n > 1 && !res) || (n > 1 && (!cx_pos || !cx_neg || !dk_x)) ||
        (m > 1 && (!cy_pos || !cy_neg || !dk_y)))
        return fail(WW_E_INVALID_ARG, "input or output array is NULL");
    return mcf_impl(res, m, n, cx_pos, cx_neg, cy_pos, cy_neg, dk_x, dk_y, potentials,
                    total_cost_host, stats_host, (hipStream_t)stream);
}

ww_status ww_integrate(const float *psi, const uint8_t *valid, const int8_t *dk_x,
                       const int8_t *dk_y, int32_t m, int32_t n, const ww_cost_params *cpin,
                       int32_t *K, float *phi, void *stream) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    WW_TRY(check_shape(m, n));
    ww_cost_params cp;
    if (cpin) cp = *cpin;
    else ww_default_cost_params(&cp);
    if (cp.ref_i >= 0 && (cp.ref_i >= m || cp.ref_j < 0 || cp.ref_j >= n))
        return fail(WW_E_INVALID_ARG, "reference pixel outside the image");
    if (!psi || !K || !phi || (n > 1 && !dk_x) || (m > 1 && !dk_y))
        return fail(WW_E_INVALID_ARG, "input or output array is NULL");
    return integrate_impl(psi, valid, dk_x, dk_y, m, n, cp, K, phi, (hipStream_t)stream);
}

void ww_default_cc_params(ww_cc_params *p) {
    if (!p) return;
    p->threshold = 300;
    p->min_size_frac = 0.001;
}

ww_status ww_connected_components(const int8_t *dk_x, const int8_t *dk_y, const int16_t *cx_pos,
                                  const int16_t *cx_neg, const int16_t *cy_pos,
                                  const int16_t *cy_neg, const uint8_t *valid, int32_t m,
                                  int32_t n, const ww_cc_params *pin, uint32_t *labels,
                                  int64_t *ncomp_host, void *stream) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    WW_TRY(check_shape(m, n));
    ww_cc_params p;
    if (pin) p = *pin;
    else ww_default_cc_params(&p);
    if (p.threshold < 0 || !(p.min_size_frac >= 0.0 && p.min_size_frac <= 1.0))
        return fail(WW_E_INVALID_ARG, "threshold must be >= 0 and min_size_frac in [0, 1]");
    if (!labels || !ncomp_host || (n > 1 && (!dk_x || !cx_pos || !cx_neg)) ||
        (m > 1 && (!dk_y || !cy_pos || !cy_neg)))
        return fail(WW_E_INVALID_ARG, "input or output array is NULL");
    return components_impl(dk_x, dk_y, cx_pos, cx_neg, cy_pos, cy_neg, valid, m, n, p.threshold,
                           p.min_size_frac, labels, ncomp_host, (hipStream_t)stream);
}

ww_status ww_unwrap(const float *psi, const float *coh, const uint8_t *valid, int32_t m,
                    int32_t n, int32_t looks, const ww_cost_params *cpin, int32_t *K, float *phi,
                    int64_t *total_cost_host, void *stream) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    ww_cost_params cp;
    if (cpin) cp = *cpin;
    else ww_default_cost_params(&cp);
    WW_TRY(check_unwrap_args(psi, coh, m, n, looks, K, phi, cp));
    int64_t total = 0;
    WW_TRY(unwrap_impl(psi, coh, valid, m, n, looks, cp, K, phi, &total, (hipStream_t)stream));
    if (total_cost_host) *total_cost_host = total;
    return WW_OK;
}

void ww_default_filter_params(ww_filter_params *p) {
    if (!p) return;
    p->patch = 32;
    p->smooth = 3;
    p->alpha = 0.5f;
}

static ww_status check_filter_params(const ww_filter_params &p) {
    if (p.patch != 16 && p.patch != 32 && p.patch != 64)
        return fail(WW_E_INVALID_ARG, "patch must be 16, 32 or 64");
    if (p.smooth != 1 && p.smooth != 3 && p.smooth != 5)
        return fail(WW_E_INVALID_ARG, "smooth must be 1, 3 or 5");
    if (!(p.alpha >= 0.f && p.alpha <= 4.f)) return fail(WW_E_INVALID_ARG, "alpha must lie in [0, 4]");
    return WW_OK;
}

ww_status ww_goldstein_filter(const float *psi, const uint8_t *valid, int32_t m, int32_t n,
                              const ww_filter_params *pin, float *psi_out, void *stream) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    WW_TRY(check_shape(m, n));
    ww_filter_params p;
    if (pin) p = *pin;
    else ww_default_filter_params(&p);
    WW_TRY(check_filter_params(p));
    if (!psi || !psi_out) return fail(WW_E_INVALID_ARG, "psi and psi_out must be non-NULL");
    return goldstein_impl(psi, valid, m, n, p, psi_out, (hipStream_t)stream);
}

ww_status ww_transfer_ambiguity(const float *psi, const uint8_t *valid, const float *psi_f,
                                const int32_t *K_f, int32_t m, int32_t n, int32_t ref_i,
                                int32_t ref_j, float nodata, int32_t *K, float *phi,
                                void *stream) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    WW_TRY(check_shape(m, n));
    if (!psi || !psi_f || !K_f || !K || !phi)
        return fail(WW_E_INVALID_ARG, "input or output array is NULL");
    if (ref_i >= 0 && (ref_i >= m || ref_j < 0 || ref_j >= n))
        return fail(WW_E_INVALID_ARG, "reference pixel outside the image");
    const int64_t ref = ref_i >= 0 ? (int64_t)ref_i * n + ref_j : -1;
    return transfer_impl(psi, valid, psi_f, K_f, m, n, ref, nullptr, nodata, K, phi,
                         (hipStream_t)stream);
}

ww_status ww_unwrap_filtered(const float *psi, const float *coh, const uint8_t *valid, int32_t m,
                             int32_t n, int32_t looks, const ww_cost_params *cpin,
                             const ww_filter_params *fpin, int32_t *K, float *phi,
                             int64_t *total_cost_host, void *stream) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    ww_cost_params cp;
    if (cpin) cp = *cpin;
    else ww_default_cost_params(&cp);
    WW_TRY(check_unwrap_args(psi, coh, m, n, looks, K, phi, cp));
    ww_filter_params fp;
    if (fpin) fp = *fpin;
    else ww_default_filter_params(&fp);
    WW_TRY(check_filter_params(fp));
    const hipStream_t st = (hipStream_t)stream;
    float *psi_f = nullptr;
    WW_TRY(scratch(SLOT_GS_PSI, sizeof(float) * (size_t)m * n, (void **)&psi_f));
    WW_TRY(goldstein_impl(psi, valid, m, n, fp, psi_f, st));
    int64_t total = 0;
    WW_TRY(unwrap_impl(psi_f, coh, valid, m, n, looks, cp, K, phi, &total, st));
    const int64_t ref = cp.ref_i >= 0 ? (int64_t)cp.ref_i * n + cp.ref_j : -1;
    const long long *ref_dev = cp.ref_i >= 0 ? nullptr : integrate_ref_index();
    if (cp.ref_i < 0 && !ref_dev) return fail(WW_E_DEVICE, "integration state unavailable");
    WW_TRY(transfer_impl(psi, valid, psi_f, K, m, n, ref, ref_dev, cp.nodata, K, phi, st));
    WW_HIP(hipStreamSynchronize(st));
    if (total_cost_host) *total_cost_host = total;
    return WW_OK;
}

void ww_default_bridge_params(ww_bridge_params *p) {
    if (!p) return;
    p->half_window = 32;
}

ww_status ww_bridge(const float *psi, const uint8_t *valid, const int32_t *K_in, int32_t m,
                    int32_t n, const ww_bridge_params *pin, float nodata, int32_t *K_out,
                    float *phi, uint32_t *regions, int64_t *nregions_host, void *stream) {
    std::lock_guard<std::mutex> g(lock());
    clear_error();
    WW_TRY(check_shape(m, n));
    ww_bridge_params p;
    if (pin) p = *pin;
    else ww_default_bridge_params(&p);
    if (!psi || !K_in || !K_out || !phi || !nregions_host)
        return fail(WW_E_INVALID_ARG, "input or output array is NULL");
    return bridge_impl(psi, valid, K_in, m, n, p.half_window, nodata, K_out, phi, regions,
                       nregions_host, (hipStream_t)stream);
}

}  // extern "C"
