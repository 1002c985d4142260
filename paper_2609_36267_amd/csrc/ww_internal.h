// Internal declarations of the gfx950 unwrapper library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ww.h"

namespace ww {

// ---------------------------------------------------------------- errors ---

ww_status fail(ww_status code, const char *fmt, ...);
void clear_error();

#define WW_HIP(call)                                                               \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return ::ww::fail(WW_E_DEVICE, "%s failed: %s (%s:%d)", #call,         \
                              hipGetErrorString(e_), __FILE__, __LINE__);          \
    } while (0)

#define WW_TRY(expr)                           \
    do {                                       \
        ww_status s_ = (expr);                 \
        if (s_ != WW_OK) return s_;            \
    } while (0)

#define WW_LAUNCH_CHECK() WW_HIP(hipGetLastError())

// ------------------------------------------------------------- workspace ---

// Grow-only device buffers owned by the library.  A workspace holds one
// buffer per slot, a pinned host staging area, timing events and the
// statistics of its last solve.  The plain entry points use one workspace
// per device and serialise on `lock()`; each worker of the job server owns a
// workspace of its own (installed for its thread with set_thread_workspace),
// so that concurrent jobs never share a buffer.
struct Buffer {
    void *ptr = nullptr;
    size_t bytes = 0;
    size_t clean = 0;  // leading bytes its user knows to hold its rest value
};

struct Workspace;

std::mutex &lock();
int current_device();
// Workspace used by the calling thread: its installed one, else the
// per-device default.
Workspace *current_workspace();
void set_thread_workspace(Workspace *ws);
Workspace *workspace_create(int device);
void workspace_destroy(Workspace *ws);
// Device bytes held by a workspace.
size_t workspace_bytes(const Workspace *ws);
// Returns a device buffer of at least `bytes` for (workspace, slot);
// contents are unspecified.
ww_status scratch(int slot, size_t bytes, void **out);
// The clean mark of (workspace, slot): the leading bytes that the slot's
// user left in a known rest state (reset to 0 when the buffer is replaced).
size_t *scratch_clean(int slot);
// Pinned host staging area (for counters read back by the solver loop).
ww_status host_scratch(size_t bytes, void **out);
// Coherent pinned host block of the current workspace that kernels write
// into directly (the solver's counters after each batch of rounds).
ww_status host_mirror(size_t bytes, void **out);
// Waits for all work queued on `st` so far (polls briefly, then blocks).
ww_status wait_stream(hipStream_t st);
// Serialises construction of the shared cost-table cache.
std::mutex &lut_lock();

enum Slot {
    SLOT_RES = 0, SLOT_CXP, SLOT_CXN, SLOT_CYP, SLOT_CYN, SLOT_DKX, SLOT_DKY, SLOT_LUT,
    SLOT_COUNTERS, SLOT_STEEP, SLOT_STEEP_KEYS,
    SLOT_MCF_LAB, SLOT_MCF_POT, SLOT_MCF_EX, SLOT_MCF_BEST, SLOT_MCF_TILES,
    SLOT_MCF_LISTS, SLOT_MCF_NODES, SLOT_MCF_PART, SLOT_INTEG,
    SLOT_LUT_WORK, SLOT_CC_LABEL, SLOT_CC_SIZE, SLOT_CC_SMALL,
    SLOT_GS_PLANES, SLOT_GS_SHIFT, SLOT_GS_PSI,
    SLOT_BR_LABEL, SLOT_BR_RANK, SLOT_BR_SMALL, SLOT_BR_SIZES, SLOT_BR_Q,
    SLOT_MCF_FLIP,
    SLOT_B_RES, SLOT_B_FX, SLOT_B_FY, SLOT_B_COST, SLOT_B_IO, SLOT_STEEP_PARTS,
    SLOT_COUNT
};

// ------------------------------------------------------------- constants ---

// Double nearest to pi and to 2 pi.  The double nearest pi lies below pi and
// no double lies in (PI_D, pi], so "diff > PI_D" is the exact test diff > pi.
constexpr double PI_D = 3.141592653589793115997963468544185161590576171875;
constexpr double TWO_PI_D = 6.28318530717958623199592693708837032318115234375;
constexpr int64_t PI_FIX = 3294199;  // round(pi * 2^20)

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------ device helpers ---

// Cycles removed by wrapping a phase difference into (-pi, pi].
__device__ __forceinline__ int wrap_cycles(double diff) {
    return (diff > PI_D) ? 1 : ((diff <= -PI_D) ? -1 : 0);
}

__device__ __forceinline__ double phase_at(const float *psi, const uint8_t *valid, int64_t k) {
    return (valid == nullptr || valid[k]) ? (double)psi[k] : 0.0;
}

// -------------------------------------------------------- entry helpers ---

// Cached device table at looks_q16 / 2^16 looks (built or blended on first use).
ww_status lut_device(int looks_q16, const ww_lut_params &p, hipStream_t stream, const int16_t **out);
// out[k] = floor((T0[k] (2^16 - f) + T1[k] f) / 2^16), k < n.
ww_status blend_lut_looks(const int16_t *T0, const int16_t *T1, int64_t n, int f, int16_t *out,
                          hipStream_t stream);
ww_status residues_impl(const float *psi, const uint8_t *valid, int m, int n, int8_t *res,
                        int8_t *perim, int64_t *ground_dev, hipStream_t stream);
ww_status edge_costs_impl(const float *psi, const float *coh, const uint8_t *valid, int m, int n,
                          const int16_t *lut, int n_alpha, int n_gamma, const ww_cost_params &cp,
                          int16_t *cxp, int16_t *cxn, int16_t *cyp, int16_t *cyn,
                          hipStream_t stream);
// One image of a min-cost-flow solve: shape, residues, cost planes, flow
// planes (outputs) and where its total cost goes.
struct McfJob {
    int m, n;
    const int8_t *res;
    const int16_t *cxp, *cxn, *cyp, *cyn;
    int8_t *dkx, *dky;
    int64_t *total;
};
// One image; sched NULL = the process-wide schedule.
ww_status mcf_impl(const int8_t *res, int m, int n, const int16_t *cxp, const int16_t *cxn,
                   const int16_t *cyp, const int16_t *cyn, int8_t *dkx, int8_t *dky,
                   int64_t *pot_out, int64_t *total, ww_mcf_stats *stats, hipStream_t stream,
                   const ww_mcf_params *sched = nullptr);
// Several images in one solve (their union graph).  Every job has m, n >= 2;
// the jobs' residues, x-flow planes and y-flow planes each lie in one
// contiguous array in job order (res_all, fx_all, fy_all).
ww_status mcf_multi_impl(const std::vector<McfJob> &jobs, const int8_t *res_all, int8_t *fx_all,
                         int8_t *fy_all, ww_mcf_stats *stats, const ww_mcf_params &sched,
                         hipStream_t stream);
ww_mcf_params process_mcf_params();
ww_status check_mcf_params(const ww_mcf_params &p);
ww_status integrate_impl(const float *psi, const uint8_t *valid, const int8_t *dkx,
                         const int8_t *dky, int m, int n, const ww_cost_params &cp, int32_t *K,
                         float *phi, hipStream_t stream);
ww_status build_lut_impl(int looks, const ww_lut_params &p, int16_t *lut_dev, hipStream_t stream);
ww_status components_impl(const int8_t *dkx, const int8_t *dky, const int16_t *cxp,
                          const int16_t *cxn, const int16_t *cyp, const int16_t *cyn,
                          const uint8_t *valid, int m, int n, int threshold, double min_size_frac,
                          uint32_t *labels, int64_t *ncomp, hipStream_t stream,
                          int all_edges = 0, uint32_t *sizes_out = nullptr);
// Bridging of mask-separated regions.
ww_status bridge_impl(const float *psi, const uint8_t *valid, const int32_t *K_in, int m, int n,
                      int half_window, float nodata, int32_t *K_out, float *phi,
                      uint32_t *regions, int64_t *nregions, hipStream_t stream);

ww_mcf_stats &last_mcf_stats();  // of the current workspace

// Whole unwrap (residues, costs, solve, integration) on `stream`, using the
// current workspace; the cost table comes from the shared cache.
ww_status unwrap_impl(const float *psi, const float *coh, const uint8_t *valid, int m, int n,
                      int looks, const ww_cost_params &cp, int32_t *K, float *phi,
                      int64_t *total, hipStream_t stream, const ww_mcf_params *sched = nullptr);
// Device bytes that unwrap_impl's workspace requests for an m x n image
// (every slot it and its steps ask for, with the allocator's growth margin).
int64_t unwrap_workspace_bytes(int m, int n);
ww_status check_unwrap_args(const float *psi, const float *coh, int m, int n, int looks,
                            const int32_t *K, const float *phi, const ww_cost_params &cp);

ww_status check_lut_params(const ww_lut_params &p);
// Goldstein filter of the wrapped phase (out may alias psi) and the transfer
// of cycle counts found on a filtered phase back onto psi; K may alias K_f.
// The reference pixel is *ref_dev when ref_dev is non-NULL, else ref_host;
// outside [0, m n) there is none.
ww_status goldstein_impl(const float *psi, const uint8_t *valid, int m, int n,
                         const ww_filter_params &fp, float *out, hipStream_t stream);
ww_status transfer_impl(const float *psi, const uint8_t *valid, const float *psi_f,
                        const int32_t *K_f, int m, int n, int64_t ref_host,
                        const long long *ref_dev, float nodata, int32_t *K, float *phi,
                        hipStream_t stream);
// Device address of the reference pixel index found by the last integration
// on the current workspace (first valid pixel, or m n when there is none).
const long long *integrate_ref_index();

ww_status check_cost_params(const ww_cost_params &p);

}  // namespace ww
