// Many interferograms on one device.
//
// The job server: a fixed set of worker threads, each with its own HIP
// stream and private workspace, fed from a queue with admission by
// device-memory footprint.  Jobs on different workers overlap on the GPU
// (their round kernels interleave on the device's hardware queues); every
// job runs exactly the computation of ww_unwrap.
//
// The batch call: a stack of jobs whose min-cost-flow problems are solved
// together, one solve per group of jobs over the union of their graphs
// (mcf_multi_impl), with residues, costs and integration per job.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <vector>

#include "ww_internal.h"

namespace ww {

namespace {

double now_s() {
    static const auto t0 = std::chrono::steady_clock::now();
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Device copies of a host-side job's inputs (psi, coh, mask) and outputs
// (K, phi), per pixel.
constexpr int64_t IO_BYTES_PER_PX = 4 + 4 + 1 + 4 + 4;
// a queued job older than this blocks the jobs behind it until it fits
constexpr double STARVE_S = 1.0;

int64_t footprint(const ww_job *j) {
    if (j->m < 1 || j->n < 1) return 0;
    return unwrap_workspace_bytes(j->m, j->n) + (j->host_io ? IO_BYTES_PER_PX * j->m * (int64_t)j->n : 0);
}

struct Worker {
    hipStream_t stream = nullptr;
    Workspace *ws = nullptr;
    // device copies for host-side jobs (grow-only)
    Buffer io[5];
    int64_t held = 0;     // device bytes its workspace and copies hold (grow-only)
    int64_t running = 0;  // footprint of the job it runs, 0 when idle
};

ww_status grow(Buffer &b, size_t bytes) {
    if (b.bytes >= bytes) return WW_OK;
    if (b.ptr) {
        WW_HIP(hipFree(b.ptr));
        b.ptr = nullptr;
        b.bytes = 0;
    }
    const size_t want = bytes + bytes / 8 + 256;
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        b.ptr = nullptr;
        return fail(WW_E_OOM, "device allocation of %zu bytes failed", want);
    }
    b.bytes = want;
    return WW_OK;
}

// One job on one worker (the worker's workspace is installed for the thread).
ww_status run_job(Worker &w, ww_job *j) {
    ww_cost_params cp;
    ww_default_cost_params(&cp);
    WW_TRY(check_unwrap_args(j->psi, j->coh, j->m, j->n, j->looks, j->K, j->phi, cp));
    if (j->use_sched) WW_TRY(check_mcf_params(j->sched));
    const size_t px = (size_t)j->m * j->n;
    hipStream_t st = w.stream;
    const float *psi = j->psi, *coh = j->coh;
    const uint8_t *valid = j->valid;
    int32_t *K = j->K;
    float *phi = j->phi;
    if (j->host_io) {
        WW_TRY(grow(w.io[0], 4 * px));
        WW_TRY(grow(w.io[1], 4 * px));
        WW_TRY(grow(w.io[2], px));
        WW_TRY(grow(w.io[3], 4 * px));
        WW_TRY(grow(w.io[4], 4 * px));
        WW_HIP(hipMemcpyAsync(w.io[0].ptr, j->psi, 4 * px, hipMemcpyHostToDevice, st));
        WW_HIP(hipMemcpyAsync(w.io[1].ptr, j->coh, 4 * px, hipMemcpyHostToDevice, st));
        if (j->valid) WW_HIP(hipMemcpyAsync(w.io[2].ptr, j->valid, px, hipMemcpyHostToDevice, st));
        psi = (const float *)w.io[0].ptr;
        coh = (const float *)w.io[1].ptr;
        valid = j->valid ? (const uint8_t *)w.io[2].ptr : nullptr;
        K = (int32_t *)w.io[3].ptr;
        phi = (float *)w.io[4].ptr;
    }
    int64_t total = 0;
    WW_TRY(unwrap_impl(psi, coh, valid, j->m, j->n, j->looks, cp, K, phi, &total, st,
                       j->use_sched ? &j->sched : nullptr));
    if (j->host_io) {
        WW_HIP(hipMemcpyAsync(j->K, K, 4 * px, hipMemcpyDeviceToHost, st));
        WW_HIP(hipMemcpyAsync(j->phi, phi, 4 * px, hipMemcpyDeviceToHost, st));
        WW_HIP(hipStreamSynchronize(st));
    }
    j->total_cost = total;
    return WW_OK;
}

// ------------------------------------------------------------- batches ---

inline size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// One group of valid jobs (each m, n >= 2), solved together on stream st
// with the current workspace.  Totals go into the jobs; nothing else of
// the jobs is touched.
ww_status batch_group(ww_job *const *jobs, int nj, const ww_mcf_params &sp, hipStream_t st) {
    ww_cost_params cp;
    ww_default_cost_params(&cp);
    ww_lut_params lp;
    ww_default_lut_params(&lp);
    size_t res_bytes = 0, nx_all = 0, ny_all = 0, cost_bytes = 0, io_bytes = 0;
    std::vector<size_t> coff(nj), ioff(nj);
    for (int k = 0; k < nj; ++k) {
        const ww_job *j = jobs[k];
        const size_t px = (size_t)j->m * j->n, nx = (size_t)j->m * (j->n - 1), ny = (size_t)(j->m - 1) * j->n;
        res_bytes += (size_t)(j->m - 1) * (j->n - 1);
        nx_all += nx;
        ny_all += ny;
        coff[k] = cost_bytes;
        cost_bytes += 2 * up256(2 * nx) + 2 * up256(2 * ny);
        ioff[k] = io_bytes;
        if (j->host_io) io_bytes += 4 * up256(4 * px) + up256(px);
    }
    int8_t *res_all = nullptr, *fx_all = nullptr, *fy_all = nullptr;
    char *costs = nullptr, *io = nullptr;
    int64_t *gdev = nullptr;
    WW_TRY(scratch(SLOT_B_RES, res_bytes + 64, (void **)&res_all));
    WW_TRY(scratch(SLOT_B_FX, nx_all + 64, (void **)&fx_all));
    WW_TRY(scratch(SLOT_B_FY, ny_all + 64, (void **)&fy_all));
    WW_TRY(scratch(SLOT_B_COST, cost_bytes + 256, (void **)&costs));
    if (io_bytes) WW_TRY(scratch(SLOT_B_IO, io_bytes, (void **)&io));
    WW_TRY(scratch(SLOT_COUNTERS, 64, (void **)&gdev));
    std::vector<McfJob> mj(nj);
    std::vector<int64_t> totals(nj, 0);
    std::vector<const float *> P(nj);
    std::vector<const uint8_t *> V(nj);
    std::vector<int32_t *> KK(nj);
    std::vector<float *> PH(nj);
    size_t noff = 0, xoff = 0, yoff = 0;
    for (int k = 0; k < nj; ++k) {
        ww_job *j = jobs[k];
        const size_t px = (size_t)j->m * j->n, nx = (size_t)j->m * (j->n - 1), ny = (size_t)(j->m - 1) * j->n;
        const float *psi = j->psi, *coh = j->coh;
        const uint8_t *valid = j->valid;
        int32_t *K = j->K;
        float *phi = j->phi;
        if (j->host_io) {
            char *b = io + ioff[k];
            float *dpsi = (float *)b, *dcoh = (float *)(b + up256(4 * px));
            K = (int32_t *)(b + 2 * up256(4 * px));
            phi = (float *)(b + 3 * up256(4 * px));
            uint8_t *dval = (uint8_t *)(b + 4 * up256(4 * px));
            WW_HIP(hipMemcpyAsync(dpsi, j->psi, 4 * px, hipMemcpyHostToDevice, st));
            WW_HIP(hipMemcpyAsync(dcoh, j->coh, 4 * px, hipMemcpyHostToDevice, st));
            if (j->valid) WW_HIP(hipMemcpyAsync(dval, j->valid, px, hipMemcpyHostToDevice, st));
            psi = dpsi;
            coh = dcoh;
            valid = j->valid ? dval : nullptr;
        }
        P[k] = psi;
        V[k] = valid;
        KK[k] = K;
        PH[k] = phi;
        int16_t *cxp = (int16_t *)(costs + coff[k]);
        int16_t *cxn = (int16_t *)(costs + coff[k] + up256(2 * nx));
        int16_t *cyp = (int16_t *)(costs + coff[k] + 2 * up256(2 * nx));
        int16_t *cyn = (int16_t *)(costs + coff[k] + 2 * up256(2 * nx) + up256(2 * ny));
        const int16_t *lut = nullptr;
        WW_TRY(lut_device(j->looks << 16, lp, st, &lut));
        WW_TRY(residues_impl(psi, valid, j->m, j->n, res_all + noff, nullptr, gdev, st));
        WW_TRY(edge_costs_impl(psi, coh, valid, j->m, j->n, lut, lp.n_alpha, lp.n_gamma, cp, cxp, cxn, cyp,
                               cyn, st));
        mj[k] = McfJob{j->m, j->n, res_all + noff, cxp, cxn, cyp, cyn, fx_all + xoff, fy_all + yoff, &totals[k]};
        noff += (size_t)(j->m - 1) * (j->n - 1);
        xoff += nx;
        yoff += ny;
    }
    WW_TRY(mcf_multi_impl(mj, res_all, fx_all, fy_all, nullptr, sp, st));
    for (int k = 0; k < nj; ++k) {
        ww_job *j = jobs[k];
        const size_t px = (size_t)j->m * j->n;
        WW_TRY(integrate_impl(P[k], V[k], mj[k].dkx, mj[k].dky, j->m, j->n, cp, KK[k], PH[k], st));
        if (j->host_io) {
            WW_HIP(hipMemcpyAsync(j->K, KK[k], 4 * px, hipMemcpyDeviceToHost, st));
            WW_HIP(hipMemcpyAsync(j->phi, PH[k], 4 * px, hipMemcpyDeviceToHost, st));
        }
    }
    WW_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < nj; ++k) jobs[k]->total_cost = totals[k];
    return WW_OK;
}

// Jobs per group and pixels per group at most.
constexpr int GROUP_MAX_JOBS = 256;
constexpr int64_t GROUP_MAX_PX = 400ll << 20;

}  // namespace

}  // namespace ww

using namespace ww;

struct ww_server {
    int device = 0;
    int64_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work;  // workers: a job was queued or memory freed
    std::condition_variable cv_done;  // pollers: a job finished
    std::deque<ww_job *> pending;
    std::deque<ww_job *> done;
    int running = 0;
    int64_t in_flight = 0;  // submitted, not yet polled
    bool stopping = false;
    std::vector<Worker> workers;
    std::vector<std::thread> threads;

    // Device bytes held or reserved by every worker but w (lock held).
    int64_t others(int w) const {
        int64_t s = 0;
        for (int k = 0; k < (int)workers.size(); ++k)
            if (k != w) s += std::max(workers[k].held, workers[k].running);
        return s;
    }

    // Picks the job for worker w to start (lock held): the first queued job
    // that fits beside what the other workers hold, unless the head has
    // waited past the starvation bound; a job runs alone when nothing else
    // runs, whatever its size.
    ww_job *pick(int w, double t) {
        if (pending.empty()) return nullptr;
        const bool head_only = t - pending.front()->t_submit > STARVE_S;
        const int64_t rest = others(w);
        for (auto it = pending.begin(); it != pending.end(); ++it) {
            const int64_t f = std::max(footprint(*it), workers[w].held);
            if (rest + f <= budget || running == 0) {
                ww_job *j = *it;
                pending.erase(it);
                return j;
            }
            if (head_only) break;
        }
        return nullptr;
    }

    void worker_main(int k) {
        (void)hipSetDevice(device);
        Worker &w = workers[k];
        set_thread_workspace(w.ws);
        for (;;) {
            ww_job *j = nullptr;
            {
                std::unique_lock<std::mutex> g(mu);
                for (;;) {
                    j = pick(k, now_s());
                    if (j || (stopping && pending.empty())) break;
                    // a starving head re-checks periodically
                    cv_work.wait_for(g, std::chrono::milliseconds(50));
                }
                if (!j) break;
                j->footprint_bytes = footprint(j);
                w.running = j->footprint_bytes;
                ++running;
            }
            j->t_start = now_s();
            clear_error();
            const ww_status s = run_job(w, j);
            j->status = s;
            j->error[0] = 0;
            if (s != WW_OK) {
                strncpy(j->error, ww_last_error(), sizeof(j->error) - 1);
                j->error[sizeof(j->error) - 1] = 0;
            }
            j->t_end = now_s();
            int64_t held = (int64_t)workspace_bytes(w.ws);
            for (auto &b : w.io) held += (int64_t)b.bytes;
            {
                std::lock_guard<std::mutex> g(mu);
                w.held = held;
                w.running = 0;
                --running;
                done.push_back(j);
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
        set_thread_workspace(nullptr);
    }
};

extern "C" {

double ww_clock(void) { return now_s(); }

ww_status ww_server_create(int32_t slots, int64_t hbm_budget_bytes, ww_server **out) {
    clear_error();
    if (!out || slots < 1 || slots > 64)
        return fail(WW_E_INVALID_ARG, "slots must lie in [1, 64] and out must be non-NULL");
    *out = nullptr;
    ww_server *s = new ww_server();
    s->device = current_device();
    if (hbm_budget_bytes <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return fail(WW_E_DEVICE, "hipMemGetInfo failed");
        }
        hbm_budget_bytes = (int64_t)(fr / 4 * 3);
    }
    s->budget = hbm_budget_bytes;
    s->workers.resize(slots);
    for (int k = 0; k < slots; ++k) {
        Worker &w = s->workers[k];
        if (hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess) {
            for (int q = 0; q < k; ++q) {
                (void)hipStreamDestroy(s->workers[q].stream);
                workspace_destroy(s->workers[q].ws);
            }
            delete s;
            return fail(WW_E_DEVICE, "stream creation failed");
        }
        w.ws = workspace_create(s->device);
    }
    for (int k = 0; k < slots; ++k) s->threads.emplace_back(&ww_server::worker_main, s, k);
    *out = s;
    return WW_OK;
}

ww_status ww_server_submit(ww_server *s, ww_job *job) {
    if (!s || !job) return fail(WW_E_INVALID_ARG, "server and job must be non-NULL");
    job->status = WW_OK;
    job->total_cost = 0;
    job->t_start = job->t_end = 0.0;
    job->footprint_bytes = 0;
    job->error[0] = 0;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stopping) return fail(WW_E_INVALID_ARG, "server is stopping");
        job->t_submit = now_s();
        s->pending.push_back(job);
        ++s->in_flight;
    }
    s->cv_work.notify_all();
    return WW_OK;
}

int32_t ww_server_poll(ww_server *s, ww_job **out, int32_t max_done, int32_t wait_ms) {
    if (!s || !out || max_done < 1) return 0;
    std::unique_lock<std::mutex> g(s->mu);
    auto ready = [&] {
        return !s->done.empty() || (wait_ms < 0 && s->pending.empty() && s->running == 0);
    };
    if (wait_ms < 0) s->cv_done.wait(g, ready);
    else if (wait_ms > 0) s->cv_done.wait_for(g, std::chrono::milliseconds(wait_ms), ready);
    int32_t k = 0;
    while (k < max_done && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
        --s->in_flight;
    }
    return k;
}

int64_t ww_server_in_flight(ww_server *s) {
    if (!s) return 0;
    std::lock_guard<std::mutex> g(s->mu);
    return s->in_flight;
}

ww_status ww_server_destroy(ww_server *s) {
    if (!s) return WW_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->threads) t.join();
    for (auto &w : s->workers) {
        (void)hipStreamSynchronize(w.stream);
        (void)hipStreamDestroy(w.stream);
        for (auto &b : w.io)
            if (b.ptr) (void)hipFree(b.ptr);
        workspace_destroy(w.ws);
    }
    delete s;
    return WW_OK;
}

ww_status ww_unwrap_batch(ww_job *jobs, int32_t njobs, int32_t group, const ww_mcf_params *sched) {
    std::lock_guard<std::mutex> lk(lock());
    clear_error();
    if (njobs < 0 || (njobs > 0 && !jobs)) return fail(WW_E_INVALID_ARG, "bad job array");
    if (group < 0) return fail(WW_E_INVALID_ARG, "group must be >= 0");
    if (sched) WW_TRY(check_mcf_params(*sched));
    if (njobs == 0) return WW_OK;
    const int gmax = (group == 0 || group > GROUP_MAX_JOBS) ? GROUP_MAX_JOBS : group;
    const ww_mcf_params sp = sched ? *sched : process_mcf_params();
    ww_cost_params cp;
    ww_default_cost_params(&cp);
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
        return fail(WW_E_DEVICE, "stream creation failed");
    auto finish = [&](ww_job *j, ww_status s, double t0) {
        j->status = s;
        j->error[0] = 0;
        if (s != WW_OK) {
            strncpy(j->error, ww_last_error(), sizeof(j->error) - 1);
            j->error[sizeof(j->error) - 1] = 0;
        }
        j->t_start = t0;
        j->t_end = now_s();
    };
    const double t_sub = now_s();
    std::vector<ww_job *> valid_jobs;
    for (int k = 0; k < njobs; ++k) {
        ww_job *j = &jobs[k];
        j->t_submit = t_sub;
        j->total_cost = 0;
        j->footprint_bytes = footprint(j);
        clear_error();
        ww_status s = check_unwrap_args(j->psi, j->coh, j->m, j->n, j->looks, j->K, j->phi, cp);
        if (s != WW_OK) {
            finish(j, s, t_sub);
            continue;
        }
        if (j->m < 2 || j->n < 2) {  // no loops: nothing to solve
            const double t0 = now_s();
            if (j->host_io) s = fail(WW_E_INVALID_ARG, "batch: host-side jobs need m, n >= 2");
            else s = unwrap_impl(j->psi, j->coh, j->valid, j->m, j->n, j->looks, cp, j->K, j->phi,
                                 &j->total_cost, st, &sp);
            finish(j, s, t0);
            continue;
        }
        valid_jobs.push_back(j);
    }
    size_t a = 0;
    while (a < valid_jobs.size()) {
        size_t b = a;
        int64_t px = 0, loops = 0;
        while (b < valid_jobs.size() && (int)(b - a) < gmax) {
            const ww_job *j = valid_jobs[b];
            const int64_t p = (int64_t)j->m * j->n, l = (int64_t)(j->m - 1) * (j->n - 1);
            if (b > a && (px + p > GROUP_MAX_PX || loops + l >= (1ll << 31) - 512)) break;
            px += p;
            loops += l;
            ++b;
        }
        const double t0 = now_s();
        clear_error();
        ww_status s = batch_group(valid_jobs.data() + a, (int)(b - a), sp, st);
        if (s == WW_OK) {
            for (size_t k = a; k < b; ++k) finish(valid_jobs[k], WW_OK, t0);
        } else {
            // isolate the failure: every job of the group alone
            (void)hipStreamSynchronize(st);
            for (size_t k = a; k < b; ++k) {
                const double t1 = now_s();
                clear_error();
                ww_status s1 = batch_group(valid_jobs.data() + k, 1, sp, st);
                finish(valid_jobs[k], s1, t1);
            }
        }
        a = b;
    }
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    for (int k = 0; k < njobs; ++k)
        if (jobs[k].status != WW_OK) return fail(jobs[k].status, "job %d: %s", k, jobs[k].error);
    return WW_OK;
}

}  // extern "C"
