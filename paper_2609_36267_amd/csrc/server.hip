// Job server for many interferograms on one device: a fixed set of worker
// threads, each with its own HIP stream and private workspace, fed from a
// queue with admission by device-memory footprint.  Jobs on different
// workers overlap on the GPU (their round kernels interleave on the device's
// hardware queues); every job runs exactly the computation of ww_unwrap.
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

// Device bytes one job holds while it runs: the workspace of the whole path
// per pixel (residues 1, four cost planes 8, two flow planes 2, solver
// labels 8 + root picks 8 + potentials 4 + excess 1 + node lists 16) and,
// for host-side jobs, the device copies of the inputs (9) and outputs (8).
constexpr int64_t WS_BYTES_PER_PX = 1 + 8 + 2 + 8 + 8 + 4 + 1 + 16;
constexpr int64_t IO_BYTES_PER_PX = 4 + 4 + 1 + 4 + 4;
constexpr int64_t WS_FIXED_BYTES = 8 << 20;
// a queued job older than this blocks the jobs behind it until it fits
constexpr double STARVE_S = 1.0;

int64_t footprint(const ww_job *j) {
    const int64_t px = (int64_t)j->m * j->n;
    return WS_FIXED_BYTES + px * (WS_BYTES_PER_PX + (j->host_io ? IO_BYTES_PER_PX : 0));
}

struct Worker {
    hipStream_t stream = nullptr;
    Workspace *ws = nullptr;
    // device copies for host-side jobs (grow-only)
    Buffer io[5];
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
    WW_TRY(unwrap_impl(psi, coh, valid, j->m, j->n, j->looks, cp, K, phi, &total, st));
    if (j->host_io) {
        WW_HIP(hipMemcpyAsync(j->K, K, 4 * px, hipMemcpyDeviceToHost, st));
        WW_HIP(hipMemcpyAsync(j->phi, phi, 4 * px, hipMemcpyDeviceToHost, st));
        WW_HIP(hipStreamSynchronize(st));
    }
    j->total_cost = total;
    return WW_OK;
}

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
    int64_t reserved = 0;  // footprint of the running jobs
    int running = 0;
    int64_t in_flight = 0;  // submitted, not yet polled
    bool stopping = false;
    std::vector<Worker> workers;
    std::vector<std::thread> threads;

    // Picks the job to start (lock held): the first queued job that fits
    // beside the running ones, unless the head has waited past the
    // starvation bound; a job larger than the budget runs alone.
    ww_job *pick(double t) {
        if (pending.empty()) return nullptr;
        const bool head_only = t - pending.front()->t_submit > STARVE_S;
        for (auto it = pending.begin(); it != pending.end(); ++it) {
            const int64_t f = footprint(*it);
            if (reserved + f <= budget || running == 0) {
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
                    j = pick(now_s());
                    if (j || (stopping && pending.empty())) break;
                    // a starving head re-checks periodically
                    cv_work.wait_for(g, std::chrono::milliseconds(50));
                }
                if (!j) break;
                j->footprint_bytes = footprint(j);
                reserved += j->footprint_bytes;
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
            {
                std::lock_guard<std::mutex> g(mu);
                reserved -= j->footprint_bytes;
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

ww_status ww_unwrap_batch(ww_job *jobs, int32_t njobs, int32_t slots) {
    clear_error();
    if (njobs < 0 || (njobs > 0 && !jobs)) return fail(WW_E_INVALID_ARG, "bad job array");
    if (njobs == 0) return WW_OK;
    ww_server *s = nullptr;
    WW_TRY(ww_server_create(slots, 0, &s));
    std::vector<int> order(njobs);
    for (int k = 0; k < njobs; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)jobs[a].m * jobs[a].n > (int64_t)jobs[b].m * jobs[b].n;
    });
    for (int k : order) {
        ww_status st = ww_server_submit(s, &jobs[k]);
        if (st != WW_OK) {
            (void)ww_server_destroy(s);
            return st;
        }
    }
    std::vector<ww_job *> buf(njobs);
    int64_t got = 0;
    while (got < njobs) got += ww_server_poll(s, buf.data(), njobs, -1);
    (void)ww_server_destroy(s);
    for (int k = 0; k < njobs; ++k)
        if (jobs[k].status != WW_OK) return fail(jobs[k].status, "job %d: %s", k, jobs[k].error);
    return WW_OK;
}

}  // extern "C"
