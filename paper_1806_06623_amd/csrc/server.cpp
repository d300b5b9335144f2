// Serving loop with continuous batching.
//
// Requests (grid class, device rho/phi, G, optional scheduled arrival time)
// are queued by any host thread.  One scheduler thread admits them in arrival
// order as soon as (a) their arrival time has passed, (b) a stream slot is
// free and (c) their workspace fits in the caller's device memory pool
// (first-fit free-list allocator; the plans and their eigenbases stay
// resident).  Admitted solves run concurrently on the slot streams; the
// scheduler polls their completion events, returns workspace and slot, and
// records arrival / admission / completion times.  A request is never split
// or reordered across kernels, so its result is bitwise the one of a lone
// spp_solve of the same plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) with coalescing frees; offsets are
// multiples of 256 bytes.
class PoolAllocator {
public:
    explicit PoolAllocator(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;   // offset -> length
};

// Workspace bytes of one request.
size_t request_workspace(const spp_plan_s* p, const spp_request& r)
{
    return spp_align256(r.precision == SPP_MIXED_FP32 ? spp_mixed_workspace_bytes(p)
                                                     : spp_path_workspace_bytes(p, spp_plan_fused(p)));
}

struct Pending {
    spp_request req;
    double arrival;   // seconds on the server clock
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    Pending job{};
    size_t ws_off = 0, ws_bytes = 0;
    double admitted = 0.0;
};

}  // namespace

struct spp_server_s {
    std::vector<const spp_plan_s*> plans;
    char* pool = nullptr;
    size_t pool_bytes = 0;
    int device = 0;
    PoolAllocator alloc{0};
    std::vector<Slot> slots;
    Clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Pending> queue;
    std::vector<spp_completion> done;
    long long submitted = 0, completed = 0;
    bool stop = false;
    std::string error;
    std::thread worker;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run();
};

void spp_server_s::run()
{
    (void)hipSetDevice(device);
    std::vector<Pending> admitted_now;
    for (;;) {
        bool idle = true;
        // 1. completions
        for (auto& sl : slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            const double t = now();
            std::lock_guard<std::mutex> lock(mu);
            if (q != hipSuccess && error.empty()) error = std::string("solve failed: ") + hipGetErrorString(q);
            alloc.release(sl.ws_off, sl.ws_bytes);
            sl.busy = false;
            done.push_back({sl.job.req.request_id, sl.job.req.plan_index, sl.job.arrival, sl.admitted, t,
                            q == hipSuccess ? 0 : int(SPP_EDEVICE)});
            ++completed;
            idle = false;
            cv.notify_all();
        }
        // 2. admissions in arrival order
        {
            std::unique_lock<std::mutex> lock(mu);
            if (stop && queue.empty()) {
                bool any = false;
                for (auto& sl : slots) any = any || sl.busy;
                if (!any) return;
            }
            const double t = now();
            while (!queue.empty() && queue.front().arrival <= t) {
                Slot* free_slot = nullptr;
                for (auto& sl : slots)
                    if (!sl.busy) {
                        free_slot = &sl;
                        break;
                    }
                if (!free_slot) break;
                const Pending job = queue.front();
                const spp_plan_s* p = plans[job.req.plan_index];
                // the workspace of the request (FP64: the plan's current path, the
                // fused path needing one spectral field, the staged path two;
                // mixed: the refinement's fields)
                const size_t need = request_workspace(p, job.req);
                size_t off = 0;
                if (!alloc.alloc(need, &off)) break;   // wait for memory
                queue.pop_front();
                free_slot->busy = true;
                free_slot->job = job;
                free_slot->ws_off = off;
                free_slot->ws_bytes = need;
                free_slot->admitted = t;
                lock.unlock();
                spp_status st = SPP_OK;
                if (job.req.ready_event &&
                    hipStreamWaitEvent(free_slot->stream, static_cast<hipEvent_t>(job.req.ready_event), 0) !=
                        hipSuccess)
                    st = spp_fail(SPP_EDEVICE, "spp_server: hipStreamWaitEvent on the request's ready_event failed");
                if (st == SPP_OK && job.req.precision == SPP_MIXED_FP32)
                    st = spp_launch_solve_mixed(p, SPP_MIXED_FP32, job.req.n_refine, 1, job.req.rho_dev,
                                                job.req.phi_dev, job.req.G, pool + off, free_slot->stream);
                else if (st == SPP_OK)
                    st = spp_launch_solve_f64(p, job.req.rho_dev, job.req.phi_dev, job.req.G, pool + off,
                                              free_slot->stream);
                if (st == SPP_OK && hipEventRecord(free_slot->done, free_slot->stream) != hipSuccess)
                    st = SPP_EDEVICE;
                lock.lock();
                if (st != SPP_OK) {
                    if (error.empty()) error = std::string("launch failed: ") + spp_last_error();
                    alloc.release(off, free_slot->ws_bytes);
                    free_slot->busy = false;
                    done.push_back({job.req.request_id, job.req.plan_index, job.arrival, t, now(), int(st)});
                    ++completed;
                    cv.notify_all();
                }
                idle = false;
            }
            if (idle) {
                // nothing changed: sleep briefly unless work is in flight
                bool busy = false;
                for (auto& sl : slots) busy = busy || sl.busy;
                if (!busy) {
                    if (queue.empty())
                        cv.wait_for(lock, std::chrono::milliseconds(2));
                    else {
                        const double wait = queue.front().arrival - now();
                        if (wait > 0) cv.wait_for(lock, std::chrono::duration<double>(std::min(wait, 0.002)));
                    }
                }
            }
        }
        if (idle) std::this_thread::yield();
    }
}

extern "C" spp_status spp_server_create(int n_plans, const spp_plan* plans, void* pool_dev, size_t pool_bytes,
                                        int n_slots, spp_server* out)
{
    if (!out) return spp_fail(SPP_EINVAL, "spp_server_create: NULL out");
    *out = nullptr;
    if (n_plans <= 0 || !plans || !pool_dev || n_slots <= 0 || n_slots > 64)
        return spp_fail(SPP_EINVAL, "spp_server_create: bad arguments");
    if (reinterpret_cast<uintptr_t>(pool_dev) & 255)
        return spp_fail(SPP_EINVAL, "spp_server_create: pool must be 256-byte aligned");
    for (int k = 0; k < n_plans; ++k) {
        if (!plans[k]) return spp_fail(SPP_EINVAL, "spp_server_create: NULL plan");
        if (!plans[k]->dev) return spp_fail(SPP_ESTATE, "spp_server_create: plan not uploaded");
        spp_prewarm_launch_caches(plans[k]);
    }
    auto* s = new (std::nothrow) spp_server_s;
    if (!s) return spp_fail(SPP_ENOMEM, "spp_server_create: out of host memory");
    s->plans.assign(plans, plans + n_plans);
    s->pool = static_cast<char*>(pool_dev);
    s->pool_bytes = pool_bytes & ~size_t(255);
    s->alloc = PoolAllocator(s->pool_bytes);
    (void)hipGetDevice(&s->device);
    s->slots.resize(n_slots);
    for (auto& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            for (auto& x : s->slots) {
                if (x.done) (void)hipEventDestroy(x.done);
                if (x.stream) (void)hipStreamDestroy(x.stream);
            }
            delete s;
            return spp_fail(SPP_EDEVICE, "spp_server_create: stream/event creation failed");
        }
    }
    s->t0 = Clock::now();
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return SPP_OK;
}

extern "C" spp_status spp_server_submit(spp_server s, const spp_request* req, double not_before)
{
    if (!s || !req) return spp_fail(SPP_EINVAL, "spp_server_submit: NULL pointer");
    if (req->plan_index < 0 || req->plan_index >= int(s->plans.size()))
        return spp_fail(SPP_EINVAL, "spp_server_submit: plan_index out of range");
    const spp_plan_s* p = s->plans[req->plan_index];
    const spp_status st = spp_validate_solve("spp_server_submit", p, req->rho_dev, req->phi_dev, req->G, s->pool);
    if (st != SPP_OK) return st;
    if (req->precision != SPP_FP64 && req->precision != SPP_MIXED_FP32)
        return spp_fail(SPP_ENOTSUP, "spp_server_submit: precision must be SPP_FP64 or SPP_MIXED_FP32");
    if (req->precision == SPP_MIXED_FP32 && (req->n_refine < 0 || req->n_refine > SPP_MAX_REFINE || p->proj_rn == 0))
        return spp_fail(SPP_EINVAL, "spp_server_submit: mixed requests need n_refine in [0, 16] and N_theta <= 128");
    if (request_workspace(p, *req) > s->pool_bytes)
        return spp_fail(SPP_ENOMEM, "spp_server_submit: request larger than the memory pool");
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) return spp_fail(SPP_ESTATE, "spp_server_submit: server is shutting down");
    const double t = s->now();
    s->queue.push_back({*req, not_before > t ? not_before : t});
    ++s->submitted;
    s->cv.notify_all();
    return SPP_OK;
}

extern "C" spp_status spp_server_poll(spp_server s, spp_completion* out, int max_out, int* n_out)
{
    if (!s || !n_out || (max_out > 0 && !out)) return spp_fail(SPP_EINVAL, "spp_server_poll: bad arguments");
    std::lock_guard<std::mutex> lock(s->mu);
    const int n = std::min<int>(max_out, int(s->done.size()));
    std::copy(s->done.begin(), s->done.begin() + n, out);
    s->done.erase(s->done.begin(), s->done.begin() + n);
    *n_out = n;
    if (!s->error.empty()) return spp_fail(SPP_EDEVICE, "spp_server: " + s->error);
    return SPP_OK;
}

extern "C" spp_status spp_server_drain(spp_server s, double timeout_s)
{
    if (!s) return spp_fail(SPP_EINVAL, "spp_server_drain: NULL server");
    std::unique_lock<std::mutex> lock(s->mu);
    const bool ok = s->cv.wait_for(lock, std::chrono::duration<double>(timeout_s),
                                   [s] { return s->completed == s->submitted; });
    if (!ok) return spp_fail(SPP_ESTATE, "spp_server_drain: timed out");
    return SPP_OK;
}

extern "C" spp_status spp_server_now(spp_server s, double* t)
{
    if (!s || !t) return spp_fail(SPP_EINVAL, "spp_server_now: NULL pointer");
    *t = s->now();
    return SPP_OK;
}

extern "C" void spp_server_destroy(spp_server s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->queue.clear();
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto& sl : s->slots) {
        (void)hipStreamSynchronize(sl.stream);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
    delete s;
}
