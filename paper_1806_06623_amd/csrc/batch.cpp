// Batched solves: many right-hand sides on grids of uneven size, captured
// once into a HIP graph whose per-solve chains are independent branches (the
// solves share nothing but read-only plans), then replayed with one launch.
#include <hip/hip_runtime.h>

#include <new>
#include <string>
#include <vector>

#include "internal.h"

struct spp_batch_s {
    int n = 0;
    std::vector<hipStream_t> streams;   // capture branches (default priority)
    std::vector<hipEvent_t> events;     // fork + joins
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~spp_batch_s()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto e : events) (void)hipEventDestroy(e);
        for (auto s : streams) (void)hipStreamDestroy(s);
    }
};

static constexpr int kMaxBranches = 8;

extern "C" spp_status spp_batch_workspace_bytes(int n, const spp_plan* plans, size_t* bytes)
{
    if (n < 0 || (n > 0 && !plans) || !bytes) return spp_fail(SPP_EINVAL, "spp_batch_workspace_bytes: bad arguments");
    size_t total = 0;
    for (int r = 0; r < n; ++r) {
        if (!plans[r]) return spp_fail(SPP_EINVAL, "spp_batch_workspace_bytes: NULL plan");
        total += spp_align256(plans[r]->workspace_bytes);
    }
    *bytes = total;
    return SPP_OK;
}

extern "C" spp_status spp_batch_create(int n, const spp_plan* plans, const double* const* rho_dev,
                                       double* const* phi_dev, const double* G, void* workspace_dev,
                                       spp_batch* out)
{
    if (!out) return spp_fail(SPP_EINVAL, "spp_batch_create: NULL out");
    *out = nullptr;
    if (n <= 0 || !plans || !rho_dev || !phi_dev || !G || !workspace_dev)
        return spp_fail(SPP_EINVAL, "spp_batch_create: bad arguments");
    if (reinterpret_cast<uintptr_t>(workspace_dev) & 255)
        return spp_fail(SPP_EINVAL, "spp_batch_create: workspace must be 256-byte aligned");
    std::vector<void*> ws(n);
    size_t off = 0;
    for (int r = 0; r < n; ++r) {
        ws[r] = static_cast<char*>(workspace_dev) + off;
        const spp_status st = spp_validate_solve("spp_batch_create", plans[r], rho_dev[r], phi_dev[r], G[r], ws[r]);
        if (st != SPP_OK) return st;
        off += spp_align256(plans[r]->workspace_bytes);
    }
    for (int r = 0; r < n; ++r) spp_prewarm_launch_caches(plans[r]);

    auto* b = new (std::nothrow) spp_batch_s;
    if (!b) return spp_fail(SPP_ENOMEM, "spp_batch_create: out of host memory");
    b->n = n;
    const int nb = n < kMaxBranches ? n : kMaxBranches;
    auto fail = [&](const char* what, hipError_t e) {
        delete b;
        return spp_fail(SPP_EDEVICE, std::string("spp_batch_create: ") + what + ": " + hipGetErrorString(e));
    };
    for (int k = 0; k < nb; ++k) {
        hipStream_t s = nullptr;
        const hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return fail("hipStreamCreateWithFlags", e);
        b->streams.push_back(s);
    }
    for (int k = 0; k < nb; ++k) {
        hipEvent_t ev = nullptr;
        const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return fail("hipEventCreate", e);
        b->events.push_back(ev);
    }

    // capture: fork from branch 0, solves round-robin over the branches, join into branch 0
    hipStream_t s0 = b->streams[0];
    hipError_t e = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail("hipStreamBeginCapture", e);
    spp_status st = SPP_OK;
    (void)hipEventRecord(b->events[0], s0);
    for (int k = 1; k < nb; ++k) (void)hipStreamWaitEvent(b->streams[k], b->events[0], 0);
    for (int r = 0; r < n && st == SPP_OK; ++r)
        st = spp_launch_solve_f64(plans[r], rho_dev[r], phi_dev[r], G[r], ws[r], b->streams[r % nb]);
    for (int k = 1; k < nb; ++k) {
        (void)hipEventRecord(b->events[k], b->streams[k]);
        (void)hipStreamWaitEvent(s0, b->events[k], 0);
    }
    e = hipStreamEndCapture(s0, &b->graph);
    if (st != SPP_OK) {
        delete b;
        return st;
    }
    if (e != hipSuccess) return fail("hipStreamEndCapture", e);
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail("hipGraphInstantiate", e);
    *out = b;
    return SPP_OK;
}

extern "C" spp_status spp_batch_launch(spp_batch b, void* stream)
{
    if (!b) return spp_fail(SPP_EINVAL, "spp_batch_launch: NULL batch");
    const hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("spp_batch_launch: ") + hipGetErrorString(e));
    return SPP_OK;
}

extern "C" void spp_batch_destroy(spp_batch b) { delete b; }

extern "C" spp_status spp_solve_batched(int n, const spp_plan* plans, const double* const* rho_dev,
                                        double* const* phi_dev, const double* G, void* workspace_dev, void* stream)
{
    spp_batch b = nullptr;
    spp_status st = spp_batch_create(n, plans, rho_dev, phi_dev, G, workspace_dev, &b);
    if (st != SPP_OK) return st;
    st = spp_batch_launch(b, stream);
    const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    spp_batch_destroy(b);
    if (st == SPP_OK && e != hipSuccess)
        st = spp_fail(SPP_EDEVICE, std::string("spp_solve_batched: ") + hipGetErrorString(e));
    return st;
}
