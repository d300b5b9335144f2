// Batched solves: many right-hand sides on grids of uneven size.
//
// The right-hand sides are grouped by plan (grid class).  For an FP64 class on
// the fused path each kernel of the solve -- folded forward FFT, per-mode
// kernel, folded inverse FFT -- is one launch over all of the class's
// right-hand sides (or over each half of them, if the tuner prefers two
// concurrent chains), so that small grids fill the device; other classes
// (staged path, mixed precision) run one solve per right-hand side.  All
// chains are captured once into one HIP graph, spread over up to 8 branches
// (largest work first onto the least-loaded branch), and replayed with one
// graph launch.  The per-class tuner times the variants the batch launches
// (the per-mode kernel's unit order, one or two launch groups) on the real
// inputs before capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

namespace {

constexpr int kMaxBranches = 8;

// One grid class of a batch.
struct ClassInfo {
    const spp_plan_s* plan = nullptr;
    std::vector<int> rhs;          // indices into the batch
    bool fused = false;            // FP64 class on the fused path: batched launches
    size_t tables = 0;             // offset of rho/phi/scale tables (fused)
    size_t region = 0;             // offset of the class's records, fields and sink (fused)
    int paired = 1, groups = 1;    // tuned launch variant (fused)
    double tuned_ms = 0.0;
    std::string candidates;        // tuner's timings
};

struct Layout {
    std::vector<ClassInfo> classes;
    std::vector<size_t> ws_off;    // per RHS: its workspace (non-batched classes)
    size_t total = 0;
};

size_t class_tables_bytes(int n) { return spp_align256(size_t(n) * 3 * sizeof(void*)); }

Layout make_layout(int n, const spp_plan* plans, spp_precision prec)
{
    Layout L;
    L.ws_off.assign(n, 0);
    for (int r = 0; r < n; ++r) {
        auto it = std::find_if(L.classes.begin(), L.classes.end(),
                               [&](const ClassInfo& c) { return c.plan == plans[r]; });
        if (it == L.classes.end()) {
            ClassInfo c;
            c.plan = plans[r];
            c.fused = prec == SPP_FP64 && spp_plan_fused(plans[r]);
            L.classes.push_back(c);
            it = L.classes.end() - 1;
        }
        it->rhs.push_back(r);
    }
    size_t off = 0;
    for (auto& c : L.classes) {
        // the per-mode kernel reaches its store sink by 32-bit offsets: a class
        // whose fields exceed that takes one solve per right-hand side
        if (c.fused && spp_class_batch_bytes(c.plan, int(c.rhs.size())) > (size_t(1) << 32)) c.fused = false;
        if (c.fused) {
            c.tables = off;
            off += class_tables_bytes(int(c.rhs.size()));
            c.region = off;
            off += spp_align256(spp_class_batch_bytes(c.plan, int(c.rhs.size())));
        } else {
            for (int r : c.rhs) {
                L.ws_off[r] = off;
                off += spp_align256(prec == SPP_FP64 ? c.plan->workspace_bytes : spp_mixed_workspace_bytes(c.plan));
            }
        }
    }
    L.total = off;
    return L;
}

}  // namespace

struct spp_batch_s {
    int n = 0;
    spp_precision prec = SPP_FP64;
    Layout layout;
    char* ws = nullptr;
    std::vector<spp_status_record*> rec;   // per RHS
    std::vector<hipStream_t> streams;      // capture branches (default priority)
    std::vector<hipEvent_t> events;        // fork + joins
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

namespace {

// The launches of class c's group [g0, g1) of its right-hand sides on s.
spp_status launch_group(const ClassInfo& c, char* ws, int g0, int g1, hipStream_t s)
{
    const int n = int(c.rhs.size());
    const size_t field = spp_align256(size_t(c.plan->nr) * c.plan->nth * c.plan->nphi * sizeof(double));
    auto* tab = reinterpret_cast<char*>(ws + c.tables);
    auto* rho_tab = reinterpret_cast<const double* const*>(tab);
    auto* phi_tab = reinterpret_cast<double* const*>(tab + size_t(n) * sizeof(void*));
    auto* scale_tab = reinterpret_cast<const double*>(tab + 2 * size_t(n) * sizeof(void*));
    char* reg = ws + c.region;
    auto* recs = reinterpret_cast<spp_status_record*>(reg);
    double* X = reinterpret_cast<double*>(reg + size_t(n) * SPP_STATUS_BYTES);
    double* sink = reinterpret_cast<double*>(reg + size_t(n) * (SPP_STATUS_BYTES + field));
    return spp_launch_class_batch(c.plan, g1 - g0, rho_tab + g0, phi_tab + g0, scale_tab + g0, recs + g0,
                                  X + size_t(g0) * (field / sizeof(double)), sink, c.paired, s);
}

// A chain of work for one graph branch: a launch group of a fused class, or
// one solve.
struct Chain {
    int cls = 0, g0 = 0, g1 = 0;   // fused class group
    int rhs = -1;                  // single solve (rhs >= 0)
    double work = 0.0;             // zones, for balancing the branches
};

}  // namespace

extern "C" spp_status spp_batch_workspace_bytes(int n, const spp_plan* plans, spp_precision prec, size_t* bytes)
{
    if (n <= 0 || !plans || !bytes) return spp_fail(SPP_EINVAL, "spp_batch_workspace_bytes: bad arguments");
    if (prec != SPP_FP64 && prec != SPP_MIXED_FP32)
        return spp_fail(SPP_ENOTSUP, "spp_batch_workspace_bytes: precision not supported");
    for (int r = 0; r < n; ++r)
        if (!plans[r]) return spp_fail(SPP_EINVAL, "spp_batch_workspace_bytes: NULL plan");
    *bytes = make_layout(n, plans, prec).total;
    return SPP_OK;
}

extern "C" spp_status spp_batch_create(int n, const spp_plan* plans, const double* const* rho_dev,
                                       double* const* phi_dev, const double* G, spp_precision prec, int n_refine,
                                       int autotune, void* workspace_dev, void* stream, spp_batch* out)
{
    if (!out) return spp_fail(SPP_EINVAL, "spp_batch_create: NULL out");
    *out = nullptr;
    if (n <= 0 || !plans || !rho_dev || !phi_dev || !G || !workspace_dev)
        return spp_fail(SPP_EINVAL, "spp_batch_create: bad arguments");
    if (prec != SPP_FP64 && prec != SPP_MIXED_FP32)
        return spp_fail(SPP_ENOTSUP, "spp_batch_create: precision not supported");
    if (prec == SPP_MIXED_FP32 && (n_refine < 0 || n_refine > SPP_MAX_REFINE))
        return spp_fail(SPP_EINVAL, "spp_batch_create: n_refine must be in [0, 16]");
    if (reinterpret_cast<uintptr_t>(workspace_dev) & 255)
        return spp_fail(SPP_EINVAL, "spp_batch_create: workspace must be 256-byte aligned");
    for (int r = 0; r < n; ++r)
        if (!plans[r]) return spp_fail(SPP_EINVAL, "spp_batch_create: NULL plan");
    auto* b = new (std::nothrow) spp_batch_s;
    if (!b) return spp_fail(SPP_ENOMEM, "spp_batch_create: out of host memory");
    b->n = n;
    b->prec = prec;
    b->layout = make_layout(n, plans, prec);
    b->ws = static_cast<char*>(workspace_dev);
    auto& classes = b->layout.classes;
    auto fail = [&](spp_status st, const std::string& what) {
        delete b;
        return spp_fail(st, "spp_batch_create: " + what);
    };
    auto fail_hip = [&](const char* what, hipError_t e) { return fail(SPP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)); };

    // validate every entry against the space it will use
    b->rec.assign(n, nullptr);
    for (auto& c : classes) {
        if (c.plan->proj_rn == 0 && prec == SPP_MIXED_FP32) return fail(SPP_ENOTSUP, "mixed needs N_theta <= 128");
        const size_t field = spp_align256(size_t(c.plan->nr) * c.plan->nth * c.plan->nphi * sizeof(double));
        for (size_t k = 0; k < c.rhs.size(); ++k) {
            const int r = c.rhs[k];
            void* ws = c.fused ? b->ws + c.region : b->ws + b->layout.ws_off[r];
            const spp_status st = spp_validate_solve("spp_batch_create", c.plan, rho_dev[r], phi_dev[r], G[r], ws);
            if (st != SPP_OK) {
                delete b;
                return st;
            }
            b->rec[r] = c.fused ? reinterpret_cast<spp_status_record*>(b->ws + c.region) + k
                                : reinterpret_cast<spp_status_record*>(ws);
            (void)field;
        }
        spp_prewarm_launch_caches(c.plan);
    }
    hipStream_t s0 = static_cast<hipStream_t>(stream);

    // per-RHS tables of the fused classes
    for (auto& c : classes) {
        if (!c.fused) continue;
        const int nc = int(c.rhs.size());
        std::vector<unsigned char> tab(class_tables_bytes(nc), 0);
        auto* rp = reinterpret_cast<const double**>(tab.data());
        auto* pp = reinterpret_cast<double**>(tab.data() + size_t(nc) * sizeof(void*));
        auto* sp = reinterpret_cast<double*>(tab.data() + 2 * size_t(nc) * sizeof(void*));
        for (int k = 0; k < nc; ++k) {
            rp[k] = rho_dev[c.rhs[k]];
            pp[k] = phi_dev[c.rhs[k]];
            sp[k] = 4.0 * M_PI * G[c.rhs[k]] / c.plan->nphi;   // the scale of spp_solve
        }
        hipError_t e = hipMemcpyAsync(b->ws + c.tables, tab.data(), tab.size(), hipMemcpyHostToDevice, s0);
        if (e == hipSuccess) e = hipStreamSynchronize(s0);
        if (e != hipSuccess) return fail_hip("table upload", e);
    }

    // branches
    for (int k = 0; k < kMaxBranches; ++k) {
        hipStream_t s = nullptr;
        const hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) return fail_hip("hipStreamCreateWithFlags", e);
        b->streams.push_back(s);
        hipEvent_t ev = nullptr;
        const hipError_t e2 = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e2 != hipSuccess) return fail_hip("hipEventCreate", e2);
        b->events.push_back(ev);
    }

    // tuner: time each launch variant of every fused class on the real inputs
    if (autotune) {
        hipEvent_t t0 = nullptr, t1 = nullptr, fork = nullptr, join = nullptr;
        hipError_t e = hipEventCreate(&t0);
        if (e == hipSuccess) e = hipEventCreate(&t1);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
        spp_status st = e == hipSuccess ? SPP_OK : spp_fail(SPP_EDEVICE, "tuner events");
        hipStream_t sa = b->streams[0], sb = b->streams[1];
        for (auto& c : classes) {
            if (!c.fused || st != SPP_OK) continue;
            const int nc = int(c.rhs.size());
            double best = 1e300;
            int bp = 1, bg = 1;
            for (int groups = 1; groups <= (nc >= 2 ? 2 : 1) && st == SPP_OK; ++groups)
                for (int paired = 1; paired >= 0 && st == SPP_OK; --paired) {
                    c.paired = paired;
                    float ms = 0.f;
                    for (int rep = 0; rep < 4 && st == SPP_OK; ++rep) {
                        if (rep == 1) (void)hipEventRecord(t0, sa);
                        if (groups == 1) {
                            st = launch_group(c, b->ws, 0, nc, sa);
                        } else {
                            (void)hipEventRecord(fork, sa);
                            (void)hipStreamWaitEvent(sb, fork, 0);
                            st = launch_group(c, b->ws, 0, nc / 2, sa);
                            if (st == SPP_OK) st = launch_group(c, b->ws, nc / 2, nc, sb);
                            (void)hipEventRecord(join, sb);
                            (void)hipStreamWaitEvent(sa, join, 0);
                        }
                    }
                    (void)hipEventRecord(t1, sa);
                    if (st == SPP_OK && hipEventSynchronize(t1) == hipSuccess &&
                        hipEventElapsedTime(&ms, t0, t1) == hipSuccess) {
                        const double per = ms / 3.0;
                        c.candidates += (c.candidates.empty() ? "" : " ") + std::string(paired ? "paired" : "plain") +
                                        "/" + std::to_string(groups) + "=" + std::to_string(per).substr(0, 6);
                        if (per < best) {
                            best = per;
                            bp = paired;
                            bg = groups;
                        }
                    }
                }
            c.paired = bp;
            c.groups = bg;
            c.tuned_ms = best;
        }
        for (auto ev : {t0, t1, fork, join})
            if (ev) (void)hipEventDestroy(ev);
        if (st != SPP_OK) {
            delete b;
            return st;
        }
    }

    // chains, largest first onto the least-loaded branch
    std::vector<Chain> chains;
    for (size_t ci = 0; ci < classes.size(); ++ci) {
        const auto& c = classes[ci];
        const double zones = double(c.plan->nr) * c.plan->nth * c.plan->nphi;
        if (c.fused) {
            const int nc = int(c.rhs.size());
            if (c.groups == 2) {
                chains.push_back({int(ci), 0, nc / 2, -1, zones * (nc / 2)});
                chains.push_back({int(ci), nc / 2, nc, -1, zones * (nc - nc / 2)});
            } else {
                chains.push_back({int(ci), 0, nc, -1, zones * nc});
            }
        } else {
            for (int r : c.rhs) chains.push_back({int(ci), 0, 0, r, zones});
        }
    }
    std::stable_sort(chains.begin(), chains.end(), [](const Chain& x, const Chain& y) { return x.work > y.work; });
    const int nb = std::min<int>(kMaxBranches, int(chains.size()));
    std::vector<double> load(nb, 0.0);
    std::vector<int> branch_of(chains.size());
    for (size_t k = 0; k < chains.size(); ++k) {
        const int br = int(std::min_element(load.begin(), load.end()) - load.begin());
        branch_of[k] = br;
        load[br] += chains[k].work;
    }

    // capture: fork from branch 0, chains on their branches, join into branch 0
    hipStream_t c0 = b->streams[0];
    hipError_t e = hipStreamBeginCapture(c0, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail_hip("hipStreamBeginCapture", e);
    spp_status st = SPP_OK;
    (void)hipEventRecord(b->events[0], c0);
    for (int k = 1; k < nb; ++k) (void)hipStreamWaitEvent(b->streams[k], b->events[0], 0);
    for (size_t k = 0; k < chains.size() && st == SPP_OK; ++k) {
        const Chain& ch = chains[k];
        const ClassInfo& c = classes[ch.cls];
        hipStream_t s = b->streams[branch_of[k]];
        if (ch.rhs < 0) {
            st = launch_group(c, b->ws, ch.g0, ch.g1, s);
        } else {
            void* ws = b->ws + b->layout.ws_off[ch.rhs];
            st = prec == SPP_FP64
                     ? spp_launch_solve_f64(c.plan, rho_dev[ch.rhs], phi_dev[ch.rhs], G[ch.rhs], ws, s)
                     : spp_launch_solve_mixed(c.plan, prec, n_refine, 1, rho_dev[ch.rhs], phi_dev[ch.rhs], G[ch.rhs],
                                              ws, s);
        }
    }
    for (int k = 1; k < nb; ++k) {
        (void)hipEventRecord(b->events[k], b->streams[k]);
        (void)hipStreamWaitEvent(c0, b->events[k], 0);
    }
    e = hipStreamEndCapture(c0, &b->graph);
    if (st != SPP_OK) {
        delete b;
        return st;
    }
    if (e != hipSuccess) return fail_hip("hipStreamEndCapture", e);
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail_hip("hipGraphInstantiate", e);
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

extern "C" spp_status spp_batch_describe(spp_batch b, char* buf, size_t len, size_t* needed)
{
    if (!b) return spp_fail(SPP_EINVAL, "spp_batch_describe: NULL batch");
    std::string d;
    for (const auto& c : b->layout.classes) {
        if (!d.empty()) d += "; ";
        d += std::to_string(c.plan->nr) + "x" + std::to_string(c.plan->nth) + "x" + std::to_string(c.plan->nphi) +
             " n=" + std::to_string(c.rhs.size());
        if (c.fused)
            d += std::string(" batched unit_order=") + (c.paired ? "paired" : "plain") +
                 " groups=" + std::to_string(c.groups) + (c.candidates.empty() ? "" : " tuned[" + c.candidates + " ms]");
        else
            d += b->prec == SPP_FP64 ? " per-rhs staged" : " per-rhs mixed";
    }
    if (needed) *needed = d.size() + 1;
    if (buf && len > 0) {
        const size_t k = std::min(len - 1, d.size());
        std::memcpy(buf, d.data(), k);
        buf[k] = '\0';
    }
    return SPP_OK;
}

extern "C" spp_status spp_batch_status(spp_batch b, int r, void* stream, spp_solve_info* info)
{
    if (!b || r < 0 || r >= b->n) return spp_fail(SPP_EINVAL, "spp_batch_status: bad arguments");
    // the class's plan serves only as the argument the status call expects
    const spp_plan_s* p = nullptr;
    for (const auto& c : b->layout.classes)
        if (std::find(c.rhs.begin(), c.rhs.end(), r) != c.rhs.end()) p = c.plan;
    return spp_solve_status(const_cast<spp_plan_s*>(p), b->rec[r], stream, info);
}

extern "C" void spp_batch_destroy(spp_batch b) { delete b; }

extern "C" spp_status spp_solve_batched(int n, const spp_plan* plans, const double* const* rho_dev,
                                        double* const* phi_dev, const double* G, spp_precision prec, int n_refine,
                                        void* workspace_dev, void* stream)
{
    spp_batch b = nullptr;
    spp_status st = spp_batch_create(n, plans, rho_dev, phi_dev, G, prec, n_refine, 0, workspace_dev, stream, &b);
    if (st != SPP_OK) return st;
    st = spp_batch_launch(b, stream);
    const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    spp_batch_destroy(b);
    if (st == SPP_OK && e != hipSuccess)
        st = spp_fail(SPP_EDEVICE, std::string("spp_solve_batched: ") + hipGetErrorString(e));
    return st;
}
