#!/usr/bin/env python3
"""Throughput of the exact spherical-polar Poisson solve on one MI355X.

Workload: the stellar-core grid N_r x N_theta x N_phi = 550 x 128 x 256
(18 022 400 zones; the grid size of the paper's timing table), FP64, with a
seeded synthetic density (``synthetic.stellar_case``).  One step is one full
solve: forward real FFT along phi, forward theta projection, radial
tridiagonal solves with the outer boundary condition, inverse projection,
inverse FFT.  Inputs are resident in HBM before the timed region.

Order of a run: set-up; the first solves after process start, timed as they
come (``cold_start``: the GPU's clocks are still ramping); a settling period
of back-to-back solves; the other legs (mixed form, face fluxes, momentum
source, residual, copies of one field as the bandwidth reference, batched and
served solves); another settling period (``settle``), the W warm-up solves
and the K timed ones (``value``), the latency loop and the per-stage profile;
finally the FP64 oracle timed on the host CPU.

Prints one JSON line (rank 0, N = 1) with solves/s as ``value``, Gzones/s,
per-solve latency percentiles, per-stage times and roofline fractions, the
error against the FP64 oracle, and the oracle itself timed on the host CPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X dense FP64 matrix, TFLOP/s
STAGES = ["fft_forward", "projection_forward", "radial_tridiagonal", "projection_inverse", "fft_inverse"]
FUSED_STAGES = ["fft_forward", "fused_modal", "fft_inverse"]
METRIC = "solves/s & Gzones/s at 550\u00d7128\u00d7256 (FP64 vs mixed); p50/p99 latency"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_model(nr, nth, nphi, parity, fused):
    """Algorithmic bytes and flops per launch of each stage (FP64).

    With the parity split each N_theta^2 product per Fourier component becomes
    two (N_theta/2)^2 products: half the flops and half the matrix bytes.  The
    fused per-mode kernel reads the folded spectrum once, writes the result
    once and runs both products (the radial solves' few flops per value are
    not counted).
    """
    n = nr * nth * nphi
    field = 8.0 * n                                   # one real field, bytes
    nm = nphi // 2 + 1
    basis = 8.0 * nm * nth * nth * (0.5 if parity else 1.0)
    proj_flops = 2.0 * nr * nth * nth * nphi * (0.5 if parity else 1.0)
    if fused:
        return {
            "fft_forward": {"bytes": 2 * field, "flops": None},
            "fused_modal": {"bytes": 2 * field + 2 * basis, "flops": 2 * proj_flops},
            "fft_inverse": {"bytes": 2 * field, "flops": None},
        }
    return {
        "fft_forward": {"bytes": 2 * field, "flops": None},
        "projection_forward": {"bytes": 2 * field + basis, "flops": proj_flops},
        "radial_tridiagonal": {"bytes": 2 * field, "flops": None},
        "projection_inverse": {"bytes": 2 * field + basis, "flops": proj_flops},
        "fft_inverse": {"bytes": 2 * field, "flops": None},
    }


# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes (the
# profiles/ summaries named for each kernel and workload), scaled by the same
# counters read over a device copy of known size (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0).  Each figure is valid only for the kernel sources it was
# taken with: if they have changed, it is withheld.
TRAFFIC = {
    "modal::k_modal": {"grid": (550, 128, 256),
                       "sources": ("modal.hip.h", "modal_layout.h", "radial.hip.h", "status.h", "solve.hip"),
                       "source_digest": "9387555aa5f1cb12",
                       "bytes_per_launch": (81339.4 * 2.0 + 140806.0) * 1024.0},
    "faceflux::k_face_fluxes": {"grid": (550, 128, 256), "sources": ("fluxes.hip.h", "xcd.h", "solve.hip"),
                                "source_digest": "b2a25584f1ab1bc0",
                                "bytes_per_launch": (74482.1 * 2.0 + 422617.4) * 1024.0},
    "momentum::k_momentum_rows": {"grid": (550, 128, 256), "sources": ("momentum.hip.h", "xcd.h", "solve.hip"),
                                  "source_digest": "b3a35a7931e3d9f5",
                                  "bytes_per_launch": (78505.7 * 2.0 + 422400.2) * 1024.0},
    "k_residual_rows": {"grid": (550, 128, 256), "sources": ("solve.hip", "internal.h", "xcd.h", "status.h"),
                        "source_digest": "3175b7ca1d3e8f72",
                        "bytes_per_launch": (148724.0 * 2.0 + 140800.0) * 1024.0},
}


def _kernel_source_digest(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1806_06623_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, nr, nth, nphi):
    t = TRAFFIC.get(kernel)
    if (t is None or t["bytes_per_launch"] is None or (nr, nth, nphi) != tuple(t["grid"])
            or _kernel_source_digest(t["sources"]) != t["source_digest"]):
        return None
    return round(t["bytes_per_launch"], 0)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _timed_oracle_solves(plan, case, seconds, label):
    runs, t0 = 0, time.perf_counter()
    ref = None
    while True:
        ref = plan.solve(case["rho"], case["G"])
        runs += 1
        el = time.perf_counter() - t0
        log(f"oracle ({label}) solve {runs} done at {el:.1f} s")
        if el >= seconds:
            break
    return ref, runs, el


def cpu_baseline(case, phi_gpu, seconds, single_seconds):
    """The FP64 oracle, as it stands, on the host cores (set-up excluded):
    once with the BLAS/OpenMP pools at all host threads, once single-threaded."""
    from oracle import spectral
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    plan = spectral.Plan(case["r_if"], case["th_if"], case["nphi"])
    ref, runs, el = _timed_oracle_solves(plan, case, seconds, f"{threads} threads")
    with threadpool_limits(limits=1):
        _, runs1, el1 = _timed_oracle_solves(plan, case, single_seconds, "1 thread")
    err = float(np.max(np.abs(phi_gpu - ref)) / np.max(np.abs(ref)))
    return {"value": runs / el, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{runs} full FP64 oracle solves of the 550x128x256 stellar workload "
                      f"({el:.1f} s wall, theta eigensystem set-up excluded)",
            "single_thread": {"value": runs1 / el1, "unit": "solves/s", "cores": 1,
                              "sample": f"{runs1} solves of the same workload, BLAS/OpenMP limited to one "
                                        f"thread ({el1:.1f} s wall)"},
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}, err


def batched_leg(spp, torch, synthetic, steps):
    """64 right-hand sides on grids drawn from N_r x N_theta x N_phi in
    {128,256,550} x {32,64,128} x {64,128,256} (draw seed 3; sources as the
    stellar workload with seeds 100..163), one HIP graph per precision: FP64
    (the right-hand sides of each grid class batched into one launch per
    kernel, launch variants tuned per class at creation) and mixed (one
    refinement).  Also times the same FP64 solves issued one after another on
    one stream."""
    grids = synthetic.batch_grids()
    plans, rhos, phis = {}, [], []
    t0 = time.perf_counter()
    for k, g in enumerate(grids):
        r_if, th_if, nphi = synthetic.stellar_grid(*g)
        if g not in plans:
            plans[g] = spp.Plan(r_if, th_if, nphi, device="cuda:0")
        rhos.append(torch.from_numpy(synthetic.stellar_density(r_if, th_if, nphi, 100 + k)).to("cuda:0"))
        phis.append(torch.empty_like(rhos[-1]))
    plist = [plans[g] for g in grids]
    log(f"batched: {len(grids)} RHS, {len(plans)} plans, set-up {time.perf_counter() - t0:.1f} s")
    zones = sum(a * c * d for a, c, d in grids)

    def timed(b):
        b.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.launch()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    out = {"rhs": len(grids), "plans": len(plans), "zones_per_batch": zones}
    t0 = time.perf_counter()
    b = spp.Batch(plist, rhos, phis, [1.0] * len(grids), autotune=True)
    log(f"batched fp64: created and tuned in {time.perf_counter() - t0:.1f} s: {b.description}")
    el = timed(b)
    phi64 = [y.clone() for y in phis]
    out["fp64"] = {"ms_per_batch": round(el * 1e3, 3), "rhs_per_s": round(len(grids) / el, 1),
                   "gzones_per_s": round(zones / el / 1e9, 3), "tuning": b.description}
    del b
    # the same solves one after another on the current stream (no graph, no batching)
    for p, x, y in zip(plist, rhos, phis):
        p.solve(x, out=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for p, x, y in zip(plist, rhos, phis):
            p.solve(x, out=y)
    torch.cuda.synchronize()
    el_seq = (time.perf_counter() - t0) / steps
    out["fp64"]["sequential_ms_per_batch"] = round(el_seq * 1e3, 3)
    out["fp64"]["speedup_vs_sequential"] = round(el_seq / el, 3)
    log(f"batched fp64: {el * 1e3:.2f} ms per batch, {zones / el / 1e9:.1f} Gzones/s "
        f"(sequential {el_seq * 1e3:.2f} ms)")
    bm = spp.Batch(plist, rhos, phis, [1.0] * len(grids), precision="mixed_fp32", n_refine=1)
    elm = timed(bm)
    d = max((y - y0).abs().max().item() / y0.abs().max().item() for y, y0 in zip(phis, phi64))
    out["mixed_fp32"] = {"n_refine": 1, "ms_per_batch": round(elm * 1e3, 3), "rhs_per_s": round(len(grids) / elm, 1),
                         "gzones_per_s": round(zones / elm / 1e9, 3), "max_rel_diff_vs_fp64": d}
    log(f"batched mixed: {elm * 1e3:.2f} ms per batch, diff vs FP64 {d:.2e}")
    del bm
    return out


def serving_leg(spp, torch, synthetic, n_requests, rates):
    """Poisson arrivals (seed 4) of requests drawn uniformly from the grid
    classes (128,32,64), (256,64,128), (550,128,256) with off-centre point
    mass + Gaussian sources; plans resident, workspaces from an HBM pool,
    8 concurrent slots.  For each precision (FP64, and mixed: FP32 projections
    with one FP64 refinement and the FP64 fallback armed): first the saturated
    throughput (all requests queued at once), then arrival rates at the given
    fractions of it."""
    classes = synthetic.SERVING_CLASSES
    plans, srcs, outs = [], [], []
    for c in classes:
        r_if, th_if, nphi = synthetic.stellar_grid(*c)
        plans.append(spp.Plan(r_if, th_if, nphi, device="cuda:0"))
        srcs.append([torch.from_numpy(synthetic.serving_source(r_if, th_if, nphi, seed=4000 + 10 * len(srcs) + k))
                     .to("cuda:0") for k in range(4)])
        outs.append([torch.empty_like(srcs[-1][0]) for _ in range(16)])
    n_slots = 8
    rng = np.random.default_rng(4)
    cls_of = rng.integers(0, len(classes), size=n_requests)
    gaps = rng.exponential(1.0, size=n_requests)
    zones = [a * b * c for a, b, c in classes]

    def run(rate, precision, pool):
        srv = spp.Server(plans, pool_bytes=pool, n_slots=n_slots)
        count = [0] * len(classes)
        t0 = srv.now() + 0.01
        arrivals = t0 + (np.cumsum(gaps) / rate if rate else np.zeros(n_requests))
        for k in range(n_requests):
            c = int(cls_of[k])
            j = count[c]
            count[c] += 1
            srv.submit(c, srcs[c][j % 4], outs[c][j % 16], request_id=k, not_before=float(arrivals[k]),
                       precision=precision, n_refine=1)
        srv.drain(300.0)
        done = srv.poll(n_requests + 16)
        srv.close()
        lat = np.array([d["t_done"] - d["t_arrival"] for d in done]) * 1e3
        span = max(d["t_done"] for d in done) - min(d["t_arrival"] for d in done)
        z = sum(zones[d["plan_index"]] for d in done)
        return {"offered_rate_per_s": None if not rate else round(rate, 1), "requests": len(done),
                "solves_per_s": round(len(done) / span, 1), "gzones_per_s": round(z / span / 1e9, 3),
                "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4)}

    out = {"classes": [list(c) for c in classes], "n_slots": n_slots}
    for precision in ("fp64", "mixed_fp32"):
        pool = n_slots * max(p.workspace_bytes_for(precision) for p in plans)
        run(None, precision, pool)   # warm-up
        sat = run(None, precision, pool)
        log(f"serving {precision} saturated: {sat['solves_per_s']} solves/s, p50 {sat['p50_ms']} ms, "
            f"p99 {sat['p99_ms']} ms")
        leg = {"pool_bytes": pool, "saturated": sat, "rates": []}
        for f in rates:
            r = run(f * sat["solves_per_s"], precision, pool)
            r["fraction_of_saturation"] = f
            leg["rates"].append(r)
            log(f"serving {precision} at {f:.2f} x sat: {r['solves_per_s']} solves/s, p50 {r['p50_ms']} ms, "
                f"p99 {r['p99_ms']} ms")
        out[precision] = leg
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--settle-s", type=float, default=0.5,
                    help="seconds of back-to-back solves before the headline's warm-up (clock ramp)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-single-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-fluxes", action="store_true")
    ap.add_argument("--no-momentum", action="store_true")
    ap.add_argument("--no-residual", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--n-refine", type=int, default=1)
    ap.add_argument("--nr", type=int, default=550)
    ap.add_argument("--nth", type=int, default=128)
    ap.add_argument("--nphi", type=int, default=256)
    ap.add_argument("--path", choices=["auto", "staged", "fused"], default="auto",
                    help="kernel path of the FP64 solve (auto: fused where the grid allows it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run torch's device copy of one field from 5 distinct sources, to "
                         "calibrate the FETCH_SIZE / WRITE_SIZE counters against a known byte count")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this solver is built and timed on a single MI355X "
              "(no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        # five distinct sources, all filled before the first copy: 720 MB written
        # after any source is filled, so that each copy reads its source from
        # memory rather than from the 256 MB last-level cache (as the solve's
        # kernels read their inputs)
        n = args.nr * args.nth * args.nphi
        srcs = [torch.full((n,), float(i + 1), dtype=torch.float64, device="cuda:0") for i in range(5)]
        b = torch.empty_like(srcs[0])
        torch.cuda.synchronize()
        for a in srcs:
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read_per_copy": 8 * n, "bytes_written_per_copy": 8 * n,
                                               "copies": 5}}), flush=True)
        return
    import paper_1806_06623_amd as spp
    import synthetic

    case = synthetic.stellar_case(args.nr, args.nth, args.nphi, seed=1)
    nr, nth, nphi = args.nr, args.nth, args.nphi
    zones = nr * nth * nphi
    log(f"workload {case['name']} zones={zones}")

    t0 = time.perf_counter()
    plan = spp.Plan(case["r_if"], case["th_if"], nphi, device="cuda:0")
    plan.path = args.path
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup (host eigensolves + upload) {setup_s:.3f} s")

    rho = torch.from_numpy(case["rho"]).to("cuda:0")
    phi = torch.empty_like(rho)
    phi_m = torch.empty_like(rho)
    K = args.steps
    # the FP64 solution the other legs start from (and compare with)
    plan.solve(rho, G=case["G"], out=phi)
    torch.cuda.synchronize()
    # The first solves after process start find the GPU's clocks still ramping
    # up (the compute-bound per-mode kernel runs about 10% slower there); they
    # are timed here as they come, for the record.  Everything after them is the
    # steady state a simulation sees when it calls the solver every time step:
    # a settling period of back-to-back solves precedes the other legs and
    # again the headline.
    for _ in range(args.warmup):
        plan.solve(rho, G=case["G"], out=phi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        plan.solve(rho, G=case["G"], out=phi)
    torch.cuda.synchronize()
    el_cold = time.perf_counter() - t0
    cold = {"solves_per_s": round(K / el_cold, 2), "ms_per_step": round(el_cold * 1e3 / K, 4),
            "note": f"the first {args.warmup} + {K} solves after process start (warm-up, then timed), before "
                    f"the GPU's clocks have ramped up"}
    log(f"cold start: {el_cold * 1e3 / K:.3f} ms/solve")

    def settle_clocks():
        """Back-to-back solves for args.settle_s seconds, so that the legs timed
        next run at the clocks of a busy GPU."""
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < args.settle_s:
            for _ in range(50):
                plan.solve(rho, G=case["G"], out=phi)
            n += 50
            torch.cuda.synchronize()
        return {"seconds": round(time.perf_counter() - t0, 3), "solves": n}

    settle_clocks()

    # mixed-precision form on the same workload (FP32-MFMA projections + FP64 refinement)
    mixed = None
    if not args.no_mixed:
        for _ in range(args.warmup):
            plan.solve_mixed(rho, G=case["G"], n_refine=args.n_refine, out=phi_m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            plan.solve_mixed(rho, G=case["G"], n_refine=args.n_refine, out=phi_m)
        torch.cuda.synchronize()
        el_m = time.perf_counter() - t0
        d = (phi_m - phi).abs().max().item() / phi.abs().max().item()
        mixed = {"precision": "mixed_fp32", "n_refine": args.n_refine, "solves_per_s": round(K / el_m, 2),
                 "gzones_per_s": round(zones * K / el_m / 1e9, 3), "ms_per_step": round(el_m * 1e3 / K, 4),
                 "max_rel_diff_vs_fp64_gpu": d}
        log(f"mixed: {el_m * 1e3 / K:.3f} ms/solve, diff vs FP64 {d:.2e}")

    # face fluxes of grad Phi (spp_face_fluxes) of the solution just computed:
    # one read of Phi and three fields written, HBM-bound
    face = None
    if not args.no_fluxes:
        fl = tuple(torch.empty_like(phi) for _ in range(3))
        for _ in range(20):
            plan.face_fluxes(phi, out=fl)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(K):
            plan.face_fluxes(phi, out=fl)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        fbytes = 4 * 8.0 * zones
        face = {"ms": round(ms, 5), "alg_bytes": fbytes, "GBps": round(fbytes / (ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(fbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "note": "whole entry point: outer-shell boundary term (shell FFT, per-mode beta, inverse "
                        "FFT) and the flux stencil; algorithmic bytes = Phi read once + three flux fields",
                "stencil_traffic": measured_traffic("faceflux::k_face_fluxes", nr, nth, nphi)}
        log(f"face fluxes: {ms * 1e3:.1f} us per call, {face['GBps']} GB/s")
        del fl

    # momentum source (spp_momentum_source) of the same Phi: one read of Phi
    # and three force fields written, HBM-bound
    mom = None
    if not args.no_momentum:
        F = tuple(torch.empty_like(phi) for _ in range(3))
        for _ in range(20):
            plan.momentum_source(phi, G=case["G"], out=F)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(K):
            plan.momentum_source(phi, G=case["G"], out=F)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        mbytes = 4 * 8.0 * zones
        mom = {"ms": round(ms, 5), "alg_bytes": mbytes, "GBps": round(mbytes / (ms * 1e-3) / 1e9, 1),
               "hbm_frac": round(mbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "note": "whole entry point: outer-face gradient (shell FFT, per-mode beta, inverse FFT) and the "
                       "stress-tensor face sums; algorithmic bytes = Phi read once + three force fields",
               "kernel_traffic": measured_traffic("momentum::k_momentum_rows", nr, nth, nphi)}
        log(f"momentum source: {ms * 1e3:.1f} us per call, {mom['GBps']} GB/s")
        del F

    # the FP64 residual 4 pi G rho - L Phi (spp_residual) of the same Phi: rho
    # and Phi read once, r written, HBM-bound
    resid = None
    if not args.no_residual:
        R = torch.empty_like(phi)
        for _ in range(20):
            plan.residual(rho, phi, G=case["G"], out=R)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(K):
            plan.residual(rho, phi, G=case["G"], out=R)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        rbytes = 3 * 8.0 * zones
        resid = {"ms": round(ms, 5), "alg_bytes": rbytes, "GBps": round(rbytes / (ms * 1e-3) / 1e9, 1),
                 "hbm_frac": round(rbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "note": "whole entry point: outer-shell boundary term (shell FFT, per-mode beta, inverse FFT) "
                         "and the flux stencil; algorithmic bytes = rho and Phi read once + r written",
                 "kernel_traffic": measured_traffic("k_residual_rows", nr, nth, nphi)}
        log(f"residual: {ms * 1e3:.1f} us per call, {resid['GBps']} GB/s")
        del R

    # copies of one field from five distinct sources (so that none is read
    # from the last-level cache): torch's device copy (`hbm_copy`; its
    # FETCH_SIZE/WRITE_SIZE counters calibrate the traffic figures) and the
    # library's streaming copy (`hbm_stream`, spp_stream_copy): one read and
    # one write stream, the rate the memory-bound kernels are set against
    # beside the 8 TB/s peak
    copy = stream = None
    if not args.no_copy:
        srcs = [torch.full_like(rho, float(i + 1)) for i in range(5)]
        dst = torch.empty_like(rho)
        cbytes = 2 * 8.0 * zones
        n_copy = max(5, (K // 5) * 5)

        def timed_copies(fn):
            for a in srcs:
                fn(a)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for k in range(n_copy):
                fn(srcs[k % 5])
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / n_copy
            return {"ms": round(ms, 5), "bytes": cbytes, "GBps": round(cbytes / (ms * 1e-3) / 1e9, 1),
                    "hbm_frac": round(cbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

        copy = timed_copies(lambda a: dst.copy_(a))
        stream = timed_copies(lambda a: spp.stream_copy(a, dst))
        if not torch.equal(dst, srcs[(n_copy - 1) % 5]):
            raise RuntimeError("spp_stream_copy did not reproduce its source")
        log(f"device copy of one field: {copy['ms'] * 1e3:.1f} us, {copy['GBps']} GB/s; "
            f"streaming copy: {stream['ms'] * 1e3:.1f} us, {stream['GBps']} GB/s")
        del srcs, dst

    batch = None if args.no_batch else batched_leg(spp, torch, synthetic, args.batch_steps)
    serving = None if args.no_serving else serving_leg(spp, torch, synthetic, args.serving_requests,
                                                        (0.5, 0.8, 0.95))

    settle = settle_clocks()
    for _ in range(args.warmup):
        plan.solve(rho, G=case["G"], out=phi)
    torch.cuda.synchronize()
    log(f"settle {settle['solves']} solves in {settle['seconds']} s, warmup {args.warmup} done")

    # throughput: K solves back to back, nothing else on the stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        plan.solve(rho, G=case["G"], out=phi)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    solves_s = K / elapsed
    log(f"timed {K} solves: {elapsed * 1e3 / K:.3f} ms/solve, {solves_s:.1f} solves/s")

    # latency: the same solves, each bracketed by HIP events (the event
    # records themselves add a few microseconds between solves)
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for k in range(K):
        ev0[k].record()
        plan.solve(rho, G=case["G"], out=phi)
        ev1[k].record()
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in zip(ev0, ev1)])

    # per-stage durations (HIP events recorded by the library on the solve stream)
    fused = plan.path == "fused"
    st = np.array([plan.solve_profiled(rho, phi, G=case["G"]) for _ in range(args.profile_steps)])
    stage_ms = st.mean(axis=0)
    model = stage_model(nr, nth, nphi, plan.parity_split, fused)
    # the fused path records the per-mode kernel as stage 1 (stages 2 and 3 are empty)
    names, times = (FUSED_STAGES, [stage_ms[0], stage_ms[1], stage_ms[4]]) if fused else (STAGES, list(stage_ms))
    stages = {}
    for name, ms in zip(names, times):
        m = model[name]
        d = {"ms": round(float(ms), 5), "alg_bytes": m["bytes"],
             "GBps": round(m["bytes"] / (ms * 1e-3) / 1e9, 1),
             "hbm_frac": round(m["bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        if m["flops"]:
            d["TFLOPs"] = round(m["flops"] / (ms * 1e-3) / 1e12, 3)
            d["mfma_frac"] = round(m["flops"] / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)
        stages[name] = d
    log(f"path {plan.path}; stages: " + ", ".join(f"{k}={v['ms']:.4f}ms" for k, v in stages.items()))

    # dominant kernel: the fused per-mode kernel (one launch per solve) or, on
    # the staged path, the theta projection (two launches per solve).  Its
    # roofline is the larger of the two ideal times: algorithmic bytes at the
    # HBM peak, algorithmic flops at the FP64 matrix peak.
    if fused:
        kname, k_ms, pm = "modal::k_modal (fused projection + radial + projection)", stage_ms[1], model["fused_modal"]
        per = "2 * N_r*N_theta^2*N_phi / 2 (both parity-split products)"
    else:
        kname = "proj::k_proj_par (parity split)" if plan.parity_split else "proj::k_proj_f64"
        k_ms, pm = 0.5 * (stage_ms[1] + stage_ms[3]), model["projection_forward"]
        per = "N_r*N_theta^2*N_phi, parity split" if plan.parity_split else "2*N_r*N_theta^2*N_phi"
    t_hbm = pm["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_mfma = pm["flops"] / (FP64_PEAK_TFLOPS * 1e12)
    if t_hbm >= t_mfma:
        achieved, peak, unit = pm["bytes"] / (k_ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, unit = pm["flops"] / (k_ms * 1e-3) / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"
    roofline = {"bound": "hbm" if t_hbm >= t_mfma else "mfma", "kernel": kname,
                "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(kname.split(" ")[0], nr, nth, nphi),
                "per_launch": (f"{pm['bytes']:.4g} algorithmic bytes (spectrum in, result out, eigenvector "
                               f"matrices) and {pm['flops']:.4g} flop ({per}) per launch; avg launch "
                               f"{k_ms * 1e3:.1f} us (HIP events on the solve stream); ideal {t_hbm * 1e6:.1f} us at "
                               f"the HBM peak, {t_mfma * 1e6:.1f} us at the FP64 matrix peak")}

    # memory-bound figures against the streaming copy's rate as well
    if stream is not None:
        for d in [v for k, v in stages.items() if k != "fused_modal"] + [face, mom, resid]:
            if d is not None:
                d["stream_frac"] = round(d["GBps"] / stream["GBps"], 4)
    if mixed is not None:
        mixed["speedup_vs_fp64"] = round(elapsed / (mixed["ms_per_step"] * 1e-3 * K), 3)
    phi_np = phi.cpu().numpy()
    result = {
        "metric": METRIC, "value": round(solves_s, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / K, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded stellar-core density: profile x lognormal field + point mass)",
        "config": {"workload": f"stellar_{nr}x{nth}x{nphi}_fp64", "nr": nr, "nth": nth, "nphi": nphi,
                   "zones": zones, "precision": "fp64", "path": plan.path},
        "gzones_per_s": round(zones * solves_s / 1e9, 3),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "setup_s": round(setup_s, 3),
        "settle": settle,
        "cold_start": cold,
        "stages": stages,
        "roofline": roofline,
        "mixed": mixed,
        "face_fluxes": face,
        "momentum_source": mom,
        "residual": resid,
        "hbm_copy": copy,
        "hbm_stream": stream,
        "batched": batch,
        "serving": serving,
    }
    if not args.no_cpu_baseline:
        cb, err = cpu_baseline(case, phi_np, args.cpu_seconds, args.cpu_single_seconds)
        result["cpu_baseline"] = cb
        result["max_rel_err_vs_oracle"] = err
    result["paper_context"] = ("Table 1: 0.32 s (32 cores) to 0.08 s (1024 cores) per solve on the Magnus "
                               "CPU cluster, i.e. 3.1-12.5 solves/s; 0.036 s with the parity split")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
