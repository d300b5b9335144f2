"""GPU tests of the serving loop: continuous batching, footprint admission,
and identical results alone and in the mix."""
import numpy as np
import pytest

import synthetic
from oracle import spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CLASSES = [(32, 16, 16), (64, 32, 32), (96, 48, 64)]


def _setup():
    import paper_1806_06623_amd as spp
    plans, grids = [], []
    for c in CLASSES:
        r_if, th_if, nphi = synthetic.stellar_grid(*c)
        plans.append(spp.Plan(r_if, th_if, nphi))
        grids.append((r_if, th_if, nphi))
    return spp, plans, grids


def test_results_identical_alone_and_in_the_mix():
    spp, plans, grids = _setup()
    rng = np.random.default_rng(4)
    reqs = []
    for k in range(60):
        cls = int(rng.integers(0, len(CLASSES)))
        r_if, th_if, nphi = grids[cls]
        rho = synthetic.serving_source(r_if, th_if, nphi, seed=1000 + k)
        x = torch.from_numpy(rho).to("cuda")
        reqs.append((cls, x, torch.empty_like(x), 1.0 + 0.01 * k, rho))
    # alone: each request as a single solve
    alone = []
    for cls, x, _, G, _ in reqs:
        alone.append(plans[cls].solve(x, G=G).clone())
    torch.cuda.synchronize()
    # in the mix: a pool that holds only two of the largest workspaces forces
    # admission to wait for memory; four slots overlap solves on the device
    pool = 2 * max(p.workspace_bytes for p in plans) + 4096
    srv = spp.Server(plans, pool_bytes=pool, n_slots=4)
    for k, (cls, x, y, G, _) in enumerate(reqs):
        srv.submit(cls, x, y, G=G, request_id=k)
    srv.drain(120.0)
    done = srv.poll()
    srv.close()
    assert len(done) == len(reqs)
    for c in done:
        assert c["status"] == 0
        assert c["t_arrival"] <= c["t_admit"] <= c["t_done"]
    for k, (cls, x, y, G, rho) in enumerate(reqs):
        assert torch.equal(y, alone[k]), f"request {k} differs in the mix"
    cls, x, y, G, rho = reqs[7]
    r_if, th_if, nphi = grids[cls]
    ref = spectral.solve(r_if, th_if, nphi, rho, G)
    e = float(np.max(np.abs(y.cpu().numpy() - ref)) / np.max(np.abs(ref)))
    print(f"[parity] served request 7 class {CLASSES[cls]}: {e:.3e}", flush=True)
    assert e <= 1e-12


def test_request_larger_than_pool_is_refused():
    spp, plans, grids = _setup()
    srv = spp.Server(plans, pool_bytes=plans[0].workspace_bytes + 256, n_slots=2)
    r_if, th_if, nphi = grids[2]
    x = torch.zeros((len(r_if) - 1, len(th_if) - 1, nphi), dtype=torch.float64, device="cuda")
    with pytest.raises(spp.SphPoissonError) as ei:
        srv.submit(2, x, torch.empty_like(x), request_id=1)
    assert ei.value.status == -4
    srv.close()


def test_scheduled_arrivals_are_respected():
    spp, plans, grids = _setup()
    srv = spp.Server(plans, pool_bytes=4 * max(p.workspace_bytes for p in plans), n_slots=2)
    r_if, th_if, nphi = grids[0]
    x = torch.from_numpy(synthetic.serving_source(r_if, th_if, nphi, seed=5)).to("cuda")
    y = torch.empty_like(x)
    t0 = srv.now()
    srv.submit(0, x, y, request_id=3, not_before=t0 + 0.05)
    srv.drain(30.0)
    (c,) = srv.poll()
    srv.close()
    assert c["t_arrival"] >= t0 + 0.05 - 1e-6
    assert c["t_admit"] >= c["t_arrival"]


def test_mixed_and_fp64_requests_identical_alone_and_in_the_mix():
    """Mixed-precision requests (FP32 projections, one refinement, FP64
    fallback armed) interleaved with FP64 ones on the same classes: every
    result is bitwise its lone solve of the same precision, and the mixed
    ones are within 1e-10 of the oracle."""
    spp, plans, grids = _setup()
    rng = np.random.default_rng(44)
    reqs = []
    for k in range(40):
        cls = int(rng.integers(0, len(CLASSES)))
        prec = "mixed_fp32" if k % 2 else "fp64"
        r_if, th_if, nphi = grids[cls]
        rho = synthetic.serving_source(r_if, th_if, nphi, seed=2000 + k)
        x = torch.from_numpy(rho).to("cuda")
        reqs.append((cls, prec, x, torch.empty_like(x), rho))
    alone = []
    for cls, prec, x, _, _ in reqs:
        p = plans[cls]
        alone.append((p.solve_mixed(x, n_refine=1) if prec == "mixed_fp32" else p.solve(x)).clone())
    torch.cuda.synchronize()
    pool = 3 * max(p.workspace_bytes_for("mixed_fp32") for p in plans)
    srv = spp.Server(plans, pool_bytes=pool, n_slots=4)
    for k, (cls, prec, x, y, _) in enumerate(reqs):
        srv.submit(cls, x, y, request_id=k, precision=prec, n_refine=1)
    srv.drain(120.0)
    done = srv.poll()
    srv.close()
    assert len(done) == len(reqs) and all(c["status"] == 0 for c in done)
    for k, (cls, prec, x, y, rho) in enumerate(reqs):
        assert torch.equal(y, alone[k]), f"request {k} ({prec}) differs in the mix"
    cls, prec, x, y, rho = reqs[1]
    r_if, th_if, nphi = grids[cls]
    ref = spectral.solve(r_if, th_if, nphi, rho)
    e = float(np.max(np.abs(y.cpu().numpy() - ref)) / np.max(np.abs(ref)))
    print(f"[parity] served mixed request 1 class {CLASSES[cls]}: {e:.3e}", flush=True)
    assert e <= 1e-10
