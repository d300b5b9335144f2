"""GPU tests of the batched form: the right-hand sides of a grid class run
batched (each kernel of the fused solve one launch over all of them), other
classes one solve each, all in one HIP graph; every entry must equal its lone
solve bit for bit, FP64 and mixed."""
import numpy as np
import pytest

import synthetic
from oracle import spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _entries(shapes, seed0, skewed=()):
    import paper_1806_06623_amd as spp
    cache, plans, cases = {}, [], []
    for k, shp in enumerate(shapes):
        key = (shp, shp in skewed)
        r_if, th_if, nphi = synthetic.stellar_grid(*shp)
        if shp in skewed:
            th_if = synthetic.skewed_theta(shp[1])
        if key not in cache:
            cache[key] = spp.Plan(r_if, th_if, nphi)
        cases.append(dict(r_if=r_if, th_if=th_if, nphi=nphi,
                          rho=synthetic.stellar_density(r_if, th_if, nphi, seed0 + k)))
        plans.append(cache[key])
    rhos = [torch.from_numpy(c["rho"]).to("cuda") for c in cases]
    return plans, cases, rhos


def test_fp64_batch_matches_lone_solves_bitwise_and_oracle():
    import paper_1806_06623_amd as spp
    # three classes batched (3, 2 and 2 right-hand sides), one lone fused
    # class, and a staged class (theta not symmetric about the equator)
    shapes = [(64, 32, 64), (40, 16, 32), (64, 32, 64), (128, 64, 128), (40, 16, 32), (33, 20, 16),
              (64, 32, 64), (128, 64, 128), (48, 24, 32), (32, 16, 256), (32, 16, 256)]
    plans, cases, rhos = _entries(shapes, 200, skewed={(48, 24, 32)})
    phis = [torch.empty_like(x) for x in rhos]
    Gs = [1.0 + 0.25 * k for k in range(len(shapes))]
    batch = spp.Batch(plans, rhos, phis, Gs)
    print(f"[batch] {batch.description}", flush=True)
    assert "64x32x64 n=3 batched" in batch.description and "48x24x32 n=1 per-rhs staged" in batch.description
    assert "32x16x256 n=2 batched" in batch.description
    batch.launch()
    torch.cuda.synchronize()
    first = [y.clone() for y in phis]
    batch.launch()                          # replay of the same graph
    torch.cuda.synchronize()
    for k, (p, x, y, y0, G, c) in enumerate(zip(plans, rhos, phis, first, Gs, cases)):
        lone = p.solve(x, G=G)
        torch.cuda.synchronize()
        assert torch.equal(y, y0), f"replay differs for entry {k}"
        assert torch.equal(y, lone), f"batched entry {k} differs from its lone solve"
        assert batch.status(k)["status"] == "ok"
        if k in (0, 3, 5, 8, 10):
            ref = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"], G)
            e = float(np.max(np.abs(y.cpu().numpy() - ref)) / np.max(np.abs(ref)))
            print(f"[parity] batch entry {k} shape {shapes[k]}: {e:.3e}", flush=True)
            assert e <= 1e-12


def test_batched_entry_status_is_per_rhs():
    """A NaN in one right-hand side of a batched class flags that entry only."""
    import paper_1806_06623_amd as spp
    shapes = [(64, 32, 64)] * 3
    plans, cases, rhos = _entries(shapes, 300)
    rhos[1][3, 4, 5] = float("nan")
    phis = [torch.empty_like(x) for x in rhos]
    batch = spp.Batch(plans, rhos, phis, [1.0] * 3, autotune=False)
    batch.launch()
    sts = [batch.status(k)["status"] for k in range(3)]
    print(f"[status] batch entries: {sts}", flush=True)
    assert sts == ["ok", "enonfinite", "ok"]


def test_mixed_batch_matches_lone_mixed_solves():
    import paper_1806_06623_amd as spp
    shapes = [(64, 32, 64), (40, 16, 32), (64, 32, 64), (33, 20, 16)]
    plans, cases, rhos = _entries(shapes, 400)
    phis = [torch.empty_like(x) for x in rhos]
    batch = spp.Batch(plans, rhos, phis, [1.0] * len(shapes), precision="mixed_fp32", n_refine=1)
    print(f"[batch] {batch.description}", flush=True)
    batch.launch()
    torch.cuda.synchronize()
    for k, (p, x, y, c) in enumerate(zip(plans, rhos, phis, cases)):
        lone = p.solve_mixed(x, n_refine=1)
        torch.cuda.synchronize()
        assert torch.equal(y, lone), f"mixed batched entry {k} differs from its lone solve"
        ref = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"])
        e = float(np.max(np.abs(y.cpu().numpy() - ref)) / np.max(np.abs(ref)))
        print(f"[parity] mixed batch entry {k} shape {shapes[k]}: {e:.3e}", flush=True)
        assert e <= 1e-10


def test_projection_autotuner_on_the_staged_grid_it_serves():
    """spp_autotune_projection times the LDS-image FP64 projection, which runs
    on theta grids not symmetric about the equator: the chosen row tile is the
    one the plan's solves then launch, and parity holds."""
    import paper_1806_06623_amd as spp
    r_if = synthetic.stellar_r_interfaces(96)
    th_if = synthetic.skewed_theta(64)
    rho = synthetic.stellar_density(r_if, th_if, 32, 7)
    plan = spp.Plan(r_if, th_if, 32)
    rows = plan.autotune()
    assert rows in (16, 32)
    assert plan.kernels[1] == f"proj::k_proj_f64<4,{rows // 16}>", plan.kernels
    got = plan.solve(torch.from_numpy(rho).to("cuda")).cpu().numpy()
    ref = spectral.solve(r_if, th_if, 32, rho)
    e = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"[parity] autotuned rows={rows} ({plan.kernels[1]}): {e:.3e}", flush=True)
    assert e <= 1e-12
