"""GPU tests of the batched form (one HIP graph over many solves on uneven grids)."""
import numpy as np
import pytest

import synthetic
from oracle import spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _plan_and_case(nr, nth, nphi, seed):
    import paper_1806_06623_amd as spp
    r_if, th_if, nphi = synthetic.stellar_grid(nr, nth, nphi)
    rho = synthetic.stellar_density(r_if, th_if, nphi, seed)
    return spp.Plan(r_if, th_if, nphi), dict(r_if=r_if, th_if=th_if, nphi=nphi, rho=rho)


def test_batch_matches_lone_solves_bitwise_and_oracle():
    import paper_1806_06623_amd as spp
    shapes = [(64, 32, 64), (40, 16, 32), (64, 32, 64), (128, 64, 128), (40, 16, 32), (33, 20, 16)]
    cache, plans, cases = {}, [], []
    for k, shp in enumerate(shapes):
        if shp not in cache:
            cache[shp] = _plan_and_case(*shp, seed=200 + k)[0]
        r_if, th_if, nphi = synthetic.stellar_grid(*shp)
        cases.append(dict(r_if=r_if, th_if=th_if, nphi=nphi,
                          rho=synthetic.stellar_density(r_if, th_if, nphi, 200 + k)))
        plans.append(cache[shp])
    rhos = [torch.from_numpy(c["rho"]).to("cuda") for c in cases]
    phis = [torch.empty_like(x) for x in rhos]
    Gs = [1.0 + 0.25 * k for k in range(len(shapes))]
    batch = spp.Batch(plans, rhos, phis, Gs)
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
        if k in (0, 3, 5):
            ref = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"], G)
            e = float(np.max(np.abs(y.cpu().numpy() - ref)) / np.max(np.abs(ref)))
            print(f"[parity] batch entry {k} shape {shapes[k]}: {e:.3e}", flush=True)
            assert e <= 1e-12


def test_autotuned_tiles_keep_parity():
    plan, c = _plan_and_case(96, 64, 32, seed=7)
    rows = plan.autotune()
    assert rows in (16, 32, 64)
    x = torch.from_numpy(c["rho"]).to("cuda")
    got = plan.solve(x).cpu().numpy()
    ref = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"])
    e = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"[parity] autotuned rows={rows}: {e:.3e}", flush=True)
    assert e <= 1e-12
