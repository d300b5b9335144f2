"""GPU parity of the mixed-precision solve (FP32-MFMA projections, FP64 refinement).

Metric: e = max|Phi_gpu - Phi_oracle| / max|Phi_oracle| against the FP64 oracle.
Bar for the refined mixed form: e <= 1e-10.
"""
import numpy as np
import pytest

import synthetic
from oracle import spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-10


def _err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _mixed(case, n_refine):
    import paper_1806_06623_amd as spp
    plan = spp.Plan(case["r_if"], case["th_if"], case["nphi"])
    x = torch.from_numpy(np.ascontiguousarray(case["rho"])).to("cuda")
    out = plan.solve_mixed(x, G=case["G"], precision="mixed_fp32", n_refine=n_refine)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _case(nr, nth, nphi, seed):
    rng = np.random.default_rng(seed)
    r_if = np.concatenate(([0.0], np.cumsum(rng.uniform(0.3, 1.7, nr))))
    return dict(name=f"random_{nr}x{nth}x{nphi}", r_if=r_if, th_if=synthetic.theta_interfaces(nth),
                nphi=nphi, rho=rng.standard_normal((nr, nth, nphi)), G=1.0)


@pytest.mark.parametrize("maker", [
    lambda: synthetic.gaussian_blob_case(),
    lambda: _case(37, 20, 8, 1),
    lambda: _case(65, 17, 16, 3),
    lambda: _case(130, 48, 128, 6),
])
def test_refinement_reaches_fp64_parity(maker):
    c = maker()
    print(f"[case] mixed {c['name']}", flush=True)
    ref = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"], c["G"])
    errs = [_err(_mixed(c, n), ref) for n in (0, 1, 2)]
    print(f"[parity] mixed_fp32 {c['name']}: n_refine 0/1/2 -> {errs[0]:.3e} {errs[1]:.3e} {errs[2]:.3e}",
          flush=True)
    assert errs[0] < 1e-5                     # one FP32-projection pass
    assert errs[1] <= TOL_MIXED
    assert errs[2] <= TOL_MIXED


def test_stellar_full_size_mixed():
    c = synthetic.stellar_case()
    print(f"[case] mixed {c['name']}", flush=True)
    ref = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"], c["G"])
    e = _err(_mixed(c, 1), ref)
    print(f"[parity] mixed_fp32 {c['name']} n_refine=1: {e:.3e}", flush=True)
    assert e <= TOL_MIXED
