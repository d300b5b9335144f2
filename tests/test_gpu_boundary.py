"""GPU tests of the rest of the boundary: the FP64 residual entry point, the
solve status (non-finite flag, refinement contraction, FP64 fallback) and
the regular inner condition.

Residual parity: r = 4 pi G rho - L Phi against oracle/laplacian.apply on
random fields, componentwise within 1e-12 of |L_loc||Phi| + |L_bnd Phi| +
|4 pi G rho| (both sides evaluate the same sums in FP64 in different orders).
"""
import numpy as np
import pytest

import synthetic
from oracle import laplacian, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _random_case(nr, nth, nphi, seed, r0=0.0, theta="uniform"):
    rng = np.random.default_rng(seed)
    r_if = r0 + np.concatenate(([0.0], np.cumsum(rng.uniform(0.3, 1.7, nr))))
    th_if = {"uniform": synthetic.theta_interfaces, "skewed": synthetic.skewed_theta,
             "coarsened": synthetic.axis_coarsened_theta}[theta](nth)
    return r_if, th_if, rng


@pytest.mark.parametrize("nr,nth,nphi,r0,theta,inner", [
    (37, 20, 8, 0.0, "uniform", "auto"),
    (9, 70, 32, 0.0, "skewed", "auto"),
    (24, 16, 16, 2.0, "coarsened", "zero_flux"),
    (24, 16, 16, 2.0, "coarsened", "regular"),
    (7, 6, 512, 1.0, "uniform", "regular"),   # N_phi > 256: the per-column kernel
    (550, 128, 256, 0.0, "uniform", "auto"),
])
def test_residual_matches_oracle(nr, nth, nphi, r0, theta, inner):
    import paper_1806_06623_amd as spp
    print(f"[case] residual {nr}x{nth}x{nphi} r0={r0} theta={theta} inner={inner}", flush=True)
    if nr == 550:
        c = synthetic.stellar_case()
        r_if, th_if, rho = c["r_if"], c["th_if"], c["rho"]
        rng = np.random.default_rng(5)
    else:
        r_if, th_if, rng = _random_case(nr, nth, nphi, nr + nth, r0, theta)
        rho = rng.standard_normal((nr, nth, nphi))
    phi = rng.standard_normal((nr, nth, nphi))
    G = 0.7
    plan = spp.Plan(r_if, th_if, nphi, inner=inner)
    r = plan.residual(torch.from_numpy(rho).to("cuda"), torch.from_numpy(phi).to("cuda"), G=G).cpu().numpy()
    oinner = "regular" if inner == "regular" else "zero_flux"
    LP, mag = laplacian.apply(r_if, th_if, nphi, phi, with_terms=True, inner=oinner)
    s = 4.0 * np.pi * G * rho
    ref = s - LP
    e = float(np.max(np.abs(r - ref) / (mag + np.abs(s))))
    print(f"[parity] residual {nr}x{nth}x{nphi} inner={inner}: componentwise {e:.3e} (bar 1e-12)", flush=True)
    assert e <= 1e-12


def test_solution_residual_at_roundoff():
    """The residual entry point applied to the solver's own output: the
    componentwise backward error is at rounding level (FP64 solve)."""
    import paper_1806_06623_amd as spp
    c = synthetic.stellar_case(nr=256, nth=64, nphi=128, seed=3)
    plan = spp.Plan(c["r_if"], c["th_if"], c["nphi"])
    rho = torch.from_numpy(c["rho"]).to("cuda")
    phi = plan.solve(rho)
    r = plan.residual(rho, phi).cpu().numpy()
    _, mag = laplacian.apply(c["r_if"], c["th_if"], c["nphi"], phi.cpu().numpy(), with_terms=True)
    s = 4.0 * np.pi * c["rho"]
    eta = float(np.max(np.abs(r) / (mag + np.abs(s))))
    print(f"[parity] residual of the GPU solution 256x64x128: backward error {eta:.2e}", flush=True)
    assert eta < 1e-13


@pytest.mark.parametrize("path", ["fused", "staged"])
def test_nonfinite_rho_is_reported_and_cleared(path):
    import paper_1806_06623_amd as spp
    c = synthetic.stellar_case(nr=128, nth=32, nphi=64, seed=2)
    plan = spp.Plan(c["r_if"], c["th_if"], c["nphi"])
    plan.path = path
    rho = torch.from_numpy(c["rho"]).to("cuda")
    plan.solve(rho)
    st = plan.status()
    assert st["status"] == "ok" and st["nonfinite"] == 0
    bad = rho.clone()
    bad[5, 7, 9] = float("nan")
    plan.solve(bad)
    st = plan.status()
    print(f"[status] {path}: NaN in rho -> {st}", flush=True)
    assert st["status"] == "enonfinite" and st["nonfinite"] == 1
    bad[5, 7, 9] = float("inf")
    plan.solve(bad)
    assert plan.status()["status"] == "enonfinite"
    plan.solve(rho)                                  # the next solve clears the flag
    assert plan.status()["status"] == "ok"


def test_mixed_status_reports_contraction():
    import paper_1806_06623_amd as spp
    c = synthetic.stellar_case(nr=128, nth=32, nphi=64, seed=4)
    plan = spp.Plan(c["r_if"], c["th_if"], c["nphi"])
    rho = torch.from_numpy(c["rho"]).to("cuda")
    ref = plan.solve(rho).clone()
    got = plan.solve_mixed(rho, n_refine=2)
    st = plan.status(workspace=plan.mixed_workspace)
    e = (got - ref).abs().max().item() / ref.abs().max().item()
    print(f"[status] mixed n_refine=2: {st}, vs FP64 {e:.2e}", flush=True)
    assert st["status"] == "ok" and st["refine_iters"] == 2 and st["not_contracted"] == 0
    # the first low-precision pass leaves a residual near 1e-3 of the source
    # (|L| amplifies the FP32 error of g), each refinement step shrinks it
    assert st["fell_back_fp64"] == 0 and 0 < st["last_residual_rel"] < 1e-3 * st["first_residual_rel"]
    assert st["first_residual_rel"] < 0.05
    assert e <= 1e-10


def test_diverging_refinement_falls_back_to_fp64_or_reports_enoconv():
    """A low-precision basis scaled by 1.5 makes each pass return 2.25 times
    its correction, so the refinement diverges: with the fallback the FP64
    solve replaces the result bit for bit; without it the status is ENOCONV."""
    import paper_1806_06623_amd as spp
    c = synthetic.stellar_case(nr=128, nth=32, nphi=64, seed=6)
    for path in ("fused", "staged"):
        plan = spp.Plan(c["r_if"], c["th_if"], c["nphi"])
        plan.path = path
        rho = torch.from_numpy(c["rho"]).to("cuda")
        ref = plan.solve(rho).clone()
        plan.scale_lowprec_basis(1.5)
        got = plan.solve_mixed(rho, n_refine=1, fallback_fp64=True)
        st = plan.status(workspace=plan.mixed_workspace)
        print(f"[status] {path} diverging, fallback: {st}", flush=True)
        assert st["status"] == "ok" and st["not_contracted"] == 1 and st["fell_back_fp64"] == 1
        assert torch.equal(got, ref)
        got = plan.solve_mixed(rho, n_refine=1, fallback_fp64=False)
        st = plan.status(workspace=plan.mixed_workspace)
        print(f"[status] {path} diverging, no fallback: {st}", flush=True)
        assert st["status"] == "enoconv" and st["fell_back_fp64"] == 0
        assert not torch.equal(got, ref)


@pytest.mark.parametrize("nr,nth,nphi,theta", [(24, 16, 16, "coarsened"), (40, 12, 8, "skewed")])
def test_regular_inner_condition_matches_oracle(nr, nth, nphi, theta):
    """r_{1/2} > 0 with the regular inner condition (staged kernels), FP64
    and mixed, against the oracle with the same condition."""
    import paper_1806_06623_amd as spp
    r_if, th_if, rng = _random_case(nr, nth, nphi, 91 + nr, 1.5, theta)
    R = r_if[-1]
    rho = synthetic.gaussian_blob(r_if, th_if, nphi, (0.5 * R, np.pi / 3, np.pi / 4), 0.15 * R)
    plan = spp.Plan(r_if, th_if, nphi, inner="regular")
    assert plan.path == "staged"
    x = torch.from_numpy(rho).to("cuda")
    got = plan.solve(x).cpu().numpy()
    mixed = plan.solve_mixed(x, n_refine=1).cpu().numpy()
    ref = spectral.solve(r_if, th_if, nphi, rho, inner="regular")
    zf = spectral.solve(r_if, th_if, nphi, rho)
    e, em, ez = _err(got, ref), _err(mixed, ref), _err(got, zf)
    print(f"[parity] regular inner {nr}x{nth}x{nphi}: fp64 {e:.3e}, mixed {em:.3e} (differs from zero flux by "
          f"{ez:.2e})", flush=True)
    assert e <= 1e-12 and em <= 1e-10 and ez > 1e-4


def test_noalloc_status():
    import paper_1806_06623_amd as spp
    c = synthetic.gaussian_blob_case()
    plan = spp.Plan(c["r_if"], c["th_if"], c["nphi"])
    rho = torch.from_numpy(c["rho"]).to("cuda")
    plan.solve_noalloc(rho)
    assert plan.status(noalloc=True)["status"] == "ok"
    bad = rho.clone()
    bad[0, 0, 0] = float("nan")
    plan.solve_noalloc(bad)
    assert plan.status(noalloc=True)["status"] == "enonfinite"


def test_stream_copy_is_exact():
    """The streaming-copy reference moves every byte: one stellar field
    (550 x 128 x 256, more elements than one sweep of its grid) and a ragged
    size."""
    import torch
    import paper_1806_06623_amd as spp
    g = torch.Generator(device="cuda").manual_seed(5)
    for n in (550 * 128 * 256, 2 * 1037):
        print(f"[case] stream copy of {n} doubles", flush=True)
        src = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        dst = torch.full_like(src, float("nan"))
        spp.stream_copy(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
