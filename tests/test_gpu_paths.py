"""GPU parity of every kernel path the library selects on valid inputs.

Each case asserts which kernels a solve of its plan launches (spp_plan_kernels)
and compares the result element by element with the FP64 oracle:
e = max|Phi_gpu - Phi_oracle| / max|Phi_oracle| <= 1e-12 (printed per case).
Where FP64 itself does not determine Phi to 1e-12 -- the theta eigenvalues
carry an absolute error near eps |K| (|K| ~ 4 / dtheta^2), i.e. a relative
error near 1e-12 on lambda ~ -2 once N_theta exceeds about 100, and
non-spherical sources feel it -- the bar is twice the spread between the
oracle and the same oracle with a second LAPACK eigensolver (MRRR), printed
beside e; the componentwise backward error must stay at the oracle's level.

Paths (selection rules of the library):
  * theta grids symmetric about the equator (Sec. 4.2) with N_theta/2 even,
    N_theta <= 128 and N_r <= 576: folded FFTs and the fused per-mode kernel;
  * otherwise the staged kernels: the parity-split projection on symmetric
    grids with N_theta <= 128, the LDS-image FP64 projection on other grids
    with N_theta <= 128 (tile width 16, 32, 64 or 128 columns), the generic
    64 x 64 tiled GEMM above N_theta = 128; the partitioned radial kernel up
    to N_r = 640 (chunks of 4, 8, 18 or 20 rows), one lane per system above.
Non-uniform theta interfaces are allowed throughout (Sec. 3.1); the
axis-coarsened symmetric grid is the kind Sec. 6 mentions.
"""
import numpy as np
import pytest

import synthetic
from oracle import laplacian, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12
TOL_MIXED = 1e-10


def _err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _case(nr, nth, nphi, seed, theta):
    """Random shell widths, the theta grid named, and the Gaussian-blob
    source of the small workload (sigma = 0.1 r_out at (0.3 r_out, pi/3,
    pi/4)) plus seeded uniform noise of 1e-3."""
    rng = np.random.default_rng(seed)
    r_if = np.concatenate(([0.0], np.cumsum(rng.uniform(0.3, 1.7, nr))))
    th_if = {"uniform": synthetic.theta_interfaces, "coarsened": synthetic.axis_coarsened_theta,
             "skewed": synthetic.skewed_theta}[theta](nth)
    R = r_if[-1]
    rho = synthetic.gaussian_blob(r_if, th_if, nphi, (0.3 * R, np.pi / 3, np.pi / 4), 0.1 * R)
    return r_if, th_if, rho + rng.uniform(-1e-3, 1e-3, rho.shape)


def _compare(name, r_if, th_if, nphi, rho, got):
    """Element-wise error against the oracle, with the bar widened to twice
    the oracle's own FP64 spread where that exceeds 1e-12 (module doc)."""
    ref = spectral.solve(r_if, th_if, nphi, rho)
    spread = _err(spectral.solve(r_if, th_if, nphi, rho, driver="stemr"), ref)
    e = _err(got, ref)
    eta = laplacian.backward_error(r_if, th_if, nphi, got, rho)
    eta_ref = laplacian.backward_error(r_if, th_if, nphi, ref, rho)
    tol = max(TOL_FP64, 2.0 * spread)
    print(f"[parity] {name}: max rel err {e:.3e} (bar {tol:.1e}; oracle FP64 spread {spread:.2e}); "
          f"backward error {eta:.2e} (oracle {eta_ref:.2e})", flush=True)
    assert np.all(np.isfinite(got))
    assert e <= tol
    assert eta <= max(4.0 * eta_ref, 1e-13)


# (name, nr, nth, nphi, theta, expected kernels of the solve)
PATHS = [
    ("generic GEMM, N_theta > 128", 12, 144, 16, "uniform",
     ["k_rfft_fwd<16>", "k_proj_f64", "radial::k_radial_part<4>", "k_proj_f64", "k_rfft_inv<16>"]),
    ("one lane per radial system, N_r > 640", 700, 8, 8, "uniform",
     ["k_rfft_fwd<8>", "proj::k_proj_par<1>", "k_radial", "proj::k_proj_par<1>", "k_rfft_inv<8>"]),
    ("partitioned radial, 20-row chunks", 600, 16, 8, "uniform",
     ["k_rfft_fwd<8>", "proj::k_proj_par<1>", "radial::k_radial_part<20>", "proj::k_proj_par<1>",
      "k_rfft_inv<8>"]),
    ("LDS-image projection, 128-column tiles, non-symmetric theta", 30, 100, 16, "skewed",
     ["k_rfft_fwd<16>", "proj::k_proj_f64<8,1>", "radial::k_radial_part<4>", "proj::k_proj_f64<8,1>",
      "k_rfft_inv<16>"]),
    ("LDS-image projection, 64-column tiles, non-symmetric theta", 25, 40, 16, "skewed",
     ["k_rfft_fwd<16>", "proj::k_proj_f64<4,2>", "radial::k_radial_part<4>", "proj::k_proj_f64<4,2>",
      "k_rfft_inv<16>"]),
    ("LDS-image projection, 16-column tiles, non-symmetric theta", 20, 12, 8, "skewed",
     ["k_rfft_fwd<8>", "proj::k_proj_f64<1,4>", "radial::k_radial_part<4>", "proj::k_proj_f64<1,4>",
      "k_rfft_inv<8>"]),
    ("parity-split projection, symmetric theta with N_theta/2 odd", 150, 54, 32, "coarsened",
     ["k_rfft_fwd<32>", "proj::k_proj_par<2>", "radial::k_radial_part<8>", "proj::k_proj_par<2>",
      "k_rfft_inv<32>"]),
    ("fused per-mode kernel, axis-coarsened theta", 200, 64, 32, "coarsened",
     ["k_rfft_fwd<32,fold>", "modal::k_modal<2,2>", "k_rfft_inv<32,fold>"]),
]


@pytest.mark.parametrize("name,nr,nth,nphi,theta,kernels", PATHS, ids=[p[0] for p in PATHS])
def test_kernel_path_matches_oracle(name, nr, nth, nphi, theta, kernels):
    import paper_1806_06623_amd as spp
    print(f"[case] {name}: {nr}x{nth}x{nphi} theta={theta}", flush=True)
    r_if, th_if, rho = _case(nr, nth, nphi, nr + nth + nphi, theta)
    plan = spp.Plan(r_if, th_if, nphi)
    assert plan.kernels == kernels, plan.kernels
    got = plan.solve(torch.from_numpy(rho).to("cuda")).cpu().numpy()
    _compare(f"{name} {nr}x{nth}x{nphi} [{';'.join(plan.kernels)}]", r_if, th_if, nphi, rho, got)


def test_staged_path_full_size_550x128x256():
    """The five staged kernels on the headline workload, element by element."""
    import paper_1806_06623_amd as spp
    c = synthetic.stellar_case()
    print(f"[case] staged {c['name']}", flush=True)
    plan = spp.Plan(c["r_if"], c["th_if"], c["nphi"])
    plan.path = "staged"
    assert plan.kernels == ["k_rfft_fwd<256>", "proj::k_proj_par<4>", "radial::k_radial_part<18>",
                            "proj::k_proj_par<4>", "k_rfft_inv<256>"], plan.kernels
    got = plan.solve(torch.from_numpy(c["rho"]).to("cuda")).cpu().numpy()
    ref = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"])
    e = _err(got, ref)
    print(f"[parity] staged {c['name']}: max rel err {e:.3e}", flush=True)
    assert e <= TOL_FP64


def test_fused_axis_coarsened_theta_full_size():
    """The headline radial grid and source with an axis-coarsened theta grid
    (cells twice as wide at the poles as at the equator, symmetric about the
    equator): the parity split and the fused per-mode kernel apply."""
    import paper_1806_06623_amd as spp
    r_if = synthetic.stellar_r_interfaces(550)
    th_if = synthetic.axis_coarsened_theta(128)
    rho = synthetic.stellar_density(r_if, th_if, 256, 31)
    print("[case] fused axis-coarsened 550x128x256", flush=True)
    plan = spp.Plan(r_if, th_if, 256)
    assert plan.kernels == ["k_rfft_fwd<256,fold>", "modal::k_modal<4,3>", "k_rfft_inv<256,fold>"], plan.kernels
    got = plan.solve(torch.from_numpy(rho).to("cuda")).cpu().numpy()
    _compare("fused axis-coarsened 550x128x256", r_if, th_if, 256, rho, got)


def test_mixed_with_one_lane_radial():
    """The mixed form with N_r > 640 (one-lane radial kernel) reaches the FP64
    solution after one refinement."""
    import paper_1806_06623_amd as spp
    r_if, th_if, rho = _case(700, 8, 8, 5, "uniform")
    print("[case] mixed 700x8x8", flush=True)
    plan = spp.Plan(r_if, th_if, 8)
    got = plan.solve_mixed(torch.from_numpy(rho).to("cuda"), n_refine=1).cpu().numpy()
    ref = spectral.solve(r_if, th_if, 8, rho)
    e = _err(got, ref)
    print(f"[parity] mixed_fp32 700x8x8 n_refine=1: max rel err {e:.3e}", flush=True)
    assert e <= TOL_MIXED
