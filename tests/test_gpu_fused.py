"""GPU parity of the fused per-mode path (equator-symmetric theta grids).

The fused path folds the theta parity in the FFTs and runs the forward
projection, the radial solves and the inverse projection in one kernel per
(Fourier component, parity).  Each case (the stellar workload's grid and
source at that size) is compared with the FP64 oracle
(e = max|Phi_gpu - Phi_oracle| / max|Phi_oracle| <= 1e-12) and with the staged
five-kernel path on the same plan.  The shapes cross the kernel's tiling:
one to three row tiles of 16 per wave (12 waves, 192 rows per tile level),
a partial last partition, and column widths h = N_theta/2 of 2 to 64,
including widths that are not a multiple of 16.
"""
import numpy as np
import pytest

import synthetic
from oracle import laplacian, spectral

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12


def _err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _grid(nr, nth, seed):
    rng = np.random.default_rng(seed)
    r_if = np.concatenate(([0.0], np.cumsum(rng.uniform(0.3, 1.7, nr))))
    th_if = np.pi * np.arange(nth + 1) / nth
    return rng, r_if, th_if


def _case(nr, nth, nphi, seed):
    """The stellar workload's grid and source at this size (N_r > 20), else a
    random-width grid with a normal source."""
    if nr > 20:
        r_if, th_if, _ = synthetic.stellar_grid(nr, nth, nphi)
        return r_if, th_if, synthetic.stellar_density(r_if, th_if, nphi, seed)
    rng, r_if, th_if = _grid(nr, nth, seed)
    return r_if, th_if, rng.standard_normal((nr, nth, nphi))


def _both_paths(r_if, th_if, nphi, rho):
    import paper_1806_06623_amd as spp
    plan = spp.Plan(r_if, th_if, nphi)
    assert plan.path == "fused"
    x = torch.from_numpy(rho).to("cuda")
    fused = plan.solve(x).cpu().numpy()
    plan.path = "staged"
    assert plan.path == "staged"
    staged = plan.solve(x).cpu().numpy()
    plan.path = "auto"
    return fused, staged


@pytest.mark.parametrize("nr,nth,nphi,seed", [
    (2, 4, 4, 11),        # smallest fused grid: h = 2, one partition
    (7, 12, 16, 12),      # h = 6, one partial chunk
    (192, 32, 32, 13),    # one row tile per wave, h = 16
    (193, 64, 64, 14),    # one row past it: two tiles, h = 32
    (384, 100, 16, 15),   # two full tiles, h = 50 (padded columns)
    (385, 128, 8, 16),    # three tiles, h = 64
    (576, 128, 32, 17),   # largest N_r of the fused kernel
    (40, 16, 1024, 18),   # 2048 workgroups: the paired unit order far past one round
    (7, 12, 256, 19),     # register-pass folded FFTs: 42 pairs, blocks span rows, ragged last block
    (9, 100, 256, 20),    # 450 pairs, h = 50
    (64, 16, 256, 21),    # 32 blocks of 16 pairs: the XCD-ordered block range of the inverse
    (300, 24, 16, 22),    # one column tile, two row tiles per wave (8-row chunks)
    (500, 32, 8, 23),     # one column tile, three row tiles
    (100, 48, 16, 24),    # two column tiles, one row tile (4-row chunks)
    (450, 60, 8, 25),     # two column tiles, three row tiles, h = 30 (padded columns)
])
def test_fused_matches_oracle_and_staged(nr, nth, nphi, seed):
    print(f"[case] fused {nr}x{nth}x{nphi} seed {seed}", flush=True)
    r_if, th_if, rho = _case(nr, nth, nphi, seed)
    fused, staged = _both_paths(r_if, th_if, nphi, rho)
    ref = spectral.solve(r_if, th_if, nphi, rho)
    e, d = _err(fused, ref), _err(fused, staged)
    print(f"[parity] fused {nr}x{nth}x{nphi}: vs oracle {e:.3e}, vs staged {d:.3e}", flush=True)
    assert np.all(np.isfinite(fused))
    assert e <= TOL_FP64
    assert d <= TOL_FP64


def test_fused_white_noise_on_random_widths():
    """A stress input outside the paper's workloads: normal noise on 385
    random-width shells.  Its conditioning puts every FP64 method about 1e-12
    apart, so the check is the residual: the componentwise backward error
    max|s - L Phi| / (|L||Phi| + |s|) stays at the oracle's level, and both GPU
    paths agree."""
    nr, nth, nphi = 385, 128, 8
    rng, r_if, th_if = _grid(nr, nth, 16)
    rho = rng.standard_normal((nr, nth, nphi))
    fused, staged = _both_paths(r_if, th_if, nphi, rho)
    ref = spectral.solve(r_if, th_if, nphi, rho)
    eta_ref = laplacian.backward_error(r_if, th_if, nphi, ref, rho)
    eta = laplacian.backward_error(r_if, th_if, nphi, fused, rho)
    d = _err(fused, staged)
    print(f"[parity] white noise {nr}x{nth}x{nphi}: backward error {eta:.3e} (oracle {eta_ref:.3e}), "
          f"vs oracle {_err(fused, ref):.3e}, vs staged {d:.3e}", flush=True)
    assert eta <= max(4.0 * eta_ref, 1e-13)
    assert d <= TOL_FP64


def test_fused_extreme_radial_widths():
    """Shells ten times wider than their inner radius (r = 0, 1, 10, ..., 1e39)
    with a 128-cell theta grid: radial coefficients spanning 80 orders of
    magnitude, angular eigenvalues up to 2.8e6, and outer-boundary
    coefficients beta(lambda) that underflow to zero for the largest ones.
    The fused path's continuants stay in range here (the plan selects it);
    the source is the stellar profile on this grid."""
    nr, nth, nphi = 40, 128, 64
    r_if = np.concatenate(([0.0], 10.0 ** np.arange(0, nr, dtype=np.float64)))
    th_if = synthetic.theta_interfaces(nth)
    rho = synthetic.stellar_density(r_if, th_if, nphi, 21, r0=1e20)
    fused, staged = _both_paths(r_if, th_if, nphi, rho)
    ref = spectral.solve(r_if, th_if, nphi, rho)
    e, d = _err(fused, ref), _err(fused, staged)
    print(f"[parity] extreme widths {nr}x{nth}x{nphi}: vs oracle {e:.3e}, vs staged {d:.3e}", flush=True)
    assert np.all(np.isfinite(fused))
    assert e <= TOL_FP64
    assert d <= TOL_FP64


def test_path_selection_rules():
    import paper_1806_06623_amd as spp
    rng, r_if, th_if = _grid(16, 16, 1)
    # theta grid not symmetric about the equator: staged only
    th_ns = np.concatenate(([0.0], np.sort(rng.uniform(0.1, np.pi - 0.1, 15)), [np.pi]))
    p = spp.Plan(r_if, th_ns, 8)
    assert p.path == "staged"
    with pytest.raises(spp.SphPoissonError):
        p.path = "fused"
    # h = N_theta / 2 odd, and N_r above the fused range: staged
    assert spp.Plan(r_if, np.pi * np.arange(19) / 18, 8).path == "staged"
    _, r_big, _ = _grid(577, 4, 2)
    assert spp.Plan(r_big, th_if, 8).path == "staged"
    assert spp.Plan(r_if, th_if, 8).path == "fused"


def test_fused_profiled_stages():
    import paper_1806_06623_amd as spp
    rng, r_if, th_if = _grid(64, 32, 3)
    plan = spp.Plan(r_if, th_if, 64)
    x = torch.from_numpy(rng.standard_normal((64, 32, 64))).to("cuda")
    out = torch.empty_like(x)
    st = plan.solve_profiled(x, out)
    ref = plan.solve(x).cpu().numpy()
    assert np.array_equal(out.cpu().numpy(), ref)
    assert st[1] > 0 and st[2] < 0.05 and st[3] < 0.05
