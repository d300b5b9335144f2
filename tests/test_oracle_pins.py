"""Pins of the FP64 oracle to facts the paper and the mathematics fix.

None of these checks re-types the oracle's own formulas: each compares it with
something independent (a closed form, a worked example the paper prints, a
dense direct solve of the operator assembled from the flux form, an invariant
of the exact discrete problem).  ``test_planted_mistakes_are_caught`` shows
that plausible slips in the oracle fail at least one of them.
"""
import json
import os

import numpy as np
import pytest

from oracle import analytic, dense, fluxes, geometry, laplacian, momentum, spectral
import synthetic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def random_r_if(rng, nr, r0=0.0):
    return np.concatenate(([r0], r0 + np.cumsum(rng.uniform(0.4, 1.6, nr))))


def random_th_if(rng, nth):
    inner = np.sort(rng.uniform(0.15, np.pi - 0.15, nth - 1))
    return np.concatenate(([0.0], inner, [np.pi]))


# ---------------------------------------------------------------- geometry
def test_worked_example_cell_centres():
    """Sec. 5.1: zone (j, k) = (32, 128) of 128 x 256 sits at (0.246 pi, 0.996 pi)."""
    with open(os.path.join(GOLDEN, "point_source_zone.json")) as fh:
        g = json.load(fh)
    _, th, phi = geometry.cell_centres([0.0, 1.0], synthetic.theta_interfaces(g["nth"]), g["nphi"])
    assert round(th[g["j_one_based"] - 1] / np.pi, 3) == g["theta_over_pi"]
    assert round(phi[g["k_one_based"] - 1] / np.pi, 3) == g["phi_over_pi"]


def test_volumes_sum_to_ball():
    """Sum of delta V over all cells is the ball volume 4/3 pi r_out^3."""
    rng = np.random.default_rng(1)
    r_if = random_r_if(rng, 17)
    th_if = random_th_if(rng, 9)
    vol = geometry.cell_volumes(r_if, th_if, 12).sum() * 12
    assert abs(vol / (4.0 / 3.0 * np.pi * r_if[-1] ** 3) - 1.0) < 1e-14


def test_factored_coefficients_continuum_limits():
    """R_i -> 1/r_i^2 and S_j -> 1/sin^2 theta_j at second order in the spacing."""
    errs_r, errs_s = [], []
    for n in (64, 128, 256):
        g = geometry.grid_geometry(synthetic.uniform_interfaces(n, 1.0, 2.0),
                                   synthetic.theta_interfaces(n), 8)
        errs_r.append(np.max(np.abs(g["R"] * g["r"] ** 2 - 1.0)))
        errs_s.append(np.max(np.abs(g["S"] * np.sin(g["th"]) ** 2 - 1.0)[n // 4: 3 * n // 4]))
    for e in (errs_r, errs_s):
        assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5


# ------------------------------------------------------------ eigensystems
def test_phi_eigenvalues_match_circulant_spectrum():
    """lambda_{phi,m} are the eigenvalues of the periodic second difference / dphi^2."""
    for n in (6, 7, 16):
        dphi = 2 * np.pi / n
        C = (np.roll(np.eye(n), 1, 1) + np.roll(np.eye(n), -1, 1) - 2 * np.eye(n)) / dphi ** 2
        ev = np.sort(np.linalg.eigvalsh(C))
        lam = spectral.phi_eigenvalues(n)
        full = np.concatenate((lam, lam[1:(n + 1) // 2]))     # m and N - m
        assert np.allclose(np.sort(full), ev, rtol=0, atol=1e-12 * np.abs(ev).max())


@pytest.mark.parametrize("m", [0, 1, 5, 40, 128])
def test_theta_eigensystem_orthonormal_and_exact(m):
    """H^T D H = I and K H = D H Lambda to rounding, for uniform 128-zone theta."""
    g = geometry.grid_geometry([0.0, 1.0], synthetic.theta_interfaces(128), 256)
    lam, H = spectral.theta_eigensystem(g, m)
    D = g["dmu"]
    assert np.max(np.abs(H.T @ (D[:, None] * H) - np.eye(128))) < 1e-13
    # K assembled here from the flux form on the unit sphere, not from the oracle
    A, omega = dense.shell_angular_operator(synthetic.theta_interfaces(128), 256)
    # restrict A to the m-th Fourier mode: apply to H_l(j) cos(m phi_k)
    phi = (np.arange(256) + 0.5) * 2 * np.pi / 256
    for l in (0, 7, 127):
        v = np.outer(H[:, l], np.cos(m * phi)).reshape(-1)
        Av = A @ v
        assert np.max(np.abs(Av - lam[l] * v)) < 1e-10 * np.max(np.abs(lam))


def test_theta_eigenvalues_continuum_limit():
    """lambda_Omega -> -(m + k)(m + k + 1) (Y_lm eigenvalues) at second order."""
    errs = []
    for n in (32, 64, 128):
        g = geometry.grid_geometry([0.0, 1.0], synthetic.theta_interfaces(n), 2 * n)
        e = []
        for m in (0, 1, 3):
            lam = np.sort(spectral.theta_eigensystem(g, m)[0])[::-1]
            exact = np.array([-(m + k) * (m + k + 1) for k in range(4)])
            if m == 0:
                assert abs(lam[0]) < 1e-11 * abs(lam).max()   # constant mode, exactly 0
                lam, exact = lam[1:4], exact[1:4]
            else:
                lam, exact = lam[:4], exact
            e.append(np.max(np.abs(lam / exact - 1.0)))
        errs.append(max(e))
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


# ------------------------------------------------------ whole-method pins
CASES = [
    # (nr, nth, nphi, r0, uniform_theta)
    (5, 4, 6, 0.0, True),
    (6, 6, 8, 0.0, True),
    (4, 5, 5, 0.7, False),
    (7, 3, 4, 0.0, False),
    (3, 6, 7, 2.0, True),
]


@pytest.mark.parametrize("driver", ["stev", "stemr"])
@pytest.mark.parametrize("nr,nth,nphi,r0,uni", CASES)
def test_spectral_matches_dense_brute_force(nr, nth, nphi, r0, uni, driver):
    """The spectral method reaches the unique solution of the dense system,
    with either of the oracle's two LAPACK eigensolvers."""
    rng = np.random.default_rng(nr * 100 + nth * 10 + nphi)
    r_if = random_r_if(rng, nr, r0)
    th_if = synthetic.theta_interfaces(nth) if uni else random_th_if(rng, nth)
    rho = rng.standard_normal((nr, nth, nphi))
    ref = dense.solve(r_if, th_if, nphi, rho)
    got = spectral.solve(r_if, th_if, nphi, rho, driver=driver)
    assert rel(got, ref) < 1e-13


@pytest.mark.parametrize("nr,nth,nphi,r0,uni", [c for c in CASES if c[3] > 0] + [(5, 4, 6, 0.3, False)])
def test_regular_inner_condition_matches_dense_brute_force(nr, nth, nphi, r0, uni):
    """With r_{1/2} > 0 and the regular inner condition, the spectral method
    (gamma(lambda) per eigenmode on the innermost row) reaches the solution of
    the dense system whose inner face is a matrix function of the directly
    assembled shell operator; and it differs from the zero-flux solution."""
    rng = np.random.default_rng(nr * 100 + nth * 10 + nphi + 3)
    r_if = random_r_if(rng, nr, r0)
    th_if = synthetic.theta_interfaces(nth) if uni else random_th_if(rng, nth)
    rho = rng.standard_normal((nr, nth, nphi))
    ref = dense.solve(r_if, th_if, nphi, rho, inner="regular")
    assert rel(spectral.solve(r_if, th_if, nphi, rho, inner="regular"), ref) < 1e-13
    assert rel(spectral.solve(r_if, th_if, nphi, rho), ref) > 1e-3


def test_regular_inner_condition_converges_to_free_space_potential():
    """A Gaussian mass (sigma = 0.18 at r = 0.95) on a grid with a hole
    r < 0.4: the continuum potential inside the source-free hole is the
    regular (finite-at-centre) solution, so with the regular inner condition
    the discrete potential converges at second order to the free-space
    potential -G M erf(d / (sqrt 2 sigma)) / d; with zero flux through the
    inner face it does not converge."""
    from scipy.special import erf

    def err(n, inner):
        r_if = synthetic.uniform_interfaces(3 * n, 0.4, 2.0)
        th_if, nphi = synthetic.theta_interfaces(n), 2 * n
        sig, c = 0.18, (0.95, np.pi / 2, np.pi)
        rho = synthetic.gaussian_blob(r_if, th_if, nphi, c, sig)
        phi = spectral.solve(r_if, th_if, nphi, rho, inner=inner)
        r, th, ph = geometry.cell_centres(r_if, th_if, nphi)
        R, T, P = np.meshgrid(r, th, ph, indexing="ij")
        cart = lambda a, b, e: np.array([a * np.sin(b) * np.cos(e), a * np.sin(b) * np.sin(e), a * np.cos(b)])
        d = np.linalg.norm(cart(R, T, P) - cart(*c)[:, None, None, None], axis=0)
        exact = -(2 * np.pi * sig ** 2) ** 1.5 * erf(d / (np.sqrt(2) * sig)) / d
        return float(np.max(np.abs(phi - exact)) / np.max(np.abs(exact)))

    reg = [err(n, "regular") for n in (16, 32, 64)]
    assert reg[2] < 3e-3
    assert 3.0 < reg[0] / reg[1] < 4.5 and 3.5 < reg[1] / reg[2] < 4.5
    zf = [err(n, "zero_flux") for n in (16, 64)]
    assert zf[1] > 0.05 and zf[1] > 0.5 * zf[0]


def test_regular_inner_pin_catches_planted_mistakes(monkeypatch):
    """Slips in the inner-face coefficient fail the dense pin."""
    rng = np.random.default_rng(99)
    r_if, th_if, nphi = random_r_if(rng, 4, 0.6), random_th_if(rng, 4), 5
    rho = rng.standard_normal((4, 4, nphi))
    ref = dense.solve(r_if, th_if, nphi, rho, inner="regular")
    ok = lambda: rel(spectral.solve(r_if, th_if, nphi, rho, inner="regular"), ref) < 1e-13
    assert ok()
    orig = spectral.inner_gamma
    for slip in (lambda g, lam, inner="zero_flux": -orig(g, lam, inner),
                 lambda g, lam, inner="zero_flux": orig(g, lam, inner) * g["r"][0] / g["r_if"][0],
                 lambda g, lam, inner="zero_flux": orig(g, 2.0 * np.asarray(lam), inner)):
        monkeypatch.setattr(spectral, "inner_gamma", slip)
        assert not ok()
        monkeypatch.undo()
    assert ok()


def test_dense_operator_is_volume_symmetric():
    """delta V * L is symmetric: the flux form is self-adjoint (reciprocity)."""
    rng = np.random.default_rng(7)
    r_if, th_if, nphi = random_r_if(rng, 4), random_th_if(rng, 4), 5
    L = dense.assemble(r_if, th_if, nphi)
    dV = np.repeat(geometry.cell_volumes(r_if, th_if, nphi).reshape(-1), nphi)
    S = dV[:, None] * L
    assert np.max(np.abs(S - S.T)) < 1e-13 * np.max(np.abs(S))


def test_reciprocity_of_spectral_solutions():
    """Phi of a unit mass at b, read at a, equals Phi of a unit mass at a, read at b."""
    rng = np.random.default_rng(11)
    r_if, th_if, nphi = random_r_if(rng, 8), synthetic.theta_interfaces(6), 8
    dV = geometry.cell_volumes(r_if, th_if, nphi)
    plan = spectral.Plan(r_if, th_if, nphi)
    a, b = (1, 2, 3), (6, 4, 0)
    ra = np.zeros((8, 6, nphi)); ra[a] = 1.0 / dV[a[:2]]
    rb = np.zeros((8, 6, nphi)); rb[b] = 1.0 / dV[b[:2]]
    pa, pb = plan.solve(ra), plan.solve(rb)
    assert abs(pa[b] - pb[a]) < 1e-13 * abs(pa[b])


@pytest.mark.parametrize("nr,nth,nphi", [(128, 16, 16), (385, 128, 8)])
def test_spherical_source_closed_form(nr, nth, nphi):
    """A spherically symmetric source excites only l = m = 0: discrete Gauss's
    law.  At N_theta = 128 a computed (not exact) m = 0 null eigenvector is off
    by about 1e-12 and fails this bar."""
    r_if = synthetic.stellar_r_interfaces(nr)
    th_if = synthetic.theta_interfaces(nth)
    r = 0.5 * (r_if[:-1] + r_if[1:])
    rho_r = (1 + (r / 20.0) ** 2) ** -1.5
    rho = np.broadcast_to(rho_r[:, None, None], (nr, nth, nphi)).copy()
    phi = spectral.solve(r_if, th_if, nphi, rho)
    f = analytic.spherical_discrete_potential(r_if, 4 * np.pi * rho_r)
    assert rel(phi, np.broadcast_to(f[:, None, None], phi.shape)) < 1e-13
    spread = np.max(phi.max(axis=(1, 2)) - phi.min(axis=(1, 2)))
    assert spread < 1e-13 * np.max(np.abs(phi))


def test_uniform_sphere_second_order():
    """Homogeneous sphere: the discrete solution converges to the Newtonian
    potential at second order in the radial spacing."""
    errs = []
    for nr in (32, 64, 128):
        r_if = synthetic.uniform_interfaces(nr, 0.0, 1.0)
        th_if = synthetic.theta_interfaces(8)
        r = 0.5 * (r_if[:-1] + r_if[1:])
        rho = np.broadcast_to((r < 0.5)[:, None, None].astype(float), (nr, 8, 8)).copy()
        phi = spectral.solve(r_if, th_if, 8, rho)
        ex = analytic.uniform_sphere_potential(r, 0.5)
        errs.append(np.max(np.abs(phi[:, 0, 0] - ex)) / np.max(np.abs(ex)))
    assert errs[0] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


@pytest.mark.parametrize("inner", ["zero_flux", "regular"])
@pytest.mark.parametrize("nr,nth,nphi,r0,uni", CASES)
def test_stencil_and_backward_error_denominator_match_dense_operator(nr, nth, nphi, r0, uni, inner):
    """laplacian.apply against the operator assembled cell by cell (dense):
    L Phi = (L_local + L_outer) Phi, and the denominator of the componentwise
    backward error is |L_local| |Phi| + |L_outer Phi| (the nonlocal outer-face
    term enters as one term, its value's magnitude) -- on random fields,
    including the outer shell, offset inner radii and non-uniform theta."""
    rng = np.random.default_rng(nr * 100 + nth * 10 + nphi + 7)
    r_if = random_r_if(rng, nr, r0)
    th_if = synthetic.theta_interfaces(nth) if uni else random_th_if(rng, nth)
    P = rng.standard_normal((nr, nth, nphi))
    Lloc, Lout = dense.assemble_parts(r_if, th_if, nphi, inner)
    x = P.reshape(-1)
    LP, mag = laplacian.apply(r_if, th_if, nphi, P, with_terms=True, inner=inner)
    want_mag = np.abs(Lloc) @ np.abs(x) + np.abs(Lout @ x)
    assert np.max(np.abs(LP.reshape(-1) - (Lloc + Lout) @ x)) < 1e-13 * np.max(want_mag)
    assert np.max(np.abs(mag.reshape(-1) - want_mag) / want_mag) < 1e-13
    # the outer shell's denominator carries the boundary term: it differs
    # from the local part alone
    outer = slice((nr - 1) * nth * nphi, None)
    assert np.max(np.abs(Lout @ x)[outer]) > 1e-3 * np.max(want_mag[outer])


def test_backward_error_denominator_pin_catches_slips(monkeypatch):
    """A slip in the outer-face term of laplacian (mirrored shell, or the
    term dropped from the denominator) fails the dense pin above."""
    rng = np.random.default_rng(17)
    nr, nth, nphi = 4, 5, 6
    r_if, th_if = random_r_if(rng, nr), random_th_if(rng, nth)
    P = rng.standard_normal((nr, nth, nphi))
    Lloc, Lout = dense.assemble_parts(r_if, th_if, nphi)
    x = P.reshape(-1)
    want_mag = np.abs(Lloc) @ np.abs(x) + np.abs(Lout @ x)

    def ok():
        LP, mag = laplacian.apply(r_if, th_if, nphi, P, with_terms=True)
        return (np.max(np.abs(LP.reshape(-1) - (Lloc + Lout) @ x)) < 1e-13 * np.max(want_mag)
                and np.max(np.abs(mag.reshape(-1) - want_mag) / want_mag) < 1e-13)

    assert ok()
    orig = laplacian.outer_flux
    for slip in (lambda g, s: orig(g, s[:, ::-1]), lambda g, s: 2.0 * orig(g, s)):
        monkeypatch.setattr(laplacian, "outer_flux", slip)
        assert not ok()
        monkeypatch.undo()
    assert ok()


def test_componentwise_backward_error_at_roundoff():
    """|s - L Phi| is at rounding level of |L||Phi| + |s| on a stellar grid."""
    c = synthetic.stellar_case(nr=96, nth=32, nphi=32, seed=5)
    phi = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"])
    eta = laplacian.backward_error(c["r_if"], c["th_if"], c["nphi"], phi, c["rho"])
    assert eta < 1e-14


def test_shift_and_reflection_equivariance():
    """Rolling rho in phi rolls Phi; mirroring rho in theta mirrors Phi."""
    rng = np.random.default_rng(3)
    r_if, th_if, nphi = random_r_if(rng, 12), synthetic.theta_interfaces(10), 12
    rho = rng.standard_normal((12, 10, nphi))
    plan = spectral.Plan(r_if, th_if, nphi)
    phi = plan.solve(rho)
    assert rel(plan.solve(np.roll(rho, 3, axis=2)), np.roll(phi, 3, axis=2)) < 1e-13
    assert rel(plan.solve(rho[:, ::-1, :]), phi[:, ::-1, :]) < 1e-12


# ------------------------------------------------------------ face fluxes
def _cell_balance_by_loops(r_if, th_if, nphi, Fr, Ft, Fp):
    """Net outward flux of every cell, summed face by face (brute force)."""
    nr, nth = len(r_if) - 1, len(th_if) - 1
    out = np.zeros((nr, nth, nphi))
    for i in range(nr):
        for j in range(nth):
            for k in range(nphi):
                v = Fr[i, j, k] + Ft[i, j, k] + Fp[i, j, k]      # outer r, theta, phi faces
                if i > 0:
                    v -= Fr[i - 1, j, k]
                if j > 0:
                    v -= Ft[i, j - 1, k]
                v -= Fp[i, j, (k - 1) % nphi]
                out[i, j, k] = v
    return out


def _cell_volumes_full(r_if, th_if, nphi):
    r_if, th_if = np.asarray(r_if), np.asarray(th_if)
    v = np.outer((r_if[1:] ** 3 - r_if[:-1] ** 3) / 3.0, np.cos(th_if[:-1]) - np.cos(th_if[1:]))
    return v[:, :, None] * (2.0 * np.pi / nphi)


@pytest.mark.parametrize("nr,nth,nphi,r0,uni", CASES)
def test_face_fluxes_gauss_law_per_cell(nr, nth, nphi, r0, uni):
    """For the exact discrete solution (dense direct solve of the operator
    assembled from the flux form), the six face fluxes of every cell add up
    to 4 pi G rho delta V (Gauss's law on the grid)."""
    rng = np.random.default_rng(nr * 100 + nth * 10 + nphi + 1)
    r_if = random_r_if(rng, nr, r0)
    th_if = synthetic.theta_interfaces(nth) if uni else random_th_if(rng, nth)
    rho = rng.standard_normal((nr, nth, nphi))
    G = 0.7
    phi = dense.solve(r_if, th_if, nphi, rho, G=G)
    Fr, Ft, Fp = fluxes.face_fluxes(r_if, th_if, nphi, phi)
    src = 4.0 * np.pi * G * rho * _cell_volumes_full(r_if, th_if, nphi)
    bal = _cell_balance_by_loops(r_if, th_if, nphi, Fr, Ft, Fp)
    assert np.max(np.abs(bal - src)) < 1e-12 * np.max(np.abs(src))
    assert np.max(np.abs(fluxes.net_outward_flux(Fr, Ft, Fp) - bal)) < 1e-14 * np.max(np.abs(src))
    assert np.all(Ft[:, -1, :] == 0.0)           # pole face theta = pi


def test_face_fluxes_spherical_closed_form():
    """A spherically symmetric source: the radial flux through the sphere
    r_{i+1/2}, per unit of dmu dphi, is 4 pi G times the enclosed mass over
    4 pi (the enclosed mass sum_{i' <= i} rho_{i'} 4 pi (r_+^3 - r_-^3)/3);
    the outer face carries the total; theta and phi fluxes vanish."""
    nr, nth, nphi, G = 128, 16, 8, 1.3
    r_if = synthetic.stellar_r_interfaces(nr)
    th_if = synthetic.theta_interfaces(nth)
    r = 0.5 * (r_if[:-1] + r_if[1:])
    rho_r = (1 + (r / 20.0) ** 2) ** -1.5
    phi_r = analytic.spherical_discrete_potential(r_if, 4 * np.pi * G * rho_r)
    phi = np.broadcast_to(phi_r[:, None, None], (nr, nth, nphi)).copy()
    Fr, Ft, Fp = fluxes.face_fluxes(r_if, th_if, nphi, phi)
    m_enc = np.cumsum(rho_r * 4.0 * np.pi * (r_if[1:] ** 3 - r_if[:-1] ** 3) / 3.0)
    dmu = np.cos(th_if[:-1]) - np.cos(th_if[1:])
    want = G * m_enc[:, None, None] * dmu[None, :, None] * (2.0 * np.pi / nphi) * np.ones((1, 1, nphi))
    assert rel(Fr, want) < 1e-12
    assert np.max(np.abs(Ft)) == 0.0 and np.max(np.abs(Fp)) == 0.0


def test_face_fluxes_total_outer_flux_is_enclosed_mass():
    """Off-centre source on a stellar grid: the outer-face fluxes sum to
    4 pi G M (global Gauss's law), and every cell balances."""
    c = synthetic.stellar_case(nr=96, nth=32, nphi=32, seed=5)
    G = 1.0
    phi = spectral.solve(c["r_if"], c["th_if"], c["nphi"], c["rho"], G=G)
    Fr, Ft, Fp = fluxes.face_fluxes(c["r_if"], c["th_if"], c["nphi"], phi)
    dV = _cell_volumes_full(c["r_if"], c["th_if"], c["nphi"])
    mass = float(np.sum(c["rho"] * dV))
    assert abs(Fr[-1].sum() - 4.0 * np.pi * G * mass) < 1e-12 * 4.0 * np.pi * G * mass
    src = 4.0 * np.pi * G * c["rho"] * dV
    bal = fluxes.net_outward_flux(Fr, Ft, Fp)
    # per cell, on the scale of the componentwise backward error:
    # |L| |Phi| delta V + |s| delta V
    _, mag = laplacian.apply(c["r_if"], c["th_if"], c["nphi"], phi, with_terms=True)
    assert np.max(np.abs(bal - src) / (mag * dV + np.abs(src))) < 1e-13


def test_face_fluxes_constant_potential():
    """Phi = c: no flux through interior faces; the constant is the exact
    (l, m) = (0, 0) eigenmode (lambda = 0, exponent p = 1), so the outer face
    carries -c r_N dmu_j dphi with r_N the outermost cell centre."""
    rng = np.random.default_rng(21)
    r_if, th_if, nphi, c = random_r_if(rng, 6, 1.0), random_th_if(rng, 8), 12, -2.5
    Fr, Ft, Fp = fluxes.face_fluxes(r_if, th_if, nphi, np.full((6, 8, nphi), c))
    rN = 0.5 * (r_if[-2] + r_if[-1])
    dmu = np.cos(th_if[:-1]) - np.cos(th_if[1:])
    want = -c * rN * dmu[:, None] * (2.0 * np.pi / nphi) * np.ones((1, nphi))
    assert np.all(Fr[:-1] == 0.0) and np.all(Ft == 0.0) and np.all(Fp == 0.0)
    assert rel(Fr[-1], want) < 1e-13


def test_face_flux_pins_catch_planted_mistakes(monkeypatch):
    """Slips in the outer-face term fail the Gauss-law pin."""
    rng = np.random.default_rng(5)
    r_if, th_if, nphi = random_r_if(rng, 5), random_th_if(rng, 4), 6
    rho = rng.standard_normal((5, 4, nphi))
    phi = dense.solve(r_if, th_if, nphi, rho)
    src = 4.0 * np.pi * rho * _cell_volumes_full(r_if, th_if, nphi)

    def ok():
        F = fluxes.face_fluxes(r_if, th_if, nphi, phi)
        return np.max(np.abs(_cell_balance_by_loops(r_if, th_if, nphi, *F) - src)) < 1e-12 * np.max(np.abs(src))

    assert ok()
    orig = fluxes.outer_flux
    for slip in (lambda g, s: -orig(g, s), lambda g, s: orig(g, s) * g["r"][-1] / g["r_if"][-1],
                 lambda g, s: orig(g, s[:, ::-1])):
        monkeypatch.setattr(fluxes, "outer_flux", slip)
        assert not ok()
        monkeypatch.undo()
    assert ok()


# --------------------------------------------------- sensitivity of the pins
def _pins_pass():
    rng = np.random.default_rng(123)
    r_if, th_if, nphi = random_r_if(rng, 5), random_th_if(rng, 4), 6
    rho = rng.standard_normal((5, 4, nphi))
    with np.errstate(invalid="ignore"):
        try:
            got = spectral.solve(r_if, th_if, nphi, rho)
        except ValueError:        # a slip that produces NaN is caught too
            return False
    return rel(got, dense.solve(r_if, th_if, nphi, rho)) < 1e-13


def test_planted_mistakes_are_caught(monkeypatch):
    """Each plausible slip in the oracle breaks the dense-solve pin."""
    assert _pins_pass()
    orig_beta, orig_phi = spectral.outer_beta, spectral.phi_eigenvalues
    orig_op, orig_geom = spectral.theta_operator, spectral.grid_geometry

    slips = {
        "lambda_phi sign dropped": ("phi_eigenvalues", lambda n: -orig_phi(n)),
        "outer exponent dropped": ("outer_beta", lambda g, lam: orig_beta(g, lam) * (g["r_if"][-1] / g["r"][-1]) ** (
            0.5 * (1 + np.sqrt(1 - 4 * np.asarray(lam))))),
        "outer face at cell centre": ("outer_beta", lambda g, lam: orig_beta(g, lam) * g["r"][-1] / g["r_if"][-1]),
        "1/dmu dropped in theta operator": ("theta_operator", lambda g, lp: (
            orig_op(g, lp)[0] / g["dmu"], orig_op(g, lp)[1])),
        "R_i taken as 1/r_i^2": ("grid_geometry", lambda *a: dict(orig_geom(*a), R=1.0 / orig_geom(*a)["r"] ** 2)),
    }
    for name, (attr, fn) in slips.items():
        monkeypatch.setattr(spectral, attr, fn)
        assert not _pins_pass(), name
        monkeypatch.undo()
    assert _pins_pass()


# ------------------------------------------------- paper-printed results
def test_displaced_point_source_adjacent_error():
    """Sec. 5.1: a unit-density zone on the 550 x 128 x 256 log grid; the
    discrete potential stays within the printed 10% of -G m / |x - x_s| in
    all 26 zones adjacent to the source and close to it far away."""
    with open(os.path.join(GOLDEN, "displaced_point_source.json")) as fh:
        g = json.load(fh)
    nr, nth, nphi = g["nr"], g["nth"], g["nphi"]
    i, j, k = (v - 1 for v in g["zone_one_based"])
    q = np.exp(0.01976)
    r0 = g["r_source"] / (0.5 * (q ** i + q ** (i + 1)))
    r_if = r0 * q ** np.arange(nr + 1)
    th_if = synthetic.theta_interfaces(nth)
    geo = geometry.grid_geometry(r_if, th_if, nphi)
    mass = geo["V"][i] * geo["dmu"][j] * geo["dphi"]
    assert abs(mass / g["mass"] - 1.0) < 1e-3
    rho = np.zeros((nr, nth, nphi))
    rho[i, j, k] = 1.0
    phi = spectral.solve(r_if, th_if, nphi, rho)

    def cart(ii, jj, kk):
        r, th, ph = geo["r"][ii], geo["th"][jj], geo["phi"][kk % nphi]
        return np.array([r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)])

    xs = cart(i, j, k)
    worst = 0.0
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for dk in (-1, 0, 1):
                if di == dj == dk == 0:
                    continue
                ana = -mass / np.linalg.norm(cart(i + di, j + dj, k + dk) - xs)
                worst = max(worst, abs(phi[i + di, j + dj, (k + dk) % nphi] / ana - 1.0))
    assert worst <= g["max_rel_err_adjacent"]
    assert worst > 0.01        # the source zone is resolved by one cell only
    # twenty cells away along the radial line through the source: close agreement
    far = -mass / np.linalg.norm(cart(i + 20, j, k) - xs)
    assert abs(phi[i + 20, j, k] / far - 1.0) < 2e-3


def _ellipsoid_error(r_if, nth, nphi, axes):
    th_if = synthetic.theta_interfaces(nth)
    rho = synthetic.ellipsoid_density(r_if, th_if, nphi, axes)
    phi = spectral.solve(r_if, th_if, nphi, rho)
    r, th, ph = geometry.cell_centres(r_if, th_if, nphi)
    R, TH, PH = np.meshgrid(r, th, ph, indexing="ij")
    st = np.sin(TH)
    exact = analytic.ellipsoid_potential(R * st * np.cos(PH), R * st * np.sin(PH), R * np.cos(TH), *axes)
    return float(np.max(np.abs(phi - exact) / np.abs(exact)))


def test_ellipsoid_accuracy_matches_paper():
    """Sec. 5.2: second-order convergence at N_r : N_theta : N_phi = 4 : 1 : 2 and
    the printed maximum relative error 3.2e-5 at 512 x 128 x 256 (within 30%)."""
    with open(os.path.join(GOLDEN, "ellipsoid_convergence.json")) as fh:
        g = json.load(fh)
    axes = tuple(g["axes"])
    e1 = _ellipsoid_error(synthetic.uniform_interfaces(128, 0.0, g["r_out"]), 32, 64, axes)
    e2 = _ellipsoid_error(synthetic.uniform_interfaces(256, 0.0, g["r_out"]), 64, 128, axes)
    assert 3.0 < e1 / e2 < 4.5
    nr, nth, nphi = g["grid"]
    e3 = _ellipsoid_error(synthetic.uniform_interfaces(nr, 0.0, g["r_out"]), nth, nphi, axes)
    assert abs(e3 / g["max_rel_err"] - 1.0) <= g["tolerance_fraction"], e3


def test_ellipsoid_radial_jump_matches_paper():
    """Sec. 5.2: 50% larger radial spacing outside r = 1.5 -> 3.6e-5 (within 30%)."""
    with open(os.path.join(GOLDEN, "ellipsoid_convergence.json")) as fh:
        g = json.load(fh)
    nr, nth, nphi = g["grid"]
    dr = g["r_out"] / nr
    i15 = int(round(1.5 / dr))
    base = dr * np.arange(i15 + 1)
    r_if = np.concatenate((base, base[-1] + 1.5 * dr * np.arange(1, nr - i15 + 1)))
    e = _ellipsoid_error(r_if, nth, nphi, tuple(g["axes"]))
    assert abs(e / g["max_rel_err_jump_at_1p5"] - 1.0) <= g["tolerance_fraction"], e


# ------------------------------------------------------ momentum source
def _unit_vectors(th, ph):
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    return (np.stack([st * cp, st * sp, ct], -1), np.stack([ct * cp, ct * sp, -st], -1),
            np.stack([-sp, cp, 0.0 * st], -1))


def test_momentum_face_integrals_match_quadrature():
    """The exact face integrals of e_r, e_theta, e_phi against a 24 x 24
    Gauss-Legendre rule over each curved face (brute force, no closed form)."""
    rng = np.random.default_rng(8)
    r_if, th_if, nphi = random_r_if(rng, 3, 0.5), random_th_if(rng, 4), 5
    fv = momentum._face_vectors(r_if, th_if, nphi)
    x, w = np.polynomial.legendre.leggauss(24)
    ph_if = 2 * np.pi * np.arange(nphi + 1) / nphi

    def quad(lo1, hi1, lo2, hi2, f):
        u = 0.5 * (hi1 + lo1) + 0.5 * (hi1 - lo1) * x
        v = 0.5 * (hi2 + lo2) + 0.5 * (hi2 - lo2) * x
        U, Vv = np.meshgrid(u, v, indexing="ij")
        W = np.outer(w, w) * 0.25 * (hi1 - lo1) * (hi2 - lo2)
        return np.einsum("ab,abc->c", W, f(U, Vv))

    i, j, k = 2, 1, 3
    R = r_if[i]                                   # r-face i - 1/2, column (j, k)
    er = quad(th_if[j], th_if[j + 1], ph_if[k], ph_if[k + 1],
              lambda t, p: _unit_vectors(t, p)[0] * (R * R * np.sin(t))[..., None])
    et = quad(th_if[j], th_if[j + 1], ph_if[k], ph_if[k + 1],
              lambda t, p: _unit_vectors(t, p)[1] * (R * R * np.sin(t))[..., None])
    ep = quad(th_if[j], th_if[j + 1], ph_if[k], ph_if[k + 1],
              lambda t, p: _unit_vectors(t, p)[2] * (R * R * np.sin(t))[..., None])
    for got, want in ((fv["r"]["N"][i, j, k], er), (fv["r"]["T1"][i, j, k], et), (fv["r"]["T2"][i, j, k], ep)):
        assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))
    TH = th_if[j]                                 # theta-face j - 1/2, row i, column k
    f = lambda idx: quad(r_if[i], r_if[i + 1], ph_if[k], ph_if[k + 1],
                         lambda r, p: _unit_vectors(TH + 0 * r, p)[idx] * (r * np.sin(TH))[..., None])
    for got, idx in ((fv["t"]["N"][i, j, k], 1), (fv["t"]["T1"][i, j, k], 0), (fv["t"]["T2"][i, j, k], 2)):
        want = f(idx)
        assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))
    PH = ph_if[k + 1]                             # phi-face k + 1/2, row i, column j
    g = lambda idx: quad(r_if[i], r_if[i + 1], th_if[j], th_if[j + 1],
                         lambda r, t: _unit_vectors(t, PH + 0 * t)[idx] * r[..., None])
    for got, idx in ((fv["p"]["N"][i, j, k], 2), (fv["p"]["T1"][i, j, k], 0), (fv["p"]["T2"][i, j, k], 1)):
        want = g(idx)
        assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


def test_momentum_cell_surfaces_close_and_interior_faces_cancel():
    """Each cell's six integrated normals sum to zero (a closed surface), and
    for any field the cell forces add up to the boundary faces' terms alone:
    interior faces cancel (total momentum conserved to rounding)."""
    rng = np.random.default_rng(9)
    r_if, th_if, nphi = random_r_if(rng, 5, 0.4), random_th_if(rng, 6), 8
    fv = momentum._face_vectors(r_if, th_if, nphi)
    N = fv
    close = ((N["r"]["N"][1:] - N["r"]["N"][:-1]) + (N["t"]["N"][:, 1:] - N["t"]["N"][:, :-1])
             + (N["p"]["N"] - np.roll(N["p"]["N"], 1, axis=2)))
    assert np.max(np.abs(close)) < 1e-14 * np.max(np.abs(N["r"]["N"]))
    P = rng.standard_normal((5, 6, nphi))
    F, Sr = momentum.cell_forces(r_if, th_if, nphi, P, G=0.8)
    total = F.sum(axis=(0, 1, 2))
    boundary = -(Sr[-1].sum(axis=(0, 1)) - Sr[0].sum(axis=(0, 1)))
    assert np.max(np.abs(total - boundary)) < 1e-14 * np.abs(F).sum()


def test_momentum_spherical_source_has_zero_net_force_and_radial_cell_forces():
    """A spherically symmetric Phi (the discrete Gauss-law solution): every
    shell's forces sum to zero and each cell's force is along the integral of
    e_r over its solid angle, pointing inwards."""
    nr, nth, nphi = 48, 12, 16
    r_if, th_if = synthetic.stellar_r_interfaces(nr), synthetic.skewed_theta(nth)
    r = 0.5 * (r_if[:-1] + r_if[1:])
    rho_r = (1 + (r / 20.0) ** 2) ** -1.5
    phi = np.broadcast_to(analytic.spherical_discrete_potential(r_if, 4 * np.pi * rho_r)[:, None, None],
                          (nr, nth, nphi)).copy()
    F, _ = momentum.cell_forces(r_if, th_if, nphi, phi)
    scale = np.abs(F).max()
    assert np.max(np.abs(F.sum(axis=(1, 2)))) < 1e-13 * scale * nth * nphi
    dirs = momentum._face_vectors(r_if, th_if, nphi)["r"]["N"][-1]     # int e_r over the outer sphere's cells
    dirs = dirs / np.linalg.norm(dirs, axis=-1, keepdims=True)
    along = np.einsum("ijkc,jkc->ijk", F, dirs)
    perp = F - along[..., None] * dirs[None]
    assert np.max(np.abs(perp)) < 1e-12 * scale
    assert np.all(along < 0)


def _momentum_convergence(n):
    from scipy.special import erf
    nr, nth, nphi = 2 * n, n, 2 * n
    r_if, th_if = synthetic.uniform_interfaces(nr, 0.0, 2.0), synthetic.theta_interfaces(nth)
    sig, c = 0.2, (0.6, np.pi / 2, np.pi)
    rho = synthetic.gaussian_blob(r_if, th_if, nphi, c, sig)
    phi = spectral.solve(r_if, th_if, nphi, rho)
    F, _ = momentum.cell_forces(r_if, th_if, nphi, phi)
    r, t, p = geometry.cell_centres(r_if, th_if, nphi)
    R, T, Pp = np.meshgrid(r, t, p, indexing="ij")
    X = np.stack([R * np.sin(T) * np.cos(Pp), R * np.sin(T) * np.sin(Pp), R * np.cos(T)], -1)
    C = np.array([c[0] * np.sin(c[1]) * np.cos(c[2]), c[0] * np.sin(c[1]) * np.sin(c[2]), c[0] * np.cos(c[1])])
    D = X - C
    d = np.linalg.norm(D, axis=-1)
    u = d / (np.sqrt(2) * sig)
    dphidd = (2 * np.pi * sig ** 2) ** 1.5 * (erf(u) / d ** 2 - np.sqrt(2 / np.pi) / sig * np.exp(-u * u) / d)
    grad = dphidd[..., None] * D / d[..., None]          # gradient of -G M erf(u) / d (G = 1)
    dV = geometry.cell_volumes(r_if, th_if, nphi)[:, :, None] * np.ones(nphi)
    want = -(rho * dV)[..., None] * grad
    return float(np.max(np.abs(F - want)) / np.max(np.abs(want)))


def test_momentum_source_converges_to_minus_rho_grad_phi():
    """The cell forces of the exact discrete potential of a Gaussian mass
    converge at second order to -rho grad Phi delta V of the continuum
    potential -G M erf(d / (sqrt 2 sigma)) / d."""
    e = [_momentum_convergence(n) for n in (16, 32, 64)]
    assert e[2] < 5e-3
    assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5


def test_momentum_pins_catch_planted_mistakes(monkeypatch):
    """Slips in the stress vector or the face integrals fail the pins above:
    the sign of the shear terms, the factor 1/2, and a face's integrated
    normal off by 1 %."""
    orig_vec = momentum._face_vectors

    def scaled_normals(r_if, th_if, nphi):      # the r-faces' integrated normals off by 1 %
        out = orig_vec(r_if, th_if, nphi)
        out["r"]["N"] = out["r"]["N"] * 1.01
        return out

    assert _momentum_convergence(16) < 0.06
    for slip in ("shear", "half"):
        def bad(r_if, th_if, nphi, Phi, G=1.0, _slip=slip):
            gr, gt, gp = momentum.face_gradients(r_if, th_if, nphi, Phi)
            sign = -1.0 if _slip == "shear" else 1.0
            half = 1.0 if _slip == "half" else 0.5
            cr = 0.5 * (gr[:-1] + gr[1:])
            ct = 0.5 * (gt[:, :-1] + gt[:, 1:])
            cp = 0.5 * (gp + np.roll(gp, 1, axis=2))

            def pad_mean(x, axis):
                x0, x1 = np.take(x, [0], axis=axis), np.take(x, [-1], axis=axis)
                mid = 0.5 * (np.take(x, range(0, x.shape[axis] - 1), axis=axis)
                             + np.take(x, range(1, x.shape[axis]), axis=axis))
                return np.concatenate((x0, mid, x1), axis=axis)
            fv = momentum._face_vectors(r_if, th_if, nphi)
            k4 = 1.0 / (4.0 * np.pi * G)

            def stress(gn, g1, g2, f):
                return k4 * ((half * (gn * gn - g1 * g1 - g2 * g2))[..., None] * f["N"]
                             + sign * (gn * g1)[..., None] * f["T1"] + sign * (gn * g2)[..., None] * f["T2"])
            Sr = stress(gr, pad_mean(ct, 0), pad_mean(cp, 0), fv["r"])
            St = stress(gt, pad_mean(cr, 1), pad_mean(cp, 1), fv["t"])
            Sp = stress(gp, 0.5 * (cr + np.roll(cr, -1, axis=2)), 0.5 * (ct + np.roll(ct, -1, axis=2)), fv["p"])
            F = -((Sr[1:] - Sr[:-1]) + (St[:, 1:] - St[:, :-1]) + (Sp - np.roll(Sp, 1, axis=2)))
            return F, Sr
        monkeypatch.setattr(momentum, "cell_forces", bad)
        assert _momentum_convergence(16) > 0.1, slip
        monkeypatch.undo()
    monkeypatch.setattr(momentum, "_face_vectors", scaled_normals)
    rng = np.random.default_rng(9)
    r_if, th_if, nphi = random_r_if(rng, 5, 0.4), random_th_if(rng, 6), 8
    fv = momentum._face_vectors(r_if, th_if, nphi)
    close = ((fv["r"]["N"][1:] - fv["r"]["N"][:-1]) + (fv["t"]["N"][:, 1:] - fv["t"]["N"][:, :-1])
             + (fv["p"]["N"] - np.roll(fv["p"]["N"], 1, axis=2)))
    assert np.max(np.abs(close)) > 1e-6 * np.max(np.abs(fv["r"]["N"]))
