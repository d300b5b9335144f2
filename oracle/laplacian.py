"""Apply the discrete operator L to a field, and residual diagnostics.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

L Phi is evaluated with the local stencil of Sec. 3.1 (radial, theta and phi
fluxes between neighbouring cells, divided by the cell volume).  On the
outermost shell the outward radial flux is the boundary term of Sec. 3.2,
-beta(lambda_Omega) f_N per angular eigenmode; it is evaluated by
transforming that one shell with the FFT and the theta eigenvectors of the
spectral oracle, multiplying each mode by beta, and transforming back.  The
inner face of the innermost shell carries gamma(lambda_Omega) f_1 in the same
way (zero for the zero-flux condition and for r_{1/2} = 0).
"""
import numpy as np

from .geometry import grid_geometry
from .spectral import inner_gamma, outer_beta, theta_eigensystem


def _mode_function(geom, shell, coef_of_lambda, driver="stev"):
    """coef(A) shell: per Fourier mode m and theta eigenmode l, times coef(lambda)."""
    nphi = geom["nphi"]
    c = np.fft.rfft(shell, axis=1) / nphi
    out = np.empty_like(c)
    for m in range(c.shape[1]):
        lam, H = theta_eigensystem(geom, m, driver)
        coef = (H.T * geom["dmu"][None, :]) @ c[:, m]
        out[:, m] = H @ (coef_of_lambda(lam) * coef)
    return np.fft.irfft(out, n=nphi, axis=1) * nphi


def outer_flux(geom, shell, driver="stev"):
    """Outer-face term beta(A) Phi_shell for one (nth, nphi) shell (`driver`:
    the LAPACK tridiagonal eigensolver of the theta eigensystems)."""
    return _mode_function(geom, shell, lambda lam: outer_beta(geom, lam), driver)


def inner_flux(geom, shell, inner="zero_flux"):
    """Inner-face term gamma(A) Phi_shell for the innermost (nth, nphi) shell."""
    return _mode_function(geom, shell, lambda lam: inner_gamma(geom, lam, inner))


def apply(r_if, th_if, nphi, Phi, with_terms=False, inner="zero_flux"):
    """L Phi (and, if asked, the absolute stencil terms for backward errors).

    With ``with_terms`` the second return value is |L| |Phi| evaluated term
    by term (each flux contribution in absolute value; each boundary face
    term, which couples a whole shell, as the magnitude of its value), the
    denominator of the componentwise backward error.
    """
    g = grid_geometry(r_if, th_if, nphi)
    P = np.asarray(Phi, dtype=np.float64)
    nr = g["nr"]
    V, R, S, al, sig, dmu = g["V"], g["R"], g["S"], g["alpha"], g["sigma"], g["dmu"]
    out = np.zeros_like(P)
    mag = np.zeros_like(P)

    # radial fluxes through interior faces i+1/2 (i = 0..nr-2)
    fr = al[:, None, None] * (P[1:] - P[:-1])
    ar = al[:, None, None] * (np.abs(P[1:]) + np.abs(P[:-1]))
    out[:-1] += fr / V[:-1, None, None]
    out[1:] -= fr / V[1:, None, None]
    mag[:-1] += ar / V[:-1, None, None]
    mag[1:] += ar / V[1:, None, None]
    # outer face: -beta(A) Phi_N
    fo = outer_flux(g, P[-1])
    out[-1] -= fo / V[-1]
    mag[-1] += np.abs(fo) / V[-1]
    # inner face (regular condition, r_{1/2} > 0): flux gamma(A) Phi_1 into the
    # innermost shell along +r
    if inner != "zero_flux" and g["r_if"][0] > 0.0:
        fi = inner_flux(g, P[0], inner)
        out[0] -= fi / V[0]
        mag[0] += np.abs(fi) / V[0]

    # theta fluxes through interior faces j+1/2, times R_i / dmu_j
    ft = sig[1:-1][None, :, None] * (P[:, 1:] - P[:, :-1])
    at = sig[1:-1][None, :, None] * (np.abs(P[:, 1:]) + np.abs(P[:, :-1]))
    wt = R[:, None, None]
    out[:, :-1] += wt * ft / dmu[None, :-1, None]
    out[:, 1:] -= wt * ft / dmu[None, 1:, None]
    mag[:, :-1] += wt * at / dmu[None, :-1, None]
    mag[:, 1:] += wt * at / dmu[None, 1:, None]

    # phi second difference, times R_i S_j / dphi^2
    wp = (R[:, None] * S[None, :] / g["dphi"] ** 2)[:, :, None]
    Pp, Pm = np.roll(P, -1, axis=2), np.roll(P, 1, axis=2)
    out += wp * (Pp - 2.0 * P + Pm)
    mag += wp * (np.abs(Pp) + 2.0 * np.abs(P) + np.abs(Pm))
    if with_terms:
        return out, mag
    return out


def backward_error(r_if, th_if, nphi, Phi, rho, G=1.0, inner="zero_flux"):
    """Componentwise backward error max |s - L Phi| / (|L||Phi| + |s|)."""
    s = 4.0 * np.pi * G * np.asarray(rho, dtype=np.float64)
    LP, mag = apply(r_if, th_if, nphi, Phi, with_terms=True, inner=inner)
    return float(np.max(np.abs(s - LP) / (mag + np.abs(s))))
