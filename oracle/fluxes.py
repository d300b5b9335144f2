"""Face fluxes of grad Phi through every cell face (Sec. 3.1 and 3.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The discrete operator of Sec. 3.1 is a finite-volume divergence: for each
cell, (Delta Phi) delta V is the sum over its six faces of the face area
times the difference quotient of Phi across that face.  Because the solver
returns the exact solution of that discrete system, these face terms are the
fluxes of the discrete gravitational field: summed over the faces of any
cell they give 4 pi G rho delta V to rounding, which is what lets a
hydrodynamics code write its gravitational momentum and energy sources in
conservative form (Sec. 1, Sec. 3.1, Sec. 6).  This module evaluates them:

  Fr[i, j, k]  through the radial face i+1/2 (outer face of cell i):
               r_{i+1/2}^2 (cos th_{j-1/2} - cos th_{j+1/2}) dphi
               * (Phi_{i+1,j,k} - Phi_{i,j,k}) / (r_{i+1} - r_i);
               for i = N_r - 1 the outer boundary face, where the difference
               quotient is the extrapolated derivative of Sec. 3.2, applied
               per angular eigenmode;
  Ft[i, j, k]  through the theta face j+1/2:
               (r_{i+1/2}^2 - r_{i-1/2}^2)/2 sin th_{j+1/2} dphi
               * (Phi_{i,j+1,k} - Phi_{i,j,k}) / (r_i (th_{j+1} - th_j));
               zero for j = N_theta - 1 (the pole face theta = pi);
  Fp[i, j, k]  through the phi face k+1/2 (periodic: k = N_phi - 1 couples
               to k = 0):
               (r_{i+1/2}^2 - r_{i-1/2}^2)/2 (th_{j+1/2} - th_{j-1/2})
               * (Phi_{i,j,k+1} - Phi_{i,j,k}) / (r_i sin th_j dphi).

Each flux is signed along its increasing coordinate.  The inner face r = 0
of the first shell and the pole face theta = 0 have zero area and are not
stored.  The areas, volumes and centres are those of Sec. 3.1 with the
readings of ``geometry`` (area factor (r_{i+1/2}^2 - r_{i-1/2}^2)/2, centres
at interface midpoints); they are computed here from the interfaces, not
from the solver's factored coefficients R_i, S_j.
"""
import numpy as np

from .geometry import grid_geometry
from .laplacian import outer_flux


def face_fluxes(r_if, th_if, nphi, Phi):
    """(Fr, Ft, Fp), each of the shape of Phi, as defined in the module doc."""
    r_if = np.asarray(r_if, dtype=np.float64)
    th_if = np.asarray(th_if, dtype=np.float64)
    P = np.asarray(Phi, dtype=np.float64)
    nr, nth = r_if.size - 1, th_if.size - 1
    assert P.shape == (nr, nth, nphi)
    r = 0.5 * (r_if[:-1] + r_if[1:])
    th = 0.5 * (th_if[:-1] + th_if[1:])
    dphi = 2.0 * np.pi / nphi
    # cos th_{j-1/2} - cos th_{j+1/2} and (r_{i+1/2}^2 - r_{i-1/2}^2)/2 in
    # factored form: the same quantities without the cancellation of the plain
    # differences next to the poles and on thin outer shells
    tm, tp = th_if[:-1], th_if[1:]
    dmu = 2.0 * np.sin(0.5 * (tp + tm)) * np.sin(0.5 * (tp - tm))
    ring = 0.5 * (r_if[1:] - r_if[:-1]) * (r_if[1:] + r_if[:-1])

    Fr = np.zeros_like(P)
    area_r = (r_if[1:-1] ** 2)[:, None] * dmu[None, :] * dphi
    Fr[:-1] = (area_r / (r[1:] - r[:-1])[:, None])[:, :, None] * (P[1:] - P[:-1])
    # outer face: area r_o^2 dmu dphi times the extrapolated derivative
    # -(1/r_o) p (r_o/r_N)^-p f_N of each eigenmode, i.e. -dmu dphi beta(A) Phi_N
    g = grid_geometry(r_if, th_if, nphi)
    Fr[-1] = -(dmu * dphi)[:, None] * outer_flux(g, P[-1])

    Ft = np.zeros_like(P)
    area_t = ring[:, None] * np.sin(th_if[1:-1])[None, :] * dphi
    dist_t = r[:, None] * (th[1:] - th[:-1])[None, :]
    Ft[:, :-1] = (area_t / dist_t)[:, :, None] * (P[:, 1:] - P[:, :-1])

    area_p = ring[:, None] * (th_if[1:] - th_if[:-1])[None, :]
    dist_p = r[:, None] * np.sin(th)[None, :] * dphi
    Fp = (area_p / dist_p)[:, :, None] * (np.roll(P, -1, axis=2) - P)
    return Fr, Ft, Fp


def net_outward_flux(Fr, Ft, Fp):
    """Sum of the fluxes out of every cell through its six faces."""
    out = Fr.copy()
    out[1:] -= Fr[:-1]
    out += Ft
    out[:, 1:] -= Ft[:, :-1]
    out += Fp - np.roll(Fp, 1, axis=2)
    return out
