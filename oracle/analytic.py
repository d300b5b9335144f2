"""Closed forms used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
import numpy as np


def uniform_sphere_potential(r, R, rho0=1.0, G=1.0):
    """Newtonian potential of a homogeneous sphere of radius R and density rho0.

    -2 pi G rho0 (R^2 - r^2/3) inside, -G M / r outside, M = 4/3 pi R^3 rho0
    (the continuum solution of Delta Phi = 4 pi G rho, Sec. 2).
    """
    r = np.asarray(r, dtype=np.float64)
    M = 4.0 / 3.0 * np.pi * R ** 3 * rho0
    inside = -2.0 * np.pi * G * rho0 * (R * R - r * r / 3.0)
    with np.errstate(divide="ignore"):
        outside = -G * M / r
    return np.where(r < R, inside, outside)


def spherical_discrete_potential(r_if, s_radial):
    """Exact discrete solution for a spherically symmetric source.

    Only the (l = 0, m = 0) mode is present: constant theta eigenvector,
    lambda_Omega = 0, so p = 1 and the outer condition gives the face flux
    -r_N f_N.  The radial flux form telescopes (Gauss's law on the grid):
      Q_i = sum_{i' <= i} s_{i'} V_{i'},   V_i = (r_{i+1/2}^3 - r_{i-1/2}^3)/3,
      r_{i+1/2}^2 (f_{i+1} - f_i) / (r_{i+1} - r_i) = Q_i   (interior faces),
      -r_N f_N = Q_N                                       (outer face).
    Returns f_i for every radial cell.
    """
    r_if = np.asarray(r_if, dtype=np.float64)
    r = 0.5 * (r_if[:-1] + r_if[1:])
    V = (r_if[1:] ** 3 - r_if[:-1] ** 3) / 3.0
    Q = np.cumsum(np.asarray(s_radial, dtype=np.float64) * V)
    f = np.empty_like(r)
    f[-1] = -Q[-1] / r[-1]
    for i in range(r.size - 2, -1, -1):
        f[i] = f[i + 1] - Q[i] * (r[i + 1] - r[i]) / r_if[i + 1] ** 2
    return f
