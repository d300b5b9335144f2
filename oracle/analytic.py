"""Closed forms used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
import numpy as np
from scipy.special import elliprd, elliprf


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


def ellipsoid_potential(x, y, z, a, b, c, rho0=1.0, G=1.0):
    """Potential of a homogeneous ellipsoid with semi-axes a, b, c along x, y, z
    (the closed form quoted in Sec. 5.2, Chandrasekhar 1969):

        Phi = pi G rho0 a b c (A x^2 + B y^2 + C z^2 - D),

    A, B, C, D the integrals over lambda from u to infinity of
    [(a^2+l)^3 (b^2+l)(c^2+l)]^-1/2, ... and [(a^2+l)(b^2+l)(c^2+l)]^-1/2, with u = 0
    inside and u the root of x^2/(a^2+u) + y^2/(b^2+u) + z^2/(c^2+u) = 1 outside.
    The integrals are Carlson's symmetric forms: D = 2 R_F(a^2+u, b^2+u, c^2+u),
    A = (2/3) R_D(b^2+u, c^2+u, a^2+u) and cyclically for B, C.
    """
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    a2, b2, c2 = a * a, b * b, c * c
    u = np.zeros(np.broadcast(x, y, z).shape)
    x, y, z = np.broadcast_arrays(x, y, z)
    out = x * x / a2 + y * y / b2 + z * z / c2 > 1.0
    xo, yo, zo = x[out], y[out], z[out]
    # the left side decreases monotonically in u; Newton from u = r^2 - a^2,
    # until the steps stop shrinking at rounding level (two more steps after
    # the largest relative step falls below 1e-13)
    uo = np.maximum(xo * xo + yo * yo + zo * zo - a2, 0.0)
    extra = 2
    for _ in range(60):
        f = xo * xo / (a2 + uo) + yo * yo / (b2 + uo) + zo * zo / (c2 + uo) - 1.0
        df = -(xo * xo / (a2 + uo) ** 2 + yo * yo / (b2 + uo) ** 2 + zo * zo / (c2 + uo) ** 2)
        un = np.maximum(uo - f / df, 0.0)
        step = float(np.max(np.abs(un - uo) / (1.0 + un))) if un.size else 0.0
        uo = un
        if step < 1e-13:
            extra -= 1
            if extra < 0:
                break
    u[out] = uo
    A = 2.0 / 3.0 * elliprd(b2 + u, c2 + u, a2 + u)
    B = 2.0 / 3.0 * elliprd(a2 + u, c2 + u, b2 + u)
    C = 2.0 / 3.0 * elliprd(a2 + u, b2 + u, c2 + u)
    D = 2.0 * elliprf(a2 + u, b2 + u, c2 + u)
    return np.pi * G * rho0 * a * b * c * (A * x * x + B * y * y + C * z * z - D)
