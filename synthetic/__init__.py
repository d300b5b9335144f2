"""Seeded synthetic grids and densities for tests and benchmarks.

This package holds input generation only: interface coordinates, densities
sampled at cell centres, and seeded random draws.  It contains none of the
solver's arithmetic, and both the oracle's tests and the HIP library's tests
and benchmarks draw their inputs from it.

Workloads (all in non-dimensional units with G = 1; lengths of the stellar
workloads are in km):

* ``gaussian_blob_case``: N_r = 64 uniform zones on r in [0, 1], N_theta = 32,
  N_phi = 64; a Gaussian blob (sigma = 0.1, amplitude 1, Cartesian distance)
  centred at (r, theta, phi) = (0.3, pi/3, pi/4) plus uniform noise in
  [-1e-3, 1e-3] (seed 0).
* ``stellar_case``: N_r = 550 (20 uniform 0.5 km zones to 10 km, then a
  geometric progression whose ratio puts the outer face at exactly 1e4 km),
  N_theta = 128, N_phi = 256.  rho = rho0 (1 + (r/r0)^2)^-1.5 with r0 = 20 km,
  times (1 + 0.05 X) with X = exp(Z), Z ~ N(0, 1) i.i.d. per zone, plus a point
  mass of 5% of the profile mass in the zone containing (r, theta, phi) =
  (30 km, 0.246 pi, 0.996 pi).  This is the grid size of the paper's timing
  table and the angular position of its displaced point-source test.
* ``batch_grids``: 64 grids drawn i.i.d. from N_r in {128, 256, 550},
  N_theta in {32, 64, 128}, N_phi in {64, 128, 256} (draw seed 3), stellar
  sources with per-grid seeds 100..163.
* ``serving_classes`` / ``serving_source``: three grid classes
  (128, 32, 64), (256, 64, 128), (550, 128, 256), each with an off-centre
  point mass plus a Gaussian blob at seeded random positions.

All random numbers come from numpy's PCG64 ``default_rng(seed)``.
"""
import numpy as np


# --------------------------------------------------------------------------
# interfaces
# --------------------------------------------------------------------------
def uniform_interfaces(n, lo, hi):
    """n uniform cells on [lo, hi] -> n + 1 interfaces (end points exact)."""
    x = lo + (hi - lo) * np.arange(n + 1, dtype=np.float64) / n
    x[0], x[-1] = lo, hi
    return x


def theta_interfaces(nth):
    """Uniform theta interfaces on [0, pi]."""
    return uniform_interfaces(nth, 0.0, np.pi)


def axis_coarsened_theta(nth, ratio=2.0):
    """Theta interfaces symmetric about the equator whose cells widen towards
    the poles: the width grows smoothly from the equator to `ratio` times that
    at the poles (the kind of axis coarsening that relaxes a hydrodynamics
    code's time step near the axis).  On the northern half, u = j / (nth/2)
    maps to theta = pi/2 (b u + (1 - b) u^2) with b = 2 ratio / (1 + ratio), whose
    slope is b at the pole and 2 - b at the equator; the southern half is the
    mirror image pi - theta (nth even)."""
    if nth % 2:
        raise ValueError("nth must be even")
    h = nth // 2
    b = 2.0 * ratio / (1.0 + ratio)
    u = np.arange(h + 1, dtype=np.float64) / h
    north = 0.5 * np.pi * (b * u + (1.0 - b) * u * u)
    north[0], north[-1] = 0.0, 0.5 * np.pi
    return np.concatenate((north, np.pi - north[-2::-1]))


def skewed_theta(nth, c=0.3):
    """Theta interfaces that are smooth but not symmetric about the equator:
    theta = pi (u + c u (1 - u)) at u = j / nth, so the cells widen from the
    south pole (width ratio (1 + c)/(1 - c) to the north pole)."""
    u = np.arange(nth + 1, dtype=np.float64) / nth
    th = np.pi * (u + c * u * (1.0 - u))
    th[0], th[-1] = 0.0, np.pi
    return th


def stellar_r_interfaces(nr, n_uniform=20, dr=0.5, r_out=1.0e4):
    """n_uniform zones of width dr from r = 0, then nr - n_uniform zones whose
    widths grow geometrically, dr*q, dr*q^2, ..., with q chosen (by bisection)
    so that the last interface lands exactly on r_out."""
    n_geo = nr - n_uniform
    if n_geo <= 0:
        raise ValueError("nr must exceed n_uniform")
    r_uni = n_uniform * dr

    def outer(q):
        return r_uni + dr * q * (q ** n_geo - 1.0) / (q - 1.0)

    lo, hi = 1.0 + 1e-12, 2.0
    while outer(hi) < r_out:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if outer(mid) < r_out:
            lo = mid
        else:
            hi = mid
    q = 0.5 * (lo + hi)
    widths = np.concatenate((np.full(n_uniform, dr), dr * q ** np.arange(1, n_geo + 1)))
    r_if = np.concatenate(([0.0], np.cumsum(widths)))
    r_if[-1] = r_out
    return r_if


# --------------------------------------------------------------------------
# helpers on cell centres (midpoints of interfaces)
# --------------------------------------------------------------------------
def _centres(r_if, th_if, nphi):
    r = 0.5 * (r_if[:-1] + r_if[1:])
    th = 0.5 * (th_if[:-1] + th_if[1:])
    phi = (np.arange(nphi) + 0.5) * (2.0 * np.pi / nphi)
    return r, th, phi


def _cartesian(r, th, phi):
    R, T, P = np.meshgrid(r, th, phi, indexing="ij")
    st = np.sin(T)
    return R * st * np.cos(P), R * st * np.sin(P), R * np.cos(T)


def _cell_volume(r_if, th_if, nphi, i, j):
    dphi = 2.0 * np.pi / nphi
    return ((r_if[i + 1] ** 3 - r_if[i] ** 3) / 3.0
            * (np.cos(th_if[j]) - np.cos(th_if[j + 1])) * dphi)


def _zone_of(r_if, th_if, nphi, r0, th0, phi0):
    i = int(np.searchsorted(r_if, r0, side="right") - 1)
    j = int(np.searchsorted(th_if, th0, side="right") - 1)
    k = int(np.floor(phi0 / (2.0 * np.pi / nphi))) % nphi
    return min(max(i, 0), r_if.size - 2), min(max(j, 0), th_if.size - 2), k


def gaussian_blob(r_if, th_if, nphi, centre, width, amplitude=1.0):
    r, th, phi = _centres(r_if, th_if, nphi)
    x, y, z = _cartesian(r, th, phi)
    cx, cy, cz = _cartesian(np.array([centre[0]]), np.array([centre[1]]), np.array([centre[2]]))
    d2 = (x - cx[0, 0, 0]) ** 2 + (y - cy[0, 0, 0]) ** 2 + (z - cz[0, 0, 0]) ** 2
    return amplitude * np.exp(-0.5 * d2 / width ** 2)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def gaussian_blob_case(seed=0):
    """Small uniform grid with a Gaussian blob and seeded noise (see module doc)."""
    nr, nth, nphi = 64, 32, 64
    r_if = uniform_interfaces(nr, 0.0, 1.0)
    th_if = theta_interfaces(nth)
    rho = gaussian_blob(r_if, th_if, nphi, (0.3, np.pi / 3, np.pi / 4), 0.1)
    rho += np.random.default_rng(seed).uniform(-1e-3, 1e-3, rho.shape)
    return dict(name="gaussian_blob_64x32x64", r_if=r_if, th_if=th_if, nphi=nphi,
                rho=rho, G=1.0)


def stellar_density(r_if, th_if, nphi, seed, rho0=1.0, r0=20.0,
                    point=(30.0, 0.246 * np.pi, 0.996 * np.pi), point_frac=0.05):
    """Stellar-core-like profile times a lognormal field, plus a point mass."""
    r, th, phi = _centres(r_if, th_if, nphi)
    prof = rho0 * (1.0 + (r / r0) ** 2) ** -1.5
    rng = np.random.default_rng(seed)
    lognorm = np.exp(rng.standard_normal((r.size, th.size, nphi)))
    rho = prof[:, None, None] * (1.0 + 0.05 * lognorm)
    dphi = 2.0 * np.pi / nphi
    vol = np.outer((r_if[1:] ** 3 - r_if[:-1] ** 3) / 3.0,
                   np.cos(th_if[:-1]) - np.cos(th_if[1:])) * dphi
    m_prof = float(np.sum(prof[:, None] * vol) * nphi)
    i, j, k = _zone_of(r_if, th_if, nphi, *point)
    rho[i, j, k] += point_frac * m_prof / _cell_volume(r_if, th_if, nphi, i, j)
    return rho


def stellar_grid(nr, nth, nphi):
    return stellar_r_interfaces(nr), theta_interfaces(nth), nphi


def stellar_case(nr=550, nth=128, nphi=256, seed=1):
    """Stellar-core grid and source (see module doc)."""
    r_if, th_if, nphi = stellar_grid(nr, nth, nphi)
    rho = stellar_density(r_if, th_if, nphi, seed)
    return dict(name=f"stellar_{nr}x{nth}x{nphi}", r_if=r_if, th_if=th_if,
                nphi=nphi, rho=rho, G=1.0)


def batch_grids(n=64, seed=3):
    """(nr, nth, nphi) for each right-hand side of the batched workload."""
    rng = np.random.default_rng(seed)
    nrs = rng.choice([128, 256, 550], size=n)
    nths = rng.choice([32, 64, 128], size=n)
    nphis = rng.choice([64, 128, 256], size=n)
    return [(int(a), int(b), int(c)) for a, b, c in zip(nrs, nths, nphis)]


SERVING_CLASSES = ((128, 32, 64), (256, 64, 128), (550, 128, 256))


def serving_source(r_if, th_if, nphi, seed):
    """Off-centre point mass plus a Gaussian blob at seeded random positions."""
    rng = np.random.default_rng(seed)
    r_out = r_if[-1]
    rb = rng.uniform(5.0, 60.0)
    cb = (rb, np.arccos(rng.uniform(-1, 1)), rng.uniform(0, 2 * np.pi))
    rho = gaussian_blob(r_if, th_if, nphi, cb, width=rng.uniform(5.0, 15.0))
    dphi = 2.0 * np.pi / nphi
    vol = np.outer((r_if[1:] ** 3 - r_if[:-1] ** 3) / 3.0,
                   np.cos(th_if[:-1]) - np.cos(th_if[1:])) * dphi
    m_blob = float(np.sum(rho * vol[:, :, None]))
    pos = (rng.uniform(10.0, min(100.0, 0.5 * r_out)), np.arccos(rng.uniform(-1, 1)),
           rng.uniform(0, 2 * np.pi))
    i, j, k = _zone_of(r_if, th_if, nphi, *pos)
    rho[i, j, k] += 0.2 * m_blob / _cell_volume(r_if, th_if, nphi, i, j)
    return rho


def ellipsoid_density(r_if, th_if, nphi, axes=(1.0, 1.5, 2.0), n_quad=16):
    """Cell-averaged density of a homogeneous ellipsoid (rho = 1 inside).

    Along each direction the boundary radius is R(mu, phi); the volume of the
    cell inside the ellipsoid is the integral over the cell's solid angle of
    (min(r_+, R)^3 - r_-^3)_+ / 3, evaluated with an n_quad x n_quad
    Gauss-Legendre rule in (mu = cos theta, phi).  Cells entirely inside or
    outside the range of R over their solid angle are 1 or 0 without
    quadrature.  (The convergence study of the paper uses recursive sub-cell
    refinement for the same quantity.)
    """
    a, b, c = axes
    r_if = np.asarray(r_if, dtype=np.float64)
    nr, nth = r_if.size - 1, len(th_if) - 1
    dphi = 2.0 * np.pi / nphi
    rho = np.zeros((nr, nth, nphi))
    xg, wg = np.polynomial.legendre.leggauss(n_quad)
    mu_if = np.cos(np.asarray(th_if, dtype=np.float64))
    for j in range(nth):
        mu = 0.5 * (mu_if[j] + mu_if[j + 1]) + 0.5 * (mu_if[j] - mu_if[j + 1]) * xg
        wm = 0.5 * (mu_if[j] - mu_if[j + 1]) * wg
        st2 = 1.0 - mu * mu
        for k in range(nphi):
            ph = (k + 0.5 * (1.0 + xg)) * dphi
            W = np.outer(wm, 0.5 * dphi * wg)
            R = 1.0 / np.sqrt(np.outer(st2, np.cos(ph) ** 2) / a ** 2 + np.outer(st2, np.sin(ph) ** 2) / b ** 2
                              + np.outer(mu * mu, np.ones_like(ph)) / c ** 2)
            rlo, rhi = R.min(), R.max()
            rho[r_if[1:] <= rlo, j, k] = 1.0
            dom = W.sum()
            for i in np.nonzero((r_if[1:] > rlo) & (r_if[:-1] < rhi))[0]:
                rm, rp = r_if[i], r_if[i + 1]
                vol = np.sum(W * np.clip(np.minimum(rp, R) ** 3 - rm ** 3, 0.0, None)) / 3.0
                rho[i, j, k] = vol / ((rp ** 3 - rm ** 3) / 3.0 * dom)
    return rho
