"""Grid geometry of the finite-volume discretisation (paper Sec. 3.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Indices here are 0-based: radial cells i = 0..nr-1 (paper i = 1..N_r),
theta cells j = 0..nth-1, phi cells k = 0..nphi-1.  Interface arrays have one
more entry than the cells they bound.

Readings of the paper's text used here:
* the radial and theta interface areas carry (r_{i+1/2}^2 - r_{i-1/2}^2)/2;
  the printed formula repeats r_{i+1/2} and would be identically zero;
* cell centres are arithmetic midpoints of their interfaces (this reproduces
  the worked example of Sec. 5.1: zone (j, k) = (32, 128) of a 128 x 256
  angular grid sits at theta = 0.246 pi, phi = 0.996 pi);
* the pole faces theta = 0 and theta = pi have zero area exactly.
"""
import numpy as np


def cell_centres(r_if, th_if, nphi):
    """Cell centres as interface midpoints; phi is uniform on [0, 2 pi)."""
    r_if = np.asarray(r_if, dtype=np.float64)
    th_if = np.asarray(th_if, dtype=np.float64)
    r = 0.5 * (r_if[:-1] + r_if[1:])
    th = 0.5 * (th_if[:-1] + th_if[1:])
    dphi = 2.0 * np.pi / nphi
    phi = (np.arange(nphi) + 0.5) * dphi
    return r, th, phi


def grid_geometry(r_if, th_if, nphi):
    """All geometric factors the discrete operator needs (Sec. 3.1).

    Returns a dict with
      r, th, phi     cell centres
      dphi           uniform phi spacing
      dth[j]         theta_{j+1/2} - theta_{j-1/2}
      dmu[j]         cos theta_{j-1/2} - cos theta_{j+1/2}
      V[i]           (r_{i+1/2}^3 - r_{i-1/2}^3)/3  (delta V = V dmu dphi)
      R[i]           3 (r_{i+1/2}^2 - r_{i-1/2}^2) / (2 r_i (r_{i+1/2}^3 - r_{i-1/2}^3))
      S[j]           dth_j / (sin theta_j dmu_j)
      alpha[i]       r_{i+1/2}^2 / (r_{i+1} - r_i) for the interior radial
                     faces i+1/2, i = 0..nr-2 (the dmu dphi factor of the
                     face area cancels against delta V)
      sigma[j]       sin theta_{j+1/2} / (theta_{j+1} - theta_j) for the nth+1
                     theta faces; the two pole entries are exactly 0
    The differences of cubes and of cosines are evaluated in factored form
    (a^3 - b^3 = (a - b)(a^2 + ab + b^2); cos a - cos b =
    2 sin((a + b)/2) sin((b - a)/2)), which are the same quantities without
    the cancellation of the plain differences on thin cells.
    """
    r_if = np.asarray(r_if, dtype=np.float64)
    th_if = np.asarray(th_if, dtype=np.float64)
    nr, nth = r_if.size - 1, th_if.size - 1
    r, th, phi = cell_centres(r_if, th_if, nphi)
    rm, rp = r_if[:-1], r_if[1:]
    tm, tp = th_if[:-1], th_if[1:]

    V = (rp - rm) * (rp * rp + rp * rm + rm * rm) / 3.0
    R = (rp * rp - rm * rm) / (2.0 * r * V)
    dth = tp - tm
    dmu = 2.0 * np.sin(0.5 * (tp + tm)) * np.sin(0.5 * (tp - tm))
    S = dth / (np.sin(th) * dmu)

    alpha = rp[:-1] ** 2 / (r[1:] - r[:-1])            # faces 1/2+i, i=0..nr-2
    sigma = np.zeros(nth + 1)
    sigma[1:-1] = np.sin(th_if[1:-1]) / (th[1:] - th[:-1])
    return dict(nr=nr, nth=nth, nphi=nphi, r_if=r_if, th_if=th_if,
                r=r, th=th, phi=phi, dphi=2.0 * np.pi / nphi,
                dth=dth, dmu=dmu, V=V, R=R, S=S, alpha=alpha, sigma=sigma)


def cell_volumes(r_if, th_if, nphi):
    """delta V_{ijk} = V_i dmu_j dphi as an (nr, nth) array (same for all k)."""
    g = grid_geometry(r_if, th_if, nphi)
    return np.outer(g["V"], g["dmu"]) * g["dphi"]
