"""Momentum-conserving gravitational source term from the exact potential.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper notes that the exact solution of the discrete Poisson equation lets
a hydrodynamics code write its gravitational source terms in conservative form
(Sec. 1, Sec. 6) without giving one.  The momentum form used here is the
gravitational stress tensor, the gravitational analogue of the Maxwell stress
tensor (a textbook identity):

    T = (grad Phi grad Phi - |grad Phi|^2 I / 2) / (4 pi G),
    div T = rho grad Phi   wherever  Laplacian Phi = 4 pi G rho,

so the force on a cell, -integral of rho grad Phi over its volume, is the
surface integral -sum over its faces of T . n dA.  Evaluating T . n once per
face and giving it to both cells that share the face makes every interior face
cancel in the total: the grid's total momentum changes only through its outer
boundary (conservation to rounding).

Discretisation (per face, with n along the increasing coordinate):
  * the normal gradient component G_n is the face difference quotient of the
    flux form of Sec. 3.1 (the outer face: the extrapolated derivative of
    Sec. 3.2 per eigenmode; the inner face: zero flux, and no area at r = 0;
    pole faces have no area);
  * each tangential component is the mean of the two adjacent cells'
    cell-centred components, a cell's component being the mean of its two face
    difference quotients in that direction (pole faces and the inner face
    taken as 0; a boundary face takes its one cell's component);
  * the stress vector integrated over the curved face is
        (1/4piG) [ (G_n^2 - G_t1^2 - G_t2^2)/2 N + G_n G_t1 T1 + G_n G_t2 T2 ],
    N, T1, T2 the exact integrals over the face of the local unit vectors
    (e_r, e_theta, e_phi in Cartesian components), so that they sum to zero
    over every closed cell surface.
The result is the force on each cell in Cartesian components (x, y, z) with
phi measured from x, theta from z.
"""
import numpy as np

from .geometry import grid_geometry
from .laplacian import outer_flux


def _face_vectors(r_if, th_if, nphi):
    """Exact integrals of e_r, e_theta, e_phi over every face (Cartesian).

    Returns dicts keyed 'r', 't', 'p' (r-, theta-, phi-faces); each maps the
    normal and tangential unit vectors to arrays of shape (..., 3):
      r-faces  [nr + 1][nth][nphi]: N = int e_r, T1 = int e_theta, T2 = int e_phi
      t-faces  [nr][nth + 1][nphi]: N = int e_theta, T1 = int e_r, T2 = int e_phi
      p-faces  [nr][nth][nphi]    : N = int e_phi (face k + 1/2), T1 = int e_r, T2 = int e_theta
    """
    r_if = np.asarray(r_if, dtype=np.float64)
    th_if = np.asarray(th_if, dtype=np.float64)
    a, b = th_if[:-1], th_if[1:]
    ph_if = 2.0 * np.pi * np.arange(nphi + 1) / nphi
    c, d = ph_if[:-1], ph_if[1:]
    # theta integrals over [a, b]
    i_s2 = 0.5 * (b - a) - 0.25 * (np.sin(2 * b) - np.sin(2 * a))        # int sin^2
    i_sc = 0.5 * (np.sin(b) ** 2 - np.sin(a) ** 2)                        # int sin cos
    i_s = np.cos(a) - np.cos(b)                                           # int sin
    i_c = np.sin(b) - np.sin(a)                                           # int cos
    # phi integrals over [c, d]
    j_c = np.sin(d) - np.sin(c)       # int cos
    j_s = np.cos(c) - np.cos(d)       # int sin
    dp = d - c
    R2 = (r_if ** 2)[:, None, None]
    ring = (0.5 * (r_if[1:] ** 2 - r_if[:-1] ** 2))[:, None, None]

    def vec(x, y, z):
        return np.stack(np.broadcast_arrays(x, y, z), axis=-1)

    out = {}
    # r-faces: dA = R^2 sin th dth dph
    out["r"] = dict(
        N=R2[..., None] * vec(i_s2[:, None] * j_c[None, :], i_s2[:, None] * j_s[None, :],
                              i_sc[:, None] * dp[None, :])[None],
        T1=R2[..., None] * vec(i_sc[:, None] * j_c[None, :], i_sc[:, None] * j_s[None, :],
                               -i_s2[:, None] * dp[None, :])[None],
        T2=R2[..., None] * vec(i_s[:, None] * -j_s[None, :], i_s[:, None] * j_c[None, :],
                               0.0 * i_s[:, None] * dp[None, :])[None])
    # theta-faces at th_if[j]: dA = r sin TH dr dph
    st, ct = np.sin(th_if), np.cos(th_if)
    st[0] = st[-1] = 0.0                      # the pole faces have no area
    out["t"] = dict(
        N=ring[..., None] * vec((st * ct)[:, None] * j_c[None, :], (st * ct)[:, None] * j_s[None, :],
                                -(st * st)[:, None] * dp[None, :])[None],
        T1=ring[..., None] * vec((st * st)[:, None] * j_c[None, :], (st * st)[:, None] * j_s[None, :],
                                 (st * ct)[:, None] * dp[None, :])[None],
        T2=ring[..., None] * vec(st[:, None] * -j_s[None, :], st[:, None] * j_c[None, :],
                                 0.0 * st[:, None] * dp[None, :])[None])
    # phi-faces at ph_if[k + 1]: dA = r dr dth
    p1 = ph_if[1:]
    out["p"] = dict(
        N=ring[..., None] * vec((b - a)[:, None] * -np.sin(p1)[None, :], (b - a)[:, None] * np.cos(p1)[None, :],
                                0.0 * (b - a)[:, None] * p1[None, :])[None],
        T1=ring[..., None] * vec(i_s[:, None] * np.cos(p1)[None, :], i_s[:, None] * np.sin(p1)[None, :],
                                 i_c[:, None] * np.ones_like(p1)[None, :])[None],
        T2=ring[..., None] * vec(i_c[:, None] * np.cos(p1)[None, :], i_c[:, None] * np.sin(p1)[None, :],
                                 -i_s[:, None] * np.ones_like(p1)[None, :])[None])
    return out


def face_gradients(r_if, th_if, nphi, Phi, driver="stev"):
    """Face difference quotients of Phi (Sec. 3.1 flux form, Sec. 3.2 outer face;
    `driver` selects the LAPACK eigensolver of the outer face's eigenmodes).

    gr [nr + 1][nth][nphi]  at r-faces (index i: face i - 1/2; inner face 0),
    gt [nr][nth + 1][nphi]  at theta-faces (pole faces 0),
    gp [nr][nth][nphi]      at phi-faces k + 1/2 (periodic).
    """
    g = grid_geometry(r_if, th_if, nphi)
    P = np.asarray(Phi, dtype=np.float64)
    nr, nth = g["nr"], g["nth"]
    r, th = g["r"], g["th"]
    gr = np.zeros((nr + 1, nth, nphi))
    gr[1:-1] = (P[1:] - P[:-1]) / (r[1:] - r[:-1])[:, None, None]
    # outer face: flux / (r_o^2 dmu dphi) = -beta(A) Phi_N / r_o^2
    gr[-1] = -outer_flux(g, P[-1], driver) / g["r_if"][-1] ** 2
    gt = np.zeros((nr, nth + 1, nphi))
    gt[:, 1:-1] = (P[:, 1:] - P[:, :-1]) / (r[:, None, None] * (th[1:] - th[:-1])[None, :, None])
    gp = (np.roll(P, -1, axis=2) - P) / (r[:, None, None] * np.sin(th)[None, :, None] * g["dphi"])
    return gr, gt, gp


def cell_forces(r_if, th_if, nphi, Phi, G=1.0, with_terms=False, driver="stev"):
    """Force on every cell, -sum over its faces of the integrated T . n_out,
    as an array [nr][nth][nphi][3] (Cartesian x, y, z); also returns the
    integrated stress vectors of the r-faces [nr + 1][nth][nphi][3] (for the
    boundary terms).  With `with_terms`, a third array of F's shape holds the
    scale of the rounding error of any evaluation of the sum: per component,
    the sum over the six faces of |k4| (|G_n^2 + G_t1^2 + G_t2^2|/2 |N| +
    |G_n G_t1| |T1| + |G_n G_t2| |T2|)."""
    gr, gt, gp = face_gradients(r_if, th_if, nphi, Phi, driver)
    # cell-centred components: mean of the two face quotients
    cr = 0.5 * (gr[:-1] + gr[1:])
    ct = 0.5 * (gt[:, :-1] + gt[:, 1:])
    cp = 0.5 * (gp + np.roll(gp, 1, axis=2))
    nr, nth = cr.shape[:2]

    def pad_mean(x, axis):
        """Mean of the two cells adjacent to each face along `axis` (faces 0..n,
        boundary faces take their one cell)."""
        x0 = np.take(x, [0], axis=axis)
        x1 = np.take(x, [-1], axis=axis)
        mid = 0.5 * (np.take(x, range(0, x.shape[axis] - 1), axis=axis)
                     + np.take(x, range(1, x.shape[axis]), axis=axis))
        return np.concatenate((x0, mid, x1), axis=axis)

    fv = _face_vectors(r_if, th_if, nphi)
    k4 = 1.0 / (4.0 * np.pi * G)

    def stress(gn, g1, g2, f):
        return k4 * ((0.5 * (gn * gn - g1 * g1 - g2 * g2))[..., None] * f["N"]
                     + (gn * g1)[..., None] * f["T1"] + (gn * g2)[..., None] * f["T2"])

    def scale(gn, g1, g2, f):
        A = np.abs
        return A(k4) * ((0.5 * (gn * gn + g1 * g1 + g2 * g2))[..., None] * A(f["N"])
                        + A(gn * g1)[..., None] * A(f["T1"]) + A(gn * g2)[..., None] * A(f["T2"]))

    cr_p = 0.5 * (cr + np.roll(cr, -1, axis=2))                             # periodic in phi
    ct_p = 0.5 * (ct + np.roll(ct, -1, axis=2))
    args_r = (gr, pad_mean(ct, 0), pad_mean(cp, 0), fv["r"])                # [nr + 1][nth][nphi]
    args_t = (gt, pad_mean(cr, 1), pad_mean(cp, 1), fv["t"])                # [nr][nth + 1][nphi]
    args_p = (gp, cr_p, ct_p, fv["p"])                                      # face k + 1/2
    Sr, St, Sp = stress(*args_r), stress(*args_t), stress(*args_p)
    F = -((Sr[1:] - Sr[:-1]) + (St[:, 1:] - St[:, :-1]) + (Sp - np.roll(Sp, 1, axis=2)))
    if not with_terms:
        return F, Sr
    Mr, Mt, Mp = scale(*args_r), scale(*args_t), scale(*args_p)
    M = (Mr[1:] + Mr[:-1]) + (Mt[:, 1:] + Mt[:, :-1]) + (Mp + np.roll(Mp, 1, axis=2))
    return F, Sr, M
