"""Dense brute-force form of the discrete operator L (tiny grids only).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

L is assembled cell by cell from the flux form of Sec. 3.1: for every face,
(area) x (difference of neighbouring values) / (distance between centres),
summed and divided by the cell volume, with the areas and volumes integrated
analytically on the spherical polar cell.  Nothing here uses the factored
coefficients R_i, S_j, the FFT or the per-m eigensystems of the spectral
oracle.  The outer radial face carries the asymptotic boundary condition of
Sec. 3.2, which acts per angular eigenmode; here it is built as a matrix
function of the unit-sphere angular operator A assembled directly on the
whole (theta, phi) shell:

    outward face derivative = -(1/r_o) P(A) Phi_shell,
    P(lambda) = p (r_o / r_N)^-p,   p = (1 + sqrt(1 - 4 lambda))/2,

with r_o the outer interface and r_N the outermost cell centre.  A is
self-adjoint in the solid-angle-weighted inner product, so P(A) is formed
from the symmetric eigendecomposition of W^1/2 A W^-1/2, W = diag(cell solid
angles).  Under the regular inner condition (r_i = r_{1/2} > 0) the inner face
is built the same way:

    face derivative along +r = (1/r_i) Q(A) Phi_shell,
    Q(lambda) = p' (r_i / r_1)^p',   p' = (-1 + sqrt(1 - 4 lambda))/2,

with r_1 the innermost cell centre.  The unknown ordering is C order over
(i, j, k).
"""
import numpy as np


def _cells(r_if, th_if, nphi):
    r_if = np.asarray(r_if, dtype=np.float64)
    th_if = np.asarray(th_if, dtype=np.float64)
    r = 0.5 * (r_if[:-1] + r_if[1:])
    th = 0.5 * (th_if[:-1] + th_if[1:])
    dphi = 2.0 * np.pi / nphi
    return r_if, th_if, r, th, dphi


def shell_angular_operator(th_if, nphi):
    """Unit-sphere finite-volume angular operator A on an (nth*nphi) shell.

    Cell solid angle (cos th_- - cos th_+) dphi; theta face "length"
    sin(th_face) dphi at centre distance th_{j+1} - th_j; phi face length
    (th_+ - th_-) at centre distance sin(th_j) dphi.  Pole faces have zero
    length.  Returns (A, solid_angles).
    """
    th_if = np.asarray(th_if, dtype=np.float64)
    nth = th_if.size - 1
    th = 0.5 * (th_if[:-1] + th_if[1:])
    dphi = 2.0 * np.pi / nphi
    n = nth * nphi
    A = np.zeros((n, n))
    omega = np.empty(n)
    idx = lambda j, k: j * nphi + (k % nphi)
    for j in range(nth):
        dom = (np.cos(th_if[j]) - np.cos(th_if[j + 1])) * dphi
        for k in range(nphi):
            c = idx(j, k)
            omega[c] = dom
            coup = []
            if j + 1 < nth:
                coup.append((idx(j + 1, k), np.sin(th_if[j + 1]) * dphi / (th[j + 1] - th[j])))
            if j > 0:
                coup.append((idx(j - 1, k), np.sin(th_if[j]) * dphi / (th[j] - th[j - 1])))
            w_phi = (th_if[j + 1] - th_if[j]) / (np.sin(th[j]) * dphi)
            coup.append((idx(j, k + 1), w_phi))
            coup.append((idx(j, k - 1), w_phi))
            for nb, w in coup:
                A[c, nb] += w / dom
                A[c, c] -= w / dom
    return A, omega


def _shell_matrix_function(th_if, nphi, fn):
    """fn(A) for the unit-sphere angular operator A of the shell."""
    A, omega = shell_angular_operator(th_if, nphi)
    sw = np.sqrt(omega)
    Asym = sw[:, None] * A / sw[None, :]
    Asym = 0.5 * (Asym + Asym.T)
    lam, Q = np.linalg.eigh(Asym)
    Psym = (Q * fn(lam)) @ Q.T
    return Psym / sw[:, None] * sw[None, :]


def outer_face_operator(r_if, th_if, nphi):
    """Matrix P(A) of the outer boundary condition (see module docstring)."""
    r_if = np.asarray(r_if, dtype=np.float64)
    ro = r_if[-1]
    rn = 0.5 * (r_if[-2] + r_if[-1])

    def P(lam):
        p = 0.5 * (1.0 + np.sqrt(1.0 - 4.0 * lam))
        return p * (ro / rn) ** (-p)
    return _shell_matrix_function(th_if, nphi, P)


def inner_face_operator(r_if, th_if, nphi):
    """Matrix Q(A) of the regular inner condition (see module docstring)."""
    r_if = np.asarray(r_if, dtype=np.float64)
    ri = r_if[0]
    r1 = 0.5 * (r_if[0] + r_if[1])

    def Q(lam):
        pp = 0.5 * (-1.0 + np.sqrt(np.maximum(1.0 - 4.0 * lam, 1.0)))
        return pp * (ri / r1) ** pp
    return _shell_matrix_function(th_if, nphi, Q)


def assemble_parts(r_if, th_if, nphi, inner="zero_flux"):
    """Dense L = L_local + L_boundary (Sec. 3.1), each (nr*nth*nphi)^2.

    L_local holds the face couplings between neighbouring cells (the local
    stencil of the flux form); L_boundary the outer boundary face of the
    outermost shell, which couples every cell of that shell to the whole
    shell through P(A), and, for inner="regular" with r_{1/2} > 0, the inner
    face of the innermost shell through Q(A) (see the module docstring).
    """
    if inner not in ("zero_flux", "regular"):
        raise ValueError("inner must be 'zero_flux' or 'regular'")
    r_if, th_if, r, th, dphi = _cells(r_if, th_if, nphi)
    nr, nth = r.size, th.size
    n = nr * nth * nphi
    L = np.zeros((n, n))
    Lo = np.zeros((n, n))
    idx = lambda i, j, k: (i * nth + j) * nphi + (k % nphi)
    P = outer_face_operator(r_if, th_if, nphi)
    Q = inner_face_operator(r_if, th_if, nphi) if inner == "regular" and r_if[0] > 0.0 else None
    for i in range(nr):
        rm, rp = r_if[i], r_if[i + 1]
        for j in range(nth):
            tm, tp = th_if[j], th_if[j + 1]
            dV = (rp ** 3 - rm ** 3) / 3.0 * (np.cos(tm) - np.cos(tp)) * dphi
            for k in range(nphi):
                c = idx(i, j, k)
                coup = []
                # radial faces: area r_f^2 (cos tm - cos tp) dphi
                if i + 1 < nr:
                    coup.append((idx(i + 1, j, k),
                                 rp ** 2 * (np.cos(tm) - np.cos(tp)) * dphi / (r[i + 1] - r[i])))
                if i > 0:
                    coup.append((idx(i - 1, j, k),
                                 rm ** 2 * (np.cos(tm) - np.cos(tp)) * dphi / (r[i] - r[i - 1])))
                # theta faces: area (rp^2 - rm^2)/2 sin(th_f) dphi, distance r_i dth_c
                if j + 1 < nth:
                    coup.append((idx(i, j + 1, k),
                                 0.5 * (rp ** 2 - rm ** 2) * np.sin(tp) * dphi
                                 / (r[i] * (th[j + 1] - th[j]))))
                if j > 0:
                    coup.append((idx(i, j - 1, k),
                                 0.5 * (rp ** 2 - rm ** 2) * np.sin(tm) * dphi
                                 / (r[i] * (th[j] - th[j - 1]))))
                # phi faces: area (rp^2 - rm^2)/2 (tp - tm), distance r_i sin(th_j) dphi
                wphi = 0.5 * (rp ** 2 - rm ** 2) * (tp - tm) / (r[i] * np.sin(th[j]) * dphi)
                coup.append((idx(i, j, k + 1), wphi))
                coup.append((idx(i, j, k - 1), wphi))
                for nb, w in coup:
                    L[c, nb] += w / dV
                    L[c, c] -= w / dV
                if i == nr - 1:
                    # outer face: area ro^2 dOmega_jk times -(1/ro) P(A) Phi_shell
                    area = rp ** 2 * (np.cos(tm) - np.cos(tp)) * dphi
                    row = (j * nphi + k)
                    base = idx(i, 0, 0)
                    Lo[c, base:base + nth * nphi] -= area / rp * P[row] / dV
                if i == 0 and Q is not None:
                    # inner face: flux along +r = area ri^2 dOmega_jk times
                    # (1/ri) Q(A) Phi_shell; it enters cell 0, so -flux / dV
                    area = rm ** 2 * (np.cos(tm) - np.cos(tp)) * dphi
                    row = (j * nphi + k)
                    Lo[c, 0:nth * nphi] -= area / rm * Q[row] / dV
    return L, Lo


def assemble(r_if, th_if, nphi, inner="zero_flux"):
    """Dense L of size (nr*nth*nphi)^2 from the flux form (Sec. 3.1)."""
    L, Lo = assemble_parts(r_if, th_if, nphi, inner)
    return L + Lo


def solve(r_if, th_if, nphi, rho, G=1.0, inner="zero_flux"):
    """Phi = L^-1 (4 pi G rho) by a dense LU solve."""
    rho = np.asarray(rho, dtype=np.float64)
    L = assemble(r_if, th_if, nphi, inner)
    s = 4.0 * np.pi * G * rho.reshape(-1)
    return np.linalg.solve(L, s).reshape(rho.shape)
