"""The exact discrete solver as the paper states it (Sec. 3.2), in plain FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Steps, in the paper's order:
  1. s = 4 pi G rho (Sec. 3.1, source of the discretised Poisson equation);
  2. Fourier coefficients s~_{ijm} of s along phi, with synthesis
     s_k = sum_m s~_m exp(+2 pi i m k / N_phi) (Sec. 3.2, phi eigenvectors h_m);
  3. for every m, the eigenvectors H_{l,m}(j) and eigenvalues lambda_{Omega,l,m}
     of the theta operator hat-Delta_theta + S_j lambda_{phi,m} (Sec. 3.2),
     orthonormal in the dmu-weighted inner product, so that the inverse of H
     is H^T D with D = diag(dmu_j);
  4. forward projection s^_{ilm} = sum_j (H^-1)_{lj} s~_{ijm};
  5. one tridiagonal radial system per (l, m):
        Delta_r f + R_i lambda_Omega f = s^,
     with the outer face derivative replaced by the extrapolated power-law
     decay f ~ r^{-(1 + sqrt(1 - 4 lambda_Omega))/2} (Sec. 3.2, outer boundary);
  6. inverse projection g_{ijm} = sum_l H_{l,m}(j) f_{ilm};
  7. inverse FFT of g along phi.

Readings of the paper's text used here:
* hat-Delta_theta carries the factor 1/dmu_j that delta V contributes; without
  it the operator would not be the theta part of the flux form divided by R_i;
* hat-Delta_phi is the second difference divided by dphi^2, and its eigenvalue
  is lambda_{phi,m} = -(sin(m dphi/2)/(dphi/2))^2 -- negative: the printed
  formula drops the sign, which would make sqrt(1 - 4 lambda_Omega) complex;
* the radial equation reads Delta_r f + R_i lambda_Omega f = s^ (the printed
  equation drops the f after lambda_Omega);
* the outer condition uses the value f_N in the outermost zone, extrapolated
  to the outer face with the decay law, and the discrete lambda_Omega;
* the inner radial face (the paper is silent on it): zero area when
  r_{1/2} = 0; otherwise either zero flux, or -- the "regular" condition --
  the decay law's counterpart for the source-free region r < r_{1/2}: each
  angular mode is the solution f ~ r^p', p' = (-1 + sqrt(1 - 4 lambda))/2, that
  stays finite at the centre, extrapolated from the innermost zone to the
  face.  Both agree for lambda = 0 (p' = 0).
"""
import numpy as np
from scipy.linalg import eigh_tridiagonal, solve_banded

from .geometry import grid_geometry


def phi_eigenvalues(nphi):
    """lambda_{phi,m} for m = 0..nphi//2 (Sec. 3.2, eigenvalues of hat-Delta_phi)."""
    dphi = 2.0 * np.pi / nphi
    m = np.arange(nphi // 2 + 1)
    return -(np.sin(m * dphi / 2.0) / (dphi / 2.0)) ** 2


def theta_operator(geom, lam_phi):
    """K = D (hat-Delta_theta + S_j lambda_phi) as (diagonal, off-diagonal).

    K is symmetric: off-diagonal K_{j,j+1} = sigma_{j+1/2}; diagonal
    -(sigma_{j-1/2} + sigma_{j+1/2}) + dmu_j S_j lambda_phi.
    """
    sig = geom["sigma"]
    diag = -(sig[:-1] + sig[1:]) + geom["dmu"] * geom["S"] * lam_phi
    off = sig[1:-1].copy()
    return diag, off


def theta_eigensystem(geom, m, driver="stev"):
    """(lambda_Omega[l], H[j, l]) for azimuthal mode m (Sec. 3.2).

    Solves K H = lambda D H through the symmetric tridiagonal matrix
    D^-1/2 K D^-1/2 (scipy's eigh_tridiagonal with LAPACK's implicit QL/QR
    driver 'stev', whose eigenvectors are orthonormal to rounding), then
    H = D^-1/2 V, which makes H^T D H = I.  For m = 0 the null pair is exact
    (see below).  ``driver='stemr'`` (LAPACK's MRRR) is a second, independent
    FP64 eigensolver: the spread between the two measures how well FP64
    determines the solution on a given grid (eigenvalues come with an
    absolute error near eps |K|, a relative one near eps |K| / |lambda| on
    the small eigenvalues that dominate Phi).
    """
    lam_phi = phi_eigenvalues(geom["nphi"])[m]
    diag, off = theta_operator(geom, lam_phi)
    dmu = geom["dmu"]
    w = 1.0 / np.sqrt(dmu)
    lam, vec = eigh_tridiagonal(diag * w * w, off * w[:-1] * w[1:], lapack_driver=driver)
    H = w[:, None] * vec
    if m == 0:
        # No flux crosses the poles (Sec. 3.1), so for m = 0 every row of K
        # sums to zero: the constant is an exact eigenvector with eigenvalue
        # 0, the largest (K is negative semidefinite).  It is used exactly;
        # a computed one is off by about eps |K| / gap, which the large radial
        # response of this mode would carry into Phi.  The other eigenvectors
        # are made exactly D-orthogonal to it.
        i = int(np.argmax(lam))
        c = np.full(dmu.size, 1.0 / np.sqrt(np.sum(dmu)))
        rest = np.arange(dmu.size) != i
        Hr = H[:, rest]
        Hr = Hr - np.outer(c, c @ (dmu[:, None] * Hr))
        H[:, rest] = Hr / np.sqrt(np.sum(dmu[:, None] * Hr * Hr, axis=0))
        H[:, i] = c
        lam = lam.copy()
        lam[i] = 0.0
    return lam, H


def outer_beta(geom, lam):
    """beta(lambda) with  (face flux)/(dmu dphi) = -beta f_N  at the outer face.

    With p = (1 + sqrt(1 - 4 lambda))/2 the derivative at r_{N+1/2} is
    -p f_N (r_{N+1/2}/r_N)^-p / r_{N+1/2}; times the face area r_{N+1/2}^2
    this is -beta f_N with beta = p r_{N+1/2} (r_{N+1/2}/r_N)^-p.
    """
    lam = np.asarray(lam, dtype=np.float64)
    p = 0.5 * (1.0 + np.sqrt(1.0 - 4.0 * lam))
    ro, rn = geom["r_if"][-1], geom["r"][-1]
    return p * ro * (ro / rn) ** (-p)


INNER_CONDITIONS = ("zero_flux", "regular")


def inner_gamma(geom, lam, inner="zero_flux"):
    """gamma(lambda) with (face flux)/(dmu dphi) = gamma f_1 at the inner face.

    Zero for the zero-flux condition and for r_{1/2} = 0 (the face has no
    area).  For the regular condition, with p' = (-1 + sqrt(1 - 4 lambda))/2
    the derivative at r_{1/2} is p' f_1 (r_{1/2}/r_1)^p' / r_{1/2}; times the
    face area r_{1/2}^2 this is gamma f_1, gamma = p' r_{1/2} (r_{1/2}/r_1)^p'.
    """
    if inner not in INNER_CONDITIONS:
        raise ValueError(f"inner condition must be one of {INNER_CONDITIONS}")
    lam = np.asarray(lam, dtype=np.float64)
    ri, r1 = geom["r_if"][0], geom["r"][0]
    if inner == "zero_flux" or ri == 0.0:
        return np.zeros_like(lam)
    pp = 0.5 * (-1.0 + np.sqrt(1.0 - 4.0 * lam))
    return pp * ri * (ri / r1) ** pp


def radial_banded(geom, lam, inner="zero_flux"):
    """The radial operator Delta_r + R_i lambda as a (3, nr) banded matrix.

    Row i: a_i f_{i-1} + b_i f_i + c_i f_{i+1} with a_i = alpha_{i-1}/V_i,
    c_i = alpha_i/V_i, b_i = -(alpha_{i-1} + alpha_i)/V_i + R_i lambda, where
    on the innermost row alpha_{-1} is replaced by gamma(lambda) (zero for the
    zero-flux condition) and a is absent, and on the outermost row alpha_{N}
    is replaced by beta(lambda) and c is absent.
    """
    nr, V, R, al = geom["nr"], geom["V"], geom["R"], geom["alpha"]
    lower = np.concatenate(([inner_gamma(geom, lam, inner)], al))   # alpha_{i-1} / gamma
    upper = np.concatenate((al, [outer_beta(geom, lam)]))   # alpha_i / beta
    ab = np.zeros((3, nr))
    ab[0, 1:] = al / V[:-1]                   # super-diagonal c_i, i = 0..nr-2
    ab[1, :] = -(lower + upper) / V + R * lam
    ab[2, :-1] = al / V[1:]                   # sub-diagonal a_{i+1}
    return ab


class Plan:
    """Set-up part of the method: geometry and all per-m theta eigensystems.

    The paper computes the eigenvectors once when the solver is set up
    (Sec. 3.2); ``solve`` then repeats steps 1-7 for any source.
    """

    def __init__(self, r_if, th_if, nphi, driver="stev", inner="zero_flux"):
        self.geom = grid_geometry(r_if, th_if, nphi)
        self.nphi = nphi
        self.inner = inner
        self.modes = [theta_eigensystem(self.geom, m, driver) for m in range(nphi // 2 + 1)]

    def forward_fft(self, s):
        """s~_{ijm}, m = 0..nphi//2, normalised for synthesis without 1/N."""
        return np.fft.rfft(s, axis=2) / self.nphi

    def inverse_fft(self, g):
        """Phi_k = sum over all m of g_m exp(+2 pi i m k/N) for real Phi."""
        return np.fft.irfft(g, n=self.nphi, axis=2) * self.nphi

    def solve_modes(self, st):
        """Steps 4-6 for every m: s~ (nr, nth, M) complex -> g, same shape."""
        geom = self.geom
        g = np.empty_like(st)
        for m, (lam, H) in enumerate(self.modes):
            Hinv = H.T * geom["dmu"][None, :]             # H^-1 = H^T D
            sh = Hinv @ st[:, :, m].T                      # (l, i)
            f = np.empty_like(sh)
            for l in range(lam.size):
                rhs = np.stack([sh[l].real, sh[l].imag], axis=1)
                sol = solve_banded((1, 1), radial_banded(geom, lam[l], self.inner), rhs)
                f[l] = sol[:, 0] + 1j * sol[:, 1]
            g[:, :, m] = (H @ f).T
        return g

    def solve(self, rho, G=1.0):
        """Phi for density rho of shape (nr, nth, nphi)."""
        s = 4.0 * np.pi * G * np.asarray(rho, dtype=np.float64)
        return self.inverse_fft(self.solve_modes(self.forward_fft(s)))


def solve(r_if, th_if, nphi, rho, G=1.0, driver="stev", inner="zero_flux"):
    """One-shot convenience wrapper: Plan(r_if, th_if, nphi).solve(rho, G)."""
    return Plan(r_if, th_if, nphi, driver, inner).solve(rho, G)
