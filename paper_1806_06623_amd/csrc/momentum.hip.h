// Momentum-conserving gravitational source term: the force on every cell as
// the surface integral of the gravitational stress tensor
//   T = (grad Phi grad Phi - |grad Phi|^2 I / 2) / (4 pi G),   div T = rho grad Phi
// where Laplacian Phi = 4 pi G rho (the exact discrete solution satisfies the
// flux form of Sec. 3.1 to rounding, the reason the paper gives for writing
// the source terms in conservative form, Sec. 1 and Sec. 6).
//
// Per face (n along the increasing coordinate): the normal component G_n is
// the face difference quotient of the flux form (the outer face: the
// extrapolated derivative of Sec. 3.2, -T_out / r_o^2; the inner face: zero
// flux); each tangential component is the mean of the two adjacent cells'
// centred components (a cell's centred component being the mean of its two
// face quotients in that direction; pole faces and the inner face count as 0;
// a boundary face takes its one cell's).  The face's stress vector is
//   k4 [ (G_n^2 - G_t1^2 - G_t2^2)/2 N + G_n G_t1 T1 + G_n G_t2 T2 ],
// N, T1, T2 the exact integrals of the local unit vectors over the curved face
// (products of the plan's per-index factors), and the force on a cell is
// minus the sum of its outer faces' vectors plus the sum of its inner faces'.
// Every face is evaluated by the same code from the same loads in both cells
// that share it, with floating-point contraction off, so the two values are
// bitwise equal and interior faces cancel exactly in the grid's total.
//
// Thread per (j, k) column and MROWS radial rows; the 3 x 3 (j, k)
// neighbourhoods of three consecutive rows are held in registers and rolled
// down the rows.  HBM-bound: Phi once (neighbours from cache), three fields
// written.
#pragma once
#include <hip/hip_runtime.h>

namespace momentum {

constexpr int THREADS = 256;
constexpr int MROWS = 8;

// Per-index factors of the face integrals and difference quotients (device
// tables of the plan).  Index conventions: r-faces i = 0..N_r (face i - 1/2),
// theta-faces j = 0..N_theta (face j - 1/2), phi-faces k (face k + 1/2).
struct Tables {
    const double* R2;       // [N_r + 1] r_{i-1/2}^2
    const double* ring;     // [N_r]     (r_{i+1/2}^2 - r_{i-1/2}^2) / 2
    const double* invr;     // [N_r]     1 / r_i
    const double* invdr;    // [N_r + 1] 1 / (r_i - r_{i-1}) at interior r-faces, 0 at the inner and outer faces
    const double* is2;      // [N_theta] int sin^2 over the cell
    const double* isc;      // [N_theta] int sin cos
    const double* is;       // [N_theta] int sin (dmu)
    const double* ic;       // [N_theta] int cos
    const double* dth;      // [N_theta] theta_{j+1/2} - theta_{j-1/2}
    const double* invsdp;   // [N_theta] 1 / (sin theta_j dphi)
    const double* invdthc;  // [N_theta + 1] 1 / (theta_j - theta_{j-1}) at interior faces, 0 at the poles
    const double* fst;      // [N_theta + 1] sin theta_{j-1/2} (0 at the poles)
    const double* fct;      // [N_theta + 1] cos theta_{j-1/2}
    const double* jc;       // [N_phi]   sin phi_{k+1/2} - sin phi_{k-1/2}
    const double* js;       // [N_phi]   cos phi_{k-1/2} - cos phi_{k+1/2}
    const double* cp1;      // [N_phi]   cos phi_{k+1/2}
    const double* sp1;      // [N_phi]   sin phi_{k+1/2}
};

struct V3 {
    double x, y, z;
};

#pragma clang fp contract(off)

// The integrated stress vector of one face.
__device__ __forceinline__ V3 stress(double gn, double g1, double g2, V3 N, V3 T1, V3 T2, double k4)
{
    const double a = 0.5 * (gn * gn - g1 * g1 - g2 * g2), b = gn * g1, c = gn * g2;
    return V3{k4 * (a * N.x + b * T1.x + c * T2.x), k4 * (a * N.y + b * T1.y + c * T2.y),
              k4 * (a * N.z + b * T1.z + c * T2.z)};
}

__device__ __forceinline__ double avg(double a, double b) { return 0.5 * (a + b); }

// 3 x 3 neighbourhood of one row: v[dj + 1][dk + 1] = Phi(i, j + dj, k + dk)
// (theta neighbours clamped at the poles, phi periodic).
struct Patch {
    double v[3][3];
};

__global__ __launch_bounds__(THREADS) void k_momentum(const double* __restrict__ phi, const double* __restrict__ tout,
                                                      double* __restrict__ fx, double* __restrict__ fy,
                                                      double* __restrict__ fz, Tables t, int nr, int nth, int nphi,
                                                      double dphi, double k4, double inv_ro2, int gx)
{
    const int plane = nth * nphi;
    const int chunk = blockIdx.x / gx;
    const int e = (blockIdx.x - chunk * gx) * THREADS + threadIdx.x;
    if (e >= plane) return;
    const int j = e / nphi, k = e - j * nphi;
    const int jm = j > 0 ? j - 1 : 0, jp = j + 1 < nth ? j + 1 : nth - 1;
    const int km = k > 0 ? k - 1 : nphi - 1, kp = k + 1 < nphi ? k + 1 : 0;
    const int cols[3] = {jm * nphi, j * nphi, jp * nphi};
    const int kk[3] = {km, k, kp};
    const int i0 = chunk * MROWS;
    const int i1 = i0 + MROWS < nr ? i0 + MROWS : nr;

    auto load = [&](int i, Patch& p) {
        const size_t base = size_t(i < 0 ? 0 : (i < nr ? i : nr - 1)) * plane;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) p.v[a][b] = phi[base + cols[a] + kk[b]];
    };
    // the outer face's normal gradient at the five columns of the plus stencil
    double go[3][3] = {};
    if (i1 == nr) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) go[a][b] = -tout[cols[a] + kk[b]] * inv_ro2;
    }

    // centred components of cell (i, j + a - 1, k + b - 1)
    auto ct_of = [&](const Patch& p, int i, int a, int b) {
        // theta faces j' - 1/2 and j' + 1/2 of column j' = j + a - 1; the
        // neighbour beyond the patch is only needed for a = 0 / 2, which the
        // force never asks for
        const int jj = a == 0 ? jm : a == 1 ? j : jp;
        const double lo = (p.v[a][b] - p.v[a > 0 ? a - 1 : 0][b]) * t.invr[i] * t.invdthc[jj];
        const double hi = (p.v[a < 2 ? a + 1 : 2][b] - p.v[a][b]) * t.invr[i] * t.invdthc[jj + 1];
        return avg(lo, hi);
    };
    auto cp_of = [&](const Patch& p, int i, int a, int b) {
        const int jj = a == 0 ? jm : a == 1 ? j : jp;
        const double lo = (p.v[a][b] - p.v[a][b > 0 ? b - 1 : 0]) * t.invr[i] * t.invsdp[jj];
        const double hi = (p.v[a][b < 2 ? b + 1 : 2] - p.v[a][b]) * t.invr[i] * t.invsdp[jj];
        return avg(lo, hi);
    };
    // radial centred component of cell i at column (a, b): the rows below and
    // above; the inner face's quotient is 0 (invdr[0] = 0), the outer face's
    // comes from go
    auto cr_of = [&](const Patch& below, const Patch& here, const Patch& above, int i, int a, int b) {
        const double lo = (here.v[a][b] - below.v[a][b]) * t.invdr[i];
        const double hi = i + 1 < nr ? (above.v[a][b] - here.v[a][b]) * t.invdr[i + 1] : go[a][b];
        return avg(lo, hi);
    };

    // exact face integrals
    auto rface = [&](int i, V3& N, V3& T1, V3& T2) {   // r-face i - 1/2 of column (j, k)
        const double R2 = t.R2[i], dp = dphi;
        N = V3{R2 * (t.is2[j] * t.jc[k]), R2 * (t.is2[j] * t.js[k]), R2 * (t.isc[j] * dp)};
        T1 = V3{R2 * (t.isc[j] * t.jc[k]), R2 * (t.isc[j] * t.js[k]), R2 * (-(t.is2[j] * dp))};
        T2 = V3{R2 * (t.is[j] * -t.js[k]), R2 * (t.is[j] * t.jc[k]), 0.0};
    };
    auto tface = [&](int i, int jf, V3& N, V3& T1, V3& T2) {   // theta-face jf - 1/2 of row i, column k
        const double rg = t.ring[i], st = t.fst[jf], ct = t.fct[jf];
        N = V3{rg * ((st * ct) * t.jc[k]), rg * ((st * ct) * t.js[k]), rg * (-((st * st) * dphi))};
        T1 = V3{rg * ((st * st) * t.jc[k]), rg * ((st * st) * t.js[k]), rg * ((st * ct) * dphi)};
        T2 = V3{rg * (st * -t.js[k]), rg * (st * t.jc[k]), 0.0};
    };
    auto pface = [&](int i, int kf, V3& N, V3& T1, V3& T2) {   // phi-face kf + 1/2 of row i, column j
        const double rg = t.ring[i], c1 = t.cp1[kf], s1 = t.sp1[kf];
        N = V3{rg * (t.dth[j] * -s1), rg * (t.dth[j] * c1), 0.0};
        T1 = V3{rg * (t.is[j] * c1), rg * (t.is[j] * s1), rg * t.ic[j]};
        T2 = V3{rg * (t.ic[j] * c1), rg * (t.ic[j] * s1), rg * (-t.is[j])};
    };

    Patch pb, ph, pa;   // rows i - 1, i, i + 1
    load(i0 - 1, pb);
    load(i0, ph);
    load(i0 + 1, pa);
    // the lower r-face of the first row (face i0 - 1/2): its tangential parts
    // are the means of cells i0 - 1 and i0 (cell i0's alone at the inner face)
    V3 lowr;
    {
        V3 N, T1, T2;
        rface(i0, N, T1, T2);
        const double gn = (ph.v[1][1] - pb.v[1][1]) * t.invdr[i0];
        double g1, g2;
        if (i0 == 0) {
            g1 = ct_of(ph, i0, 1, 1);
            g2 = cp_of(ph, i0, 1, 1);
        } else {
            g1 = avg(ct_of(pb, i0 - 1, 1, 1), ct_of(ph, i0, 1, 1));
            g2 = avg(cp_of(pb, i0 - 1, 1, 1), cp_of(ph, i0, 1, 1));
        }
        lowr = stress(gn, g1, g2, N, T1, T2, k4);
    }
    for (int i = i0; i < i1; ++i) {
        Patch pn;
        load(i + 2, pn);   // the next row ahead (clamped)
        V3 N, T1, T2;
        // upper r-face i + 1/2 (face index i + 1)
        V3 upr;
        {
            rface(i + 1, N, T1, T2);
            double gn, g1, g2;
            if (i + 1 < nr) {
                gn = (pa.v[1][1] - ph.v[1][1]) * t.invdr[i + 1];
                g1 = avg(ct_of(ph, i, 1, 1), ct_of(pa, i + 1, 1, 1));
                g2 = avg(cp_of(ph, i, 1, 1), cp_of(pa, i + 1, 1, 1));
            } else {
                gn = go[1][1];
                g1 = ct_of(ph, i, 1, 1);
                g2 = cp_of(ph, i, 1, 1);
            }
            upr = stress(gn, g1, g2, N, T1, T2, k4);
        }
        // theta-faces j - 1/2 (face index j) and j + 1/2 (face index j + 1):
        // normal quotient, radial and phi parts as means of the two cells
        V3 lowt, upt;
        {
            tface(i, j, N, T1, T2);
            const double gn = (ph.v[1][1] - ph.v[0][1]) * t.invr[i] * t.invdthc[j];
            const double g1 = avg(cr_of(pb, ph, pa, i, 0, 1), cr_of(pb, ph, pa, i, 1, 1));
            const double g2 = avg(cp_of(ph, i, 0, 1), cp_of(ph, i, 1, 1));
            lowt = stress(gn, g1, g2, N, T1, T2, k4);
        }
        {
            tface(i, j + 1, N, T1, T2);
            const double gn = (ph.v[2][1] - ph.v[1][1]) * t.invr[i] * t.invdthc[j + 1];
            const double g1 = avg(cr_of(pb, ph, pa, i, 1, 1), cr_of(pb, ph, pa, i, 2, 1));
            const double g2 = avg(cp_of(ph, i, 1, 1), cp_of(ph, i, 2, 1));
            upt = stress(gn, g1, g2, N, T1, T2, k4);
        }
        // phi-faces k - 1/2 (that of column k - 1) and k + 1/2
        V3 lowp, upp;
        {
            pface(i, km, N, T1, T2);
            const double gn = (ph.v[1][1] - ph.v[1][0]) * t.invr[i] * t.invsdp[j];
            const double g1 = avg(cr_of(pb, ph, pa, i, 1, 0), cr_of(pb, ph, pa, i, 1, 1));
            const double g2 = avg(ct_of(ph, i, 1, 0), ct_of(ph, i, 1, 1));
            lowp = stress(gn, g1, g2, N, T1, T2, k4);
        }
        {
            pface(i, k, N, T1, T2);
            const double gn = (ph.v[1][2] - ph.v[1][1]) * t.invr[i] * t.invsdp[j];
            const double g1 = avg(cr_of(pb, ph, pa, i, 1, 1), cr_of(pb, ph, pa, i, 1, 2));
            const double g2 = avg(ct_of(ph, i, 1, 1), ct_of(ph, i, 1, 2));
            upp = stress(gn, g1, g2, N, T1, T2, k4);
        }
        const size_t at = size_t(i) * plane + e;
        __builtin_nontemporal_store(-(((upr.x - lowr.x) + (upt.x - lowt.x)) + (upp.x - lowp.x)), fx + at);
        __builtin_nontemporal_store(-(((upr.y - lowr.y) + (upt.y - lowt.y)) + (upp.y - lowp.y)), fy + at);
        __builtin_nontemporal_store(-(((upr.z - lowr.z) + (upt.z - lowt.z)) + (upp.z - lowp.z)), fz + at);
        lowr = upr;
        pb = ph;
        ph = pa;
        pa = pn;
    }
}

#pragma clang fp contract(on)

}  // namespace momentum
