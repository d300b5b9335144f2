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
// Thread per (j, k) column and MROWS radial rows (plane blocks in the
// XCD-aware order of spp_plane_block).  Per row a thread forms every centred
// component it needs once (radial ones at the five columns of its plus
// stencil, theta and phi ones at the three cells along each direction), the
// radial quotients of a face are carried from one row to the next, and the
// r-face between two rows is evaluated once; the theta- and phi-faces are
// evaluated by both cells that share them.  Phi is read once from HBM (the
// neighbours' values from cache), three fields are written.
#pragma once
#include <hip/hip_runtime.h>

#include "xcd.h"

namespace momentum {

constexpr int THREADS = 256;
constexpr int MROWS = 8;        // radial rows per thread (k_momentum)
constexpr int ROWS_LDS = 8;     // radial rows per thread (k_momentum_rows)

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

// The scalars of a face's stress vector: with s = k4 times the face's radial
// factor (r^2 of an r-face, the ring factor of a theta- or phi-face),
//   a = s (G_n^2 - G_t1^2 - G_t2^2) / 2,  b = s G_n G_t1,  c = s G_n G_t2,
// so that the integrated vector is a N + b T1 + c T2 (N, T1, T2 the angular
// parts of the face's unit-vector integrals).
struct Abc {
    double a, b, c;
};

__device__ __forceinline__ Abc scalars(double gn, double g1, double g2, double s, double hs)
{
    const double sg = s * gn;
    return Abc{hs * ((gn * gn - g1 * g1) - g2 * g2), sg * g1, sg * g2};
}

// r-face of column (j, k): N = (S2 jc, S2 js, SC dphi), T1 = (SC jc, SC js,
// -S2 dphi), T2 = (-SN js, SN jc, 0) with S2, SC, SN the integrals of sin^2,
// sin cos and sin over the cell's theta range and jc, js the differences of
// sin and cos phi over its phi range, collected as
//   x = jc u - js v,  y = js u + jc v,  z = dphi (a SC - b S2),  u = a S2 + b SC,  v = c SN.
__device__ __forceinline__ V3 rvec(const Abc& q, double S2, double SC, double SN, double jc, double js, double dphi)
{
    const double u = q.a * S2 + q.b * SC, v = q.c * SN;
    return V3{jc * u - js * v, js * u + jc * v, dphi * (q.a * SC - q.b * S2)};
}

// theta-face at theta_f (st = sin, ct = cos): N = (st ct jc, st ct js,
// -st^2 dphi), T1 = (st^2 jc, st^2 js, st ct dphi), T2 = (-st js, st jc, 0).
__device__ __forceinline__ V3 tvec(const Abc& q, double sct, double ss, double st, double jc, double js, double dphi)
{
    const double u = q.a * sct + q.b * ss, v = q.c * st;
    return V3{jc * u - js * v, js * u + jc * v, dphi * (q.b * sct - q.a * ss)};
}

// phi-face at phi_f (c1 = cos, s1 = sin) of a cell with theta width D and
// sin / cos integrals SN, CS: N = (-D s1, D c1, 0), T1 = (SN c1, SN s1, CS),
// T2 = (CS c1, CS s1, -SN).
__device__ __forceinline__ V3 pvec(const Abc& q, double D, double SN, double CS, double c1, double s1)
{
    const double w = q.b * SN + q.c * CS, ad = q.a * D;
    return V3{c1 * w - s1 * ad, s1 * w + c1 * ad, q.b * CS - q.c * SN};
}

__device__ __forceinline__ double avg(double a, double b) { return 0.5 * (a + b); }

// Centred gradient components of the cells a thread needs in one row i:
// radial ones at the five columns of the plus stencil (0 own, 1 j-1, 2 j+1,
// 3 k-1, 4 k+1), theta ones at (j, k-1), (j, k), (j, k+1), phi ones at
// (j-1, k), (j, k), (j+1, k); the own column's face quotients in theta and
// phi (the normal components of its theta- and phi-faces) and the radial
// quotients of the upper face i + 1/2 at the five columns (the lower face's
// for row i + 1).
struct RowComps {
    double cr[5], ct[3], cp[3];
    double gtl, gth, gpl, gph;
    double grh[5];
};

// ROW_WAVES: every wave lies within one theta row (N_phi a multiple of 64),
// so j and everything that depends on it are wave-uniform and live in
// scalar registers.
// At most 168 VGPRs (three waves per SIMD, a few values spilled): the
// arithmetic chains of a row need the latency hiding more than the registers.
template <bool ROW_WAVES>
__global__ __launch_bounds__(THREADS, 3) void k_momentum(const double* __restrict__ phi, const double* __restrict__ tout,
                                                      double* __restrict__ fx, double* __restrict__ fy,
                                                      double* __restrict__ fz, Tables t, int nr, int nth, int nphi,
                                                      double dphi, double k4, double inv_ro2, int gx)
{
    const int plane = nth * nphi;
    const int chunk = blockIdx.x / gx;
    const int e = spp_plane_block(blockIdx.x - chunk * gx, gx) * THREADS + threadIdx.x;
    if (e >= plane) return;
    const int jl = e / nphi, k = e - jl * nphi;
    const int j = ROW_WAVES ? __builtin_amdgcn_readfirstlane(jl) : jl;
    const int jm = j > 0 ? j - 1 : 0, jp = j + 1 < nth ? j + 1 : nth - 1;
    const int km = k > 0 ? k - 1 : nphi - 1, kp = k + 1 < nphi ? k + 1 : 0;
    // 32-bit byte offsets of the 3 x 3 patch within a row of the field (a row
    // of at most 2^29 elements)
    unsigned off[3][3];
    {
        const unsigned rowo[3] = {unsigned(jm * nphi), unsigned(j * nphi), unsigned(jp * nphi)};
        const unsigned colo[3] = {unsigned(km), unsigned(k), unsigned(kp)};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) off[a][b] = (rowo[a] + colo[b]) * 8u;   // bytes
    }
    const int i0 = chunk * MROWS;
    const int i1 = i0 + MROWS < nr ? i0 + MROWS : nr;
    // plus-stencil column c as (theta row a, phi column b) of the 3 x 3 patch
    constexpr int PA[5] = {1, 0, 2, 1, 1}, PB[5] = {1, 1, 1, 0, 2};

    // the per-column factors, read once (the table pointers may alias the
    // outputs as far as the compiler knows)
    const double jck = t.jc[k], jsk = t.js[k];
    const double S2 = t.is2[j], SC = t.isc[j], SN = t.is[j], CS = t.ic[j], D = t.dth[j];
    const double stl = t.fst[j], sth = t.fst[j + 1];
    const double sctl = stl * t.fct[j], ssl = stl * stl, scth = sth * t.fct[j + 1], ssh = sth * sth;
    const double c1l = t.cp1[km], s1l = t.sp1[km], c1h = t.cp1[k], s1h = t.sp1[k];
    const double qtl = t.invdthc[j], qth = t.invdthc[j + 1];
    const double qp[3] = {t.invsdp[jm], t.invsdp[j], t.invsdp[jp]};


    // the components of row i from its 3 x 3 patch P, the radial quotients of
    // its lower face (grl) and of its upper face (grh) at the five columns
    auto comps = [&](int i, const double (&P)[3][3], const double (&grl)[5], const double (&grh)[5], RowComps& C) {
        const double ir = t.invr[i];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            C.grh[c] = grh[c];
            C.cr[c] = avg(grl[c], grh[c]);
        }
        const double rtl = ir * qtl, rth = ir * qth;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double lo = (P[1][b] - P[0][b]) * rtl, hi = (P[2][b] - P[1][b]) * rth;
            C.ct[b] = avg(lo, hi);
            if (b == 1) {
                C.gtl = lo;
                C.gth = hi;
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double rp = ir * qp[a];
            const double lo = (P[a][1] - P[a][0]) * rp, hi = (P[a][2] - P[a][1]) * rp;
            C.cp[a] = avg(lo, hi);
            if (a == 1) {
                C.gpl = lo;
                C.gph = hi;
            }
        }
    };
    // row i of the field (clamped into range: rows outside are never used)
    auto load_patch = [&](int i, double (&P)[3][3]) {
        const char* __restrict__ row =
            reinterpret_cast<const char*>(phi + size_t(i < 0 ? 0 : (i < nr ? i : nr - 1)) * plane);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) P[a][b] = *reinterpret_cast<const double*>(row + off[a][b]);
    };
    // radial quotients of face i + 1/2 (rows i and i + 1 at the five columns;
    // the outer face's extrapolated derivative for i = N_r - 1)
    auto rquot = [&](int i, const double (&P)[3][3], const double (&Q)[3][3], double (&g)[5]) {
        if (i + 1 < nr) {
            const double f = t.invdr[i + 1];
#pragma unroll
            for (int c = 0; c < 5; ++c) g[c] = (Q[PA[c]][PB[c]] - P[PA[c]][PB[c]]) * f;
        } else {
#pragma unroll
            for (int c = 0; c < 5; ++c)
                g[c] = -*reinterpret_cast<const double*>(reinterpret_cast<const char*>(tout) + off[PA[c]][PB[c]]) * inv_ro2;
        }
    };

    // prologue: rows i0 - 1, i0 and i0 + 1 (each later row's patch is loaded in
    // the iteration that first uses it: a patch kept in flight across
    // iterations would cost the third wave per SIMD)
    double Pb[3][3], P[3][3], Pn[3][3], grl[5], grh[5];
    RowComps C;
    V3 lowr;
    load_patch(i0 - 1, Pb);
    load_patch(i0, P);
    load_patch(i0 + 1, Pn);
    {
        const double f = t.invdr[i0];   // 0 at the inner face
#pragma unroll
        for (int c = 0; c < 5; ++c) grl[c] = (P[PA[c]][PB[c]] - Pb[PA[c]][PB[c]]) * f;
        rquot(i0, P, Pn, grh);
        comps(i0, P, grl, grh, C);
        // the chunk's lower r-face i0 - 1/2: tangential parts the means of
        // cells i0 - 1 and i0 (cell i0's alone at the inner face)
        double g1 = C.ct[1], g2 = C.cp[1];
        if (i0 > 0) {
            RowComps Cb;
            comps(i0 - 1, Pb, grl, grl, Cb);   // its theta and phi parts only are used
            g1 = avg(Cb.ct[1], C.ct[1]);
            g2 = avg(Cb.cp[1], C.cp[1]);
        }
        const double s = k4 * t.R2[i0];
        lowr = rvec(scalars(grl[0], g1, g2, s, 0.5 * s), S2, SC, SN, jck, jsk, dphi);
    }

    for (int i = i0; i < i1; ++i) {
        // theta- and phi-faces of row i
        const double sr = k4 * t.ring[i], hsr = 0.5 * sr;
        const V3 lowt = tvec(scalars(C.gtl, avg(C.cr[1], C.cr[0]), avg(C.cp[0], C.cp[1]), sr, hsr), sctl, ssl, stl,
                             jck, jsk, dphi);
        const V3 upt = tvec(scalars(C.gth, avg(C.cr[0], C.cr[2]), avg(C.cp[1], C.cp[2]), sr, hsr), scth, ssh, sth,
                            jck, jsk, dphi);
        const V3 lowp = pvec(scalars(C.gpl, avg(C.cr[3], C.cr[0]), avg(C.ct[0], C.ct[1]), sr, hsr), D, SN, CS, c1l, s1l);
        const V3 upp = pvec(scalars(C.gph, avg(C.cr[0], C.cr[4]), avg(C.ct[1], C.ct[2]), sr, hsr), D, SN, CS, c1h, s1h);
        const V3 side{(upt.x - lowt.x) + (upp.x - lowp.x), (upt.y - lowt.y) + (upp.y - lowp.y),
                      (upt.z - lowt.z) + (upp.z - lowp.z)};
        // upper r-face i + 1/2: the next row's components first (the outer
        // face of the last row takes its one cell's tangential parts)
        double g1 = C.ct[1], g2 = C.cp[1];
        const double gn = C.grh[0];
        if (i + 1 < nr) {
            double Pnn[3][3], gnx[5];
            load_patch(i + 2, Pnn);
            rquot(i + 1, Pn, Pnn, gnx);
            RowComps Cn;
            comps(i + 1, Pn, C.grh, gnx, Cn);
            g1 = avg(C.ct[1], Cn.ct[1]);
            g2 = avg(C.cp[1], Cn.cp[1]);
            C = Cn;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) Pn[a][b] = Pnn[a][b];
        }
        const double s = k4 * t.R2[i + 1];
        const V3 upr = rvec(scalars(gn, g1, g2, s, 0.5 * s), S2, SC, SN, jck, jsk, dphi);
        const size_t o = size_t(i) * plane + e;
        __builtin_nontemporal_store(-((upr.x - lowr.x) + side.x), fx + o);
        __builtin_nontemporal_store(-((upr.y - lowr.y) + side.y), fy + o);
        __builtin_nontemporal_store(-((upr.z - lowr.z) + side.z), fz + o);
        lowr = upr;
    }
}

// Workgroups that hold whole theta rows (64 <= N_phi <= THREADS, N_phi
// dividing THREADS): every cell's phi neighbours are in its workgroup.  The
// cells of a row then exchange through LDS what both sides of a phi-face need,
// instead of each recomputing its neighbours': Phi of its column at theta rows
// j-1, j, j+1 (the neighbours' phi quotients), its radial and theta centred
// components, and its upper phi-face's stress vector, which the next cell
// takes as its lower one (each phi-face evaluated once).  Theta-faces are
// still evaluated by both cells, by the same code from the same values; the
// r-face between two rows once.  Two barriers per row: after the centred
// components (the row's Phi having been exchanged in the previous row's
// step), and after the phi-faces.  Phi is double-buffered in LDS by row.
// Threads past the end of the plane (a last workgroup with whole rows past
// N_theta; PARTIAL launches only) take part in the barriers and store nothing.
// The row loop is unrolled and reads its per-row factors from LDS, and with
// PARTIAL = false the stores are unconditional: the only global loads after
// the prologue are the rows of Phi, so that waiting for them never waits for
// a store as well.
template <bool PARTIAL>
__global__ __launch_bounds__(THREADS) void k_momentum_rows(const double* __restrict__ phi,
                                                           const double* __restrict__ tout, double* __restrict__ fx,
                                                           double* __restrict__ fy, double* __restrict__ fz, Tables t,
                                                           int nr, int nth, int nphi, double dphi, double k4,
                                                           double inv_ro2, int gx)
{
    __shared__ double sphi[2][3][THREADS];   // Phi of row i (buffer i % 2) at theta rows j-1, j, j+1, per cell
    __shared__ double scomp[2][THREADS];     // radial and theta centred components of the current row, per cell
    __shared__ double sface[3][THREADS];     // the upper phi-face's stress vector, per cell
    // per-row factors of the chunk, rows i0 .. i0 + ROWS_LDS (clamped):
    // 1/r_i, 1/dr of face i + 1/2, the ring factor of row i, r^2 of face i + 1/2
    __shared__ double srow[4][ROWS_LDS + 1];
    const int plane = nth * nphi;
    const int chunk = blockIdx.x / gx;
    const int tid = threadIdx.x;
    const int e = spp_plane_block(blockIdx.x - chunk * gx, gx) * THREADS + tid;
    const bool valid = e < plane;
    const int jl = e / nphi, k = e - jl * nphi;
    const int jw = __builtin_amdgcn_readfirstlane(jl);   // every wave lies within one theta row
    const int j = jw < nth ? jw : nth - 1;
    const int jm = j > 0 ? j - 1 : 0, jp = j + 1 < nth ? j + 1 : nth - 1;
    const int ln = k > 0 ? tid - 1 : tid + nphi - 1;      // LDS slot of the cell k - 1 (periodic)
    const int rn = k + 1 < nphi ? tid + 1 : tid - nphi + 1;
    const int ec = valid ? k : 0;
    const int col[3] = {jm * nphi + ec, j * nphi + ec, jp * nphi + ec};
    const int i0 = chunk * ROWS_LDS;
    const int i1 = i0 + ROWS_LDS < nr ? i0 + ROWS_LDS : nr;
    if (tid < 4 * (ROWS_LDS + 1)) {
        const int a = tid / (ROWS_LDS + 1), ii = i0 + tid - a * (ROWS_LDS + 1);
        const int c0 = ii < nr ? ii : nr - 1, c1 = ii + 1 < nr ? ii + 1 : nr;
        srow[a][tid - a * (ROWS_LDS + 1)] =
            a == 0 ? t.invr[c0] : a == 1 ? t.invdr[c1] : a == 2 ? t.ring[c0] : t.R2[c1];
    }

    const double jck = t.jc[ec], jsk = t.js[ec], c1 = t.cp1[ec], s1 = t.sp1[ec];
    const double S2 = t.is2[j], SC = t.isc[j], SN = t.is[j], CS = t.ic[j], D = t.dth[j];
    const double stl = t.fst[j], sth = t.fst[j + 1];
    const double sctl = stl * t.fct[j], ssl = stl * stl, scth = sth * t.fct[j + 1], ssh = sth * sth;
    const double qtl = t.invdthc[j], qth = t.invdthc[j + 1];
    const double qp[3] = {t.invsdp[jm], t.invsdp[j], t.invsdp[jp]};

    auto column = [&](int i, double (&v)[3]) {
        const double* __restrict__ row = phi + size_t(i < 0 ? 0 : (i < nr ? i : nr - 1)) * plane;
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] = row[col[a]];
    };
    auto publish = [&](int i, const double (&v)[3]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) sphi[i & 1][a][tid] = v[a];
    };
    // the own column's theta and phi centred components of row i (ir = 1/r_i)
    // from its column values v and the neighbours' published ones
    auto own_tp = [&](int i, double ir, const double (&v)[3], double& ct, double& cp, double& gtl, double& gth,
                      double& gpl, double& gph) {
        gtl = (v[1] - v[0]) * (ir * qtl);
        gth = (v[2] - v[1]) * (ir * qth);
        ct = avg(gtl, gth);
        const double rp = ir * qp[1];
        gpl = (v[1] - sphi[i & 1][1][ln]) * rp;
        gph = (sphi[i & 1][1][rn] - v[1]) * rp;
        cp = avg(gpl, gph);
    };
    // radial quotients of face i + 1/2 at the three columns (f = its 1/dr;
    // the outer face: the extrapolated derivative, from to[])
    double to[3] = {0.0, 0.0, 0.0};
    if (i1 == nr) {
#pragma unroll
        for (int a = 0; a < 3; ++a) to[a] = tout[col[a]];
    }
    auto rquot = [&](int i, double f, const double (&v)[3], const double (&w)[3], double (&g)[3]) {
        if (i + 1 < nr) {
#pragma unroll
            for (int a = 0; a < 3; ++a) g[a] = (w[a] - v[a]) * f;
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) g[a] = -to[a] * inv_ro2;
        }
    };

    // prologue: rows i0 - 1, i0 (published) and i0 + 1; the chunk's lower
    // r-face i0 - 1/2 (tangential parts the means of cells i0 - 1 and i0,
    // cell i0's alone at the inner face)
    double prev[3], cur[3], nxt[3], grl[3];
    // theta and phi components of the current row (and its face quotients),
    // computed once: as the next row's while the row below forms its upper
    // r-face, then carried into that row's own iteration
    double o_ct, o_cp, o_gtl, o_gth, o_gpl, o_gph;
    column(i0 - 1, prev);
    column(i0, cur);
    column(i0 + 1, nxt);
    publish(i0 - 1, prev);
    publish(i0, cur);
    __syncthreads();
    V3 lowr;
    {
        const double f = t.invdr[i0];   // 0 at the inner face
#pragma unroll
        for (int a = 0; a < 3; ++a) grl[a] = (cur[a] - prev[a]) * f;
        own_tp(i0, t.invr[i0], cur, o_ct, o_cp, o_gtl, o_gth, o_gpl, o_gph);
        const double ct0 = o_ct, cp0 = o_cp;
        double g1 = ct0, g2 = cp0;
        if (i0 > 0) {
            double ctb, cpb, x0, x1, x2, x3;
            own_tp(i0 - 1, t.invr[i0 - 1], prev, ctb, cpb, x0, x1, x2, x3);
            g1 = avg(ctb, ct0);
            g2 = avg(cpb, cp0);
        }
        const double sr = k4 * t.R2[i0];
        lowr = rvec(scalars(grl[1], g1, g2, sr, 0.5 * sr), S2, SC, SN, jck, jsk, dphi);
    }
    __syncthreads();   // the buffer of row i0 - 1 is rewritten with row i0 + 1 below

#pragma unroll
    for (int r = 0; r < ROWS_LDS; ++r) {
        const int i = i0 + r;
        if (i >= i1) break;
        double nn[3];
        column(i + 2, nn);    // in flight through this row
        publish(i + 1, nxt);
        // row i: radial components at the three columns, theta and phi ones
        // of the own column, phi ones of the columns j -+ 1
        double grh[3], cr[3], cp[3];
        rquot(i, srow[1][r], cur, nxt, grh);
#pragma unroll
        for (int a = 0; a < 3; ++a) cr[a] = avg(grl[a], grh[a]);
        const double ct = o_ct, gtl = o_gtl, gth = o_gth, gph = o_gph;
        cp[1] = o_cp;
        const double ir = srow[0][r];
#pragma unroll
        for (int a = 0; a < 3; a += 2) {
            const double rp = ir * qp[a];
            cp[a] = avg((cur[a] - sphi[i & 1][a][ln]) * rp, (sphi[i & 1][a][rn] - cur[a]) * rp);
        }
        scomp[0][tid] = cr[1];
        scomp[1][tid] = ct;
        __syncthreads();

        const double sr = k4 * srow[2][r], hsr = 0.5 * sr;
        // upper phi-face k + 1/2, evaluated here once
        const V3 upp = pvec(scalars(gph, avg(cr[1], scomp[0][rn]), avg(ct, scomp[1][rn]), sr, hsr), D, SN, CS, c1, s1);
        sface[0][tid] = upp.x;
        sface[1][tid] = upp.y;
        sface[2][tid] = upp.z;
        // theta-faces j - 1/2 and j + 1/2
        const V3 lowt = tvec(scalars(gtl, avg(cr[0], cr[1]), avg(cp[0], cp[1]), sr, hsr), sctl, ssl, stl, jck, jsk,
                             dphi);
        const V3 upt = tvec(scalars(gth, avg(cr[1], cr[2]), avg(cp[1], cp[2]), sr, hsr), scth, ssh, sth, jck, jsk,
                            dphi);
        // upper r-face i + 1/2: the next row's own theta and phi components
        // (its Phi published above), or the cell's own at the outer face
        double g1 = ct, g2 = cp[1];
        if (i + 1 < nr) {
            own_tp(i + 1, srow[0][r + 1], nxt, o_ct, o_cp, o_gtl, o_gth, o_gpl, o_gph);
            g1 = avg(ct, o_ct);
            g2 = avg(cp[1], o_cp);
        }
        const double srr = k4 * srow[3][r];
        const V3 upr = rvec(scalars(grh[1], g1, g2, srr, 0.5 * srr), S2, SC, SN, jck, jsk, dphi);
        __syncthreads();

        // lower phi-face k - 1/2: the cell k - 1's upper one
        const V3 lowp{sface[0][ln], sface[1][ln], sface[2][ln]};
        if (!PARTIAL || valid) {
            const size_t o = size_t(i) * plane + e;
            __builtin_nontemporal_store(-(((upr.x - lowr.x) + (upt.x - lowt.x)) + (upp.x - lowp.x)), fx + o);
            __builtin_nontemporal_store(-(((upr.y - lowr.y) + (upt.y - lowt.y)) + (upp.y - lowp.y)), fy + o);
            __builtin_nontemporal_store(-(((upr.z - lowr.z) + (upt.z - lowt.z)) + (upp.z - lowp.z)), fz + o);
        }
        lowr = upr;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            grl[a] = grh[a];
            cur[a] = nxt[a];
            nxt[a] = nn[a];
        }
    }
}

#pragma clang fp contract(on)

}  // namespace momentum
