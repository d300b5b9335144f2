// Face fluxes of grad Phi through every cell face: the terms of the
// finite-volume operator of Sec. 3.1, whose sum over the faces of a cell is
// (Delta Phi) delta V.  For the exact discrete solution that sum is
// 4 pi G rho delta V, the property that conservative gravitational source
// terms rest on (Sec. 1, Sec. 3.1).  With the plan's tables
//   Fr[i][j][k] = alpha_i dmu_j dphi (Phi[i+1][j][k] - Phi[i][j][k])     i < N_r - 1
//   Fr[N_r-1][j][k] = -dmu_j dphi T[j][k]    (outer face, Sec. 3.2; T = beta(A) Phi_shell)
//   Ft[i][j][k] = (V R)_i sigma_{j+1/2} dphi (Phi[i][j+1][k] - Phi[i][j][k])   (0 at the pole face)
//   Fp[i][j][k] = (V R)_i S_j dmu_j / dphi (Phi[i][j][k+1] - Phi[i][j][k])    (k + 1 periodic)
// where alpha_i = r_{i+1/2}^2 / (r_{i+1} - r_i), (V R)_i = (r_{i+1/2}^2 -
// r_{i-1/2}^2) / (2 r_i), sigma_{j+1/2} = sin th_{j+1/2} / (th_{j+1} - th_j)
// and S_j dmu_j = (th_{j+1/2} - th_{j-1/2}) / sin th_j.
//
// HBM-bound: one read of Phi, three fields written.  A thread owns one
// (j, k) column and ROWS consecutive radial rows: it issues the loads of all
// its rows (plus the next row) and of their theta and phi neighbours before
// the first store, so each thread keeps ~3 ROWS loads in flight.  The
// neighbours are rows that adjacent threads load and come from cache.
// Consecutive threads run along phi, so every load and store of a wave
// covers 512 contiguous bytes.  The flux fields are stored non-temporally
// (three times the size of Phi, nothing rereads them here), which keeps them
// from evicting the rows of Phi that neighbouring workgroups still read.
#pragma once
#include <hip/hip_runtime.h>

#include "xcd.h"

namespace faceflux {

constexpr int THREADS = 256;
constexpr int ROWS = 8;    // radial rows per thread (k_face_fluxes)
constexpr int BATCH = 16;  // matrix loads in flight per thread (k_shell_apply)

struct Tables {
    const double* alpha;   // [N_r], alpha[N_r - 1] = 0
    const double* VR;      // [N_r]
    const double* sig;     // [N_theta + 1], faces j - 1/2 (both poles 0)
    const double* dmu;     // [N_theta]
    const double* Sj;      // [N_theta]
};

// One-dimensional grid of gx * ceil(N_r / ROWS) workgroups, gx =
// ceil(N_theta N_phi / THREADS) blocks of the (j, k) plane per chunk of rows,
// in the XCD-aware order of spp_plane_block.  `outer` holds the boundary
// term T[j][k] of the outermost shell.  Row indices past N_r - 1 are clamped
// for the loads (those values are never used) and skipped for the stores.
__global__ __launch_bounds__(THREADS) void k_face_fluxes(const double* __restrict__ phi,
                                                         const double* __restrict__ outer,
                                                         double* __restrict__ fr, double* __restrict__ ft,
                                                         double* __restrict__ fp, Tables t, int nr, int nth,
                                                         int nphi, double dphi, int gx)
{
    const int plane = nth * nphi;
    const int chunk = blockIdx.x / gx;
    const int e = spp_plane_block(blockIdx.x - chunk * gx, gx) * THREADS + threadIdx.x;
    if (e >= plane) return;
    const int j = e / nphi;
    const int k = e - j * nphi;
    const int ek = k + 1 < nphi ? e + 1 : e + 1 - nphi;   // phi neighbour k + 1, periodic
    const int ej = j + 1 < nth ? e + nphi : e;            // theta neighbour (itself at the pole face)
    const int i0 = chunk * ROWS;

    double c[ROWS + 1], nk[ROWS], nj[ROWS];
#pragma unroll
    for (int r = 0; r <= ROWS; ++r) c[r] = phi[size_t(min(i0 + r, nr - 1)) * plane + e];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const size_t row = size_t(min(i0 + r, nr - 1)) * plane;
        nk[r] = phi[row + ek];
        nj[r] = phi[row + ej];
    }
    const double ob = i0 + ROWS >= nr ? outer[e] : 0.0;   // only the chunk with the last row uses it

    const double cr = t.dmu[j] * dphi;
    const double ct = t.sig[j + 1] * dphi;
    const double cp = t.Sj[j] * t.dmu[j] / dphi;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int i = i0 + r;
        if (i < nr) {
            const size_t at = size_t(i) * plane + e;
            const double vr = t.VR[i];
            __builtin_nontemporal_store(i + 1 < nr ? t.alpha[i] * cr * (c[r + 1] - c[r]) : -cr * ob, fr + at);
            __builtin_nontemporal_store(vr * ct * (nj[r] - c[r]), ft + at);
            __builtin_nontemporal_store(vr * cp * (nk[r] - c[r]), fp + at);
        }
    }
}

// Boundary term of Sec. 3.2 on a shell, per Fourier mode m:
//   ob_q = H_m diag(c_m) H_m^T D g_q
// (c = beta on the outermost shell; c = gamma on the innermost one with the
// regular inner condition) for the components q = m and q = N_phi - m of m
// (one component for m = 0 and m = N_phi / 2).  The plan stores each
// B_m = H_m diag(c_m) H_m^T D as one N_theta x N_theta matrix, transposed, so
// that k_shell_apply forms ob_q = B_m g_q in one product; workgroup (m, b)
// computes the 32 outputs 32 b .. 32 b + 31 of both components of m from one
// pass over 32 columns of the stored matrix, so the (N_phi/2 + 1) x
// ceil(N_theta/32) workgroups share the matrix bytes.  Vectors are
// [q][N_theta] (g_q may be strided: g + q gq).  Dynamic LDS: (2 N_theta +
// 512) doubles.

// y = A^T x for the 32 outputs o0 .. o0 + 31 and two vectors x0, x1 (LDS):
// thread (o, sp) = (tid % 32, tid / 32) sums the rows x = sp, sp + 8, ...
// with BATCH loads in flight, and the 8 partial sums meet in LDS.  Columns
// past N_theta are clamped for the loads and their results dropped.
__device__ __forceinline__ void cols32(const double* __restrict__ A, const double* x0, const double* x1, int o0,
                                       int nth, double* part, double& y0, double& y1)
{
    const int tid = threadIdx.x, o = tid & 31, sp = tid >> 5;
    const int col = min(o0 + o, nth - 1);
    double a0 = 0.0, a1 = 0.0;
    for (int xb = sp; xb < nth; xb += 8 * BATCH) {
        double a[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int x = xb + 8 * u;
            a[u] = x < nth ? A[size_t(x) * nth + col] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int x = min(xb + 8 * u, nth - 1);   // a[u] = 0 past the end
            a0 += a[u] * x0[x];
            a1 += a[u] * x1[x];
        }
    }
    part[sp * 32 + o] = a0;
    part[256 + sp * 32 + o] = a1;
    __syncthreads();
    y0 = 0.0;
    y1 = 0.0;
    if (tid < 32) {
        for (int y = 0; y < 8; ++y) {
            y0 += part[y * 32 + tid];
            y1 += part[256 + y * 32 + tid];
        }
    }
}

__global__ __launch_bounds__(256) void k_shell_apply(const double* __restrict__ g, size_t gq,
                                                     double* __restrict__ ob, const double* __restrict__ B, int nth,
                                                     int nphi)
{
    extern __shared__ double sh[];
    double* x0 = sh;
    double* x1 = sh + nth;
    const int m = blockIdx.x, o0 = blockIdx.y * 32;
    const bool two = m > 0 && 2 * m < nphi;
    const int q1 = nphi - m;
    for (int j = threadIdx.x; j < nth; j += 256) {
        x0[j] = g[size_t(m) * gq + j];
        x1[j] = two ? g[size_t(q1) * gq + j] : 0.0;
    }
    __syncthreads();
    double y0, y1;
    cols32(B + size_t(m) * nth * nth, x0, x1, o0, nth, sh + 2 * nth, y0, y1);
    const int j = o0 + int(threadIdx.x);
    if (threadIdx.x < 32 && j < nth) {
        ob[size_t(m) * nth + j] = y0;
        if (two) ob[size_t(q1) * nth + j] = y1;
    }
}

// The shell term of every component on `stream`: g (strided by gq) -> ob
// ([q][N_theta], a different buffer: workgroups of one mode all read g_q).
inline void launch_outer(const double* g, size_t gq, double* ob, const double* B, int nth, int nphi, hipStream_t s)
{
    const dim3 grid(nphi / 2 + 1, (nth + 31) / 32);
    const size_t lds = (2 * size_t(nth) + 512) * sizeof(double);
    hipLaunchKernelGGL(k_shell_apply, grid, dim3(256), lds, s, g, gq, ob, B, nth, nphi);
}

// LDS bound of launch_outer: (2 N_theta + 512) doubles within 64 KB.
constexpr int OUTER_NTH_MAX = (65536 / 8 - 512) / 2;

}  // namespace faceflux
