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
// covers 512 contiguous bytes.
#pragma once
#include <hip/hip_runtime.h>

namespace faceflux {

constexpr int THREADS = 256;
constexpr int ROWS = 8;    // radial rows per thread (k_face_fluxes)
constexpr int BATCH = 16;  // matrix loads in flight per thread (k_outer_modes)

struct Tables {
    const double* alpha;   // [N_r], alpha[N_r - 1] = 0
    const double* VR;      // [N_r]
    const double* sig;     // [N_theta + 1], faces j - 1/2 (both poles 0)
    const double* dmu;     // [N_theta]
    const double* Sj;      // [N_theta]
};

// grid (ceil(N_theta N_phi / THREADS), ceil(N_r / ROWS)); `outer` holds the
// boundary term T[j][k] of the outermost shell.  Row indices past N_r - 1 are
// clamped for the loads (those values are never used) and skipped for the
// stores.
__global__ __launch_bounds__(THREADS) void k_face_fluxes(const double* __restrict__ phi,
                                                         const double* __restrict__ outer,
                                                         double* __restrict__ fr, double* __restrict__ ft,
                                                         double* __restrict__ fp, Tables t, int nr, int nth,
                                                         int nphi, double dphi)
{
    const int plane = nth * nphi;
    const int e = blockIdx.x * THREADS + threadIdx.x;
    if (e >= plane) return;
    const int j = e / nphi;
    const int k = e - j * nphi;
    const int ek = k + 1 < nphi ? e + 1 : e + 1 - nphi;   // phi neighbour k + 1, periodic
    const int ej = j + 1 < nth ? e + nphi : e;            // theta neighbour (itself at the pole face)
    const int i0 = blockIdx.y * ROWS;

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
            fr[at] = i + 1 < nr ? t.alpha[i] * cr * (c[r + 1] - c[r]) : -cr * ob;
            ft[at] = vr * ct * (nj[r] - c[r]);
            fp[at] = vr * cp * (nk[r] - c[r]);
        }
    }
}

// Outer boundary term of Sec. 3.2 on the outermost shell, per Fourier mode m:
//   ob_q = H_m diag(beta_m) H_m^T D g_q
// for the components q = m and q = N_phi - m of m (one component for m = 0
// and m = N_phi / 2), one workgroup per m, so both components share one pass
// over the stored matrices (W_m = H_m^T D, so H_m = diag(1/dmu) W_m^T):
//   c_l  = beta_l sum_j H[j][l] dmu_j g_j,     ob_j = (1/dmu_j) sum_l W[l][j] c_l.
// Each sum is split over 256 / (outputs) threads, reading the matrices along
// contiguous rows, and reduced in LDS.  g_q starts at g + q gq, ob_q at
// ob + q N_theta.  Dynamic LDS: (4 N_theta + 512) doubles.
__global__ __launch_bounds__(256) void k_outer_modes(const double* __restrict__ g, size_t gq,
                                                     double* __restrict__ ob, const double* __restrict__ W,
                                                     const double* __restrict__ H,
                                                     const double* __restrict__ beta,
                                                     const double* __restrict__ dmu, int nth, int nphi)
{
    extern __shared__ double sh[];
    double* gs = sh;               // [2][nth]  dmu-weighted inputs
    double* cs = sh + 2 * nth;     // [2][nth]  coefficients
    double* part = sh + 4 * nth;   // [2][256]  partial sums
    const int m = blockIdx.x;
    const bool two = m > 0 && 2 * m < nphi;
    const int q1 = nphi - m;
    const int tid = threadIdx.x;
    for (int j = tid; j < nth; j += 256) {
        gs[j] = g[size_t(m) * gq + j] * dmu[j];
        gs[nth + j] = two ? g[size_t(q1) * gq + j] * dmu[j] : 0.0;
    }
    __syncthreads();
    const double* Hm = H + size_t(m) * nth * nth;   // [j][l]
    const double* Wm = W + size_t(m) * nth * nth;   // [l][j]
    for (int pass = 0; pass < 2; ++pass) {
        const double* A = pass == 0 ? Hm : Wm;      // both read as A[x][o] for output o
        const double* in = pass == 0 ? gs : cs;
        for (int base = 0; base < nth; base += 256) {
            const int nout = min(256, nth - base);
            const int S = 256 / nout;
            const int o = tid % nout, sp = tid / nout;
            if (sp < S) {
                // BATCH independent matrix loads in flight per thread (the
                // sums are latency-bound otherwise: 129 workgroups at N_phi = 256)
                double a0 = 0.0, a1 = 0.0;
                for (int x0 = sp; x0 < nth; x0 += BATCH * S) {
                    double a[BATCH];
#pragma unroll
                    for (int u = 0; u < BATCH; ++u) {
                        const int x = x0 + u * S;
                        a[u] = x < nth ? A[size_t(x) * nth + base + o] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < BATCH; ++u) {
                        const int x = min(x0 + u * S, nth - 1);   // a[u] = 0 past the end
                        a0 += a[u] * in[x];
                        a1 += a[u] * in[nth + x];
                    }
                }
                part[sp * nout + o] = a0;
                part[256 + sp * nout + o] = a1;
            }
            __syncthreads();
            if (tid < nout) {
                double v0 = 0.0, v1 = 0.0;
                for (int y = 0; y < S; ++y) {
                    v0 += part[y * nout + tid];
                    v1 += part[256 + y * nout + tid];
                }
                const int idx = base + tid;
                if (pass == 0) {
                    const double b = beta[size_t(m) * nth + idx];
                    cs[idx] = v0 * b;
                    cs[nth + idx] = v1 * b;
                } else {
                    const double w = 1.0 / dmu[idx];
                    ob[size_t(m) * nth + idx] = v0 * w;
                    if (two) ob[size_t(q1) * nth + idx] = v1 * w;
                }
            }
            __syncthreads();
        }
    }
}

}  // namespace faceflux
