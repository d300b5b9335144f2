// FP64 solve path for gfx950: the five stages of Sec. 3.2 as HIP kernels.
//
//   k_rfft_fwd   s = 4 pi G rho, real FFT along phi       rho[i][j][k] -> X[q][i][j]
//   k_proj_f64   s^_q = W_m s~_q  (MFMA, batched over q)  X[q][i][j]   -> Y[q][i][l]
//   k_radial     Delta_r f + R_i lambda f = s^ per (q,l)   Y[q][i][l]   -> Y (in place)
//   k_proj_f64   g_q = H_m f_q                             Y[q][i][l]   -> X[q][i][j]
//   k_rfft_inv   inverse real FFT along phi                X[q][i][j]   -> phi[i][j][k]
//
// q runs over the N_phi real Fourier components (cos and sin parts of every
// mode m, see fft.hip.h); both parts of a mode share the eigensystem of m.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fft.hip.h"
#include "fftfold.hip.h"
#include "fluxes.hip.h"
#include "internal.h"
#include "modal.hip.h"
#include "momentum.hip.h"
#include "proj.hip.h"
#include "radial.hip.h"
#include "status.h"

namespace {

// True unless both values are finite (a NaN fails every comparison).
__device__ __forceinline__ bool nonfinite2(double a, double b)
{
    return !(__builtin_fabs(a) <= 1.7976931348623157e308 && __builtin_fabs(b) <= 1.7976931348623157e308);
}

// ------------------------------------------------------------------ FFT
// Persistent workgroups: each one loops over blocks of JB lines and keeps the
// global loads of its next block in flight (in registers) while the current
// block is transformed in LDS.
// With FOLD (equator-symmetric theta grids, Sec. 4.2) a block holds JB/2
// line pairs (i, k), (i, N_theta-1-k), k < h = N_theta/2; it transforms the
// even fold (sum) and the odd fold (difference) and stores them as lines
// (i, k) and (i, h+k).
// PERSIST: a grid of resident workgroups loops over the blocks, keeping the
// loads of its next block in flight; otherwise one block per workgroup, two
// workgroups per CU, and the hardware overlaps one block's loads with the
// other's transform and stores.
template <int N, bool FOLD = false, bool PERSIST = true>
__global__ __launch_bounds__(FOLD ? 512 : 256, PERSIST ? 1 : 4) void k_rfft_fwd(const double* __restrict__ rho, double* __restrict__ X,
                                                  const c64* __restrict__ tw_g, double scale, int nlines,
                                                  int nblocks, int nth, spp_status_record* __restrict__ reset,
                                                  const unsigned* __restrict__ gate, spp_batch_view bv)
{
    if (spp_gate_closed(gate)) return;
    // batched launch (one block per workgroup only): RHS r owns the nblocks
    // workgroups from r * nblocks
    int blk0 = blockIdx.x;
    if (!PERSIST && bv.rho) {
        const int r = blk0 / nblocks;
        blk0 -= r * nblocks;
        rho = bv.rho[r];
        X += r * bv.xstride;
        scale = bv.scale[r];
        if (reset) reset += r;
    }
    spp_status_clear(reset, blk0 == 0);
    constexpr int TH = FOLD ? 512 : 256;         // 16 line pairs per block for N_phi = 256
    using S = FftShape<N, TH>;
    constexpr int N2 = S::N2, T = S::T, JB = S::JB, LS = LineStride<N2>::LS;
    constexpr int PER = JB * N2 / TH;           // complex values loaded per thread and block
    __shared__ c64 lds[JB * LS];
    __shared__ c64 tws[N];
    for (int t = threadIdx.x; t < N; t += TH) tws[t] = tw_g[t];

    // a real line of N doubles is read as N2 complex values; indices past the
    // end are clamped (those lines are never stored)
    const double2* src = reinterpret_cast<const double2*>(rho);
    const size_t total = size_t(nlines) * N2;
    constexpr int PB = FOLD ? JB / 2 : JB;       // line pairs (FOLD) or lines per block
    const int h = nth >> 1;
    const size_t npairs = size_t(nlines) / 2;
    double2 pre[PER];
    auto prefetch = [&](int blk) {
        if constexpr (FOLD) {
#pragma unroll
            for (int u = 0; u < PER / 2; ++u) {
                // 32-bit pair arithmetic: the folded layout serves the grids of
                // the fused per-mode kernel (N_r N_theta <= 576 x 128), and a
                // 64-bit division per load would hold the loads back
                const int e = threadIdx.x + TH * u;
                unsigned P = unsigned(blk) * PB + unsigned(e / N2);
                P = P < unsigned(npairs) ? P : unsigned(npairs) - 1;
                const unsigned i = P / unsigned(h), k = P - i * unsigned(h);
                pre[2 * u] = src[size_t(i * unsigned(nth) + k) * N2 + e % N2];
                pre[2 * u + 1] = src[size_t(i * unsigned(nth) + unsigned(nth) - 1 - k) * N2 + e % N2];
            }
        } else {
            const size_t base = size_t(blk) * JB * N2 + threadIdx.x;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const size_t e = base + TH * u;
                pre[u] = src[e < total ? e : total - 1];
            }
        }
    };

    const int line = threadIdx.x / T, tid = threadIdx.x % T;
    const int l = threadIdx.x % JB, grp = threadIdx.x / JB;
    const size_t plane = size_t(nlines);
    int blk = blk0;
    if (blk < nblocks) prefetch(blk);
    for (; blk < nblocks; blk += gridDim.x) {
        if constexpr (FOLD) {
#pragma unroll
            for (int u = 0; u < PER / 2; ++u) {
                const int e = threadIdx.x + TH * u;
                const double2 a = pre[2 * u], b = pre[2 * u + 1];
                lds[(e / N2) * LS + pidx(e % N2)] = {(a.x + b.x) * scale, (a.y + b.y) * scale};
                lds[(PB + e / N2) * LS + pidx(e % N2)] = {(a.x - b.x) * scale, (a.y - b.y) * scale};
            }
        } else {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = threadIdx.x + TH * u;
                lds[(e / N2) * LS + pidx(e % N2)] = {pre[u].x * scale, pre[u].y * scale};
            }
        }
        __syncthreads();
        if constexpr (PERSIST) {
            if (blk + int(gridDim.x) < nblocks) prefetch(blk + gridDim.x);
        }
        fft_passes<N2, 1, T, S::E>(lds + line * LS, tid, tws);

        // split Z into the half spectrum X_m and store halfcomplex planes
        bool valid;
        size_t oline;
        if constexpr (FOLD) {
            const unsigned P = unsigned(blk) * PB + unsigned(l % PB);
            valid = P < unsigned(npairs);
            const unsigned i = valid ? P / unsigned(h) : 0, k = P - i * unsigned(h);
            oline = size_t(i * unsigned(nth) + unsigned(l / PB) * unsigned(h) + k);
        } else {
            oline = size_t(blk) * JB + l;
            valid = oline < size_t(nlines);
        }
        if (valid) {
            const c64* Z = lds + l * LS;
            double* out = X + oline;
            for (int p = grp; p <= N2 / 2; p += T) {
                const c64 a = Z[pidx(p)];
                const c64 b = Z[pidx((N2 - p) & (N2 - 1))];
                // X_p = (a + conj b)/2 + w^p (a - conj b)/(2i)
                const c64 A = {0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
                const c64 B = {0.5 * (a.y + b.y), -0.5 * (a.x - b.x)};
                const c64 w = tws[p];
                const c64 Xp = cadd(A, cmul(w, B));
                // partner X_{N2-p} = conj(A) - conj(w) conj(B)
                const c64 Xq = csub(cconj(A), cmul(cconj(w), cconj(B)));
                if (p == 0) {
                    out[0] = Xp.x;                         // Re X_0
                    out[size_t(N2) * plane] = Xq.x;        // Re X_{N/2}
                } else if (2 * p == N2) {
                    out[size_t(p) * plane] = Xp.x;
                    out[size_t(N - p) * plane] = Xp.y;
                } else {
                    out[size_t(p) * plane] = Xp.x;
                    out[size_t(N - p) * plane] = Xp.y;
                    out[size_t(N2 - p) * plane] = Xq.x;
                    out[size_t(N2 + p) * plane] = Xq.y;
                }
            }
        }
        __syncthreads();
        if constexpr (!PERSIST) break;
    }
}

// With FOLD the block's lines are the even and odd folds (i, k), (i, h+k)
// of JB/2 pairs; it stores their sum as line (i, k) and their difference as
// line (i, N_theta-1-k).
// A workgroup that stores a non-finite value sets flag->nonfinite (when
// flag is not NULL).
template <int N, bool FOLD = false, bool PERSIST = true>
__global__ __launch_bounds__(FOLD ? 512 : 256, PERSIST ? 1 : 4) void k_rfft_inv(const double* __restrict__ X, double* __restrict__ phi,
                                                  const c64* __restrict__ tw_g, int nlines, int nblocks, int nth,
                                                  spp_status_record* __restrict__ flag,
                                                  const unsigned* __restrict__ gate, spp_batch_view bv)
{
    if (spp_gate_closed(gate)) return;
    bool bad = false;
    int blk0 = blockIdx.x;
    if (!PERSIST && bv.phi) {
        const int r = blk0 / nblocks;
        blk0 -= r * nblocks;
        phi = bv.phi[r];
        X += r * bv.xstride;
        if (flag) flag += r;
    }
    constexpr int TH = FOLD ? 512 : 256;         // 16 line pairs per block for N_phi = 256
    using S = FftShape<N, TH>;
    constexpr int N2 = S::N2, T = S::T, JB = S::JB, LS = LineStride<N2>::LS;
    constexpr int NT = (N2 / 2 + T) / T;         // split tasks p = 0..N2/2 per thread
    constexpr int PER = JB * N2 / TH;
    __shared__ c64 lds[JB * LS];
    __shared__ c64 tws[N];
    for (int t = threadIdx.x; t < N; t += TH) tws[t] = tw_g[t];

    const int line = threadIdx.x / T, tid = threadIdx.x % T;
    const int l = threadIdx.x % JB, grp = threadIdx.x / JB;
    const size_t plane = size_t(nlines);

    // raw halfcomplex values of task p: Re X_p, Im X_p, Re X_{N2-p}, Im X_{N2-p}
    // (for p = 0 the imaginary slots hold Re X_0 and are discarded)
    constexpr int PB = FOLD ? JB / 2 : JB;
    const int h = nth >> 1;
    const size_t npairs = size_t(nlines) / 2;
    double pre[NT][4];
    auto prefetch = [&](int blk) {
        size_t L;
        if constexpr (FOLD) {
            unsigned P = unsigned(blk) * PB + unsigned(l % PB);
            P = P < unsigned(npairs) ? P : unsigned(npairs) - 1;
            const unsigned i = P / unsigned(h), k = P - i * unsigned(h);
            L = size_t(i * unsigned(nth) + unsigned(l / PB) * unsigned(h) + k);
        } else {
            L = size_t(min(blk * JB + l, nlines - 1));
        }
        const double* in = X + L;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            int p = grp + T * u;
            p = p <= N2 / 2 ? p : N2 / 2;
            pre[u][0] = in[size_t(p) * plane];
            pre[u][1] = in[size_t(p == 0 ? 0 : N - p) * plane];
            pre[u][2] = in[size_t(N2 - p) * plane];
            pre[u][3] = in[size_t(p == 0 ? 0 : N2 + p) * plane];
        }
    };

    int blk = blk0;
    if (blk < nblocks) prefetch(blk);
    __syncthreads();   // twiddles
    for (; blk < nblocks; blk += gridDim.x) {
        // Z_m = [X_m + conj X_{N2-m}] + i w^-m [X_m - conj X_{N2-m}], stored as
        // conj(Z): the inverse transform is conj(FFT(conj Z)).
        c64* Z = lds + l * LS;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int p = grp + T * u;
            if (p <= N2 / 2) {
                const c64 xp = {pre[u][0], p == 0 ? 0.0 : pre[u][1]};
                const c64 xq = {pre[u][2], p == 0 ? 0.0 : pre[u][3]};
                const c64 wc = cconj(tws[p]);                 // w^-p
                const c64 Ep = cadd(xp, cconj(xq)), Dp = csub(xp, cconj(xq));
                Z[pidx(p)] = cconj(cadd(Ep, cmul({-wc.y, wc.x}, Dp)));
                if (p != 0 && 2 * p != N2) {
                    // Z_{N2-p} with w^-(N2-p) = -w^p
                    const c64 Eq = cadd(xq, cconj(xp)), Dq = csub(xq, cconj(xp));
                    const c64 w = tws[p];
                    Z[pidx(N2 - p)] = cconj(cadd(Eq, cmul({w.y, -w.x}, Dq)));
                }
            }
        }
        __syncthreads();
        if constexpr (PERSIST) {
            if (blk + int(gridDim.x) < nblocks) prefetch(blk + gridDim.x);
        }
        fft_passes<N2, 1, T, S::E>(lds + line * LS, tid, tws);

        // x_{2n} = Re z_n, x_{2n+1} = Im z_n with z = conj(FFT(conj Z))
        if constexpr (FOLD) {
            double2* dst = reinterpret_cast<double2*>(phi);
#pragma unroll
            for (int u = 0; u < PER / 2; ++u) {
                const int e = threadIdx.x + TH * u;
                const unsigned P = unsigned(blk) * PB + unsigned(e / N2);
                if (P < unsigned(npairs)) {
                    const unsigned i = P / unsigned(h), k = P - i * unsigned(h);
                    const c64 ve = lds[(e / N2) * LS + pidx(e % N2)];
                    const c64 vo = lds[(PB + e / N2) * LS + pidx(e % N2)];
                    bad = bad || nonfinite2(ve.x + vo.x, ve.y + vo.y) || nonfinite2(ve.x - vo.x, ve.y - vo.y);
                    dst[(size_t(i) * nth + k) * N2 + e % N2] = double2{ve.x + vo.x, -(ve.y + vo.y)};
                    dst[(size_t(i) * nth + nth - 1 - k) * N2 + e % N2] = double2{ve.x - vo.x, -(ve.y - vo.y)};
                }
            }
        } else {
            const int L0 = blk * JB;
            const int nl = min(JB, nlines - L0);
            double2* dst = reinterpret_cast<double2*>(phi + size_t(L0) * N);
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = threadIdx.x + TH * u;
                if (e < nl * N2) {
                    const c64 v = lds[(e / N2) * LS + pidx(e % N2)];
                    bad = bad || nonfinite2(v.x, v.y);
                    dst[e] = double2{v.x, -v.y};
                }
            }
        }
        __syncthreads();
        if constexpr (!PERSIST) break;
    }
    if (bad && flag) atomicOr(&flag->nonfinite, 1u);
}

// ------------------------------------------------------------------ projection GEMM (MFMA f64)
// C[q][i][n] = sum_k A[q][i][k] * B[m(q)][n][k], i < M, n, k < K (= N_theta).
// Workgroup tile 64 x 64, four waves of 32 x 32, v_mfma_f64_16x16x4 with
// K staged through LDS in chunks of 16 (k-major, padded against bank
// conflicts).  Operand layouts of the 16x16x4 f64 MFMA: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; the 16x16 result lives in 4
// registers per lane, register v holding row (l / 16) + 4 v, column l % 16.
constexpr int PBM = 64, PBN = 64, PBK = 16, PPAD = 16;

__global__ __launch_bounds__(256) void k_proj_f64(const double* __restrict__ A, const double* __restrict__ B,
                                                  double* __restrict__ C, int M, int K, int nphi,
                                                  const unsigned* __restrict__ gate)
{
    if (spp_gate_closed(gate)) return;
    const int q = blockIdx.z;
    const int m = q <= nphi / 2 ? q : nphi - q;
    const double* Aq = A + size_t(q) * M * K;
    const double* Bm = B + size_t(m) * K * K;
    double* Cq = C + size_t(q) * M * K;
    const int i0 = blockIdx.y * PBM, n0 = blockIdx.x * PBN;

    __shared__ double As[PBK][PBM + PPAD];
    __shared__ double Bs[PBK][PBN + PPAD];

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lrow = t >> 2, lk = (t & 3) * 4;   // loader: one row, four k

    using d4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < K; k0 += PBK) {
        {
            const int gi = i0 + lrow, gn = n0 + lrow;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int gk = k0 + lk + c;
                As[lk + c][lrow] = (gi < M && gk < K) ? Aq[size_t(gi) * K + gk] : 0.0;
                Bs[lk + c][lrow] = (gn < K && gk < K) ? Bm[size_t(gn) * K + gk] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < PBK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double a[2], b[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) a[r] = As[kr][wm * 32 + r * 16 + (lane & 15)];
#pragma unroll
            for (int c = 0; c < 2; ++c) b[c] = Bs[kr][wn * 32 + c * 16 + (lane & 15)];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], b[c], acc[r][c], 0, 0, 0);
        }
        __syncthreads();
    }

#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int col = n0 + wn * 32 + c * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = i0 + wm * 32 + r * 16 + (lane >> 4) + 4 * v;
                if (row < M && col < K) Cq[size_t(row) * K + col] = acc[r][c][v];
            }
        }
}

// ------------------------------------------------------------------ radial tridiagonal
// One lane per (q, l) system; rows scaled by V_i so the matrix is symmetric:
//   alpha_{i-1} f_{i-1} + (-(alpha_{i-1} + alpha_i) + V_i R_i lambda) f_i
//     + alpha_i f_{i+1} = V_i s^_i,
// with alpha_{-1} replaced by gamma(lambda) (0 unless the regular inner
// condition) and the outermost alpha by beta(lambda).
// Forward elimination stores y_i in place and 1/w_i in `piv`; the back
// substitution then runs from the outer shell inwards.
__global__ __launch_bounds__(256) void k_radial(double* __restrict__ Y, double* __restrict__ piv,
                                                const double* __restrict__ lam, const double* __restrict__ beta,
                                                const double* __restrict__ gamma,
                                                const double* __restrict__ alpha, const double* __restrict__ V,
                                                const double* __restrict__ VR, int nr, int nth, int nphi,
                                                const unsigned* __restrict__ gate)
{
    if (spp_gate_closed(gate)) return;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nphi * nth) return;
    const int q = gid / nth, l = gid - q * nth;
    const int m = q <= nphi / 2 ? q : nphi - q;
    const double lm = lam[m * nth + l];
    const double bo = beta[m * nth + l];
    const double gi = gamma[m * nth + l];
    const size_t stride = size_t(nth);
    double* y = Y + size_t(q) * nr * nth + l;
    double* pv = piv + size_t(q) * nr * nth + l;

    double a_prev = 0.0, w_prev = 1.0, y_prev = 0.0, inv_prev = 0.0;
    for (int i = 0; i < nr; ++i) {
        const double ai = (i + 1 < nr) ? alpha[i] : bo;
        const double diag = -((i == 0 ? gi : a_prev) + ai) + VR[i] * lm;
        const double rhs = V[i] * y[i * stride];
        const double lf = a_prev * inv_prev;          // a_prev / w_prev
        const double w = diag - lf * a_prev;
        const double yi = rhs - lf * y_prev;
        const double inv = 1.0 / w;
        y[i * stride] = yi;
        pv[i * stride] = inv;
        a_prev = ai;
        w_prev = w;
        y_prev = yi;
        inv_prev = inv;
    }
    (void)w_prev;
    double f_next = 0.0;
    for (int i = nr - 1; i >= 0; --i) {
        const double ai = (i + 1 < nr) ? alpha[i] : 0.0;
        const double f = (y[i * stride] - ai * f_next) * pv[i * stride];
        y[i * stride] = f;
        f_next = f;
    }
}

// Compute units of the current device (queried once).
int device_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

// Rows per wave tile (16 RM) of the projection kernel.  The default depends on
// the tile width; spp_autotune_projection may record a measured choice per
// (N_theta, N_r), which then takes precedence.
std::mutex g_tune_mu;
std::map<std::pair<int, int>, int> g_tuned_rm;

int proj_rm_default(int rn) { return rn == 8 ? 1 : rn == 4 ? 2 : 4; }

int proj_rm(int K, int M)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tuned_rm.find({K, M});
    return it != g_tuned_rm.end() ? it->second : proj_rm_default(projimg::rn_for(K));
}

// Candidate RM values per tile width (each one an instantiated kernel).
std::vector<int> proj_rm_candidates(int rn)
{
    switch (rn) {
    case 8: return {1, 2};
    case 4: return {1, 2};   // RM = 4 spills at this tile width
    default: return {2, 4};
    }
}

bool launch_proj_rm(const double* A, const double* B, double* C, int M, int K, int nphi, int rm, hipStream_t s,
                    const unsigned* gate = nullptr)
{
    if (K > 128) return false;
    const int rn = projimg::rn_for(K);
    const int groups = (M + 16 * rm - 1) / (16 * rm);
    // one workgroup per CU at a time for the largest tile (B_m fills most of
    // the LDS): split the rows of a component only when there are fewer
    // components than CUs
    int splits = (device_cus() + nphi - 1) / nphi;
    const int maxsplits = (groups + proj::NWAVES - 1) / proj::NWAVES;
    if (splits > maxsplits) splits = maxsplits;
    if (splits < 1) splits = 1;
    const dim3 grid(splits, nphi), block(64 * proj::NWAVES);
    const bool kvec = (K % 32) == 0;
#define SPP_PROJ(RN, RM)                                                                                       \
    do {                                                                                                       \
        if (kvec)                                                                                              \
            hipLaunchKernelGGL((proj::k_proj_f64<RN, RM, true>), grid, block, 0, s, A, B, C, M, K, nphi, splits,   \
                               gate);                                                                          \
        else                                                                                                   \
            hipLaunchKernelGGL((proj::k_proj_f64<RN, RM, false>), grid, block, 0, s, A, B, C, M, K, nphi, splits,  \
                               gate);                                                                          \
    } while (0)
    if (rn == 8) {
        if (rm == 2) SPP_PROJ(8, 2); else SPP_PROJ(8, 1);
    } else if (rn == 4) {
        if (rm == 1) SPP_PROJ(4, 1); else SPP_PROJ(4, 2);
    } else if (rn == 2) {
        if (rm == 2) SPP_PROJ(2, 2); else SPP_PROJ(2, 4);
    } else {
        if (rm == 2) SPP_PROJ(1, 2); else SPP_PROJ(1, 4);
    }
#undef SPP_PROJ
    return true;
}

// Parity-split projection for equator-symmetric theta grids (h = N_theta/2 <= 64).
bool launch_proj_par(const double* A, const double* Bpar, double* C, int M, int N, int nphi, bool fwd, int rn,
                     hipStream_t s, const unsigned* gate = nullptr)
{
    if (rn == 0) return false;
    const int h = N / 2;
    const int rm = 1;
    const int groups = (M + 16 * rm - 1) / (16 * rm);
    int splits = (device_cus() + nphi - 1) / nphi;
    const int maxsplits = (groups + proj::NWAVES - 1) / proj::NWAVES;
    if (splits > maxsplits) splits = maxsplits;
    if (splits < 1) splits = 1;
    const dim3 grid(splits, nphi), block(64 * proj::NWAVES);
    const bool kvec = (h % 32) == 0;
#define SPP_PAR(RN, KV)                                                                                        \
    do {                                                                                                       \
        if (fwd)                                                                                               \
            hipLaunchKernelGGL((proj::k_proj_par<RN, 1, KV, true>), grid, block, 0, s, A, Bpar, C, M, N, nphi, splits,   \
                               gate);                                                                          \
        else                                                                                                   \
            hipLaunchKernelGGL((proj::k_proj_par<RN, 1, KV, false>), grid, block, 0, s, A, Bpar, C, M, N, nphi, splits,  \
                               gate);                                                                          \
    } while (0)
    switch (rn) {
    case 1: if (kvec) SPP_PAR(1, true); else SPP_PAR(1, false); break;
    case 2: if (kvec) SPP_PAR(2, true); else SPP_PAR(2, false); break;
    default: if (kvec) SPP_PAR(4, true); else SPP_PAR(4, false); break;
    }
#undef SPP_PAR
    return true;
}

// Projection GEMM with B_m staged in LDS for N_theta <= 128; false above.
bool launch_proj(const double* A, const double* B, double* C, int M, int K, int nphi, hipStream_t s,
                 const unsigned* gate = nullptr)
{
    return launch_proj_rm(A, B, C, M, K, nphi, K <= 128 ? proj_rm(K, M) : 0, s, gate);
}

// Rows per chunk of the instantiated partitioned radial kernel for N_r
// (capacities whose register arrays stay in VGPRs, no scratch), 0 above
// N_r = 32 * 20 (then the one-lane kernel k_radial runs).
int radial_part_capacity(int nr)
{
    if (nr > radial::NRMAX) return 0;
    const int P = nr < radial::PMAX ? nr : radial::PMAX;
    const int ch = (nr + P - 1) / P;
    for (int c : {4, 8, 18, 20})
        if (ch <= c) return c;
    return 0;
}

// Partitioned radial solve for N_r <= 32 * 20; returns false above that.
bool launch_radial_part(double* Y, const double* lam, const double* beta, const radial::Coef& cf, int nth,
                        int nphi, hipStream_t s, const unsigned* gate = nullptr)
{
    const int nr = cf.nr;
    const int cap = radial_part_capacity(nr);
    if (cap == 0) return false;
    const int P = nr < radial::PMAX ? nr : radial::PMAX;
    const int nsys = nphi * nth;
    const dim3 grid((nsys + radial::SYS - 1) / radial::SYS), block(radial::THREADS);
    switch (cap) {
    case 4: hipLaunchKernelGGL(radial::k_radial_part<4>, grid, block, 0, s, Y, lam, beta, cf, nth, nphi, P, gate); break;
    case 8: hipLaunchKernelGGL(radial::k_radial_part<8>, grid, block, 0, s, Y, lam, beta, cf, nth, nphi, P, gate); break;
    case 18: hipLaunchKernelGGL(radial::k_radial_part<18>, grid, block, 0, s, Y, lam, beta, cf, nth, nphi, P, gate); break;
    default: hipLaunchKernelGGL(radial::k_radial_part<20>, grid, block, 0, s, Y, lam, beta, cf, nth, nphi, P, gate); break;
    }
    return true;
}

// Fused per-mode kernel (projection, radial solves, inverse projection) on
// the folded spectrum X, in place; false when the grid is outside its range.
// Template arguments (column tiles RN, row tiles T) of the fused kernel for
// this grid; false when it is outside the kernel's range.
bool modal_variant(int nr, int nth, int* rn, int* T)
{
    const int h = nth / 2;
    *rn = modalimg::rn_for(h);
    *T = (nr + 16 * modal::NW - 1) / (16 * modal::NW);
    return !(h % 2 != 0 || h > 64 || *T < 1 || *T > modalimg::TMAX);
}

// nrhs > 1: a batched launch over the spectral fields X + r * xstride.
bool launch_modal(double* X, const double* Fimg, const double* Iimg, const double* Rimg, const double* lam,
                  const double* beta, const radial::Coef& cf, int nr, int nth, int nphi, double* sink,
                  hipStream_t s, const unsigned* gate = nullptr, int nrhs = 1, size_t xstride = 0, int paired = 1)
{
    int rn = 0, T = 0;
    if (!modal_variant(nr, nth, &rn, &T)) return false;
    // one workgroup per (RHS, q, parity), see modal::unit_of
    const dim3 grid(2 * nphi * nrhs), block(modal::THREADS);
#define SPP_MODAL(RN, TT)                                                                                      \
    case RN * 4 + TT:                                                                                          \
        hipLaunchKernelGGL((modal::k_modal<RN, TT>), grid, block, 0, s, X, Fimg, Iimg, Rimg, lam, beta, cf, nth, nphi, \
                           sink, gate, nrhs > 1 ? xstride : size_t(0), paired);                               \
        return true;
    switch (rn * 4 + T) {
        SPP_MODAL(1, 1)
        SPP_MODAL(1, 2)
        SPP_MODAL(1, 3)
        SPP_MODAL(2, 1)
        SPP_MODAL(2, 2)
        SPP_MODAL(2, 3)
        SPP_MODAL(4, 1)
        SPP_MODAL(4, 2)
        SPP_MODAL(4, 3)
    }
#undef SPP_MODAL
    return false;
}

// Workgroups of the FFT kernel for N that fit on the device at once (cached).
template <int N>
int fft_resident(bool forward, bool fold)
{
    static int resident[4] = {0, 0, 0, 0};
    int& res = resident[(forward ? 0 : 1) + (fold ? 2 : 0)];
    if (res == 0) {
        int per_cu = 0;
        if (forward && fold)
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rfft_fwd<N, true>, 512, 0);
        else if (forward)
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rfft_fwd<N, false>, 256, 0);
        else if (fold)
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rfft_inv<N, true>, 512, 0);
        else
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rfft_inv<N, false>, 256, 0);
        res = (per_cu > 0 ? per_cu : 1) * device_cus();
    }
    return res;
}

// rec: the forward FFT clears this status record first, the inverse FFT sets
// its non-finite flag (either may be NULL); gate: see status.h.
struct FftExtra {
    spp_status_record* rec = nullptr;
    const unsigned* gate = nullptr;
    spp_batch_view bv{};       // batched launch over nrhs right-hand sides (folded FFTs only)
    int nrhs = 1;
};

template <int N>
void launch_fft_pair(bool forward, const double* in, double* out, const c64* tw, double scale, int nlines,
                     bool fold, int nth, hipStream_t s, FftExtra x)
{
    const int per_block = fold ? FftShape<N, 512>::JB / 2 : FftShape<N, 256>::JB;
    const int units = fold ? nlines / 2 : nlines;
    const int nblocks = (units + per_block - 1) / per_block;
    // persistent grid: as many workgroups as can be resident, blocks spread evenly
    const int res = fft_resident<N>(forward, fold);
    const int per = (nblocks + res - 1) / res;
    const int grid = (nblocks + per - 1) / per;
    if (fold && N == fftfold::N) {   // one block of 16 line pairs per workgroup
        if (forward)
            hipLaunchKernelGGL(fftfold::k_rfft_fwd_fold, dim3(nblocks * x.nrhs), dim3(fftfold::THREADS), 0, s, in, out,
                               tw, scale, nlines, nblocks, nth, x.rec, x.gate, x.bv);
        else
            hipLaunchKernelGGL(fftfold::k_rfft_inv_fold, dim3(nblocks * x.nrhs), dim3(fftfold::THREADS), 0, s, in, out,
                               tw, nlines, nblocks, nth, x.rec, x.gate, x.bv);
        return;
    }
    if (forward) {
        if (fold)   // one block per workgroup (see k_rfft_fwd)
            hipLaunchKernelGGL((k_rfft_fwd<N, true, false>), dim3(nblocks * x.nrhs), dim3(512), 0, s, in, out, tw,
                               scale, nlines, nblocks, nth, x.rec, x.gate, x.bv);
        else
            hipLaunchKernelGGL((k_rfft_fwd<N, false>), dim3(grid), dim3(256), 0, s, in, out, tw, scale, nlines,
                               nblocks, nth, x.rec, x.gate, spp_batch_view{});
    } else {
        if (fold)
            hipLaunchKernelGGL((k_rfft_inv<N, true, false>), dim3(nblocks * x.nrhs), dim3(512), 0, s, in, out, tw,
                               nlines, nblocks, nth, x.rec, x.gate, x.bv);
        else
            hipLaunchKernelGGL((k_rfft_inv<N, false>), dim3(grid), dim3(256), 0, s, in, out, tw, nlines, nblocks,
                               nth, x.rec, x.gate, spp_batch_view{});
    }
}

// fold: the line-pair layout of the fused per-mode path (equator-symmetric grids)
bool launch_fft(int nphi, bool forward, const double* in, double* out, const c64* tw, double scale, int nlines,
                hipStream_t s, bool fold = false, int nth = 0, FftExtra x = {})
{
    switch (nphi) {
#define SPP_FFT_CASE(n) \
    case n: launch_fft_pair<n>(forward, in, out, tw, scale, nlines, fold, nth, s, x); return true;
        SPP_FFT_CASE(4)
        SPP_FFT_CASE(8)
        SPP_FFT_CASE(16)
        SPP_FFT_CASE(32)
        SPP_FFT_CASE(64)
        SPP_FFT_CASE(128)
        SPP_FFT_CASE(256)
        SPP_FFT_CASE(512)
        SPP_FFT_CASE(1024)
        SPP_FFT_CASE(2048)
#undef SPP_FFT_CASE
    default: return false;
    }
}

// Fill n 64-bit words with zero (a kernel, so that the fill can be captured
// into a graph).
__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long* __restrict__ x, size_t n)
{
    const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) x[i] = 0ull;
}

// ------------------------------------------------------------------ residuals
// The refinement of the mixed form works on the Fourier components: the phi
// operator is diagonal there (eigenvalue lambda_{phi,m}), so the discrete
// Laplacian of component q is a local operator in (i, j) plus, on the
// outermost shell, the boundary term of Sec. 3.2 (and on the innermost shell
// the regular inner condition's term), which act per theta eigenmode.

struct ResidualTables {
    const double* alpha;   // [nr], alpha[nr-1] = 0
    const double* V;       // [nr]
    const double* VR;      // [nr]
    const double* sig;     // [nth + 1]
    const double* dmu;     // [nth]
    const double* Sj;      // [nth]
    const double* lamphi;  // [nphi/2 + 1]
};

// Largest |x| over a workgroup of 256 threads, NaN winning (a NaN compares
// false, so it is tracked apart); the result as IEEE-754 bits, which order
// non-negative doubles and put NaN above infinity.
__device__ __forceinline__ unsigned long long block_absmax_bits(double v, bool nan, double* red)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double m = nan ? __builtin_nan("") : v;
    unsigned long long bits = __double_as_longlong(m);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_xor(bits, o, 64);
        bits = other > bits ? other : bits;
    }
    if (lane == 0) red[w] = __longlong_as_double(bits);
    __syncthreads();
    unsigned long long out = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) {
            const unsigned long long b = __double_as_longlong(red[k]);
            out = b > out ? b : out;
        }
    return out;
}

// r = s~ - L_q g for every element (q, i, j), FP64.  Workgroup (x, q) covers
// 256 (row chunk, j) columns of component q, a thread RES_ROWS consecutive
// rows of one j: all its loads (the column with one row beyond each end, the
// j -+ 1 neighbours, s~) are issued before the first result, so that about
// 4 RES_ROWS loads are in flight per thread.  Each workgroup adds max |r| of
// its elements into rmax_q[q] (and max |s~| into smax_q[q] when not NULL) with
// one atomic.
constexpr int RES_ROWS = 8;

__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ St, const double* __restrict__ Gf,
                                                  const double* __restrict__ ob, const double* __restrict__ ib,
                                                  double* __restrict__ R, ResidualTables t, int nr, int nth,
                                                  int nphi, unsigned long long* __restrict__ rmax_q,
                                                  unsigned long long* __restrict__ smax_q)
{
    __shared__ double red[4];
    const int q = blockIdx.y;
    const int m = q <= nphi / 2 ? q : nphi - q;
    const size_t plane = size_t(nr) * nth;
    const int nchunks = (nr + RES_ROWS - 1) / RES_ROWS;
    const int item = blockIdx.x * 256 + threadIdx.x;
    double mr = 0.0, ms = 0.0;
    bool nr_nan = false, ns_nan = false;
    if (item < nth * nchunks) {
        const int chunk = item / nth, j = item - chunk * nth;
        const int i0 = chunk * RES_ROWS;
        const double* __restrict__ G = Gf + size_t(q) * plane + j;
        const double* __restrict__ Sq = St + size_t(q) * plane + j;
        auto at = [&](int i) { return size_t(i < 0 ? 0 : (i < nr ? i : nr - 1)) * nth; };
        // g of rows i0 - 1 .. i0 + RES_ROWS (clamped; the values past the ends are not used)
        double c[RES_ROWS + 2], lj[RES_ROWS], rj[RES_ROWS], sv[RES_ROWS];
#pragma unroll
        for (int r = 0; r < RES_ROWS + 2; ++r) c[r] = G[at(i0 - 1 + r)];
        const int dl = j > 0 ? -1 : 0, dr = j + 1 < nth ? 1 : 0;   // in-range neighbour offsets
#pragma unroll
        for (int r = 0; r < RES_ROWS; ++r) {
            const size_t o = at(i0 + r);
            lj[r] = G[o + dl];
            rj[r] = G[o + dr];
            sv[r] = Sq[o];
        }
        // the row tables of the chunk, also loaded up front (al[r] = alpha of
        // row i0 - 1 + r), so that no row waits on a load
        double al[RES_ROWS + 1], vv[RES_ROWS], vrr[RES_ROWS];
#pragma unroll
        for (int r = 0; r <= RES_ROWS; ++r) {
            const int i = i0 - 1 + r;
            al[r] = t.alpha[i < 0 ? 0 : (i < nr ? i : nr - 1)];
        }
#pragma unroll
        for (int r = 0; r < RES_ROWS; ++r) {
            const int i = i0 + r < nr ? i0 + r : nr - 1;
            vv[r] = t.V[i];
            vrr[r] = t.VR[i];
        }
        const double obj = i0 + RES_ROWS >= nr ? ob[size_t(q) * nth + j] : 0.0;
        const double ibj = i0 == 0 && ib ? ib[size_t(q) * nth + j] : 0.0;
        const double sig_l = t.sig[j], sig_h = t.sig[j + 1], dmu = t.dmu[j], sjl = t.Sj[j] * t.lamphi[m];
        // every load is awaited here, once: the rows below store between
        // their computations, and a wait for a later row's load would
        // otherwise also wait for the stores issued before it
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt not waited
        double res[RES_ROWS];
#pragma unroll
        for (int r = 0; r < RES_ROWS; ++r) {
            const int i = i0 + r;
            const double g0 = c[r + 1];
            // radial fluxes through the faces i+1/2 and i-1/2 (outer face:
            // boundary term; inner face: the regular condition's term, 0 for
            // zero flux)
            double flux = 0.0;
            if (i + 1 < nr) flux += al[r + 1] * (c[r + 2] - g0);
            else flux -= obj;
            if (i > 0) flux -= al[r] * (g0 - c[r]);
            else if (ib) flux -= ibj;
            const double Vi = vv[r];
            // theta fluxes (pole faces have sigma = 0) and the phi eigenvalue term
            double th = 0.0;
            if (j + 1 < nth) th += sig_h * (rj[r] - g0);
            if (j > 0) th -= sig_l * (g0 - lj[r]);
            const double Ri = vrr[r] / Vi;
            const double Lg = flux / Vi + Ri * (th / dmu + sjl * g0);
            res[r] = sv[r] - Lg;
        }
#pragma unroll
        for (int r = 0; r < RES_ROWS; ++r) {
            const int i = i0 + r;
            if (i < nr) {
                R[size_t(q) * plane + size_t(i) * nth + j] = res[r];
                const double ar = __builtin_fabs(res[r]), as = __builtin_fabs(sv[r]);
                nr_nan |= ar != ar;
                mr = ar > mr ? ar : mr;
                ns_nan |= as != as;
                ms = as > ms ? as : ms;
            }
        }
    }
    const unsigned long long br = block_absmax_bits(mr, nr_nan, red);
    if (threadIdx.x == 0) atomicMax(rmax_q + q, br);
    if (smax_q) {
        __syncthreads();
        const unsigned long long bs = block_absmax_bits(ms, ns_nan, red);
        if (threadIdx.x == 0) atomicMax(smax_q + q, bs);
    }
}

// After the refinement of the mixed form: reduce the per-component maxima
// of each residual (part[k][q], k = 0: the source, k = 1..n: the residuals
// the corrections were computed from) into the status record and decide.
// Refinement step k contracted if max |r_k| <= max |r_{k-1}| / 2 (finite);
// if any step did not, the record says so and, with allow_fallback, opens
// the gate of the FP64 solve enqueued behind (whose inverse FFT then sets the
// non-finite flag afresh).  One workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_refine_gate(spp_status_record* __restrict__ rec,
                                                     const unsigned long long* __restrict__ part, int nphi,
                                                     int n_refine, int allow_fallback)
{
    __shared__ double red[4];
    __shared__ unsigned long long kmax[SPP_MAX_REFINE + 1];
    for (int k = 0; k <= n_refine; ++k) {
        unsigned long long mb = 0;
        for (int q = threadIdx.x; q < nphi; q += 256) {
            const unsigned long long b = part[size_t(k) * nphi + q];
            mb = b > mb ? b : mb;
        }
        const double v = __longlong_as_double(mb);
        const unsigned long long r = block_absmax_bits(v, v != v, red);
        if (threadIdx.x == 0) kmax[k] = r;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsigned bad = 0;
        for (int k = 1; k <= n_refine; ++k) {
            const double rk = __longlong_as_double(kmax[k]), rp = __longlong_as_double(kmax[k - 1]);
            if (!(rk <= 0.5 * rp)) bad = 1;      // NaN or infinity fail too
        }
        for (int k = 0; k <= n_refine; ++k) rec->rmax[k] = kmax[k];
        rec->refine_iters = unsigned(n_refine);
        rec->not_contracted = bad;
        const unsigned fb = bad && allow_fallback ? 1u : 0u;
        rec->fallback = fb;
        if (fb) rec->nonfinite = 0u;
    }
}

// r = 4 pi G rho - L Phi in physical space (spp_residual), FP64: the flux
// stencil of Sec. 3.1 divided by the cell volume,
//   L Phi = [F_{i+1/2} - F_{i-1/2}] / V_i
//         + R_i [sigma_{j+1/2} (Phi_{j+1} - Phi_j) - sigma_{j-1/2} (Phi_j - Phi_{j-1})] / dmu_j
//         + R_i S_j (Phi_{k+1} - 2 Phi_k + Phi_{k-1}) / dphi^2,
// F_{i+1/2} = alpha_i (Phi_{i+1} - Phi_i) inside, -T_out on the outer face and
// T_in (the regular inner condition; 0 for zero flux) on the inner face, T
// per (j, k) from the shell transforms.  A thread owns one (j, k) column and
// RROWS radial rows, with every load issued before the first store; the
// neighbour rows come from cache (adjacent threads load them; plane blocks in
// the XCD-aware order of spp_plane_block).
constexpr int RROWS = 4;
constexpr int RES_LDS_ROWS = 8;   // rows per thread of k_residual_rows

__global__ __launch_bounds__(256) void k_residual_phys(const double* __restrict__ rho, const double* __restrict__ phi,
                                                       const double* __restrict__ tout,
                                                       const double* __restrict__ tin, double* __restrict__ r,
                                                       ResidualTables t, double four_pi_g, int nr, int nth,
                                                       int nphi, double inv_dphi2, int gx)
{
    const int plane = nth * nphi;
    const int chunk = blockIdx.x / gx;
    const int e = spp_plane_block(blockIdx.x - chunk * gx, gx) * 256 + threadIdx.x;
    if (e >= plane) return;
    const int j = e / nphi, k = e - j * nphi;
    const int ekp = k + 1 < nphi ? e + 1 : e + 1 - nphi;
    const int ekm = k > 0 ? e - 1 : e - 1 + nphi;
    const int ejp = j + 1 < nth ? e + nphi : e;       // pole faces: sigma = 0
    const int ejm = j > 0 ? e - nphi : e;
    const int i0 = chunk * RROWS;
    auto row = [&](int i) { return size_t(i < 0 ? 0 : (i < nr ? i : nr - 1)) * plane; };
    double c[RROWS + 2], kp[RROWS], km[RROWS], jp[RROWS], jm[RROWS], src[RROWS];
#pragma unroll
    for (int u = 0; u < RROWS + 2; ++u) c[u] = phi[row(i0 - 1 + u) + e];
#pragma unroll
    for (int u = 0; u < RROWS; ++u) {
        const size_t b = row(i0 + u);
        kp[u] = phi[b + ekp];
        km[u] = phi[b + ekm];
        jp[u] = phi[b + ejp];
        jm[u] = phi[b + ejm];
        src[u] = rho[b + e];
    }
    const double to = i0 + RROWS >= nr ? tout[e] : 0.0;
    const double ti = (i0 == 0 && tin) ? tin[e] : 0.0;
    const double sp = t.sig[j + 1], sm = t.sig[j], idm = 1.0 / t.dmu[j], sj = t.Sj[j] * inv_dphi2;
    // the chunk's row tables, loaded up front too (al[u] = alpha of row i0 - 1 + u)
    double al[RROWS + 1], vv[RROWS], vrr[RROWS];
#pragma unroll
    for (int u = 0; u <= RROWS; ++u) {
        const int i = i0 - 1 + u;
        al[u] = t.alpha[i < 0 ? 0 : (i < nr ? i : nr - 1)];
    }
#pragma unroll
    for (int u = 0; u < RROWS; ++u) {
        const int i = i0 + u < nr ? i0 + u : nr - 1;
        vv[u] = t.V[i];
        vrr[u] = t.VR[i];
    }
    // every load is awaited here, once: the rows below store between their
    // computations, and a wait for a later row's load would otherwise also wait
    // for the stores issued before it
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt not waited
#pragma unroll
    for (int u = 0; u < RROWS; ++u) {
        const int i = i0 + u;
        if (i < nr) {
            const double x = c[u + 1];
            const double fo = i + 1 < nr ? al[u + 1] * (c[u + 2] - x) : -to;
            const double fi = i > 0 ? al[u] * (x - c[u]) : ti;
            const double Vi = vv[u], Ri = vrr[u] / Vi;
            const double th = sp * (jp[u] - x) - sm * (x - jm[u]);
            const double LP = (fo - fi) / Vi + Ri * (th * idm + sj * (kp[u] - 2.0 * x + km[u]));
            r[size_t(i) * plane + e] = four_pi_g * src[u] - LP;
        }
    }
}

// The same residual for N_phi dividing 256: every workgroup covers whole theta
// rows, so the phi neighbours of a value are values other threads of the
// workgroup have loaded.  They are exchanged through LDS instead of loaded
// again, and the per-row factors (alpha, 1/V_i and R_i = (VR)_i / V_i) are
// formed once per workgroup.  Threads past the plane (whole theta rows of
// the last workgroup) load a valid row, take part in the exchange among
// themselves and store nothing.  r is stored non-temporally (nothing here
// reads it), so that it does not evict the rows of Phi and rho that the
// neighbouring workgroups still read.
template <int ROWS>
__global__ __launch_bounds__(256) void k_residual_rows(const double* __restrict__ rho, const double* __restrict__ phi,
                                                       const double* __restrict__ tout,
                                                       const double* __restrict__ tin, double* __restrict__ r,
                                                       ResidualTables t, double four_pi_g, int nr, int nth,
                                                       int nphi, double inv_dphi2, int gx)
{
    __shared__ double cs[ROWS][256];     // this workgroup's Phi values of its ROWS rows
    __shared__ double fa[3][ROWS + 1];   // alpha of row i0 - 1 + u; 1/V and R of row i0 + u
    const int tid = threadIdx.x;
    const int plane = nth * nphi;
    const int chunk = blockIdx.x / gx;
    const int e = spp_plane_block(blockIdx.x - chunk * gx, gx) * 256 + tid;
    const bool live = e < plane;
    const int jj = e / nphi, k = e - jj * nphi;
    const int j = jj < nth ? jj : nth - 1;
    const int el = j * nphi + k;
    const int ejp = j + 1 < nth ? el + nphi : el;      // pole faces: sigma = 0
    const int ejm = j > 0 ? el - nphi : el;
    const int tkp = k + 1 < nphi ? tid + 1 : tid + 1 - nphi;
    const int tkm = k > 0 ? tid - 1 : tid - 1 + nphi;
    const int i0 = chunk * ROWS;
    auto clampr = [&](int i) { return i < 0 ? 0 : (i < nr ? i : nr - 1); };
    double c[ROWS + 2], jp[ROWS], jm[ROWS], src[ROWS];
#pragma unroll
    for (int u = 0; u < ROWS + 2; ++u) c[u] = phi[size_t(clampr(i0 - 1 + u)) * plane + el];
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const size_t b = size_t(clampr(i0 + u)) * plane;
        jp[u] = phi[b + ejp];
        jm[u] = phi[b + ejm];
        src[u] = rho[b + el];
    }
    const double to = i0 + ROWS >= nr ? tout[el] : 0.0;
    const double ti = (i0 == 0 && tin) ? tin[el] : 0.0;
    const double sp = t.sig[j + 1], sm = t.sig[j], dm = t.dmu[j], sjv = t.Sj[j];
    double fal = 0.0, fv = 1.0, fvr = 0.0;
    if (tid <= ROWS) {
        fal = t.alpha[clampr(i0 - 1 + tid)];
        fv = t.V[clampr(i0 + tid)];
        fvr = t.VR[clampr(i0 + tid)];
    }
    // every load is awaited here, once, before any store
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt not waited
#pragma unroll
    for (int u = 0; u < ROWS; ++u) cs[u][tid] = c[u + 1];
    if (tid <= ROWS) {
        const double iv = 1.0 / fv;
        fa[0][tid] = fal;
        fa[1][tid] = iv;
        fa[2][tid] = fvr * iv;
    }
    const double idm = 1.0 / dm, sj = sjv * inv_dphi2;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int i = i0 + u;
        const double x = c[u + 1];
        const double fo = i + 1 < nr ? fa[0][u + 1] * (c[u + 2] - x) : -to;
        const double fi = i > 0 ? fa[0][u] * (x - c[u]) : ti;
        const double th = sp * (jp[u] - x) - sm * (x - jm[u]);
        const double ph = cs[u][tkp] - 2.0 * x + cs[u][tkm];
        const double LP = (fo - fi) * fa[1][u] + fa[2][u] * (th * idm + sj * ph);
        if (live && i < nr) __builtin_nontemporal_store(four_pi_g * src[u] - LP, r + size_t(i) * plane + el);
    }
}

bool launch_proj_f32(const double* A, const float* B, double* C, int M, int K, int nphi, bool accum, hipStream_t s)
{
    if (K > 128) return false;
    const int rn = projimg::rn_for(K);
    const int rm = rn == 8 ? 1 : rn == 4 ? 2 : 4;
    const int groups = (M + 16 * rm - 1) / (16 * rm);
    int splits = (device_cus() + nphi - 1) / nphi;
    const int maxsplits = (groups + proj::NWAVES - 1) / proj::NWAVES;
    if (splits > maxsplits) splits = maxsplits;
    if (splits < 1) splits = 1;
    const dim3 grid(splits, nphi), block(64 * proj::NWAVES);
    const bool kvec = (K % 32) == 0;
#define SPP_PROJ32(RN, RM, KV, AC) \
    hipLaunchKernelGGL((proj::k_proj_f32<RN, RM, KV, AC>), grid, block, 0, s, A, B, C, M, K, nphi, splits)
#define SPP_PROJ32_CASE(RN, RM)                                                    \
    case RN:                                                                       \
        if (kvec) { if (accum) SPP_PROJ32(RN, RM, true, true); else SPP_PROJ32(RN, RM, true, false); }     \
        else { if (accum) SPP_PROJ32(RN, RM, false, true); else SPP_PROJ32(RN, RM, false, false); }        \
        break;
    switch (rn) {
        SPP_PROJ32_CASE(1, 4)
        SPP_PROJ32_CASE(2, 4)
        SPP_PROJ32_CASE(4, 2)
        SPP_PROJ32_CASE(8, 1)
    }
#undef SPP_PROJ32_CASE
#undef SPP_PROJ32
    return true;
}

}  // namespace

// Typed views of a plan's device tables.
struct PlanTables {
    const char* base;
    explicit PlanTables(const spp_plan_s* p) : base(static_cast<const char*>(p->dev)) {}
    const double* d(size_t off) const { return reinterpret_cast<const double*>(base + off); }
    const float* f(size_t off) const { return reinterpret_cast<const float*>(base + off); }
    const c64* c(size_t off) const { return reinterpret_cast<const c64*>(base + off); }
};

spp_status spp_launch_solve_f64(const spp_plan_s* p, const double* rho, double* phi, double G, void* ws,
                                void* stream, hipEvent_t* ev, const unsigned* gate)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const PlanTables T(p);
    const auto& L = p->lay;
    const c64* tw = T.c(L.tw);
    const double *lam = T.d(L.lam), *beta = T.d(L.beta);
    const radial::Coef cf{T.d(L.alpha), T.d(L.V), T.d(L.VR), p->nr, T.d(L.gamma)};

    const int nr = p->nr, nth = p->nth, nphi = p->nphi;
    const int nlines = nr * nth;
    const size_t field = spp_align256(size_t(nlines) * nphi * sizeof(double));
    // the status record, then the fields
    auto* rec = static_cast<spp_status_record*>(ws);
    char* fields = static_cast<char*>(ws) + SPP_STATUS_BYTES;
    double* X = reinterpret_cast<double*>(fields);
    double* Y = reinterpret_cast<double*>(fields + field);
    // a gated solve (the mixed form's fallback) keeps the record it reports into
    const FftExtra fwd{gate ? nullptr : rec, gate}, inv{rec, gate};

    // s~ scaled so that the inverse transform needs no 1/N: 4 pi G / N_phi
    const double scale = 4.0 * M_PI * G / nphi;
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], s);
    };
    if (spp_plan_fused(p)) {
        mark(0);
        if (!launch_fft(nphi, true, rho, X, tw, scale, nlines, s, true, nth, fwd))
            return spp_fail(SPP_ENOTSUP, "spp_solve: unsupported nphi");
        mark(1);
        // the workspace's region after the spectral field is the sink of the
        // per-mode kernel's stores of padding rows and columns
        static_assert(modal::THREADS * sizeof(double) <= spp_modal_sink_bytes, "sink of one workgroup");
        // the kernel reaches the sink by 32-bit byte offsets from each unit's rows
        if (field + spp_modal_sink_bytes > (size_t(1) << 32))
            return spp_fail(SPP_ENOTSUP, "spp_solve: field too large for the fused kernel");
        double* sink = reinterpret_cast<double*>(fields + field);
        if (!launch_modal(X, T.d(L.Fimg), T.d(L.Iimg), T.d(L.Rimg), lam, beta, cf, nr, nth, nphi, sink, s, gate))
            return spp_fail(SPP_ENOTSUP, "spp_solve: grid outside the fused kernel's range");
        mark(2);
        mark(3);
        mark(4);
        launch_fft(nphi, false, X, phi, tw, 1.0, nlines, s, true, nth, inv);
        mark(5);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("spp_solve: ") + hipGetErrorString(e));
        return SPP_OK;
    }
    mark(0);
    if (!launch_fft(nphi, true, rho, X, tw, scale, nlines, s, false, 0, fwd))
        return spp_fail(SPP_ENOTSUP, "spp_solve: unsupported nphi");
    mark(1);
    const dim3 pgrid((nth + PBN - 1) / PBN, (nr + PBM - 1) / PBM, nphi);
    if (!launch_proj_par(X, T.d(L.Wpar), Y, nr, nth, nphi, true, p->par_rn, s, gate) &&
        !launch_proj(X, T.d(L.Wimg), Y, nr, nth, nphi, s, gate))
        hipLaunchKernelGGL(k_proj_f64, pgrid, dim3(256), 0, s, X, T.d(L.W), Y, nr, nth, nphi, gate);
    mark(2);
    const int nsys = nphi * nth;
    if (!launch_radial_part(Y, lam, beta, cf, nth, nphi, s, gate))
        hipLaunchKernelGGL(k_radial, dim3((nsys + 255) / 256), dim3(256), 0, s, Y, X, lam, beta, cf.gamma, cf.alpha,
                           cf.V, cf.VR, nr, nth, nphi, gate);
    mark(3);
    if (!launch_proj_par(Y, T.d(L.Hpar), X, nr, nth, nphi, false, p->par_rn, s, gate) &&
        !launch_proj(Y, T.d(L.Himg), X, nr, nth, nphi, s, gate))
        hipLaunchKernelGGL(k_proj_f64, pgrid, dim3(256), 0, s, Y, T.d(L.H), X, nr, nth, nphi, gate);
    mark(4);
    launch_fft(nphi, false, X, phi, tw, 1.0, nlines, s, false, 0, inv);
    mark(5);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("spp_solve: ") + hipGetErrorString(e));
    return SPP_OK;
}

namespace {

// Workspace of the mixed form after the status record: s~, the accumulated
// g, the residual, the projections' field, the outer and inner shell terms,
// and the per-component maxima of the residuals [SPP_MAX_REFINE + 1][N_phi].
struct MixedLayout {
    size_t field, shell, St, Gf, Y, Z, ob, ib, part, total;
    explicit MixedLayout(const spp_plan_s* p)
    {
        field = spp_align256(size_t(p->nr) * p->nth * p->nphi * sizeof(double));
        shell = spp_align256(size_t(p->nphi) * p->nth * sizeof(double));
        St = SPP_STATUS_BYTES;
        Gf = St + field;
        Y = Gf + field;
        Z = Y + field;
        ob = Z + field;
        ib = ob + shell;
        part = ib + shell;
        total = part + spp_align256(size_t(SPP_MAX_REFINE + 1) * p->nphi * sizeof(unsigned long long));
    }
};

// The outer-face term beta(A) g_N (and with the regular inner condition the
// inner-face term gamma(A) g_1) of every Fourier component of the field F
// [q][i][j] into ob (ib) [q][j].
void launch_shell_terms(const spp_plan_s* p, const double* F, double* ob, double* ib, hipStream_t s)
{
    const PlanTables T(p);
    const auto& L = p->lay;
    const int nr = p->nr, nth = p->nth, nphi = p->nphi;
    faceflux::launch_outer(F + size_t(nr - 1) * nth, size_t(nr) * nth, ob, T.d(L.Bo), nth, nphi, s);
    if (ib) faceflux::launch_outer(F, size_t(nr) * nth, ib, T.d(L.Bi), nth, nphi, s);
}

}  // namespace

size_t spp_mixed_workspace_bytes(const spp_plan_s* p)
{
    const MixedLayout M(p);
    // the FP64 fallback solve runs in the same workspace
    return std::max(M.total, spp_path_workspace_bytes(p, spp_plan_fused(p)));
}

// Mixed-precision solve (iterative refinement in Fourier space):
//   s~ = FFT(4 pi G rho)                          FP64, once
//   g  = H~ F^-1 W~ s~                            FP32-MFMA projections, FP64 radial
//   repeat n_refine times:
//     r = s~ - L g                                FP64 (local stencil + boundary terms)
//     g += H~ F^-1 W~ r
//   Phi = IFFT(g)                                 FP64, once
// then the contraction check of k_refine_gate and, if a step did not contract
// and fallback_fp64 is set, the FP64 solve, gated on the device.
spp_status spp_launch_solve_mixed(const spp_plan_s* p, spp_precision, int n_refine, int fallback_fp64,
                                  const double* rho, double* phi, double G, void* ws, void* stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const PlanTables T(p);
    const auto& L = p->lay;
    const c64* tw = T.c(L.tw);
    const float* W32 = T.f(L.Wimg32);
    const float* H32 = T.f(L.Himg32);
    const radial::Coef cf{T.d(L.alpha), T.d(L.V), T.d(L.VR), p->nr, T.d(L.gamma)};

    const int nr = p->nr, nth = p->nth, nphi = p->nphi;
    const int nlines = nr * nth;
    const MixedLayout M(p);
    char* w = static_cast<char*>(ws);
    auto* rec = reinterpret_cast<spp_status_record*>(w);
    double* St = reinterpret_cast<double*>(w + M.St);   // s~ (kept for the residuals)
    double* Gf = reinterpret_cast<double*>(w + M.Gf);   // accumulated g
    double* Y = reinterpret_cast<double*>(w + M.Y);     // residual
    double* Z = reinterpret_cast<double*>(w + M.Z);     // projections / radial solves
    double* ob = reinterpret_cast<double*>(w + M.ob);   // outer-shell term
    double* ib = p->inner_regular ? reinterpret_cast<double*>(w + M.ib) : nullptr;
    auto* part = reinterpret_cast<unsigned long long*>(w + M.part);

    const ResidualTables rt{T.d(L.alpha), T.d(L.V), T.d(L.VR), T.d(L.sig), T.d(L.dmu), T.d(L.Sj), T.d(L.lamphi)};
    const double scale = 4.0 * M_PI * G / nphi;
    if (!launch_fft(nphi, true, rho, St, tw, scale, nlines, s, false, 0, FftExtra{rec, nullptr}))
        return spp_fail(SPP_ENOTSUP, "spp_solve_mixed: unsupported nphi");
    // per-component maxima start at zero (a fill kernel, capturable)
    const size_t npart = size_t(n_refine + 1) * nphi;
    hipLaunchKernelGGL(k_fill_u64, dim3((npart + 255) / 256), dim3(256), 0, s, part, npart);
    const int rgx = (nth * ((nr + RES_ROWS - 1) / RES_ROWS) + 255) / 256;
    for (int it = 0; it <= n_refine; ++it) {
        const double* src = St;
        if (it > 0) {
            // boundary terms of the current g
            launch_shell_terms(p, Gf, ob, ib, s);
            hipLaunchKernelGGL(k_residual, dim3(rgx, nphi), dim3(256), 0, s, St, Gf, ob, ib, Y, rt, nr, nth, nphi,
                               part + size_t(it) * nphi, it == 1 ? part : nullptr);
            src = Y;
        }
        launch_proj_f32(src, W32, Z, nr, nth, nphi, false, s);
        if (!launch_radial_part(Z, T.d(L.lam), T.d(L.beta), cf, nth, nphi, s))
            hipLaunchKernelGGL(k_radial, dim3((nphi * nth + 255) / 256), dim3(256), 0, s, Z, Y, T.d(L.lam),
                               T.d(L.beta), cf.gamma, cf.alpha, cf.V, cf.VR, nr, nth, nphi, nullptr);
        launch_proj_f32(Z, H32, Gf, nr, nth, nphi, it > 0, s);
    }
    launch_fft(nphi, false, Gf, phi, tw, 1.0, nlines, s, false, 0, FftExtra{rec, nullptr});
    hipLaunchKernelGGL(k_refine_gate, dim3(1), dim3(256), 0, s, rec, part, nphi, n_refine, fallback_fp64);
    if (fallback_fp64 && n_refine > 0) {
        // the FP64 solve in the same workspace (its spectral fields overlay
        // s~ and g), run only when the gate opened
        const spp_status st = spp_launch_solve_f64(p, rho, phi, G, ws, stream, nullptr, &rec->fallback);
        if (st != SPP_OK) return st;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("spp_solve_mixed: ") + hipGetErrorString(e));
    return SPP_OK;
}

// Face fluxes of grad Phi (fluxes.hip.h).  The outer face needs the boundary
// term of Sec. 3.2 on the outermost shell, T = beta(A) Phi_shell, which acts
// per angular eigenmode: the shell's Fourier components (forward FFT of its
// N_theta lines), the per-mode product of faceflux::launch_outer, and
// the inverse FFT back to [j][k].  Workspace after its status record: two
// shell-sized buffers A, B (A: spectrum, B: boundary term per component, A:
// T).
spp_status spp_launch_face_fluxes(const spp_plan_s* p, const double* phi, double* fr, double* ft, double* fp,
                                  void* ws, void* stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const PlanTables T(p);
    const auto& L = p->lay;
    const c64* tw = T.c(L.tw);
    const int nr = p->nr, nth = p->nth, nphi = p->nphi;
    const int plane = nth * nphi;
    char* w = static_cast<char*>(ws) + SPP_STATUS_BYTES;
    double* A = reinterpret_cast<double*>(w);
    double* B = reinterpret_cast<double*>(w + spp_align256(size_t(plane) * sizeof(double)));

    if (nth > faceflux::OUTER_NTH_MAX)
        return spp_fail(SPP_ENOTSUP, "spp_face_fluxes: needs N_theta <= " + std::to_string(faceflux::OUTER_NTH_MAX));
    if (p->inner_regular)
        return spp_fail(SPP_ENOTSUP, "spp_face_fluxes: the inner face flux of the regular inner condition is not "
                                     "stored (grids with r_{1/2} > 0 need the zero-flux condition here)");
    if (!launch_fft(nphi, true, phi + size_t(nr - 1) * plane, A, tw, 1.0 / nphi, nth, s))
        return spp_fail(SPP_ENOTSUP, "spp_face_fluxes: unsupported nphi");
    faceflux::launch_outer(A, size_t(nth), B, T.d(L.Bo), nth, nphi, s);
    launch_fft(nphi, false, B, A, tw, 1.0, nth, s);
    const faceflux::Tables t{T.d(L.alpha), T.d(L.VR), T.d(L.sig), T.d(L.dmu), T.d(L.Sj)};
    const int gx = (plane + faceflux::THREADS - 1) / faceflux::THREADS;
    const int chunks = (nr + faceflux::ROWS - 1) / faceflux::ROWS;
    hipLaunchKernelGGL(faceflux::k_face_fluxes, dim3(gx * chunks), dim3(faceflux::THREADS), 0, s, phi, A, fr, ft, fp,
                       t, nr, nth, nphi, 2.0 * M_PI / nphi, gx);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("spp_face_fluxes: ") + hipGetErrorString(e));
    return SPP_OK;
}

// Force on every cell from the gravitational stress tensor (momentum.hip.h).
// The outer face's normal gradient, -beta(A) Phi_shell / r_o^2, comes from the
// shell transforms as for the face fluxes.  Workspace after its status
// record: two shell buffers.
spp_status spp_launch_momentum(const spp_plan_s* p, const double* phi, double G, double* fx, double* fy, double* fz,
                               void* ws, void* stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const PlanTables T(p);
    const auto& L = p->lay;
    const c64* tw = T.c(L.tw);
    const int nr = p->nr, nth = p->nth, nphi = p->nphi;
    const int plane = nth * nphi;
    char* w = static_cast<char*>(ws) + SPP_STATUS_BYTES;
    double* A = reinterpret_cast<double*>(w);
    double* B = reinterpret_cast<double*>(w + spp_align256(size_t(plane) * sizeof(double)));
    if (nth > faceflux::OUTER_NTH_MAX)
        return spp_fail(SPP_ENOTSUP, "spp_momentum_source: needs N_theta <= " + std::to_string(faceflux::OUTER_NTH_MAX));
    if (p->inner_regular)
        return spp_fail(SPP_ENOTSUP, "spp_momentum_source: grids with the regular inner condition are not supported");
    if (!launch_fft(nphi, true, phi + size_t(nr - 1) * plane, A, tw, 1.0 / nphi, nth, s))
        return spp_fail(SPP_ENOTSUP, "spp_momentum_source: unsupported nphi");
    faceflux::launch_outer(A, size_t(nth), B, T.d(L.Bo), nth, nphi, s);
    launch_fft(nphi, false, B, A, tw, 1.0, nth, s);
    const spp_mom_layout M(nr, nth, nphi);
    const double* q = T.d(L.mom);
    const momentum::Tables t{q + M.R2, q + M.ring, q + M.invr, q + M.invdr, q + M.is2, q + M.isc, q + M.is,
                             q + M.ic, q + M.dth, q + M.invsdp, q + M.invdthc, q + M.fst, q + M.fct, q + M.jc,
                             q + M.js, q + M.cp1, q + M.sp1};
    const int gx = (plane + momentum::THREADS - 1) / momentum::THREADS;
    const int chunks = (nr + momentum::MROWS - 1) / momentum::MROWS;
    const double ro = p->r_if[nr];
    // workgroups of whole theta rows (64 <= N_phi <= 256) share the phi-faces
    // through LDS; otherwise with N_phi a multiple of 64 every wave (64
    // consecutive plane elements from a multiple of 64) still lies within one
    // theta row
    if (nphi >= 64 && momentum::THREADS % nphi == 0) {
        const int lchunks = (nr + momentum::ROWS_LDS - 1) / momentum::ROWS_LDS;
        // whole workgroups only (every thread on a cell) unless the plane ends mid-workgroup
        auto kern = (nth * nphi) % momentum::THREADS == 0 ? momentum::k_momentum_rows<false>
                                                          : momentum::k_momentum_rows<true>;
        hipLaunchKernelGGL(kern, dim3(gx * lchunks), dim3(momentum::THREADS), 0, s, phi, A, fx,
                           fy, fz, t, nr, nth, nphi, 2.0 * M_PI / nphi, 1.0 / (4.0 * M_PI * G), 1.0 / (ro * ro), gx);
    } else {
        auto kern = nphi % 64 == 0 ? momentum::k_momentum<true> : momentum::k_momentum<false>;
        hipLaunchKernelGGL(kern, dim3(gx * chunks), dim3(momentum::THREADS), 0, s, phi, A, fx, fy, fz, t, nr, nth,
                           nphi, 2.0 * M_PI / nphi, 1.0 / (4.0 * M_PI * G), 1.0 / (ro * ro), gx);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("spp_momentum_source: ") + hipGetErrorString(e));
    return SPP_OK;
}

// r = 4 pi G rho - L Phi (spp_residual).  The boundary terms of the outermost
// (and, with the regular inner condition, the innermost) shell act per angular
// eigenmode: shell FFT, the two per-mode products, inverse FFT, as for the
// face fluxes.  Workspace after its status record: four shell buffers.
spp_status spp_launch_residual(const spp_plan_s* p, const double* rho, const double* phi, double G, double* r,
                               void* ws, void* stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const PlanTables T(p);
    const auto& L = p->lay;
    const c64* tw = T.c(L.tw);
    const int nr = p->nr, nth = p->nth, nphi = p->nphi;
    const int plane = nth * nphi;
    const size_t sh = spp_align256(size_t(plane) * sizeof(double));
    char* w = static_cast<char*>(ws) + SPP_STATUS_BYTES;
    double *A = reinterpret_cast<double*>(w), *B = reinterpret_cast<double*>(w + sh);
    double *C = reinterpret_cast<double*>(w + 2 * sh), *D = reinterpret_cast<double*>(w + 3 * sh);
    if (nth > faceflux::OUTER_NTH_MAX)
        return spp_fail(SPP_ENOTSUP, "spp_residual: needs N_theta <= " + std::to_string(faceflux::OUTER_NTH_MAX));
    // shell -> spec (Fourier components) -> tmp (boundary term per component) -> spec ([j][k])
    auto shell_term = [&](const double* shell, const double* op, double* spec, double* tmp) {
        launch_fft(nphi, true, shell, spec, tw, 1.0 / nphi, nth, s);
        faceflux::launch_outer(spec, size_t(nth), tmp, op, nth, nphi, s);
        launch_fft(nphi, false, tmp, spec, tw, 1.0, nth, s);
    };
    shell_term(phi + size_t(nr - 1) * plane, T.d(L.Bo), A, B);
    if (p->inner_regular) shell_term(phi, T.d(L.Bi), C, D);
    const ResidualTables rt{T.d(L.alpha), T.d(L.V), T.d(L.VR), T.d(L.sig), T.d(L.dmu), T.d(L.Sj), T.d(L.lamphi)};
    const int gx = (plane + 255) / 256;
    const double dphi = 2.0 * M_PI / nphi;
    const double* tin = p->inner_regular ? C : nullptr;
    if (256 % nphi == 0) {
        const int chunks = (nr + RES_LDS_ROWS - 1) / RES_LDS_ROWS;
        hipLaunchKernelGGL(k_residual_rows<RES_LDS_ROWS>, dim3(gx * chunks), dim3(256), 0, s, rho, phi, A, tin, r, rt,
                           4.0 * M_PI * G, nr, nth, nphi, 1.0 / (dphi * dphi), gx);
    } else {
        const int chunks = (nr + RROWS - 1) / RROWS;
        hipLaunchKernelGGL(k_residual_phys, dim3(gx * chunks), dim3(256), 0, s, rho, phi, A, tin, r, rt,
                           4.0 * M_PI * G, nr, nth, nphi, 1.0 / (dphi * dphi), gx);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("spp_residual: ") + hipGetErrorString(e));
    return SPP_OK;
}

// Batched FP64 solves of n right-hand sides of one fused-path plan: the
// folded forward FFT, the per-mode kernel and the folded inverse FFT, each one
// launch over all n (workgroups of RHS r consecutive).  recs: n status
// records; X: n spectral fields back to back; sink: the per-mode kernel's
// store sink, after the fields and within 4 GB of X (spp_class_batch_bytes
// sizes records, fields and sink together); the tables (device) hold each
// RHS's rho, phi and 4 pi G_r / N_phi.  paired: the per-mode kernel's
// XCD-paired unit order.
size_t spp_class_batch_bytes(const spp_plan_s* p, int n)
{
    const size_t field = spp_align256(size_t(p->nr) * p->nth * p->nphi * sizeof(double));
    return size_t(n) * (SPP_STATUS_BYTES + field) + spp_modal_sink_bytes;
}

spp_status spp_launch_class_batch(const spp_plan_s* p, int n, const double* const* rho_tab,
                                  double* const* phi_tab, const double* scale_tab, spp_status_record* recs,
                                  double* X, double* sink, int paired, hipStream_t s)
{
    if (!spp_plan_fused(p)) return spp_fail(SPP_ENOTSUP, "batched launch: plan not on the fused path");
    const PlanTables T(p);
    const auto& L = p->lay;
    const int nr = p->nr, nth = p->nth, nphi = p->nphi, nlines = nr * nth;
    const size_t field = spp_align256(size_t(nlines) * nphi * sizeof(double));
    // the per-mode kernel reaches the sink by 32-bit byte offsets from each unit's rows
    const size_t reach = size_t(reinterpret_cast<char*>(sink) - reinterpret_cast<char*>(X)) + spp_modal_sink_bytes;
    if (reinterpret_cast<char*>(sink) < reinterpret_cast<char*>(X) + size_t(n) * field || reach > (size_t(1) << 32))
        return spp_fail(SPP_ENOTSUP, "batched launch: the store sink must follow the fields within 4 GB");
    const size_t xstride = field / sizeof(double);
    FftExtra fwd{recs, nullptr, spp_batch_view{rho_tab, nullptr, scale_tab, xstride}, n};
    FftExtra inv{recs, nullptr, spp_batch_view{nullptr, phi_tab, nullptr, xstride}, n};
    const radial::Coef cf{T.d(L.alpha), T.d(L.V), T.d(L.VR), nr, T.d(L.gamma)};
    if (!launch_fft(nphi, true, nullptr, X, T.c(L.tw), 0.0, nlines, s, true, nth, fwd))
        return spp_fail(SPP_ENOTSUP, "batched launch: unsupported nphi");
    if (!launch_modal(X, T.d(L.Fimg), T.d(L.Iimg), T.d(L.Rimg), T.d(L.lam), T.d(L.beta), cf, nr, nth, nphi, sink, s,
                      nullptr, n, xstride, paired))
        return spp_fail(SPP_ENOTSUP, "batched launch: grid outside the fused kernel's range");
    launch_fft(nphi, false, X, nullptr, T.c(L.tw), 1.0, nlines, s, true, nth, inv);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("batched launch: ") + hipGetErrorString(e));
    return SPP_OK;
}

// Time every candidate tile of the projection kernel on this plan's shape
// (forward projection on the workspace buffers, whose contents do not matter
// for timing) and record the fastest for (N_theta, N_r).  Synchronises the
// stream.  *chosen_rm receives the choice (may be NULL).
spp_status spp_autotune_projection_impl(const spp_plan_s* p, void* ws, void* stream, int* chosen_rm)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->nth > 128) {
        if (chosen_rm) *chosen_rm = 0;
        return SPP_OK;
    }
    const char* base = static_cast<const char*>(p->dev);
    const double* Wimg = reinterpret_cast<const double*>(base + p->lay.Wimg);
    const size_t field = spp_align256(size_t(p->nr) * p->nth * p->nphi * sizeof(double));
    const double* A = reinterpret_cast<const double*>(static_cast<char*>(ws) + SPP_STATUS_BYTES);
    double* C = reinterpret_cast<double*>(static_cast<char*>(ws) + SPP_STATUS_BYTES + field);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return spp_fail(SPP_EDEVICE, "autotune: hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return spp_fail(SPP_EDEVICE, "autotune: hipEventCreate");
    }
    int best = proj_rm_default(projimg::rn_for(p->nth));
    float best_ms = 1e30f;
    for (int rm : proj_rm_candidates(projimg::rn_for(p->nth))) {
        launch_proj_rm(A, Wimg, C, p->nr, p->nth, p->nphi, rm, s);   // warm-up
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 3; ++r) launch_proj_rm(A, Wimg, C, p->nr, p->nth, p->nphi, rm, s);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) {
            best_ms = ms;
            best = rm;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned_rm[{p->nth, p->nr}] = best;
    }
    if (chosen_rm) *chosen_rm = best;
    return SPP_OK;
}

// Evaluate the launch-configuration caches (CU count, FFT occupancy) for
// this plan outside any stream capture.
void spp_prewarm_launch_caches(const spp_plan_s* p)
{
    (void)device_cus();
    switch (p->nphi) {
#define SPP_WARM(n)                                                                                    \
    case n:                                                                                            \
        fft_resident<n>(true, false); fft_resident<n>(false, false);                                   \
        fft_resident<n>(true, true); fft_resident<n>(false, true);                                     \
        break;
        SPP_WARM(4) SPP_WARM(8) SPP_WARM(16) SPP_WARM(32) SPP_WARM(64)
        SPP_WARM(128) SPP_WARM(256) SPP_WARM(512) SPP_WARM(1024) SPP_WARM(2048)
#undef SPP_WARM
    default: break;
    }
}

// Kernels an FP64 solve of this plan launches, in order, named by the same
// selection rules as spp_launch_solve_f64 (separated by semicolons).
std::string spp_describe_solve(const spp_plan_s* p)
{
    const int nr = p->nr, nth = p->nth, nphi = p->nphi;
    const std::string n = std::to_string(nphi);
    if (spp_plan_fused(p)) {
        int rn = 0, T = 0;
        modal_variant(nr, nth, &rn, &T);
        return "k_rfft_fwd<" + n + ",fold>;modal::k_modal<" + std::to_string(rn) + "," + std::to_string(T) +
               ">;k_rfft_inv<" + n + ",fold>";
    }
    std::string proj;
    if (p->par_rn != 0)
        proj = "proj::k_proj_par<" + std::to_string(p->par_rn) + ">";
    else if (nth <= 128)
        proj = "proj::k_proj_f64<" + std::to_string(projimg::rn_for(nth)) + "," + std::to_string(proj_rm(nth, nr)) + ">";
    else
        proj = "k_proj_f64";
    const int cap = radial_part_capacity(nr);
    const std::string rad = cap ? "radial::k_radial_part<" + std::to_string(cap) + ">" : "k_radial";
    return "k_rfft_fwd<" + n + ">;" + proj + ";" + rad + ";" + proj + ";k_rfft_inv<" + n + ">";
}
