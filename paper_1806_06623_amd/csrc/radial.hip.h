// Radial tridiagonal solves (Sec. 3.2: Delta_r f + R_i lambda_Omega f = s^ for
// every (m, l), with the asymptotic outer boundary condition), float64.
//
// Every row is scaled by V_i, which makes each system symmetric:
//   alpha_{i-1} f_{i-1} + b_i f_i + alpha_i f_{i+1} = V_i s^_i,
//   b_i = -(alpha_{i-1} + alpha_i) + V_i R_i lambda   (alpha_{-1} = 0),
// and on the outermost row the missing face coefficient is beta(lambda).
//
// Partition method, one workgroup per 16 systems and P <= 32 chunks of rows:
// lane (s, p) holds rows [s_p, s_{p+1}) of system s in registers.  Row s_p is
// a separator; the interior rows of a chunk are eliminated locally, which
// expresses its first and last interior unknowns in terms of the two
// separators around it.  Substituting those into the separator rows gives a
// P x P tridiagonal system per system (the Schur complement), solved by
// parallel cyclic reduction over the P lanes of the system through LDS; each
// lane then back-substitutes its interior with the separators known.  Every
// value is read from and written to HBM once.
#pragma once
#include <hip/hip_runtime.h>

#include "status.h"

namespace radial {

constexpr int SYS = 16;     // systems per workgroup (consecutive (q, l) pairs)
constexpr int PMAX = 32;    // chunks per system
constexpr int THREADS = SYS * PMAX;

constexpr int NRMAX = 640;  // largest N_r of the partitioned kernel (PMAX * 20)

struct Coef {
    const double* alpha;    // alpha_i, coupling rows i and i+1; alpha[nr-1] = 0
    const double* V;
    const double* VR;
    int nr;
    const double* gamma;    // inner-face coefficient gamma(lambda), [M][N_theta] (zero
                            // unless the regular inner condition with r_{1/2} > 0)
};

// Per-row coefficients staged in LDS once per workgroup.
struct RowCoef {
    const double* alpha;    // LDS
    const double* VR;       // LDS
    int nr;
    __device__ __forceinline__ double off(int i) const { return alpha[i]; }
    // diagonal of row i for eigenvalue lm, outer coefficient bo and inner
    // coefficient gi (the innermost row's missing coupling is gi)
    __device__ __forceinline__ double diag(int i, double lm, double bo, double gi) const
    {
        const double am = i > 0 ? alpha[i - 1] : gi;
        double b = -(am + alpha[i]) + VR[i] * lm;
        if (i == nr - 1) b -= bo;
        return b;
    }
};

// 1/w from the hardware reciprocal estimate y0 (relative error below 2^-24
// on gfx950) and its residual e = 1 - w y0:  1/w = y0 / (1 - e)
// = y0 (1 + e + e^2) + O(e^3 y0).  The truncation term e^3 < 2^-72 lies far
// below the last bit of float64, so the error is that of the three rounded
// operations, within about one ulp (not always the correctly rounded
// reciprocal).  One fused multiply-add fewer than two Newton steps.
__device__ __forceinline__ double recip(double w)
{
    const double y = __builtin_amdgcn_rcp(w);
    const double e = __builtin_fma(-w, y, 1.0);
    return __builtin_fma(y, __builtin_fma(e, e, e), y);
}

// 512 threads and at most 128 VGPRs per lane: two workgroups per CU.
template <int CH>
__global__ __launch_bounds__(THREADS, 4) void k_radial_part(double* __restrict__ Y, const double* __restrict__ lam,
                                                      const double* __restrict__ beta, Coef tab, int nth,
                                                      int nphi, int P, const unsigned* __restrict__ gate)
{
    if (spp_gate_closed(gate)) return;
    __shared__ double own[3][PMAX][SYS];   // separator row p: B (diag part), C, D
    __shared__ double nxt[3][PMAX][SYS];   // contribution of chunk p to row p+1: A, B add, D sub
    __shared__ double red[4][PMAX][SYS];   // reduced rows (A, B, C, D) during cyclic reduction
    __shared__ double xs[PMAX + 1][SYS];
    __shared__ double c_alpha[NRMAX], c_VR[NRMAX], c_V[NRMAX];

    const int nr = tab.nr;
    for (int i = threadIdx.x; i < nr; i += THREADS) {
        c_alpha[i] = tab.alpha[i];
        c_VR[i] = tab.VR[i];
        c_V[i] = tab.V[i];
    }
    const int t = threadIdx.x;
    const int sl = t % SYS, p = t / SYS;
    const int nsys = nphi * nth;
    const int sys_raw = blockIdx.x * SYS + sl;
    const bool live = sys_raw < nsys;
    const int sys = live ? sys_raw : nsys - 1;
    const int q = sys / nth, l = sys - q * nth;
    const int m = q <= nphi / 2 ? q : nphi - q;
    const double lm = lam[m * nth + l];
    const double bo = beta[m * nth + l];
    const double gi = tab.gamma[m * nth + l];
    const bool active = p < P;

    const int s0 = active ? (p * nr) / P : 0;
    const int s1 = active ? ((p + 1) * nr) / P : 0;
    const int n = s1 - s0 - 1;                  // interior rows s0+1 .. s1-1
    const bool last = p == P - 1;
    double* col = Y + size_t(q) * nr * nth + l;

    // this lane's rows, loaded unconditionally (row index clamped; values of
    // rows beyond the chunk are never used) so that all loads are in flight
    double d[CH];
    double invw[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int row = s0 + k < nr ? s0 + k : nr - 1;
        d[k] = col[size_t(row) * nth];
        invw[k] = 0.0;
    }
    __syncthreads();   // coefficient tables in LDS
    const RowCoef cf{c_alpha, c_VR, nr};
#pragma unroll
    for (int k = 0; k < CH; ++k)
        if (k <= n) d[k] *= c_V[s0 + k];

    // ---- pass 1: eliminate the interior in both directions
    double Yf = 0.0, Uf = 0.0, Vf = 1.0, Yl = 0.0, Ul = 1.0, Vl = 0.0;
    const double oL = (active && s0 + 1 < nr) ? cf.off(s0) : 0.0;                 // s0 <-> s0+1
    const double oR = (active && !last) ? cf.off(s1 - 1) : 0.0;                  // s1-1 <-> s1
    if (active && n >= 1) {
        // forward (LU): pivots w_k, running L^-1 d and L^-1 (-oL e_1)
        double w = 1.0, zf = 0.0, uf = 0.0, iwn = 0.0;
#pragma unroll
        for (int k = 1; k < CH; ++k) {
            if (k <= n) {
                const int i = s0 + k;
                if (k == 1) {
                    w = cf.diag(i, lm, bo, gi);
                    zf = d[1];
                    uf = -oL;
                } else {
                    const double o = cf.off(i - 1);
                    const double mult = o * invw[k - 1];
                    w = cf.diag(i, lm, bo, gi) - mult * o;
                    zf = d[k] - mult * zf;
                    uf = -mult * uf;
                }
                invw[k] = recip(w);
                iwn = invw[k];
            }
        }
        Yl = zf * iwn;
        Ul = uf * iwn;
        Vl = -oR * iwn;
        // backward (UL): pivots from the last interior row upwards
        double wh = 1.0, zh = 0.0, vh = 0.0, iwh = 0.0;
#pragma unroll
        for (int k = CH - 1; k >= 1; --k) {
            if (k <= n) {
                const int i = s0 + k;
                if (k == n) {
                    wh = cf.diag(i, lm, bo, gi);
                    zh = d[k];
                    vh = -oR;
                } else {
                    const double o = cf.off(i);
                    const double mult = o * iwh;
                    wh = cf.diag(i, lm, bo, gi) - mult * o;
                    zh = d[k] - mult * zh;
                    vh = -mult * vh;
                }
                iwh = recip(wh);
            }
        }
        Yf = zh * iwh;
        Vf = vh * iwh;
        Uf = -oL * iwh;
    }

    // ---- reduced system over the separators s_0..s_{P-1}
    if (active) {
        const double bs = cf.diag(s0, lm, bo, gi);
        own[0][p][sl] = bs + oL * Uf;
        own[1][p][sl] = oL * Vf;
        own[2][p][sl] = d[0] - oL * Yf;
        nxt[0][p][sl] = oR * Ul;
        nxt[1][p][sl] = oR * Vl;
        nxt[2][p][sl] = oR * Yl;
    }
    __syncthreads();
    // row p of the reduced system, A x_{p-1} + B x_p + C x_{p+1} = D
    double rA = 0.0, rB = 1.0, rC = 0.0, rD = 0.0;
    if (active) {
        rB = own[0][p][sl];
        rC = own[1][p][sl];
        rD = own[2][p][sl];
        if (p > 0) {
            rA = nxt[0][p - 1][sl];
            rB += nxt[1][p - 1][sl];
            rD -= nxt[2][p - 1][sl];
        }
    }
    // parallel cyclic reduction: after step h every row couples only to rows
    // 2h away; rows outside 0..P-1 are absent (identity rows).
    for (int h = 1; h < P; h *= 2) {
        if (active) {
            red[0][p][sl] = rA;
            red[1][p][sl] = rB;
            red[2][p][sl] = rC;
            red[3][p][sl] = rD;
        }
        __syncthreads();
        if (active) {
            double a = 0.0, c = 0.0, nb = rB, nd = rD, na = 0.0, nc = 0.0;
            if (p >= h) {
                a = -rA * recip(red[1][p - h][sl]);
                na = a * red[0][p - h][sl];
                nb += a * red[2][p - h][sl];
                nd += a * red[3][p - h][sl];
            }
            if (p + h < P) {
                c = -rC * recip(red[1][p + h][sl]);
                nc = c * red[2][p + h][sl];
                nb += c * red[0][p + h][sl];
                nd += c * red[3][p + h][sl];
            }
            rA = na;
            rB = nb;
            rC = nc;
            rD = nd;
        }
        __syncthreads();
    }
    if (active) xs[p][sl] = rD * recip(rB);
    __syncthreads();

    // ---- pass 2: interior with both separators known
    if (active) {
        const double xL = xs[p][sl];
        const double xR = last ? 0.0 : xs[p + 1][sl];
        if (live) col[size_t(s0) * nth] = xL;
        if (n >= 1) {
            d[1] -= oL * xL;
#pragma unroll
            for (int k = 1; k < CH; ++k)
                if (k == n) d[k] -= oR * xR;
#pragma unroll
            for (int k = 2; k < CH; ++k)
                if (k <= n) d[k] -= cf.off(s0 + k - 1) * invw[k - 1] * d[k - 1];
            double xn = 0.0;
#pragma unroll
            for (int k = CH - 1; k >= 1; --k) {
                if (k <= n) {
                    const double up = k < n ? cf.off(s0 + k) * xn : 0.0;
                    xn = (d[k] - up) * invw[k];
                    if (live) col[size_t(s0 + k) * nth] = xn;
                }
            }
        }
    }
}

}  // namespace radial
