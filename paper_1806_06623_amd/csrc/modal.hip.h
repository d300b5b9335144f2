// Fused per-mode solve for equator-symmetric theta grids (Sec. 3.2 with the
// parity split of Sec. 4.2): for one real Fourier component q (mode m) and one
// theta parity, one workgroup computes
//
//   s^ = B_f^T a           forward projection of the folded spectrum,
//   radial solves          Delta_r f + R_i lambda_l f = s^ with the outer
//                          boundary condition, for every l of this parity,
//   G  = B_i^T f           inverse projection (half of the theta values),
//
// keeping the N_r x h slab in registers between the three steps, so the field
// crosses HBM once in and once out instead of three times each.
//
// Input and output share the array X[q][i][j'] (in place).  On entry the
// first h = N_theta/2 values of a row hold the even fold s_k + s_{N-1-k},
// the last h the odd fold s_k - s_{N-1-k} (written by the folded forward
// FFT); on exit they hold G_e and G_o with g_k = G_e + G_o and
// g_{N-1-k} = G_e - G_o (undone by the unfolding inverse FFT).  Each
// workgroup reads and writes only its own half rows.
//
// Work split (NW = 12 waves, T row tiles of 16 per wave, CH = 4 T):
//   wave w, lane (lr = lane % 16, g = lane / 16), accumulator register v of
//   tile rb and column tile cb holds row  w 16 T + g CH + 4 rb + v  and
//   column l = lr + 16 cb.  The MFMA row index r of tile rb is mapped to
//   that row by r = g + 4 v (A operand: lane lr supplies row
//   w 16 T + (lr % 4) CH + 4 rb + lr / 4), so every lane group owns CH
//   consecutive rows of each of its columns: a chunk of the radial
//   partition method, which runs on the accumulators without moving them.
//   The CH x 4 chunks of the 4 NW lane groups of a column are its
//   partitions; the reduced (Schur complement) system over their separator
//   rows is solved by parallel cyclic reduction in LDS, 16 columns at a time.
//   For the inverse projection each tile is transposed through a small LDS
//   buffer into the A-operand layout.
//
// v_mfma_f64_16x16x4f64 operand layout: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; result register v of lane l is C[l / 16 + 4 v][l % 16].
#pragma once
#include <hip/hip_runtime.h>

#include "modal_layout.h"
#include "radial.hip.h"

namespace modal {

using d4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;

constexpr int NW = modalimg::NW;
constexpr int THREADS = 64 * NW;
constexpr int P = 4 * NW;          // radial partitions per column
constexpr int TP = 34;             // pitch of the transpose buffer (32 columns + pad)

template <int RN> struct Geo {
    static constexpr int KP = modalimg::kp(RN);
    static constexpr int KG = KP / 4;        // MFMA steps per tile
    static constexpr int NC = KG / 8;        // load chunks (of 8 steps) per tile
    static constexpr int NP = modalimg::np(RN);
    static constexpr int ELEMS = KP * NP;
};

// A operand of one chunk (8 steps, k in [32 kc, 32 kc + 32)) of one row: four
// 16-byte loads.  k beyond the half row is clamped to h - 2 (finite values
// that meet zero rows of the image); the row index is clamped by the caller.
__device__ __forceinline__ void load_a(double (&buf)[8], const double* __restrict__ row, int kc, int g, int h)
{
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int k = 32 * kc + 8 * t + 2 * g;
        k = k <= h - 2 ? k : h - 2;
        const double2 v = *reinterpret_cast<const double2*>(row + k);
        buf[2 * t] = v.x;
        buf[2 * t + 1] = v.y;
    }
}

template <int RN>
__device__ __forceinline__ void mma_chunk(d4 (&acc)[RN], const double (&a)[8], const double* __restrict__ Bs, int kc,
                                          int g, int lr)
{
    constexpr int NP = Geo<RN>::NP;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const double* br = Bs + (4 * (8 * kc + u) + g) * NP + lr;
        double b[RN];
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) b[cb] = br[16 * cb];
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[cb], acc[cb], 0, 0, 0);
    }
}

// Contiguous copy of one image into LDS (the plan stores it in LDS layout).
template <int ELEMS>
__device__ __forceinline__ void stage_image(double* __restrict__ Bs, const double* __restrict__ img)
{
    const double2* src = reinterpret_cast<const double2*>(img);
    double2* dst = reinterpret_cast<double2*>(Bs);
    constexpr int HALF = ELEMS / 2, PER = (HALF + THREADS - 1) / THREADS;
    double2 v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = threadIdx.x + u * THREADS;
        v[u] = src[i < HALF ? i : HALF - 1];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = threadIdx.x + u * THREADS;
        if (i < HALF) dst[i] = v[u];
    }
}

template <int RN, int T>
__global__ __launch_bounds__(THREADS) void k_modal(double* __restrict__ X, const double* __restrict__ Fimg,
                                                   const double* __restrict__ Iimg, const double* __restrict__ lam,
                                                   const double* __restrict__ beta, radial::Coef tab, int nth,
                                                   int nphi)
{
    using Gm = Geo<RN>;
    constexpr int NC = Gm::NC, ELEMS = Gm::ELEMS;
    constexpr int CH = 4 * T;               // rows per lane chunk
    constexpr int ROWS = NW * 16 * T;       // row capacity
    constexpr int NCH = T * NC;             // load chunks of the forward product
    constexpr int RED = 10 * P * 16;        // own[3], nxt[3], red[4] of [P][16]
    constexpr int TRB = NW * 16 * TP;       // one 16 x 32 transpose buffer per wave
    constexpr int UN = RED > TRB ? RED : TRB;
    __shared__ __attribute__((aligned(16))) double Bs[ELEMS];
    __shared__ __attribute__((aligned(16))) double un[UN];
    __shared__ double xs[(P + 1) * 16];
    __shared__ double c_alpha[ROWS], c_VR[ROWS], c_V[ROWS];

    const int par = blockIdx.x, q = blockIdx.y;
    const int m = q <= nphi / 2 ? q : nphi - q;
    const int nr = tab.nr, h = nth >> 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, g = lane >> 4;
    double* __restrict__ Xq = X + size_t(q) * nr * nth + par * h;

    // rows supplied as A operand by this lane in tile rb (clamped into range)
    auto arow = [&](int rb) {
        const int R = w * 16 * T + (lr & 3) * CH + 4 * rb + (lr >> 2);
        return Xq + size_t(R < nr ? R : nr - 1) * nth;
    };

    // ---- forward projection: first two chunks in flight during the staging
    d4 acc[T][RN];
#pragma unroll
    for (int rb = 0; rb < T; ++rb)
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) acc[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
    double ba[8], bb[8];
    load_a(ba, arow(0), 0, g, h);
    if constexpr (NCH > 1) load_a(bb, arow(1 / NC), 1 % NC, g, h);

    stage_image<ELEMS>(Bs, Fimg + (size_t(m) * 2 + par) * ELEMS);
    for (int i = threadIdx.x; i < ROWS; i += THREADS) {
        const bool in = i < nr;
        c_alpha[i] = in ? tab.alpha[i] : 0.0;
        c_VR[i] = in ? tab.VR[i] : 0.0;
        c_V[i] = in ? tab.V[i] : 0.0;
    }
    __syncthreads();

#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int rb = c / NC, kc = c % NC;
        if (c % 2 == 0) {
            mma_chunk<RN>(acc[rb], ba, Bs, kc, g, lr);
            if (c + 2 < NCH) load_a(ba, arow((c + 2) / NC), (c + 2) % NC, g, h);
        } else {
            mma_chunk<RN>(acc[rb], bb, Bs, kc, g, lr);
            if (c + 2 < NCH) load_a(bb, arow((c + 2) / NC), (c + 2) % NC, g, h);
        }
    }

    // ---- radial solves (partition method on the accumulators)
    // lane group g of wave w owns rows s0 .. s0 + CH - 1 of its columns
    const int p = 4 * w + g;
    const int PA = (nr + CH - 1) / CH;       // partitions that hold rows
    const bool active = p < PA;
    const int s0 = p * CH;
    const int s1 = active ? (s0 + CH < nr ? s0 + CH : nr) : s0 + 1;
    const int n = s1 - s0 - 1;                // interior rows s0+1 .. s1-1
    const bool last = p == PA - 1;
    const radial::RowCoef cf{c_alpha, c_VR, nr};
#define D(k) acc[(k) >> 2][cb][(k) & 3]

#pragma unroll
    for (int cb = 0; cb < RN; ++cb)
#pragma unroll
        for (int k = 0; k < CH; ++k)
            if (k <= n) D(k) *= c_V[s0 + k];

    double* own = un;                 // [3][P][16]
    double* nxt = un + 3 * P * 16;    // [3][P][16]
    double* red = un + 6 * P * 16;    // [4][P][16]
    const double oL = (active && s0 + 1 < nr) ? cf.off(s0) : 0.0;   // s0 <-> s0+1
    const double oR = (active && !last) ? cf.off(s1 - 1) : 0.0;     // s1-1 <-> s1

#pragma unroll
    for (int cb = 0; cb < RN; ++cb) {
        const int l = lr + 16 * cb;
        const int L = par * h + (l < h ? l : h - 1);
        const double lm = lam[size_t(m) * nth + L];
        const double bo = beta[size_t(m) * nth + L];

        // pass 1: eliminate the interior in both directions
        double invw[CH];
        double Yf = 0.0, Uf = 0.0, Vf = 1.0, Yl = 0.0, Ul = 1.0, Vl = 0.0;
        if (active && n >= 1) {
            double wv = 1.0, zf = 0.0, uf = 0.0, iwn = 0.0;
#pragma unroll
            for (int k = 1; k < CH; ++k) {
                invw[k] = 0.0;
                if (k <= n) {
                    const int i = s0 + k;
                    if (k == 1) {
                        wv = cf.diag(i, lm, bo);
                        zf = D(1);
                        uf = -oL;
                    } else {
                        const double o = cf.off(i - 1);
                        const double mult = o * invw[k - 1];
                        wv = cf.diag(i, lm, bo) - mult * o;
                        zf = D(k) - mult * zf;
                        uf = -mult * uf;
                    }
                    invw[k] = radial::recip(wv);
                    iwn = invw[k];
                }
            }
            Yl = zf * iwn;
            Ul = uf * iwn;
            Vl = -oR * iwn;
            double wh = 1.0, zh = 0.0, vh = 0.0, iwh = 0.0;
#pragma unroll
            for (int k = CH - 1; k >= 1; --k) {
                if (k <= n) {
                    const int i = s0 + k;
                    if (k == n) {
                        wh = cf.diag(i, lm, bo);
                        zh = D(k);
                        vh = -oR;
                    } else {
                        const double o = cf.off(i);
                        const double mult = o * iwh;
                        wh = cf.diag(i, lm, bo) - mult * o;
                        zh = D(k) - mult * zh;
                        vh = -mult * vh;
                    }
                    iwh = radial::recip(wh);
                }
            }
            Yf = zh * iwh;
            Vf = vh * iwh;
            Uf = -oL * iwh;
        }

        // reduced system over the separators s_0 .. s_{PA-1} of these 16 columns
        if (active) {
            const double bs = cf.diag(s0, lm, bo);
            own[(0 * P + p) * 16 + lr] = bs + oL * Uf;
            own[(1 * P + p) * 16 + lr] = oL * Vf;
            own[(2 * P + p) * 16 + lr] = D(0) - oL * Yf;
            nxt[(0 * P + p) * 16 + lr] = oR * Ul;
            nxt[(1 * P + p) * 16 + lr] = oR * Vl;
            nxt[(2 * P + p) * 16 + lr] = oR * Yl;
        }
        __syncthreads();
        double rA = 0.0, rB = 1.0, rC = 0.0, rD = 0.0;
        if (active) {
            rB = own[(0 * P + p) * 16 + lr];
            rC = own[(1 * P + p) * 16 + lr];
            rD = own[(2 * P + p) * 16 + lr];
            if (p > 0) {
                rA = nxt[(0 * P + p - 1) * 16 + lr];
                rB += nxt[(1 * P + p - 1) * 16 + lr];
                rD -= nxt[(2 * P + p - 1) * 16 + lr];
            }
        }
        // parallel cyclic reduction: after step hs every row couples only to
        // rows 2 hs away; rows outside 0 .. PA-1 are absent
        for (int hs = 1; hs < PA; hs *= 2) {
            if (active) {
                red[(0 * P + p) * 16 + lr] = rA;
                red[(1 * P + p) * 16 + lr] = rB;
                red[(2 * P + p) * 16 + lr] = rC;
                red[(3 * P + p) * 16 + lr] = rD;
            }
            __syncthreads();
            if (active) {
                double nb = rB, nd = rD, na = 0.0, nc = 0.0;
                if (p >= hs) {
                    const double a = -rA * radial::recip(red[(1 * P + p - hs) * 16 + lr]);
                    na = a * red[(0 * P + p - hs) * 16 + lr];
                    nb += a * red[(2 * P + p - hs) * 16 + lr];
                    nd += a * red[(3 * P + p - hs) * 16 + lr];
                }
                if (p + hs < PA) {
                    const double c = -rC * radial::recip(red[(1 * P + p + hs) * 16 + lr]);
                    nc = c * red[(2 * P + p + hs) * 16 + lr];
                    nb += c * red[(0 * P + p + hs) * 16 + lr];
                    nd += c * red[(3 * P + p + hs) * 16 + lr];
                }
                rA = na;
                rB = nb;
                rC = nc;
                rD = nd;
            }
            __syncthreads();
        }
        if (active) xs[p * 16 + lr] = rD * radial::recip(rB);
        __syncthreads();

        // pass 2: interior with both separators known
        if (active) {
            const double xL = xs[p * 16 + lr];
            const double xR = last ? 0.0 : xs[(p + 1) * 16 + lr];
            D(0) = xL;
            if (n >= 1) {
                D(1) -= oL * xL;
#pragma unroll
                for (int k = 1; k < CH; ++k)
                    if (k == n) D(k) -= oR * xR;
#pragma unroll
                for (int k = 2; k < CH; ++k)
                    if (k <= n) D(k) -= cf.off(s0 + k - 1) * invw[k - 1] * D(k - 1);
                double xn = 0.0;
#pragma unroll
                for (int k = CH - 1; k >= 1; --k) {
                    if (k <= n) {
                        const double up = k < n ? cf.off(s0 + k) * xn : 0.0;
                        xn = (D(k) - up) * invw[k];
                        D(k) = xn;
                    }
                }
            }
        }
    }
#undef D

    // ---- inverse projection, tile by tile through the transpose buffer
    __syncthreads();   // every wave is done with the forward image and the reduced system
    stage_image<ELEMS>(Bs, Iimg + (size_t(m) * 2 + par) * ELEMS);
    __syncthreads();
    double* tb = un + w * 16 * TP;
#pragma unroll
    for (int rb = 0; rb < T; ++rb) {
        d4 out[RN];
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) out[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < NC; ++kc) {
            // columns 32 kc .. 32 kc + 31 of tile rb, row r = g + 4 v
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int cb = 2 * kc + half;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    tb[(g + 4 * v) * TP + lr + 16 * half] = cb < RN ? acc[rb][cb < RN ? cb : 0][v] : 0.0;
            }
            __syncthreads();
            double a[8];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double2 x = *reinterpret_cast<const double2*>(tb + lr * TP + 8 * t + 2 * g);
                a[2 * t] = x.x;
                a[2 * t + 1] = x.y;
            }
            __syncthreads();
            mma_chunk<RN>(out, a, Bs, kc, g, lr);
        }
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) {
            const int j = lr + 16 * cb;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int R = w * 16 * T + g * CH + 4 * rb + v;
                if (R < nr && j < h) Xq[size_t(R) * nth + j] = out[cb][v];
            }
        }
    }
}

}  // namespace modal
