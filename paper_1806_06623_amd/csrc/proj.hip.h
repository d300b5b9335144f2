// Theta projections (Sec. 3.2: s^ = H^-1 s~ and g = H f for every azimuthal
// mode m) as FP64 MFMA GEMMs on gfx950, batched over the N_phi real Fourier
// components q; both components (cos and sin) of a mode use that mode's matrix.
//
//   C[q][i][n] = sum_k A[q][i][k] * B[m(q)][n][k],   i < M (= N_r), n, k < K (= N_theta)
//
// One workgroup (8 waves) per (q, slice of rows).  The whole matrix B_m is
// staged once in LDS (copied from an image the plan prepares in that layout); every wave then streams its own rows of A straight from
// global memory into registers (double-buffered chunks of 8 k-steps) and
// keeps a 16*RM x 16*RN block of C in accumulators.  The k index is permuted
// between lanes so that both operands are contiguous per lane: in MFMA step s
// the lane group g = lane / 16 multiplies k = g * KG + s (KG = K_pad / 4);
// the LDS copy of B stores that k at row 4 s + g, and a 16-double row pad
// puts the four groups of one step on distinct bank halves.
//
// v_mfma_f64_16x16x4f64 operand layout: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; result register v of lane l is C[l / 16 + 4 v][l % 16].
#pragma once
#include <hip/hip_runtime.h>

#include "proj_layout.h"
#include "status.h"

namespace proj {

using d4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;

template <int RN> struct Shape {
    static constexpr int NMAX = projimg::nmax(RN);          // largest N_theta handled
    static constexpr int KMAX = projimg::kmax(RN);          // padded K capacity
    static constexpr int NP = projimg::np(RN);              // padded LDS row length
    static constexpr int ELEMS = KMAX * NP;                 // doubles per image
};

// Loads of A are unconditional: row and k indices are clamped into range and
// the values used as loaded.  Rows >= M only feed accumulator rows that are
// never stored, and k >= K meets the zero padding of B in LDS, so no select
// is needed -- a select right after the load would force the compiler to wait
// for it, whereas plain loads let the next chunk stay in flight while the
// MFMAs of the current chunk run (ping-pong register buffers, no copies).
template <int RM, bool KVEC>
__device__ __forceinline__ void load_chunk(double (&buf)[RM][8], const double* __restrict__ Aq, int M, int K,
                                           int rbase, int lr, int k0)
{
#pragma unroll
    for (int rb = 0; rb < RM; ++rb) {
        const int row = rbase + rb * 16 + lr;
        const double* src = Aq + size_t(row < M ? row : M - 1) * K;
        if constexpr (KVEC) {
            // K is a multiple of 32: k0 .. k0+7 are in range and 16-byte aligned
#pragma unroll
            for (int u = 0; u < 8; u += 2) {
                const double2 v = *reinterpret_cast<const double2*>(src + k0 + u);
                buf[rb][u] = v.x;
                buf[rb][u + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + u;
                buf[rb][u] = src[k < K ? k : K - 1];
            }
        }
    }
}

template <int RN, int RM>
__device__ __forceinline__ void mfma_chunk(d4 (&acc)[RM][RN], const double (&a)[RM][8], const double* __restrict__ Bs,
                                           int NP, int s0, int g, int lr)
{
    // B fragments of step u+1 are read from LDS before the MFMAs of step u
    double b[2][RN];
    const double* brow = Bs + (4 * s0 + g) * NP + lr;
#pragma unroll
    for (int cb = 0; cb < RN; ++cb) b[0][cb] = brow[cb * 16];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (u + 1 < 8) {
            const double* bn = Bs + (4 * (s0 + u + 1) + g) * NP + lr;
#pragma unroll
            for (int cb = 0; cb < RN; ++cb) b[(u + 1) & 1][cb] = bn[cb * 16];
        }
#pragma unroll
        for (int rb = 0; rb < RM; ++rb)
#pragma unroll
            for (int cb = 0; cb < RN; ++cb)
                acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][u], b[u & 1][cb], acc[rb][cb], 0, 0, 0);
    }
}

constexpr int NWAVES = 8;                 // two waves per SIMD share one LDS copy of B_m

template <int RN, int RM, bool KVEC, int NW = NWAVES>
__global__ __launch_bounds__(64 * NW) void k_proj_f64(const double* __restrict__ A, const double* __restrict__ Bimg,
                                                  double* __restrict__ C, int M, int K, int nphi, int splits,
                                                  const unsigned* __restrict__ gate)
{
    if (spp_gate_closed(gate)) return;
    using S = Shape<RN>;
    __shared__ double Bs[S::KMAX * S::NP];

    const int q = blockIdx.y;
    const int m = q <= nphi / 2 ? q : nphi - q;
    const double* __restrict__ Aq = A + size_t(q) * M * K;
    double* __restrict__ Cq = C + size_t(q) * M * K;
    const int Kp = (K + 31) & ~31;
    const int KG = Kp >> 2;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const int kb0 = g * KG;
    double pa[RM][8], pb[RM][8];
    // first A chunk of this wave's first row group: in flight during the staging
    {
        const int gi0 = blockIdx.x * NW + wave;
        load_chunk<RM, KVEC>(pa, Aq, M, K, gi0 * 16 * RM < M ? gi0 * 16 * RM : 0, lr, kb0);
    }

    // ---- stage B_m: the plan holds it already in the LDS image layout
    // (k-permuted, padded, zero-filled), so this is a contiguous copy
    {
        const double2* src = reinterpret_cast<const double2*>(Bimg + size_t(m) * S::ELEMS);
        double2* dst = reinterpret_cast<double2*>(Bs);
        constexpr int TH = 64 * NW, HALF = S::ELEMS / 2, PER = (HALF + TH - 1) / TH;
        double2 v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * TH;
            v[u] = src[i < HALF ? i : HALF - 1];
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * TH;
            if (i < HALF) dst[i] = v[u];
        }
    }
    __syncthreads();

    const int ngroups = (M + 16 * RM - 1) / (16 * RM);

    for (int gi = blockIdx.x * NW + wave; gi < ngroups; gi += NW * splits) {
        const int rbase = gi * 16 * RM;
        d4 acc[RM][RN];
#pragma unroll
        for (int a = 0; a < RM; ++a)
#pragma unroll
            for (int b = 0; b < RN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

        if (gi != blockIdx.x * NW + wave) load_chunk<RM, KVEC>(pa, Aq, M, K, rbase, lr, kb0);
        for (int s0 = 0; s0 < KG; s0 += 16) {
            const int s1 = s0 + 8 < KG ? s0 + 8 : KG - 8;
            load_chunk<RM, KVEC>(pb, Aq, M, K, rbase, lr, kb0 + s1);
            __builtin_amdgcn_sched_barrier(0);
            mfma_chunk<RN, RM>(acc, pa, Bs, S::NP, s0, g, lr);
            const int s2 = s0 + 16 < KG ? s0 + 16 : KG - 8;
            __builtin_amdgcn_sched_barrier(0);
            load_chunk<RM, KVEC>(pa, Aq, M, K, rbase, lr, kb0 + s2);
            __builtin_amdgcn_sched_barrier(0);
            const bool hb = s0 + 8 < KG;
#pragma unroll
            for (int rb = 0; rb < RM; ++rb)
#pragma unroll
                for (int u = 0; u < 8; ++u) pb[rb][u] = hb ? pb[rb][u] : 0.0;
            mfma_chunk<RN, RM>(acc, pb, Bs, S::NP, hb ? s0 + 8 : s0, g, lr);
        }

#pragma unroll
        for (int rb = 0; rb < RM; ++rb)
#pragma unroll
            for (int cb = 0; cb < RN; ++cb) {
                const int col = cb * 16 + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rbase + rb * 16 + g + 4 * v;
                    if (row < M && col < K) Cq[size_t(row) * K + col] = acc[rb][cb][v];
                }
            }
    }
}

// ---------------------------------------------------------------------------
// Parity-split projection (Sec. 4.2) for theta grids symmetric about the
// equator, N = N_theta = 2h: the eigenvectors are even or odd in j, so each
// N x N product becomes two h x h products on the folded data.
//   forward (FWD): A_e[k] = s_k + s_{N-1-k}, A_o[k] = s_k - s_{N-1-k} (k < h);
//                  C[l] = (B_e A_e)[l] for l < h, C[h + l] = (B_o A_o)[l]
//                  (modes ordered even, then odd);
//   inverse:       A_e = f[0..h), A_o = f[h..N);
//                  C[j] = G_e[j] + G_o[j], C[N-1-j] = G_e[j] - G_o[j], G_p = B_p A_p.
// B_e and B_o (images of K = h) are staged together in LDS.
template <int RM, bool KVEC, bool FWD>
__device__ __forceinline__ void load_chunk_par(double (&x)[RM][8], double (&z)[RM][8], const double* __restrict__ Aq,
                                               int M, int N, int h, int rbase, int lr, int k0)
{
#pragma unroll
    for (int rb = 0; rb < RM; ++rb) {
        const int row = rbase + rb * 16 + lr;
        const double* src = Aq + size_t(row < M ? row : M - 1) * N;
        // second operand: mirrored run N-8-k0 .. N-1-k0 (forward) or h+k0 .. (inverse)
        const int z0 = FWD ? N - 8 - k0 : h + k0;
        if constexpr (KVEC) {
#pragma unroll
            for (int u = 0; u < 8; u += 2) {
                const double2 a = *reinterpret_cast<const double2*>(src + k0 + u);
                const double2 b = *reinterpret_cast<const double2*>(src + z0 + u);
                x[rb][u] = a.x;
                x[rb][u + 1] = a.y;
                z[rb][u] = b.x;
                z[rb][u + 1] = b.y;
            }
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + u < h ? k0 + u : h - 1;   // k >= h meets zero rows of B
                x[rb][u] = src[k];
                const int kz = FWD ? N - 8 - k0 + u : h + k0 + u;
                z[rb][u] = src[kz < 0 ? 0 : (kz < N ? kz : N - 1)];
            }
        }
    }
}

template <int RN, int RM, bool FWD>
__device__ __forceinline__ void mfma_chunk_par(d4 (&ae)[RM][RN], d4 (&ao)[RM][RN], const double (&x)[RM][8],
                                               const double (&z)[RM][8], const double* __restrict__ Be,
                                               const double* __restrict__ Bo, int NP, int s0, int g, int lr)
{
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const double* re = Be + (4 * (s0 + u) + g) * NP + lr;
        const double* ro = Bo + (4 * (s0 + u) + g) * NP + lr;
        double be[RN], bo[RN];
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) {
            be[cb] = re[cb * 16];
            bo[cb] = ro[cb * 16];
        }
#pragma unroll
        for (int rb = 0; rb < RM; ++rb) {
            const double ev = FWD ? x[rb][u] + z[rb][7 - u] : x[rb][u];
            const double od = FWD ? x[rb][u] - z[rb][7 - u] : z[rb][u];
#pragma unroll
            for (int cb = 0; cb < RN; ++cb) {
                ae[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ev, be[cb], ae[rb][cb], 0, 0, 0);
                ao[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(od, bo[cb], ao[rb][cb], 0, 0, 0);
            }
        }
    }
}

template <int RN, int RM, bool KVEC, bool FWD, int NW = NWAVES>
__global__ __launch_bounds__(64 * NW) void k_proj_par(const double* __restrict__ A, const double* __restrict__ Bpar,
                                                      double* __restrict__ C, int M, int N, int nphi, int splits,
                                                      const unsigned* __restrict__ gate)
{
    if (spp_gate_closed(gate)) return;
    using S = Shape<RN>;
    __shared__ double Bs[2 * S::ELEMS];

    const int q = blockIdx.y;
    const int m = q <= nphi / 2 ? q : nphi - q;
    const int h = N / 2;
    const double* __restrict__ Aq = A + size_t(q) * M * N;
    double* __restrict__ Cq = C + size_t(q) * M * N;
    const int KG = ((h + 31) & ~31) >> 2;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const int kb0 = g * KG;
    double xa[RM][8], za[RM][8], xb[RM][8], zb[RM][8];
    {
        const int gi0 = blockIdx.x * NW + wave;
        load_chunk_par<RM, KVEC, FWD>(xa, za, Aq, M, N, h, gi0 * 16 * RM < M ? gi0 * 16 * RM : 0, lr, kb0);
    }
    {
        const double2* src = reinterpret_cast<const double2*>(Bpar + size_t(m) * 2 * S::ELEMS);
        double2* dst = reinterpret_cast<double2*>(Bs);
        constexpr int TH = 64 * NW, HALF = S::ELEMS, PER = (HALF + TH - 1) / TH;   // 2*ELEMS doubles
        double2 v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * TH;
            v[u] = src[i < HALF ? i : HALF - 1];
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * TH;
            if (i < HALF) dst[i] = v[u];
        }
    }
    __syncthreads();
    const double* Be = Bs;
    const double* Bo = Bs + S::ELEMS;

    const int ngroups = (M + 16 * RM - 1) / (16 * RM);
    for (int gi = blockIdx.x * NW + wave; gi < ngroups; gi += NW * splits) {
        const int rbase = gi * 16 * RM;
        d4 ae[RM][RN], ao[RM][RN];
#pragma unroll
        for (int a = 0; a < RM; ++a)
#pragma unroll
            for (int b = 0; b < RN; ++b) {
                ae[a][b] = d4{0.0, 0.0, 0.0, 0.0};
                ao[a][b] = d4{0.0, 0.0, 0.0, 0.0};
            }
        if (gi != blockIdx.x * NW + wave) load_chunk_par<RM, KVEC, FWD>(xa, za, Aq, M, N, h, rbase, lr, kb0);
        for (int s0 = 0; s0 < KG; s0 += 16) {
            const int s1 = s0 + 8 < KG ? s0 + 8 : KG - 8;
            load_chunk_par<RM, KVEC, FWD>(xb, zb, Aq, M, N, h, rbase, lr, kb0 + s1);
            __builtin_amdgcn_sched_barrier(0);
            mfma_chunk_par<RN, RM, FWD>(ae, ao, xa, za, Be, Bo, S::NP, s0, g, lr);
            const int s2 = s0 + 16 < KG ? s0 + 16 : KG - 8;
            __builtin_amdgcn_sched_barrier(0);
            load_chunk_par<RM, KVEC, FWD>(xa, za, Aq, M, N, h, rbase, lr, kb0 + s2);
            __builtin_amdgcn_sched_barrier(0);
            const bool hb = s0 + 8 < KG;
#pragma unroll
            for (int rb = 0; rb < RM; ++rb)
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    xb[rb][u] = hb ? xb[rb][u] : 0.0;
                    zb[rb][u] = hb ? zb[rb][u] : 0.0;
                }
            mfma_chunk_par<RN, RM, FWD>(ae, ao, xb, zb, Be, Bo, S::NP, hb ? s0 + 8 : s0, g, lr);
        }

#pragma unroll
        for (int rb = 0; rb < RM; ++rb)
#pragma unroll
            for (int cb = 0; cb < RN; ++cb) {
                const int col = cb * 16 + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rbase + rb * 16 + g + 4 * v;
                    if (row < M && col < h) {
                        double* c = Cq + size_t(row) * N;
                        if (FWD) {
                            c[col] = ae[rb][cb][v];
                            c[h + col] = ao[rb][cb][v];
                        } else {
                            c[col] = ae[rb][cb][v] + ao[rb][cb][v];
                            c[N - 1 - col] = ae[rb][cb][v] - ao[rb][cb][v];
                        }
                    }
                }
            }
    }
}

// ---------------------------------------------------------------------------
// FP32 variant for the mixed-precision solve: the same tiling, with A rounded
// to float in registers, B_m taken from an FP32 image of the same layout, and
// v_mfma_f32_16x16x4f32 products accumulated in FP32.  Its result register v
// of lane l is C[4 (l / 16) + v][l % 16].  With ACCUM the result is added to C
// (FP64) instead of overwriting it.
using f4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;

template <int RN, int RM>
__device__ __forceinline__ void mfma_chunk_f32(f4 (&acc)[RM][RN], const double (&a)[RM][8], const float* __restrict__ Bs,
                                               int NP, int s0, int g, int lr)
{
    float b[2][RN];
    const float* brow = Bs + (4 * s0 + g) * NP + lr;
#pragma unroll
    for (int cb = 0; cb < RN; ++cb) b[0][cb] = brow[cb * 16];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (u + 1 < 8) {
            const float* bn = Bs + (4 * (s0 + u + 1) + g) * NP + lr;
#pragma unroll
            for (int cb = 0; cb < RN; ++cb) b[(u + 1) & 1][cb] = bn[cb * 16];
        }
#pragma unroll
        for (int rb = 0; rb < RM; ++rb) {
            const float av = static_cast<float>(a[rb][u]);
#pragma unroll
            for (int cb = 0; cb < RN; ++cb)
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b[u & 1][cb], acc[rb][cb], 0, 0, 0);
        }
    }
}

template <int RN, int RM, bool KVEC, bool ACCUM, int NW = NWAVES>
__global__ __launch_bounds__(64 * NW) void k_proj_f32(const double* __restrict__ A, const float* __restrict__ Bimg,
                                                      double* __restrict__ C, int M, int K, int nphi, int splits)
{
    using S = Shape<RN>;
    __shared__ float Bs[S::KMAX * S::NP];

    const int q = blockIdx.y;
    const int m = q <= nphi / 2 ? q : nphi - q;
    const double* __restrict__ Aq = A + size_t(q) * M * K;
    double* __restrict__ Cq = C + size_t(q) * M * K;
    const int KG = ((K + 31) & ~31) >> 2;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const int kb0 = g * KG;
    double pa[RM][8], pb[RM][8];
    {
        const int gi0 = blockIdx.x * NW + wave;
        load_chunk<RM, KVEC>(pa, Aq, M, K, gi0 * 16 * RM < M ? gi0 * 16 * RM : 0, lr, kb0);
    }
    {
        // S::ELEMS is a multiple of 4 (KMAX is a multiple of 32)
        const float4* src = reinterpret_cast<const float4*>(Bimg + size_t(m) * S::ELEMS);
        float4* dst = reinterpret_cast<float4*>(Bs);
        constexpr int TH = 64 * NW, QUART = S::ELEMS / 4, PER = (QUART + TH - 1) / TH;
        float4 v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * TH;
            v[u] = src[i < QUART ? i : QUART - 1];
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * TH;
            if (i < QUART) dst[i] = v[u];
        }
    }
    __syncthreads();

    const int ngroups = (M + 16 * RM - 1) / (16 * RM);
    for (int gi = blockIdx.x * NW + wave; gi < ngroups; gi += NW * splits) {
        const int rbase = gi * 16 * RM;
        f4 acc[RM][RN];
#pragma unroll
        for (int a = 0; a < RM; ++a)
#pragma unroll
            for (int b = 0; b < RN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

        if (gi != blockIdx.x * NW + wave) load_chunk<RM, KVEC>(pa, Aq, M, K, rbase, lr, kb0);
        for (int s0 = 0; s0 < KG; s0 += 16) {
            const int s1 = s0 + 8 < KG ? s0 + 8 : KG - 8;
            // the loads of the next chunk are pinned ahead of this chunk's
            // products (scheduling barriers), and the second product is
            // unconditional (zeroed when past K): otherwise the compiler sinks
            // each 16-byte load next to its FP32 conversion and waits on it there
            load_chunk<RM, KVEC>(pb, Aq, M, K, rbase, lr, kb0 + s1);
            __builtin_amdgcn_sched_barrier(0);
            mfma_chunk_f32<RN, RM>(acc, pa, Bs, S::NP, s0, g, lr);
            const int s2 = s0 + 16 < KG ? s0 + 16 : KG - 8;
            __builtin_amdgcn_sched_barrier(0);
            load_chunk<RM, KVEC>(pa, Aq, M, K, rbase, lr, kb0 + s2);
            __builtin_amdgcn_sched_barrier(0);
            const bool hb = s0 + 8 < KG;
#pragma unroll
            for (int rb = 0; rb < RM; ++rb)
#pragma unroll
                for (int u = 0; u < 8; ++u) pb[rb][u] = hb ? pb[rb][u] : 0.0;
            mfma_chunk_f32<RN, RM>(acc, pb, Bs, S::NP, hb ? s0 + 8 : s0, g, lr);
        }

        // with ACCUM, every value of C the tile adds to is loaded before the
        // first store, so that the loads are in flight together instead of
        // each waiting behind the previous store
        double prior[RM][RN][4];
#pragma unroll
        for (int rb = 0; rb < RM; ++rb)
#pragma unroll
            for (int cb = 0; cb < RN; ++cb) {
                const int col = cb * 16 + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rbase + rb * 16 + 4 * g + v;
                    prior[rb][cb][v] = ACCUM && row < M && col < K ? Cq[size_t(row) * K + col] : 0.0;
                }
            }
#pragma unroll
        for (int rb = 0; rb < RM; ++rb)
#pragma unroll
            for (int cb = 0; cb < RN; ++cb) {
                const int col = cb * 16 + lr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rbase + rb * 16 + 4 * g + v;
                    if (row < M && col < K) {
                        const double val = static_cast<double>(acc[rb][cb][v]);
                        Cq[size_t(row) * K + col] = ACCUM ? prior[rb][cb][v] + val : val;
                    }
                }
            }
    }
}

}  // namespace proj
