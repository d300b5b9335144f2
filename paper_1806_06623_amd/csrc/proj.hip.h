// Theta projections (Sec. 3.2: s^ = H^-1 s~ and g = H f for every azimuthal
// mode m) as FP64 MFMA GEMMs on gfx950, batched over the N_phi real Fourier
// components q; both components (cos and sin) of a mode use that mode's matrix.
//
//   C[q][i][n] = sum_k A[q][i][k] * B[m(q)][n][k],   i < M (= N_r), n, k < K (= N_theta)
//
// One workgroup (8 waves) per (q, slice of rows).  The whole matrix B_m is
// staged once in LDS; every wave then streams its own rows of A straight from
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

namespace proj {

using d4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;

template <int RN> struct Shape {
    static constexpr int NMAX = 16 * RN;                    // largest N_theta handled
    static constexpr int KMAX = (NMAX + 31) / 32 * 32;      // padded K capacity
    static constexpr int NP = NMAX + 16;                    // padded LDS row length
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
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const double* brow = Bs + (4 * (s0 + u) + g) * NP + lr;
        double b[RN];
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) b[cb] = brow[cb * 16];
#pragma unroll
        for (int rb = 0; rb < RM; ++rb)
#pragma unroll
            for (int cb = 0; cb < RN; ++cb)
                acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][u], b[cb], acc[rb][cb], 0, 0, 0);
    }
}

constexpr int NWAVES = 8;                 // two waves per SIMD share one LDS copy of B_m
constexpr int NTHREADS = 64 * NWAVES;

template <int RN, int RM, bool KVEC>
__global__ __launch_bounds__(NTHREADS) void k_proj_f64(const double* __restrict__ A, const double* __restrict__ B,
                                                  double* __restrict__ C, int M, int K, int nphi, int splits)
{
    using S = Shape<RN>;
    __shared__ double Bs[S::KMAX * S::NP];

    const int q = blockIdx.y;
    const int m = q <= nphi / 2 ? q : nphi - q;
    const double* __restrict__ Aq = A + size_t(q) * M * K;
    const double* __restrict__ Bm = B + size_t(m) * K * K;
    double* __restrict__ Cq = C + size_t(q) * M * K;
    const int Kp = (K + 31) & ~31;
    const int KG = Kp >> 2;

    // ---- stage B_m in LDS (k-permuted rows, zero padding for k, n >= K).
    // Each thread owns one column n and a strided set of k; eight loads are
    // issued before their LDS stores.
    {
        constexpr int TPC = NTHREADS / S::NMAX;             // threads per column n
        const int n = threadIdx.x % S::NMAX, part = threadIdx.x / S::NMAX;
        const int nc = n < K ? n : K - 1;
        const double* brow = Bm + size_t(nc) * K;
        for (int kb = part; kb < Kp; kb += 8 * TPC) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = kb + u * TPC;
                // multiply by a 0/1 mask (the matrix is finite) rather than
                // select, so the load is issued unconditionally and all eight
                // stay in flight together
                const double keep = (n < K && k < K) ? 1.0 : 0.0;
                v[u] = brow[k < K ? k : K - 1] * keep;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = kb + u * TPC;
                if (k < Kp) Bs[(4 * (k % KG) + k / KG) * S::NP + n] = v[u];
            }
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const int ngroups = (M + 16 * RM - 1) / (16 * RM);

    for (int gi = blockIdx.x * NWAVES + wave; gi < ngroups; gi += NWAVES * splits) {
        const int rbase = gi * 16 * RM;
        d4 acc[RM][RN];
#pragma unroll
        for (int a = 0; a < RM; ++a)
#pragma unroll
            for (int b = 0; b < RN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

        double pa[RM][8], pb[RM][8];
        const int kb0 = g * KG;
        load_chunk<RM, KVEC>(pa, Aq, M, K, rbase, lr, kb0);
        for (int s0 = 0; s0 < KG; s0 += 16) {
            const int s1 = s0 + 8 < KG ? s0 + 8 : KG - 8;
            load_chunk<RM, KVEC>(pb, Aq, M, K, rbase, lr, kb0 + s1);
            mfma_chunk<RN, RM>(acc, pa, Bs, S::NP, s0, g, lr);
            const int s2 = s0 + 16 < KG ? s0 + 16 : KG - 8;
            load_chunk<RM, KVEC>(pa, Aq, M, K, rbase, lr, kb0 + s2);
            if (s0 + 8 < KG) mfma_chunk<RN, RM>(acc, pb, Bs, S::NP, s0 + 8, g, lr);
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

}  // namespace proj
