// Folded real FFTs along phi for N_phi = 256 (the layout of the fused
// per-mode path on equator-symmetric theta grids, Sec. 4.2), with the first
// and last radix passes held in registers.
//
// A block is 16 line pairs (i, k), (i, N_theta-1-k), k < h = N_theta/2: 32
// folded lines of N2 = 128 complex points, 16 threads per line.  The complex
// FFT of length 128 runs as three Stockham passes (same arithmetic as
// fft.hip.h): two radix-8 passes and one radix-2 pass.
//
// Forward:  each line is loaded straight into the first radix-8 butterflies
//   (thread c of a line holds points c + 16 r) and takes the first pass in
//   registers; the fold follows at the second pass (the passes are linear):
//   the two lines of a pair sit in adjacent rows of one wave, which read both
//   LDS rows, form the sum (even fold) or the difference (odd fold) and write
//   the second pass back, with no workgroup barrier.  One workgroup barrier;
//   then the radix-2 pass fused with the split into the half spectrum, in the
//   store mapping (consecutive lanes own consecutive lines, so that every
//   store instruction writes 128-byte runs of a component plane).
// Inverse:  mirror image.  Lanes l < 16 of the load mapping read the even
//   fold E of pair l, lanes l >= 16 the odd fold O; inverse split and the
//   radix-2 pass in registers; one workgroup barrier; the second pass forms
//   E + O (line (i, k)) and E - O (line (i, N_theta-1-k)) in the pair's wave;
//   both radix-8 passes stay in that wave; stores straight from registers.
//
// Store/load mapping: l = tid % 32, g = tid / 32.  The radix-2 butterflies b
// of thread g are {g, 64 - g, 32 - g, 32 + g} (g = 0: {0, 32, 16, 48}); with
// them the thread holds Z_p and Z_{N2-p} of the split tasks p in {g, 64 - g,
// 32 - g, 32 + g} (g = 0: p in {0, 64, 32, 16, 48}), i.e. every split runs in
// registers.
#pragma once
#include "fft.hip.h"
#include "internal.h"
#include "status.h"
#include "xcd.h"

namespace fftfold {

constexpr int N = 256, N2 = 128, PB = 16, THREADS = 512, LS = LineStride<N2>::LS;

// LDS ordering among the lanes of one wave: the accesses of a wave reach LDS
// in program order, so a wave-scope fence (no workgroup barrier) suffices.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// radix-2 butterflies of thread g (see above)
__device__ __forceinline__ void butterflies(int g, int* b)
{
    if (g == 0) {
        b[0] = 0; b[1] = 32; b[2] = 16; b[3] = 48;
    } else {
        b[0] = g; b[1] = 64 - g; b[2] = 32 - g; b[3] = 32 + g;
    }
}

// Pair index of block blk, slot s (clamped into range) and its (i, k).
__device__ __forceinline__ void pair_of(int blk, int s, unsigned npairs, int h, unsigned* i, unsigned* k, bool* valid)
{
    unsigned P = unsigned(blk) * PB + unsigned(s);
    *valid = P < npairs;
    P = *valid ? P : npairs - 1;
    *i = P / unsigned(h);
    *k = P - *i * unsigned(h);
}

__global__ __launch_bounds__(THREADS, 4) void k_rfft_fwd_fold(const double* __restrict__ rho, double* __restrict__ X,
                                                               const c64* __restrict__ tw_g, double scale, int nlines,
                                                               int nblocks, int nth, spp_status_record* __restrict__ reset,
                                                               const unsigned* __restrict__ gate, spp_batch_view bv)
{
    if (spp_gate_closed(gate)) return;
    int blk = blockIdx.x;
    if (bv.rho) {   // batched: RHS r owns the nblocks workgroups from r * nblocks
        const int r = blk / nblocks;
        blk -= r * nblocks;
        rho = bv.rho[r];
        X += r * bv.xstride;
        scale = bv.scale[r];
        if (reset) reset += r;
    }
    spp_status_clear(reset, blk == 0);
    // issue priority: high while a wave issues its loads, low through the
    // transform, raised again for the stores, so that the waves of the other
    // workgroup on the CU get their loads out while this one computes
    __builtin_amdgcn_s_setprio(3);
    __shared__ c64 lds[2 * PB * LS];
    __shared__ c64 tws[N];

    const int h = nth >> 1;
    const unsigned npairs = unsigned(nlines) / 2;
    // line-major mapping: rows 0, 1 of wave w hold lines (i, k), (i, N_theta-1-k)
    // of pair 2w, rows 2, 3 those of pair 2w + 1; LDS row of pair pp: pp for
    // the even fold, PB + pp for the odd fold
    const int row = (threadIdx.x >> 4) & 3, c = threadIdx.x & 15;
    const int pp = 2 * (threadIdx.x >> 6) + (row >> 1), half = row & 1;
    {
        unsigned i, k;
        bool valid;
        pair_of(blk, pp, npairs, h, &i, &k, &valid);
        const double2* src = reinterpret_cast<const double2*>(rho) +
                             size_t(i * unsigned(nth) + (half ? unsigned(nth) - 1 - k : k)) * N2 + c;
        c64 tw0 = threadIdx.x < N ? tw_g[threadIdx.x] : c64{0.0, 0.0};
        double2 a[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) a[r] = src[16 * r];
        if (threadIdx.x < N) tws[threadIdx.x] = tw0;
        __syncthreads();   // twiddles
        __builtin_amdgcn_s_setprio(0);
        // first pass of the line itself (radix 8, Ns = 1: butterfly c reads
        // points c + 16 r, no twiddles); the fold follows, the pass being linear
        c64 v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = {a[r].x * scale, a[r].y * scale};
        dft<8>(v);
        c64* own = lds + (half * PB + pp) * LS;
#pragma unroll
        for (int r = 0; r < 8; ++r) own[pidx(8 * c + r)] = v[r];
        wave_lds_sync();
        // second pass (radix 8, Ns = 8) of the even fold (sum of the pair's
        // rows) or the odd fold (difference); both rows of the pair are read
        // by the one wave before either is overwritten
        const c64* le = lds + pp * LS;
        const c64* lo = lds + (PB + pp) * LS;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const c64 x = le[pidx(c + 16 * r)], y = lo[pidx(c + 16 * r)];
            v[r] = half ? csub(x, y) : cadd(x, y);
        }
#pragma unroll
        for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], tws[r * (c & 7) * 4]);
        dft<8>(v);
        const int base = (c >> 3) * 64 + (c & 7);
#pragma unroll
        for (int r = 0; r < 8; ++r) own[pidx(base + 8 * r)] = v[r];
    }
    __syncthreads();

    // third pass (radix 2, Ns = 64) fused with the split, store mapping
    const int l = threadIdx.x & 31, g = threadIdx.x >> 5;
    unsigned i, k;
    bool valid;
    pair_of(blk, l & 15, npairs, h, &i, &k, &valid);
    if (!valid) return;
    double* out = X + size_t(i * unsigned(nth) + unsigned(l >> 4) * unsigned(h) + k);
    const size_t plane = size_t(nlines);
    const c64* Zl = lds + l * LS;
    int bf[4];
    butterflies(g, bf);
    c64 z[4][2];   // z[j][0] = Z[bf[j]], z[j][1] = Z[bf[j] + 64]
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const c64 v0 = Zl[pidx(bf[j])];
        const c64 v1 = cmul(Zl[pidx(bf[j] + 64)], tws[2 * bf[j]]);
        z[j][0] = cadd(v0, v1);
        z[j][1] = csub(v0, v1);
    }
    // X_p = (a + conj b)/2 + w^p (a - conj b)/(2i), X_{N2-p} = conj(A) - conj(w^p) conj(B)
    auto split = [&](int p, c64 a, c64 b, c64* Xp, c64* Xq) {
        const c64 A = {0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
        const c64 B = {0.5 * (a.y + b.y), -0.5 * (a.x - b.x)};
        const c64 w = tws[p];
        *Xp = cadd(A, cmul(w, B));
        *Xq = csub(cconj(A), cmul(cconj(w), cconj(B)));
    };
    auto store4 = [&](int p, c64 Xp, c64 Xq) {
        out[size_t(p) * plane] = Xp.x;
        out[size_t(N - p) * plane] = Xp.y;
        out[size_t(N2 - p) * plane] = Xq.x;
        out[size_t(N2 + p) * plane] = Xq.y;
    };
    c64 Xp, Xq;
    __builtin_amdgcn_s_setprio(2);
    if (g == 0) {
        split(0, z[0][0], z[0][0], &Xp, &Xq);
        out[0] = Xp.x;                          // Re X_0
        out[size_t(N2) * plane] = Xq.x;         // Re X_{N/2}
        split(64, z[0][1], z[0][1], &Xp, &Xq);
        out[size_t(64) * plane] = Xp.x;
        out[size_t(N - 64) * plane] = Xp.y;
        split(32, z[1][0], z[1][1], &Xp, &Xq);
        store4(32, Xp, Xq);
        split(16, z[2][0], z[3][1], &Xp, &Xq);
        store4(16, Xp, Xq);
        split(48, z[3][0], z[2][1], &Xp, &Xq);
        store4(48, Xp, Xq);
    } else {
        split(g, z[0][0], z[1][1], &Xp, &Xq);
        store4(g, Xp, Xq);
        split(64 - g, z[1][0], z[0][1], &Xp, &Xq);
        store4(64 - g, Xp, Xq);
        split(32 - g, z[2][0], z[3][1], &Xp, &Xq);
        store4(32 - g, Xp, Xq);
        split(32 + g, z[3][0], z[2][1], &Xp, &Xq);
        store4(32 + g, Xp, Xq);
    }
}

// A workgroup that stores a non-finite value sets flag->nonfinite (when
// flag is not NULL).
__global__ __launch_bounds__(THREADS, 4) void k_rfft_inv_fold(const double* __restrict__ X, double* __restrict__ phi,
                                                               const c64* __restrict__ tw_g, int nlines, int nblocks,
                                                               int nth, spp_status_record* __restrict__ flag,
                                                               const unsigned* __restrict__ gate, spp_batch_view bv)
{
    if (spp_gate_closed(gate)) return;
    int blk = blockIdx.x;
    if (bv.phi) {
        const int r = blk / nblocks;
        blk -= r * nblocks;
        phi = bv.phi[r];
        X += r * bv.xstride;
        if (flag) flag += r;
    }
    // blocks of one XCD cover a contiguous range of lines, so that the
    // 128-byte runs of a component plane read by neighbouring blocks come
    // through the same L2 at about the same time
    blk = spp_plane_block(blk, nblocks);
    __shared__ c64 lds[2 * PB * LS];
    __shared__ c64 tws[N];
    if (threadIdx.x < N) tws[threadIdx.x] = tw_g[threadIdx.x];

    const int h = nth >> 1;
    const unsigned npairs = unsigned(nlines) / 2;
    const size_t plane = size_t(nlines);
    {
        // load mapping: lanes l < 16 read the even fold E of pair l, lanes
        // l >= 16 the odd fold O of pair l - 16 (the unfold follows the first
        // pass, which is linear)
        const int l = threadIdx.x & 31, g = threadIdx.x >> 5;
        unsigned i, k;
        bool valid;
        pair_of(blk, l & 15, npairs, h, &i, &k, &valid);
        const double* F = X + size_t(i * unsigned(nth) + unsigned(l >> 4) * unsigned(h) + k);
        // planes of the raw halfcomplex values of the tasks: Re X_p, Im X_p,
        // Re X_{N2-p}, Im X_{N2-p}; for g = 0 the first four are Re X_0,
        // Re X_{N/2} and Re, Im X_64 (X_0 and X_{N/2} are real, X_64 is its
        // own partner)
        int tp[4];
        butterflies(g, tp);   // the tasks p have the same values as the butterflies
        int pl[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            pl[4 * j] = tp[j];
            pl[4 * j + 1] = N - tp[j];
            pl[4 * j + 2] = N2 - tp[j];
            pl[4 * j + 3] = N2 + tp[j];
        }
        if (g == 0) {
            pl[1] = N2;
            pl[2] = 64;
            pl[3] = N - 64;
        }
        double x[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = F[size_t(pl[j]) * plane];
        // conj(Z_p) and conj(Z_{N2-p}) from X_p, X_{N2-p}:
        // Z_m = [X_m + conj X_{N2-m}] + i w^-m [X_m - conj X_{N2-m}]
        auto zpair = [&](int p, c64 xp, c64 xq, c64* zp, c64* zq) {
            const c64 wc = cconj(tws[p]);
            const c64 Ep = cadd(xp, cconj(xq)), Dp = csub(xp, cconj(xq));
            *zp = cconj(cadd(Ep, cmul({-wc.y, wc.x}, Dp)));
            const c64 Eq = cadd(xq, cconj(xp)), Dq = csub(xq, cconj(xp));
            const c64 w = tws[p];
            *zq = cconj(cadd(Eq, cmul({w.y, -w.x}, Dq)));
        };
        c64 z[4][2];   // z[j][0] = conj Z[bf[j]], z[j][1] = conj Z[bf[j] + 64], bf = tp
        __syncthreads();   // twiddles
        c64 unused;
        if (g == 0) {
            zpair(0, {x[0], 0.0}, {x[1], 0.0}, &z[0][0], &unused);
            zpair(64, {x[2], x[3]}, {x[2], x[3]}, &z[0][1], &unused);
            zpair(32, {x[4], x[5]}, {x[6], x[7]}, &z[1][0], &z[1][1]);
            zpair(16, {x[8], x[9]}, {x[10], x[11]}, &z[2][0], &z[3][1]);
            zpair(48, {x[12], x[13]}, {x[14], x[15]}, &z[3][0], &z[2][1]);
        } else {
            zpair(g, {x[0], x[1]}, {x[2], x[3]}, &z[0][0], &z[1][1]);
            zpair(64 - g, {x[4], x[5]}, {x[6], x[7]}, &z[1][0], &z[0][1]);
            zpair(32 - g, {x[8], x[9]}, {x[10], x[11]}, &z[2][0], &z[3][1]);
            zpair(32 + g, {x[12], x[13]}, {x[14], x[15]}, &z[3][0], &z[2][1]);
        }
        // first pass (radix 2, Ns = 1): butterfly b reads points b, b + 64,
        // writes 2b, 2b + 1
        c64* Zl = lds + l * LS;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            Zl[pidx(2 * tp[j])] = cadd(z[j][0], z[j][1]);
            Zl[pidx(2 * tp[j] + 1)] = csub(z[j][0], z[j][1]);
        }
    }
    __syncthreads();

    // second (radix 8, Ns = 2) and third (radix 8, Ns = 16) passes in the
    // pair's own wave: rows 0, 1 of wave w transform E + O and E - O of pair
    // 2w, rows 2, 3 those of pair 2w + 1 (both LDS rows of the pair are read
    // by the one wave before either is overwritten)
    const int row = (threadIdx.x >> 4) & 3, c = threadIdx.x & 15;
    const int pp = 2 * (threadIdx.x >> 6) + (row >> 1), half = row & 1;
    const c64* le = lds + pp * LS;
    const c64* lo = lds + (PB + pp) * LS;
    c64 v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const c64 x = le[pidx(c + 16 * r)], y = lo[pidx(c + 16 * r)];
        v[r] = half ? csub(x, y) : cadd(x, y);
    }
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], tws[r * (c & 1) * 16]);
    dft<8>(v);
    c64* own = lds + (half * PB + pp) * LS;
    const int base = (c >> 1) * 16 + (c & 1);
#pragma unroll
    for (int r = 0; r < 8; ++r) own[pidx(base + 2 * r)] = v[r];
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = own[pidx(c + 16 * r)];
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], tws[2 * r * c]);
    dft<8>(v);

    // x_{2n} = Re z_n, x_{2n+1} = Im z_n with z = conj(FFT(conj Z)), n = c + 16 r
    unsigned i, k;
    bool valid;
    pair_of(blk, pp, npairs, h, &i, &k, &valid);
    bool bad = false;
    if (valid) {
        const unsigned j = half ? unsigned(nth) - 1 - k : k;
        double2* dst = reinterpret_cast<double2*>(phi) + size_t(i * unsigned(nth) + j) * N2 + c;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            bad = bad || !(__builtin_fabs(v[r].x) <= 1.7976931348623157e308 &&
                           __builtin_fabs(v[r].y) <= 1.7976931348623157e308);
            dst[16 * r] = double2{v[r].x, -v[r].y};
        }
    }
    if (bad && flag) atomicOr(&flag->nonfinite, 1u);
}

}  // namespace fftfold
