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
// workgroup reads and writes only its own half rows.  `sink` (THREADS
// doubles, shared by all workgroups and never read, in the same allocation as
// X and less than 4 GB after it) receives the stores of padding rows and
// columns.
//
// Work split (NW = 12 waves, T row tiles of 16 per wave, CH = 4 T):
//   wave w, lane (lr = lane % 16, g = lane / 16), accumulator register v of
//   tile rb and column tile cb holds row  w 16 T + g CH + 4 rb + v  and
//   column l = lr + 16 cb.  The MFMA row index r of tile rb is mapped to
//   that row by r = g + 4 v (A operand: lane lr supplies row
//   w 16 T + (lr % 4) CH + 4 rb + lr / 4), so every lane group owns CH
//   consecutive rows of each of its columns: a chunk of the radial
//   partition method, which runs on the accumulators without moving them.
//   The CH-row chunks of the 4 NW lane groups of a column are its
//   partitions.  Pass 1 eliminates each chunk's interior (through the
//   continuants of the interior block); the reduced (Schur complement)
//   system over the 48 separator rows of a column is solved inside one
//   16-lane row of a wave (local elimination, then cyclic reduction through
//   DPP row shifts), 16 columns per quartet of waves; pass 2 back-substitutes
//   the interiors.  The three steps are software-pipelined over the column
//   groups of 16.  For the inverse projection each tile is transposed
//   through a small per-wave LDS buffer into the A-operand layout.
//
// v_mfma_f64_16x16x4f64 operand layout: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; result register v of lane l is C[l / 16 + 4 v][l % 16].
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "modal_layout.h"
#include "radial.hip.h"
#include "status.h"

namespace modal {

using d4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;

constexpr int NW = modalimg::NW;
constexpr int THREADS = 64 * NW;
constexpr int P = 4 * NW;          // radial partitions per column
constexpr int TP = 34;             // pitch of the transpose buffer (32 columns + pad)

// Every phase of the kernel is straight-line code in one basic block; this
// keeps the instruction scheduler from interleaving neighbouring phases
// (which would keep values of several phases live at once and spill).
#define MODAL_PHASE_FENCE() __builtin_amdgcn_sched_barrier(0)

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
__device__ __forceinline__ void stage_image(double* __restrict__ Bs, const double* __restrict__ img, int tid)
{
    const double2* src = reinterpret_cast<const double2*>(img);
    double2* dst = reinterpret_cast<double2*>(Bs);
    constexpr int HALF = ELEMS / 2, PER = (HALF + THREADS - 1) / THREADS;
    double2 v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = tid + u * THREADS;
        v[u] = src[i < HALF ? i : HALF - 1];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = tid + u * THREADS;
        if (i < HALF) dst[i] = v[u];
    }
}

// Part of an image (COUNT doubles from FIRST) held in registers between its
// load and its copy into LDS.
template <int COUNT> struct ImagePart {
    static constexpr int HALF = COUNT / 2, PER = (HALF + THREADS - 1) / THREADS;
    double2 v[PER];
};

template <int FIRST, int COUNT>
__device__ __forceinline__ void load_part(ImagePart<COUNT>& part, const double* __restrict__ img, int tid)
{
    using IP = ImagePart<COUNT>;
    const double2* src = reinterpret_cast<const double2*>(img + FIRST);
#pragma unroll
    for (int u = 0; u < IP::PER; ++u) {
        const int i = tid + u * THREADS;
        part.v[u] = src[i < IP::HALF ? i : IP::HALF - 1];
    }
}

template <int FIRST, int COUNT>
__device__ __forceinline__ void store_part(double* __restrict__ Bs, const ImagePart<COUNT>& part, int tid)
{
    using IP = ImagePart<COUNT>;
    double2* dst = reinterpret_cast<double2*>(Bs + FIRST);
#pragma unroll
    for (int u = 0; u < IP::PER; ++u) {
        const int i = tid + u * THREADS;
        if (i < IP::HALF) dst[i] = part.v[u];
    }
}

// Asynchronous copy of an image into LDS without registers (gfx950 LDS DMA)
// by the NWAVES waves wq = 0 .. NWAVES-1: each copies 1 KB pieces, lane i
// moving 16 bytes from piece + 16 i to the same offset of the LDS
// destination.  Completion is awaited with s_waitcnt vmcnt(0) by every wave
// before a barrier (the compiler also waits before the wave's next LDS read).
template <int ELEMS, int NWAVES>
__device__ __forceinline__ void image_dma(double* __restrict__ Bs, const double* __restrict__ img, int wq, int lane)
{
    constexpr int PIECES = ELEMS / 128;                 // 128 doubles = 1 KB per wave and piece
    static_assert(ELEMS % 128 == 0, "image in whole 1 KB pieces");
#pragma unroll
    for (int u = 0; u < (PIECES + NWAVES - 1) / NWAVES; ++u) {
        const int pc = wq + NWAVES * u;                 // wave-uniform
        if (pc < PIECES)
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(img + pc * 128 + 2 * lane),
                                             (__attribute__((address_space(3))) void*)(Bs + pc * 128), 16, 0, 0);
    }
}

// The same for an image of any even length: the last piece moves only the
// lanes whose 16 bytes lie inside the image.
template <int ELEMS, int NWAVES>
__device__ __forceinline__ void image_dma_tail(double* __restrict__ Bs, const double* __restrict__ img, int wq,
                                               int lane)
{
    constexpr int PIECES = (ELEMS + 127) / 128;
    static_assert(ELEMS % 2 == 0, "image in whole 16-byte pairs");
#pragma unroll
    for (int u = 0; u < (PIECES + NWAVES - 1) / NWAVES; ++u) {
        const int pc = wq + NWAVES * u;                 // wave-uniform
        if (pc < PIECES && pc * 128 + 2 * lane < ELEMS)
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(img + pc * 128 + 2 * lane),
                                             (__attribute__((address_space(3))) void*)(Bs + pc * 128), 16, 0, 0);
    }
}

// Calls f(integral_constant<int, I>) for I = I0 .. N-1 in order.
template <int I0, int N, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I0 < N) {
        f(std::integral_constant<int, I0>{});
        static_for<I0 + 1, N>(f);
    }
}

// The lane index within the wave, computed afresh from the hardware lane
// counter (mbcnt over a full mask) inside an opaque asm, so that the compiler
// cannot keep one copy and reuse it.  The kernel recomputes lane-derived
// indices at the start of every phase: values derived once would stay live
// through the register-heavy phases, be spilled, and their reloads would sit
// on the critical path.
__device__ __forceinline__ int lane_now()
{
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
}

// The (component q, parity) unit of workgroup L of the 1-D grid of 2 N_phi.
// Workgroups are dispatched to the 8 XCDs in turn (L % 8), so units placed
// at L and L + 8 share an XCD's L2 and start together.  The cosine and sine
// components of one m (q and N_phi - q) with the same parity read the same
// eigenvector images; they are paired that way: in each block of 16
// workgroups, pair k = 8 (L / 16) + L % 8 has its q at L and its N_phi - q at
// L + 8.  Pairs k < N_phi - 2 are (m = k/2 + 1, parity k % 2); the last two
// hold the unpaired components q = 0 and q = N_phi/2 (one parity each at L
// and L + 8).  Grids with N_phi < 8, and launches with paired == 0, keep the
// plain order (q = L / 2, parity L % 2).
__device__ __forceinline__ void unit_of(int L, int nphi, int paired, int& q, int& par)
{
    if (nphi < 8 || !paired) {
        par = L & 1;
        q = L >> 1;
        return;
    }
    const int k = 8 * (L >> 4) + (L & 7), mem = (L >> 3) & 1;
    if (k < nphi - 2) {
        const int pm = k >> 1;
        par = k & 1;
        q = mem ? nphi - 1 - pm : pm + 1;
    } else {
        q = k == nphi - 2 ? 0 : nphi / 2;
        par = mem;
    }
}

// Issue priority of this wave among the waves of its SIMD (0..3).
template <int PRIO>
__device__ __forceinline__ void set_priority()
{
    static_assert(PRIO >= 0 && PRIO <= 3, "wave priority 0..3");
    __builtin_amdgcn_s_setprio(PRIO);
}

// Move a double between lanes of a 16-lane row (DPP row shift): with
// CTRL = 0x110 + n (row_shr) lane i receives lane i - n, with 0x100 + n
// (row_shl) lane i + n; lanes without a source in their row receive zero
// (written by the DPP bound control, with no fill value moved first).
template <int CTRL>
__device__ __forceinline__ double row_move0(double v)
{
    const long long vb = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp(int(vb), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(int(vb >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// One level of parallel cyclic reduction over the 16 lanes of a row, stride
// HS: row t (a x_{t-1} + b x_t + c x_{t+1} = d in the current stride) is
// combined with rows t - HS and t + HS; a partner outside the row contributes
// nothing (its coupling to t is zero by construction, and the select keeps a
// missing partner's value out).
template <int HS>
__device__ __forceinline__ void pcr16_level(double& ra, double& rb, double& rc, double& rd, int t)
{
    // bm and bp of a missing partner are zero; the selects below discard the
    // reciprocals formed from them
    const double am = row_move0<0x110 + HS>(ra), bm = row_move0<0x110 + HS>(rb);
    const double cm = row_move0<0x110 + HS>(rc), dm = row_move0<0x110 + HS>(rd);
    const double ap = row_move0<0x100 + HS>(ra), bp = row_move0<0x100 + HS>(rb);
    const double cp = row_move0<0x100 + HS>(rc), dp = row_move0<0x100 + HS>(rd);
    const double a = t >= HS ? -ra * radial::recip(bm) : 0.0;
    const double c = t + HS < 16 ? -rc * radial::recip(bp) : 0.0;
    rb = rb + a * cm + c * ap;
    rd = rd + a * dm + c * dp;
    ra = a * am;
    rc = c * cp;
}

template <int RN, int T>
__global__ __launch_bounds__(THREADS) void k_modal(double* __restrict__ X, const double* __restrict__ Fimg,
                                                   const double* __restrict__ Iimg, const double* __restrict__ Rimg,
                                                   const double* __restrict__ lam,
                                                   const double* __restrict__ beta, radial::Coef tab, int nth,
                                                   int nphi, double* __restrict__ sink,
                                                   const unsigned* __restrict__ gate, size_t xstride, int paired)
{
    if (spp_gate_closed(gate)) return;
    using Gm = Geo<RN>;
    constexpr int NC = Gm::NC, ELEMS = Gm::ELEMS;
    constexpr int CH = 4 * T;               // rows per lane chunk
    constexpr int ROWS = NW * 16 * T;       // row capacity
    constexpr int NCH = T * NC;             // load chunks of the forward product
    constexpr int FP = 17;                  // pitch of a partition row in the [P][16] fields (bank skew)
    constexpr int PS = P * FP;              // one reduced-system field: [P][16] with that pitch
    constexpr int RED = 12 * PS;            // two buffers of own[3], nxt[3]
    constexpr int TRB = NW * 16 * TP;       // one 16 x 32 transpose buffer per wave
    constexpr int UN = RED > TRB ? RED : TRB;
    __shared__ __attribute__((aligned(16))) double Bs[ELEMS];
    __shared__ __attribute__((aligned(16))) double un[UN];
    __shared__ double xs[2 * PS];           // two buffers of the separator values
    // per-row radial records {x, y, z, a, a^2, V}: x = -(alpha_{i-1} + alpha_i),
    // y = V_i R_i, z = [i = N_r - 1], a = alpha_i, so that the diagonal for
    // eigenvalue lambda and outer coefficient beta is x + y lambda - z beta;
    // rows >= N_r are decoupled identity rows.  Row i sits at i + i / CH; the
    // interior rows of chunk p (all but its first) are multiplied by the power
    // of two 2^-e_p (exact), which keeps the continuants of pass 1 near unit
    // size, and the free slot after each chunk holds {oL, oR, 2^-e_p, -oL oR
    // 2^-e_p prod of the chunk's scaled interior couplings}, oL and oR the
    // chunk's (unscaled) couplings to its own and to the next separator.  The
    // plan builds this image (it depends on the radial grid only).
    constexpr int RB = 8 * modalimg::RECD;  // bytes per record
    static_assert(ROWS + P == modalimg::rec_records(T), "record image of the plan");
    __shared__ __attribute__((aligned(16))) double t_rec[(ROWS + P) * (RB / 8)];
    __shared__ double t_lam[16 * RN], t_bo[16 * RN];   // lambda_l, beta_l of this (m, parity)

    // batched launch: RHS r owns the 2 N_phi workgroups from 2 N_phi r and the
    // spectral field at r * xstride (xstride = 0: a single solve)
    int L = blockIdx.x;
    if (xstride) {
        const int r = L / (2 * nphi);
        L -= r * 2 * nphi;
        X += r * xstride;
    }
    int q, par;
    unit_of(L, nphi, paired, q, par);
    const int m = q <= nphi / 2 ? q : nphi - q;
    const int nr = tab.nr, h = nth >> 1;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave index (uniform)
    const int lane = lane_now(), lr = lane & 15, g = lane >> 4;       // forward phase only
    double* __restrict__ Xq = X + size_t(q) * nr * nth + par * h;

    // rows supplied as A operand by this lane in tile rb (clamped into range)
    auto arow = [&](int rb) {
        const int R = w * 16 * T + (lr & 3) * CH + 4 * rb + (lr >> 2);
        return Xq + size_t(R < nr ? R : nr - 1) * nth;
    };

    // ---- forward projection, in chunks c of 8 MFMA steps: column block
    // kc = c / T (k in [32 kc, 32 kc + 32)) of row tile rb = c % T.  With two
    // column blocks (SPLIT) the first T chunks use only the image rows of
    // k < 32, the first half of the image: only that half and chunk 0 are
    // loaded before the first barrier, so that the first products start on
    // less data; chunk 1 and the second half follow while they run.
    constexpr bool SPLIT = NC == 2;
    constexpr int HALF_E = ELEMS / 2;
    const double* fimg = Fimg + (size_t(m) * 2 + par) * ELEMS;
    const int tid0 = w * 64 + lane;
    d4 acc[T][RN];
#pragma unroll
    for (int rb = 0; rb < T; ++rb)
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) acc[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
    double ba[8], bb[8];
    load_a(ba, arow(0), 0, g, h);
    if constexpr (SPLIT) {
        ImagePart<HALF_E> first;
        load_part<0, HALF_E>(first, fimg, tid0);
        store_part<0, HALF_E>(Bs, first, tid0);
    } else {
        stage_image<ELEMS>(Bs, fimg, tid0);
    }
    // lambda_l and beta_l of this (m, parity), one per column
    if (threadIdx.x < 16 * RN) {
        const int l = threadIdx.x, L = par * h + (l < h ? l : h - 1);
        t_lam[l] = lam[size_t(m) * nth + L];
        t_bo[l] = beta[size_t(m) * nth + L];
    }
    // the radial row records (built by the plan, the same for every unit).
    // With two column blocks they and the second half of the image are copied
    // into LDS by direct loads from quartet 2, issued here, so that no wave
    // holds them in registers through the first products (the compiler would
    // instead reload such values one after another at their stores, each load
    // waiting for every load in flight).  The barrier's release makes quartet
    // 2 wait for its copies (they are LDS writes); they overlap the other
    // waves' loads.
    constexpr int RECE = (ROWS + P) * modalimg::RECD;
    if constexpr (SPLIT) {
        if (w >> 2 == 2) {
            image_dma<HALF_E, 4>(Bs + HALF_E, fimg + HALF_E, w - 8, lane);
            image_dma_tail<RECE, 4>(t_rec, Rimg, w - 8, lane);
        }
    } else {
        stage_image<RECE>(t_rec, Rimg, tid0);
    }
    __syncthreads();
    if constexpr (SPLIT) {
        if (w >> 2 == 2) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the copies have landed
    }
    if constexpr (NCH > 1) load_a(bb, arow(1 % T), 1 / T, g, h);

    static_for<0, NCH>([&](auto cc) __attribute__((always_inline)) {
        constexpr int c = decltype(cc)::value, rb = c % T, kc = c / T;
        if constexpr (SPLIT && c == T) __syncthreads();

        // issue priority falls as a wave gets ahead, so that the three waves of
        // a SIMD share the matrix pipe evenly and finish the product together
        // (with equal priorities the oldest wave runs ahead and the radial
        // phase waits for the last one)
        set_priority<(NCH - 1 - c > 3 ? 3 : NCH - 1 - c)>();
        if constexpr (c % 2 == 0) {
            mma_chunk<RN>(acc[rb], ba, Bs, kc, g, lr);
            if constexpr (c + 2 < NCH) load_a(ba, arow((c + 2) % T), (c + 2) / T, g, h);
        } else {
            mma_chunk<RN>(acc[rb], bb, Bs, kc, g, lr);
            if constexpr (c + 2 < NCH) load_a(bb, arow((c + 2) % T), (c + 2) / T, g, h);
        }
    });

    set_priority<0>();
    MODAL_PHASE_FENCE();
    // ---- radial solves (partition method on the accumulators, no branches:
    // padding rows have diagonal 1, no coupling and a zero right-hand side,
    // and partitions past the last row reduce to identity rows)
    // the slab as scalars from here on (no MFMA register tuples to maintain)
    double sl[T][RN][4];
#pragma unroll
    for (int rb = 0; rb < T; ++rb)
#pragma unroll
        for (int cb = 0; cb < RN; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) sl[rb][cb][v] = acc[rb][cb][v];
#define D(k) sl[(k) >> 2][cb][(k) & 3]

    // partition p = 4 w + g of this lane group: rows s0 .. s0 + CH - 1, first
    // record (skewed) at sk
#define PART_INDICES()                                                  \
    const int ln_ = lane_now(), lr = ln_ & 15, p = 4 * w + (ln_ >> 4); \
    const int s0 = p * CH, sk = s0 + p;                                 \
    (void)s0; (void)sk

    // Row records are loaded behind empty asm statements that take pivots as
    // inputs, so that the records of other rows are never live at the same
    // time: pass 2 reads one row ahead (the load of row k+1 and the first use
    // of row k are pinned after the pivot of row k-1, so the load latency
    // overlaps one row of the recurrence); pass 1 loads the two rows of a step
    // after both previous pivots.
    // records addressed by a byte offset, so that every row load is one
    // immediate offset from the same register
#define REC_AT(off) (reinterpret_cast<const char*>(t_rec) + (off))
#define ROW(k) (*reinterpret_cast<const double4*>(REC_AT(rb0 + (k) * RB)))
// a^2 of a row: the record holds it as the square of its a, which is computed
// instead of loaded
#define SQ(a) ((a) * (a))
#define VOL(k) (*reinterpret_cast<const double*>(REC_AT(rb0 + (k) * RB + 40)))
#define DIAG(r) ((r).x + (r).y * lm - (r).z * bo)
#define TIE(r, dep) asm volatile("" : "+v"((r).x), "+v"((r).y), "+v"((r).z), "+v"((r).w) : "v"(dep))
#define NEXT_BASE(dep) asm volatile("" : "+v"(rb0) : "v"(dep))
#define NEXT_BASE2(d1, d2) asm volatile("" : "+v"(rb0) : "v"(d1), "v"(d2))

    // pass 1 of column group cb.  The interior rows 1..n (n = CH - 1) of the
    // chunk form a tridiagonal block A (scaled by 2^-e_p) coupled to the
    // separators on either side.  Its continuants, p_k = det of the leading
    // k x k block and q_k = det of the trailing block from row k, satisfy
    //   p_k = d_k p_{k-1} - a_{k-1}^2 p_{k-2},  q_k = d_k q_{k+1} - a_k^2 q_{k+2},
    // and the entries of A^-1 that pass 1 needs are ratios of them:
    // (A^-1)_nn = p_{n-1}/p_n, (A^-1)_11 = q_2/q_1, (A^-1)_1n = prod a / p_n.
    // The first and last entries of A^-1 D are T_1/q_1 and S_n/p_n with
    //   S_k = p_{k-1} D_k - a_{k-1} S_{k-1},  T_k = q_{k+1} D_k - a_k T_{k+1}
    // Two multiply-adds per row and recurrence, no division; one reciprocal
    // per sweep.  The partition's separator row and its contribution to the
    // next separator row go to buffer cb % 2.
    // n = CH - 1 is odd, so the sign (-1)^(n+1) of (A^-1)_1n is +1
    static_assert(CH % 2 == 0, "chunks of an even number of rows");
    auto pass1 = [&](auto cbc) __attribute__((always_inline)) {
        constexpr int cb = decltype(cbc)::value;
        PART_INDICES();
        double* own = un + (cb & 1) * 6 * PS;   // [3][P][16]
        double* nxt = own + 3 * PS;             // [3][P][16]
        const double lm = t_lam[lr + 16 * cb];
        const double bo = t_bo[lr + 16 * cb];
        unsigned rb0 = unsigned(sk) * RB;
#pragma unroll
        for (int k = 0; k < CH; ++k) D(k) *= VOL(k);
        // the forward sweep (p, S) from row 1 up and the backward sweep (q, T)
        // from row n down are independent: they run interleaved, one row of
        // each per step, whose record loads are issued together after the
        // previous step's pivots and awaited once.
        // Forward: pk = p_{k-1}, pk1 = p_{k-2}, al the coupling a of row
        // k-1; backward: qk = q_{k+1}, qk1 = q_{k+2}
        double pk, pk1 = 1.0, S = D(1), al;
        double qk, qk1 = 1.0, Tk = D(CH - 1);
        {
            const double4 cf = ROW(1), cr = ROW(CH - 1);
            pk = DIAG(cf);
            al = cf.w;
            qk = DIAG(cr);
        }
#pragma unroll
        for (int i = 0; i < CH - 2; ++i) {
            const int kf = 2 + i, kr = CH - 2 - i;
            NEXT_BASE2(pk, qk);
            const double4 cf = ROW(kf), cr = ROW(kr);
            S = pk * D(kf) - al * S;
            const double pn = DIAG(cf) * pk - SQ(al) * pk1;
            pk1 = pk;
            pk = pn;
            al = cf.w;
            Tk = qk * D(kr) - cr.w * Tk;
            const double qn = DIAG(cr) * qk - SQ(cr.w) * qk1;
            qk1 = qk;
            qk = qn;
        }
        const double ipn = radial::recip(pk);
        const double iq1 = radial::recip(qk);
        NEXT_BASE2(ipn, iq1);
        const double4 pt = ROW(CH);             // oL, oR, 2^-e_p, -oL oR 2^-e_p prod a
        nxt[(0 * P + p) * FP + lr] = pt.w * ipn;
        nxt[(1 * P + p) * FP + lr] = -(pt.y * pt.y * pt.z) * pk1 * ipn;
        nxt[(2 * P + p) * FP + lr] = pt.y * S * ipn;
        own[(0 * P + p) * FP + lr] = DIAG(ROW(0)) - (pt.x * pt.x * pt.z) * qk1 * iq1;
        own[(1 * P + p) * FP + lr] = pt.w * iq1;
        own[(2 * P + p) * FP + lr] = D(0) - pt.x * Tk * iq1;
    };

    // The separator rows of a column form a tridiagonal system of P = 48
    // rows.  A quartet of waves solves it for the 16 columns of group cb, one
    // 16-lane row per column (column 4 (w % 4) + g), lane t holding
    // partitions 3t .. 3t+2: the two interior rows of each lane are
    // eliminated locally, leaving one row per lane, which parallel cyclic
    // reduction over the 16 lanes of the row (DPP row shifts, no barriers)
    // solves in four levels.  The separator values go to xs buffer cb % 2.
    static_assert(P == 48, "the reduced solve maps 48 partitions onto 16 lanes x 3");
    auto solve = [&](auto cbc) __attribute__((always_inline)) {
        constexpr int cb = decltype(cbc)::value;
        const double* own = un + (cb & 1) * 6 * PS;
        const double* nxt = own + 3 * PS;
        double* xsb = xs + (cb & 1) * PS;
        const int ln_ = lane_now(), t = ln_ & 15, c = 4 * (w & 3) + (ln_ >> 4);
        double qa[3], qb[3], qc[3], qd[3];   // rows 3t .. 3t+2
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int pr = 3 * t + r;
            const int pq = pr > 0 ? pr - 1 : 0;
            const bool first = pr == 0;
            qa[r] = first ? 0.0 : nxt[(0 * P + pq) * FP + c];
            qb[r] = own[(0 * P + pr) * FP + c] + (first ? 0.0 : nxt[(1 * P + pq) * FP + c]);
            qc[r] = own[(1 * P + pr) * FP + c];
            qd[r] = own[(2 * P + pr) * FP + c] - (first ? 0.0 : nxt[(2 * P + pq) * FP + c]);
        }
        // rows 3t+1, 3t+2 in terms of x_{3t} and x_{3t+3}:
        //   x_{3t+1} = e1 + f1 x_{3t} + g1 x_{3t+3},  x_{3t+2} = e2 + f2 x_{3t} + g2 x_{3t+3}
        const double idet = radial::recip(qb[1] * qb[2] - qc[1] * qa[2]);
        const double e1 = (qb[2] * qd[1] - qc[1] * qd[2]) * idet, f1 = -qb[2] * qa[1] * idet, g1 = qc[1] * qc[2] * idet;
        const double e2 = (qb[1] * qd[2] - qa[2] * qd[1]) * idet, f2 = qa[2] * qa[1] * idet, g2 = -qb[1] * qc[2] * idet;
        // the previous lane's x_{3t-1} = e2' + f2' x_{3t-3} + g2' x_{3t} enters row 3t
        // (lane 0 has qa[0] = 0)
        const double e2p = row_move0<0x111>(e2), f2p = row_move0<0x111>(f2);
        const double g2p = row_move0<0x111>(g2);
        double ra = qa[0] * f2p;
        double rb = qb[0] + qa[0] * g2p + qc[0] * f1;
        double rc = qc[0] * g1;
        double rd = qd[0] - qa[0] * e2p - qc[0] * e1;
        pcr16_level<1>(ra, rb, rc, rd, t);
        pcr16_level<2>(ra, rb, rc, rd, t);
        pcr16_level<4>(ra, rb, rc, rd, t);
        pcr16_level<8>(ra, rb, rc, rd, t);
        const double x0 = rd * radial::recip(rb);
        const double x3 = row_move0<0x101>(x0);        // x_{3t+3}; lane 15 has g1 = g2 = 0
        xsb[(3 * t + 0) * FP + c] = x0;
        xsb[(3 * t + 1) * FP + c] = e1 + f1 * x0 + g1 * x3;
        xsb[(3 * t + 2) * FP + c] = e2 + f2 * x0 + g2 * x3;
    };

    // pass 2 of column group cb: the interior rows with both separators known
    // (pivots recomputed)
    auto pass2 = [&](auto cbc) __attribute__((always_inline)) {
        constexpr int cb = decltype(cbc)::value;
        const double* xsb = xs + (cb & 1) * PS;
        PART_INDICES();
        const int pp = p < P - 1 ? p + 1 : P - 1;
        const double lm = t_lam[lr + 16 * cb];
        const double bo = t_bo[lr + 16 * cb];
        unsigned rb0 = unsigned(sk) * RB;
        const double4 pt = ROW(CH);
        const double xL = xsb[p * FP + lr];
        const double xR = xsb[pp * FP + lr];     // multiplied by oR = 0 for the last partition
        D(0) = xL;
        D(1) -= (pt.x * pt.z) * xL;
        D(CH - 1) -= (pt.y * pt.z) * xR;
        // forward elimination (Thomas): pivot w_k = d_k - a_{k-1}^2 / w_{k-1};
        // D(k) becomes y_k = (D_k - a_{k-1} y_{k-1}) / w_k and cw[k] keeps
        // c_k = a_k / w_k, so that the back substitution x_k = y_k - c_k x_{k+1}
        // needs no record loads
        double cw[CH];
        NEXT_BASE(xL);
        double4 cur = ROW(1);
        double4 nx = ROW(2);
        double iw = radial::recip(DIAG(cur));
        D(1) *= iw;
        cw[1] = cur.w * iw;
        double al_prev = cur.w;
#pragma unroll
        for (int k = 2; k < CH; ++k) {
            cur = nx;
            TIE(cur, iw);
            NEXT_BASE(iw);
            if (k + 1 < CH) nx = ROW(k + 1);
            iw = radial::recip(DIAG(cur) - SQ(al_prev) * iw);
            D(k) = (D(k) - al_prev * D(k - 1)) * iw;
            if (k + 1 < CH) cw[k] = cur.w * iw;
            al_prev = cur.w;
        }
        // back substitution from x_{CH-1} = y_{CH-1}
        double xn = D(CH - 1);
#pragma unroll
        for (int k = CH - 2; k >= 1; --k) {
            xn = D(k) - cw[k] * xn;
            asm volatile("" : "+v"(xn));   // keeps the sweep ahead of the next pass's code
            D(k) = xn;
        }
    };

    // Software pipeline over the column groups, one barrier per round: in
    // round r every wave runs pass 2 of group r-2 and pass 1 of group r while
    // the quartet (r-1) % 3 first solves the reduced system of group r-1.
    // Pass 1 of a group and its reduced solve, and the solve and pass 2, are
    // one barrier apart; the double buffers keep rounds r and r+1 apart.
    const int quartet = w >> 2;
    auto round = [&](auto rc) __attribute__((always_inline)) {
        constexpr int r = decltype(rc)::value;
        MODAL_PHASE_FENCE();
        // the inverse image goes into the forward image's LDS (free since the
        // end of round 0) by direct copies from quartet 2, issued at the start
        // of round 1 so that their memory latency (a few microseconds: the
        // image comes from HBM for one of the two workgroups that share it)
        // overlaps the round's passes; the barrier that ends the round waits
        // for their completion, and the inverse phase starts without a load
        if constexpr (r == 1 && RN >= 2) {
            if (quartet == 2) image_dma<ELEMS, 4>(Bs, Iimg + (size_t(m) * 2 + par) * ELEMS, w - 8, lane_now());
        }
        if constexpr (r >= 1 && r <= RN) {
            if (quartet == (r - 1) % 3) solve(std::integral_constant<int, r - 1>{});
        }
        if constexpr (r >= 2) pass2(std::integral_constant<int, r - 2>{});
        if constexpr (r < RN) pass1(std::integral_constant<int, r>{});
        if constexpr (r <= RN) __syncthreads();
    };
    static_for<0, RN + 2>(round);
#undef PART_INDICES
#undef REC_AT
#undef ROW
#undef SQ
#undef VOL
#undef DIAG
#undef TIE
#undef NEXT_BASE
#undef NEXT_BASE2
#undef D

    // ---- inverse projection, tile by tile through a per-wave transpose
    // buffer (wave-local ordering only: LDS operations of one wave complete
    // in order, and the fences keep the compiler from reordering them)
    MODAL_PHASE_FENCE();
    if constexpr (RN >= 2) {
        __builtin_amdgcn_s_waitcnt(0);     // this wave's image pieces have landed
    } else {                               // a single column group: no round 1 to hide the copy in
        const int ln_ = lane_now();
        stage_image<ELEMS>(Bs, Iimg + (size_t(m) * 2 + par) * ELEMS, w * 64 + ln_);
    }
    __syncthreads();
    MODAL_PHASE_FENCE();
    double* tb = un + w * 16 * TP;
    const int lni = lane_now(), lri = lni & 15, gi = lni >> 4;   // inverse phase
    // Stores without branches (branches around them would split the code into
    // blocks the scheduler cannot interleave): every store addresses the
    // unit's base with a 32-bit byte offset, and the values of padding rows
    // and columns go to this lane's slot of the sink instead (the sink follows
    // the field in the same workspace; its slots are shared by all workgroups
    // and never read).
    char* const xbase = reinterpret_cast<char*>(Xq);
    const unsigned sink_off = unsigned(reinterpret_cast<char*>(sink) - xbase) + unsigned(w * 64 + lni) * 8u;
#pragma unroll
    for (int rb = 0; rb < T; ++rb) {
        d4 out[RN];
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) out[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < NC; ++kc) {
            // columns 32 kc .. 32 kc + 31 of tile rb, row r = gi + 4 v
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int cb = 2 * kc + half;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    tb[(gi + 4 * v) * TP + lri + 16 * half] = cb < RN ? sl[rb][cb < RN ? cb : 0][v] : 0.0;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            double a[8];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double2 x = *reinterpret_cast<const double2*>(tb + lri * TP + 8 * t + 2 * gi);
                a[2 * t] = x.x;
                a[2 * t + 1] = x.y;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            mma_chunk<RN>(out, a, Bs, kc, gi, lri);
        }
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) {
            const int j = lri + 16 * cb;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int R = w * 16 * T + gi * CH + 4 * rb + v;
                const unsigned off = (R < nr && j < h) ? unsigned(R * nth + j) * 8u : sink_off;
                *reinterpret_cast<double*>(xbase + off) = out[cb][v];
            }
        }
    }
}

}  // namespace modal
