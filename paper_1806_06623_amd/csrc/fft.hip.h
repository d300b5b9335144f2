// LDS-resident real FFT along phi for gfx950 (float64).
//
// A real line of N = N_phi samples is read as N/2 complex values
// z_n = x_{2n} + i x_{2n+1}; a complex Stockham FFT of length N/2 runs in LDS
// with radix-8/4/2 passes held in registers, and one split step turns Z into
// the half spectrum X_m, m = 0..N/2 (and back for the inverse).  Spectral data
// are stored as N real components per line ("halfcomplex" order):
//   q = m        : Re X_m,  m = 0..N/2
//   q = N - m    : Im X_m,  m = 1..N/2-1
// in planes [q][line], line = i * N_theta + j, so that each later stage reads
// and writes contiguous runs of lines for a fixed component q.
#pragma once
#include <hip/hip_runtime.h>

struct c64 {
    double x, y;
};

__device__ __forceinline__ c64 cadd(c64 a, c64 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c64 csub(c64 a, c64 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c64 cmul(c64 a, c64 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ c64 cconj(c64 a) { return {a.x, -a.y}; }
__device__ __forceinline__ c64 cmul_mi(c64 a) { return {a.y, -a.x}; }   // a * (-i)

// Forward DFT of size R on registers, exp(-2 pi i r s / R).
template <int R> __device__ __forceinline__ void dft(c64* v);

template <> __device__ __forceinline__ void dft<2>(c64* v)
{
    const c64 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <> __device__ __forceinline__ void dft<4>(c64* v)
{
    const c64 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const c64 s13 = cadd(v[1], v[3]), d13 = cmul_mi(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

template <> __device__ __forceinline__ void dft<8>(c64* v)
{
    c64 e[4] = {v[0], v[2], v[4], v[6]};
    c64 o[4] = {v[1], v[3], v[5], v[7]};
    dft<4>(e);
    dft<4>(o);
    const double h = 0.70710678118654752440;   // sqrt(1/2)
    const c64 o1 = {h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};    // * exp(-i pi/4)
    const c64 o2 = cmul_mi(o[2]);                                      // * exp(-i pi/2)
    const c64 o3 = {h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};   // * exp(-3 i pi/4)
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

// LDS index of complex element i of a line: one pad slot after every 8
// elements, so that the radix-8 pass (which writes 8 consecutive elements per
// thread) and the transposed accesses of the split step fall on distinct
// banks.  Lines are LS complex values apart, LS = padded length + 1.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }
template <int N2> struct LineStride {
    static constexpr int LS = N2 + N2 / 8 + 1;
};

// One Stockham autosort pass of radix R over a line of N2 complex values in
// LDS, processed by T threads (tid = 0..T-1).  Ns is the length of the
// sub-transforms already done.  tw[t] = exp(-2 pi i t / (2 N2)).
template <int N2, int R, int Ns, int T>
__device__ __forceinline__ void stockham_pass(c64* line, int tid, const c64* __restrict__ tw)
{
    constexpr int NB = N2 / R;      // butterflies per line
    constexpr int BPT = NB / T;     // butterflies per thread
    static_assert(BPT >= 1 && NB % T == 0, "thread mapping");
    constexpr int TWS = (2 * N2) / (Ns * R);   // twiddle stride in the N-point table
    c64 v[BPT][R];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int b = tid + u * T;
        const int k = b % Ns;
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = line[pidx(b + r * NB)];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[u][r] = cmul(v[u][r], tw[r * k * TWS]);
        }
        dft<R>(v[u]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int b = tid + u * T;
        const int k = b % Ns;
        const int base = (b / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) line[pidx(base + r * Ns)] = v[u][r];
    }
    __syncthreads();
}

template <int N2, int Ns, int T, int E>
__device__ __forceinline__ void fft_passes(c64* line, int tid, const c64* __restrict__ tw)
{
    if constexpr (Ns < N2) {
        constexpr int rem = N2 / Ns;
        constexpr int R = rem >= 8 ? (E >= 8 ? 8 : E) : rem;
        stockham_pass<N2, R, Ns, T>(line, tid, tw);
        fft_passes<N2, Ns * R, T, E>(line, tid, tw);
    }
}

// Thread/line mapping of the FFT kernels for a given N = N_phi.
template <int N, int THREADS_ = 256> struct FftShape {
    static constexpr int N2 = N / 2;                 // complex points per line
    static constexpr int E = N2 < 8 ? N2 : 8;        // complex values per thread
    static constexpr int T = N2 / E;                 // threads per line
    static constexpr int THREADS = THREADS_;
    static constexpr int JB = THREADS / T;           // lines per workgroup
};
