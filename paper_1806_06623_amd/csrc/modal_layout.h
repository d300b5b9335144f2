// Geometry of the LDS images read by the fused per-mode kernel (modal.hip.h);
// shared by the host code that builds the images in the plan and by the
// kernel that copies them into LDS.
//
// One image per (m, parity) and direction holds a half-size matrix B[k][n]
// (k, n < h = N_theta / 2 <= 64) in KP rows of NP doubles, KP = h rounded up
// to a multiple of 32.  In MFMA step s the lane group g = lane / 16 multiplies
// k = 8 (s / 2) + 2 g + (s % 2): the four groups of two consecutive steps
// cover eight consecutive k, so one 16-byte load per lane fetches its A
// operand for two steps and a chunk of eight steps reads 32 consecutive
// doubles (two whole 128-byte lines) of every row.  Image row 4 s + g holds
// that k; the 16-double row pad puts the four rows of one step on distinct
// bank halves.  Entries with k >= h or n >= h are zero.
#pragma once
#include <cstddef>

namespace modalimg {

constexpr int NW = 12;                       // waves per workgroup
constexpr int TMAX = 3;                      // row tiles of 16 per wave
constexpr int NRMAX = NW * 16 * TMAX;        // largest N_r of the fused kernel (576)

constexpr int rn_for(int h) { return h <= 16 ? 1 : h <= 32 ? 2 : 4; }

// Radial row records of the fused kernel, one image per plan (they depend on
// the radial grid only).  Row tiles per wave T = ceil(N_r / (16 NW)), chunks
// of CH = 4 T rows, P = 4 NW chunks; row i's record {x, y, z, a, a^2, V}
// (RECD doubles) sits at record i + i / CH, and the free record after each
// chunk holds the chunk's {oL, oR, 2^-e_p, -oL oR 2^-e_p prod a}.
constexpr int RECD = 6;
constexpr int t_for(int nr) { return (nr + 16 * NW - 1) / (16 * NW); }
constexpr int rec_records(int T) { return NW * 16 * T + 4 * NW; }
constexpr size_t rec_elems(int T) { return size_t(rec_records(T)) * RECD; }
constexpr int kp(int RN) { return RN == 4 ? 64 : 32; }
constexpr int np(int RN) { return 16 * RN + 16; }
constexpr size_t elems(int RN) { return size_t(kp(RN)) * np(RN); }
inline int row_of(int k)
{
    const int t = k >> 3, g = (k >> 1) & 3, odd = k & 1;
    return 4 * (2 * t + odd) + g;
}

}  // namespace modalimg
