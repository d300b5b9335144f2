// Geometry of the LDS image of one projection matrix B_m (shared by the host
// code that builds the images in the plan and by the projection kernel that
// copies them into LDS).
//
// For a K x K matrix B[n][k] (K = N_theta <= 16 RN) the image has KMAX rows of
// NP doubles.  Row 4 s + g holds k = g * KG + s (KG = Kp / 4, Kp = K rounded up
// to a multiple of 32): in MFMA step s the lane group g = lane / 16 reads the
// four rows of one step, and the 16-double pad puts those rows on distinct
// bank halves.  Entries with n >= K or k >= K are zero.
#pragma once
#include <cstddef>

namespace projimg {

constexpr int rn_for(int K) { return K <= 16 ? 1 : K <= 32 ? 2 : K <= 64 ? 4 : 8; }
constexpr int nmax(int RN) { return 16 * RN; }
constexpr int kmax(int RN) { return (16 * RN + 31) / 32 * 32; }
constexpr int np(int RN) { return 16 * RN + 16; }
constexpr size_t elems(int RN) { return size_t(kmax(RN)) * np(RN); }
inline int kpad(int K) { return (K + 31) & ~31; }
inline int row_of(int k, int KG) { return 4 * (k % KG) + k / KG; }

}  // namespace projimg
