// Internal declarations shared by the host set-up code and the HIP solve path.
#pragma once

#include <atomic>
#include <cstddef>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "modal_layout.h"
#include "sphpoisson.h"
#include "status.h"

struct spp_grid_s {
    int nr = 0, nth = 0, nphi = 0;
    spp_inner_bc inner = SPP_INNER_AUTO;
    std::vector<double> r_if, th_if;
};

// Byte offsets of the device-resident plan tables (all 256-byte aligned).
struct spp_plan_layout {
    size_t tw = 0;      // twiddles exp(-2 pi i t / N_phi), t < N_phi: [N_phi][2]
    size_t W = 0;       // forward projection, [M][N_theta(l)][N_theta(j)]
    size_t H = 0;       // inverse projection, [M][N_theta(j)][N_theta(l)]
    size_t lam = 0;     // lambda_Omega, [M][N_theta]
    size_t beta = 0;    // outer-boundary coefficient, [M][N_theta]
    size_t gamma = 0;   // inner-boundary coefficient (regular inner condition), [M][N_theta]
    size_t alpha = 0;   // radial face coefficients, [N_r] (last entry 0)
    size_t V = 0;       // radial volume factors, [N_r]
    size_t VR = 0;      // V_i R_i, [N_r]
    size_t Wimg = 0;    // LDS images of W_m for the projection kernel, [M][KMAX][NP]
    size_t Himg = 0;    // LDS images of H_m, [M][KMAX][NP]
    size_t Wimg32 = 0;  // FP32 copies of the images (mixed-precision projections)
    size_t Himg32 = 0;
    size_t Wpar = 0;    // parity-split images, [M][2][KMAX][NP] (even, odd)
    size_t Hpar = 0;
    size_t Fimg = 0;    // fused per-mode kernel images, [M][2][KP][NP] (forward, then inverse)
    size_t Iimg = 0;
    size_t Rimg = 0;    // radial row records of the fused kernel (modal_layout.h)
    size_t sig = 0;     // theta face coefficients sigma_{j+1/2}, [N_theta + 1] (poles 0)
    size_t dmu = 0;     // cos theta_{j-1/2} - cos theta_{j+1/2}, [N_theta]
    size_t Sj = 0;      // S_j, [N_theta]
    size_t lamphi = 0;  // lambda_{phi,m}, [M]
    size_t mom = 0;     // factors of the momentum source's face integrals (spp_mom_layout)
    size_t Bo = 0;      // outer-shell operator per mode, [M][N_theta(j')][N_theta(j)] (transposed)
    size_t Bi = 0;      // inner-shell operator (regular inner condition), same layout; empty otherwise
    size_t total = 0;
};

struct spp_plan_s {
    int nr = 0, nth = 0, nphi = 0, nm = 0;   // nm = N_phi/2 + 1 azimuthal modes
    std::vector<double> r_if, th_if;
    // host tables (float64), layouts as in spp_plan_layout
    std::vector<double> tw, W, H, lam, beta, gamma, alpha, V, VR, Wimg, Himg, sig, dmu, Sj, lamphi, mom;
    bool inner_regular = false;                // regular inner condition with r_{1/2} > 0
    std::vector<float> Wimg32, Himg32;
    std::vector<double> Ue, Uo, Wpar, Hpar;   // half-size even/odd eigenvectors and their images
    int proj_rn = 0;                           // tile width of the projection kernel (0: fallback)
    bool parity = false;                       // equator-symmetric theta grid: modes ordered even, odd
    int par_rn = 0;                            // tile width of the parity-split kernel (0: not used)
    std::vector<double> Fimg, Iimg, Rimg;      // images of the fused per-mode kernel
    std::vector<double> Bo, Bi;                // shell operators H diag(beta) H^T D (gamma for Bi)
    bool fused_ok = false;                     // the fused per-mode path can run this grid
    std::atomic<int> path{SPP_PATH_AUTO};      // requested path (spp_plan_set_path)
    spp_plan_layout lay;
    size_t workspace_bytes = 0;
    void* dev = nullptr;                       // caller-owned device copy
};

// thread-local error message helpers
spp_status spp_fail(spp_status st, const std::string& msg);

// Device entry of the FP64 solve (solve.hip).  With ev != NULL, ev[0..5]
// are recorded on the stream before the first and after every stage.
// With gate != NULL every kernel runs only if *gate != 0 (status.h); such a
// solve does not clear the workspace's status record.
spp_status spp_launch_solve_f64(const spp_plan_s* p, const double* rho, double* phi, double G,
                                void* ws, void* stream, hipEvent_t* ev = nullptr, const unsigned* gate = nullptr);

// Number of timed stages of one solve and their names.
constexpr int SPP_NUM_STAGES = 5;

// Device entry of the mixed-precision solve (solve.hip).
spp_status spp_launch_solve_mixed(const spp_plan_s* p, spp_precision prec, int n_refine, int fallback_fp64,
                                  const double* rho, double* phi, double G, void* ws, void* stream);

// Workspace of the mixed-precision solve: the status record, four fields, two
// shells and the residual maxima (and at least the FP64 fallback's workspace).
size_t spp_mixed_workspace_bytes(const spp_plan_s* p);

// Device entry of the momentum source (solve.hip): the force on every cell
// from the gravitational stress tensor; the workspace needs two shells after
// its status record.
spp_status spp_launch_momentum(const spp_plan_s* p, const double* phi, double G, double* fx, double* fy, double* fz,
                               void* ws, void* stream);

// Device entry of the FP64 residual r = 4 pi G rho - L Phi (solve.hip); the
// workspace needs four shells after its status record.
spp_status spp_launch_residual(const spp_plan_s* p, const double* rho, const double* phi, double G, double* r,
                               void* ws, void* stream);

// Device entry of the face fluxes of grad Phi (solve.hip); the workspace needs
// two shells of N_theta N_phi doubles (any FP64 solve workspace holds them).
spp_status spp_launch_face_fluxes(const spp_plan_s* p, const double* phi, double* fr, double* ft, double* fp,
                                  void* ws, void* stream);

// Batched FP64 solves of n right-hand sides of one fused-path plan, one launch
// per kernel over all of them (solve.hip): region layout and size.
size_t spp_class_batch_bytes(const spp_plan_s* p, int n);
spp_status spp_launch_class_batch(const spp_plan_s* p, int n, const double* const* rho_tab,
                                  double* const* phi_tab, const double* scale_tab, spp_status_record* recs,
                                  double* X, double* sink, int paired, hipStream_t s);

// Projection tile autotuner and launch-cache prewarm (solve.hip).
spp_status spp_autotune_projection_impl(const spp_plan_s* p, void* ws, void* stream, int* chosen_rm);
void spp_prewarm_launch_caches(const spp_plan_s* p);

// Resolve the no-allocation solve's scratch address on the current device
// (noalloc.hip; called by spp_plan_upload), and look it up.
void spp_noalloc_prepare_current_device();
spp_status spp_noalloc_scratch_current(void** ptr);

// Kernels of an FP64 solve of this plan, separated by semicolons (solve.hip).
std::string spp_describe_solve(const spp_plan_s* p);

// Argument checks shared by the solve entry points (plan.cpp).
spp_status spp_validate_solve(const char* who, const spp_plan_s* p, const double* rho_dev, const double* phi_dev,
                              double G, const void* workspace_dev);

// Symmetric tridiagonal eigensolver (eigen_ql.cpp): d[n] diagonal,
// e[n-1] off-diagonal; on return d holds the eigenvalues in ascending order
// and Z (row-major n x n) the orthonormal eigenvectors as columns.
bool spp_tridiag_eigen(int n, std::vector<double>& d, std::vector<double> e, std::vector<double>& Z);

// The solve takes the fused per-mode path (folded FFT, one kernel for
// projection + radial + inverse projection, folded inverse FFT).
inline bool spp_plan_fused(const spp_plan_s* p) { return p->fused_ok && p->path.load() != SPP_PATH_STAGED; }

constexpr size_t spp_align256(size_t x) { return (x + 255) & ~size_t(255); }

// Offsets (in doubles) of the momentum source's tables inside the plan's `mom`
// vector, in the order of momentum::Tables.
struct spp_mom_layout {
    size_t R2, ring, invr, invdr, is2, isc, is, ic, dth, invsdp, invdthc, fst, fct, jc, js, cp1, sp1, total;
    spp_mom_layout(int nr, int nth, int nphi)
    {
        size_t o = 0;
        auto take = [&](size_t n) { const size_t r = o; o += n; return r; };
        R2 = take(nr + 1); ring = take(nr); invr = take(nr); invdr = take(nr + 1);
        is2 = take(nth); isc = take(nth); is = take(nth); ic = take(nth); dth = take(nth); invsdp = take(nth);
        invdthc = take(nth + 1); fst = take(nth + 1); fct = take(nth + 1);
        jc = take(nphi); js = take(nphi); cp1 = take(nphi); sp1 = take(nphi);
        total = o;
    }
};

// Workspace bytes after the spectral field of a fused FP64 solve that the
// per-mode kernel uses as the sink of its stores of padding rows and columns:
// one double per thread of its workgroup, shared by all its workgroups
// (nothing reads them).
constexpr size_t spp_modal_sink_bytes = spp_align256(size_t(modalimg::NW) * 64 * sizeof(double));

// Workspace bytes of one FP64 solve: the status record (status.h), then on
// the fused path one spectral field, transformed in place, and the store
// sink, on the staged path two fields; either also holds the four shells of
// spp_residual (two of which spp_face_fluxes uses).
inline size_t spp_path_workspace_bytes(const spp_plan_s* p, bool fused)
{
    const size_t field = spp_align256(size_t(p->nr) * p->nth * p->nphi * sizeof(double));
    const size_t shells = 4 * spp_align256(size_t(p->nth) * p->nphi * sizeof(double));
    const size_t need = (fused && p->fused_ok) ? field + spp_modal_sink_bytes : 2 * field;
    return SPP_STATUS_BYTES + (need > shells ? need : shells);
}
