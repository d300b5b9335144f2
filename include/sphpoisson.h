/*
 * sphpoisson.h -- C ABI of the MI355X (gfx950) exact discrete Poisson solver
 * on N_r x N_theta x N_phi spherical polar finite-volume grids.
 *
 * The method (Mueller & Chan 2019, "An FFT-based solution method for the
 * Poisson equation on 3D spherical polar grids", Sec. 3):
 *   s = 4 pi G rho                                    (Sec. 3.1)
 *   real FFT of s along the uniform phi direction     (Sec. 3.2)
 *   per azimuthal mode m: projection onto the eigenvectors of the discrete
 *     theta operator hat-Delta_theta + S_j lambda_{phi,m}   (Sec. 3.2)
 *   per (m, l): tridiagonal radial solve of Delta_r f + R_i lambda_Omega f
 *     = s^ with the asymptotic outer boundary condition     (Sec. 3.2)
 *   inverse projection and inverse FFT                      (Sec. 3.2)
 * The discrete operator is the finite-volume Laplacian of Sec. 3.1 with
 * zero-area pole faces, periodic phi, the inner radial face of spp_inner_bc
 * (zero area when r_{1/2} = 0) and the outer condition above; the solver
 * returns its unique solution.
 *
 * Conventions shared by every call:
 *   - every function returns spp_status; on a non-OK status a message is
 *     available from spp_last_error() (thread-local, valid until the next
 *     call on the same thread);
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device memory of the current device; the library allocates no device
 *     memory at all: the caller provides the plan buffer and the workspace;
 *   - streams are hipStream_t passed as void*; NULL means the null stream.
 *     Device work is only enqueued; the caller synchronises the stream;
 *   - rho and Phi are row-major float64 arrays [N_r][N_theta][N_phi]
 *     (phi fastest), i.e. a contiguous float64 tensor of shape
 *     (N_r, N_theta, N_phi). Indices are 0-based (the paper's are 1-based).
 */
#ifndef SPHPOISSON_H
#define SPHPOISSON_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The enumerations below are passed as C ints.  Under C++ they get int as
 * their fixed underlying type, so that an out-of-range value a caller passes
 * is a valid value of the type (rejected with SPP_EINVAL) rather than
 * undefined behaviour. */
#ifdef __cplusplus
#define SPP_ENUM(tag) enum tag : int
#else
#define SPP_ENUM(tag) enum tag
#endif

typedef SPP_ENUM(spp_status_e) {
    SPP_OK = 0,
    SPP_EINVAL = -1,     /* invalid argument (sizes, interfaces, NULL pointers) */
    SPP_ENOTSUP = -2,    /* valid for the method, not supported by the library */
    SPP_EDEVICE = -3,    /* a HIP call failed                                   */
    SPP_ENOMEM = -4,     /* host allocation failed                              */
    SPP_ESTATE = -5,     /* object used out of order (e.g. solve before upload) */
    SPP_ENONFINITE = -6, /* non-finite value detected                           */
    SPP_ENOCONV = -7     /* refinement did not contract (FP64 fallback disabled) */
} spp_status;

/* Inner radial face r_{1/2} (the paper does not fix it; it matters only when
 * r_{1/2} > 0, since a face at r = 0 has no area). */
typedef SPP_ENUM(spp_inner_bc_e) {
    SPP_INNER_AUTO = 0,      /* zero area when r_{1/2} = 0, else zero flux             */
    SPP_INNER_ZERO_FLUX = 1, /* no flux through the inner face (exact for l = 0 when
                                no mass lies inside r_{1/2})                         */
    SPP_INNER_REGULAR = 2    /* the source-free interior's regular solution: each
                                angular eigenmode decays inwards as r^p',
                                p' = (-1 + sqrt(1 - 4 lambda_Omega))/2, extrapolated
                                from the innermost zone to the face (the counterpart of
                                the outer condition of Sec. 3.2)                     */
} spp_inner_bc;

typedef SPP_ENUM(spp_precision_e) {
    SPP_FP64 = 0,          /* all stages in float64                                */
    SPP_MIXED_FP32 = 1,    /* theta projections as FP32 MFMA products accumulated in
                              FP32; FFTs, radial solves, residual and the
                              accumulated solution in FP64 (spp_solve_mixed)       */
    SPP_MIXED_BF16X3 = 2   /* split-BF16 projections: reserved, SPP_ENOTSUP        */
} spp_precision;

typedef SPP_ENUM(spp_path_e) {
    SPP_PATH_AUTO = 0,     /* fused when the grid allows it, else staged           */
    SPP_PATH_STAGED = 1,   /* five kernels: FFT, projection, radial, projection, FFT */
    SPP_PATH_FUSED = 2     /* folded FFT, one per-mode kernel, folded inverse FFT  */
} spp_path;

/* What a solve found, read back by spp_solve_status after the stream ran. */
typedef struct {
    int refine_iters;              /* refinement steps taken (mixed form; 0 for FP64)   */
    double first_residual_rel;     /* max|s - L g_0| / max|s| after the first low-
                                      precision pass (mixed form; 0 for FP64)           */
    double last_residual_rel;      /* max|s - L g_n-1| / max|s|, the residual the last
                                      correction was computed from (mixed form)         */
    int not_contracted;            /* some refinement step had max|r_k| > max|r_k-1| / 2 */
    int fell_back_fp64;            /* the FP64 solve replaced the mixed result           */
    int nonfinite;                 /* Phi holds a NaN or an infinity                     */
} spp_solve_info;

typedef struct spp_grid_s* spp_grid;   /* host geometry, immutable        */
typedef struct spp_plan_s* spp_plan;   /* eigensystems + device layout    */
typedef struct spp_batch_s* spp_batch; /* captured graph of many solves   */
typedef struct spp_server_s* spp_server; /* serving loop                  */

/* One request of the serving loop. */
typedef struct {
    int plan_index;          /* index into the server's plans (grid class)       */
    const double* rho_dev;   /* device, [N_r][N_theta][N_phi] of that plan        */
    double* phi_dev;         /* device, same shape, written                       */
    double G;
    long long request_id;    /* caller's tag, echoed in the completion            */
    void* ready_event;       /* hipEvent_t recorded by the caller after the work
                                that writes rho (on any stream); the solve's slot
                                stream waits for it.  NULL: rho is already
                                complete on the device at submission.  The event
                                must stay valid until the completion is polled. */
    int precision;           /* SPP_FP64 (spp_solve) or SPP_MIXED_FP32
                                (spp_solve_mixed with the FP64 fallback)         */
    int n_refine;            /* refinement steps of a mixed request (0..16)      */
} spp_request;

/* Completion record; times in seconds on the server's steady clock. */
typedef struct {
    long long request_id;
    int plan_index;
    double t_arrival;        /* submission time or scheduled arrival, whichever is later */
    double t_admit;          /* admitted: memory and a stream slot were free      */
    double t_done;           /* completion observed by the scheduler              */
    int status;              /* SPP_OK or the failure                             */
} spp_completion;

/*
 * Create a grid from cell interfaces (Sec. 3.1: r_{i+-1/2}, theta_{j+-1/2},
 * and a uniform phi spacing 2 pi / N_phi).
 *   nr     >= 2 radial cells; r_if (host, nr+1 doubles) strictly increasing,
 *          r_if[0] >= 0;
 *   nth    >= 2 theta cells; th_if (host, nth+1 doubles) strictly increasing
 *          from 0 to pi (checked to 1e-12, then snapped to exactly 0 and pi);
 *          the cells need not be uniform (the separation of variables does not
 *          require it, Sec. 3.1);
 *   nphi   uniform phi cells; the GPU path needs a power of two in [4, 2048]
 *          (SPP_ENOTSUP otherwise);
 *   inner  the inner radial face condition (spp_inner_bc).
 * The interface arrays are copied. *out receives the new grid.
 * Errors: SPP_EINVAL for the conditions above, an unknown `inner` or NULL
 * pointers.
 */
spp_status spp_grid_create(int nr, const double* r_if, int nth, const double* th_if,
                           int nphi, spp_inner_bc inner, spp_grid* out);
void spp_grid_destroy(spp_grid g);

/*
 * Set-up of Sec. 3.2, done once per grid on the host in float64: geometric
 * factors (V_i, R_i, the face coefficients), lambda_{phi,m} for
 * m = 0..N_phi/2, and for each m the eigenvalues lambda_{Omega,l,m} and the
 * eigenvectors H_{l,m}(j) of the theta operator, orthonormal in the
 * dmu-weighted inner product (so H^-1 = H^T diag(dmu)), by an implicit QL
 * iteration on the symmetrised tridiagonal matrix.  Also the outer-boundary
 * coefficients of every (l, m).  The grid may be destroyed afterwards.
 * Errors: SPP_EINVAL (NULL), SPP_ENOMEM, SPP_ENOTSUP (nphi not a power of two
 * in [4, 2048]), SPP_EDEVICE (eigen iteration failed to converge).
 */
spp_status spp_plan_create(spp_grid g, spp_plan* out);
void spp_plan_destroy(spp_plan p);

/*
 * Device memory the caller must provide:
 *   *plan_bytes       one buffer per plan, written by spp_plan_upload and
 *                     read-only afterwards (eigenvector matrices, tables);
 *   *workspace_bytes  scratch for one solve in flight; concurrent solves on
 *                     different streams need separate workspaces.  Its first
 *                     256 bytes hold the status record of the last solve
 *                     enqueued on it (spp_solve_status).
 * Both are multiples of 256 bytes; buffers must be 256-byte aligned.
 */
spp_status spp_plan_device_bytes(spp_plan p, size_t* plan_bytes, size_t* workspace_bytes);

/*
 * Copy the plan's tables into caller-owned device memory plan_dev (at least
 * plan_bytes) on `stream`.  The host copy stays alive until the stream has
 * executed the copy (the call synchronises the stream before returning).
 * The plan remembers plan_dev; uploading again replaces it.
 * Errors: SPP_EINVAL (NULL, misaligned), SPP_EDEVICE.
 */
spp_status spp_plan_upload(spp_plan p, void* plan_dev, void* stream);

/*
 * Enqueue one FP64 solve Phi = L^-1 (4 pi G rho) on `stream` (Sec. 3.2):
 *   rho_dev  device, [N_r][N_theta][N_phi] float64, read-only;
 *   phi_dev  device, same shape, written (may not alias rho_dev);
 *   G        the gravitational constant in the caller's units;
 *   workspace_dev  device scratch of workspace_bytes (256-byte aligned).
 * Errors (synchronous, nothing enqueued): SPP_EINVAL (NULL/misaligned/alias),
 * SPP_ESTATE (plan not uploaded), SPP_EDEVICE (launch failure).  A non-finite
 * value of Phi (from a NaN or infinity in rho, or an overflow) is recorded on
 * the device and reported by spp_solve_status.
 */
spp_status spp_solve(spp_plan p, const double* rho_dev, double* phi_dev, double G,
                     void* workspace_dev, void* stream);

/*
 * Outcome of the last solve enqueued on `workspace_dev` (spp_solve,
 * spp_solve_mixed; spp_solve_noalloc with workspace_dev NULL): synchronises
 * `stream`, then reads the status record the solve's kernels wrote into the
 * workspace's first 256 bytes (the scratch of spp_solve_noalloc when
 * workspace_dev is NULL).
 *   info  host, may be NULL; receives the record (spp_solve_info).
 * Returns SPP_ENONFINITE if Phi holds a NaN or an infinity, SPP_ENOCONV if a
 * refinement step of the mixed form did not contract and its FP64 fallback
 * was disabled (Phi is then the unconverged mixed result), otherwise SPP_OK
 * (also when the fallback replaced the result: info->fell_back_fp64 = 1).
 * Errors: SPP_EINVAL (NULL plan), SPP_EDEVICE (synchronisation or copy).
 */
spp_status spp_solve_status(spp_plan p, const void* workspace_dev, void* stream, spp_solve_info* info);

/*
 * The FP64 residual of Phi, enqueued on `stream`:
 *   r = 4 pi G rho - L Phi,
 * L the discrete operator of Sec. 3.1 (the local flux stencil, divided by the
 * cell volume) with the outer boundary face of Sec. 3.2 (and the inner face of
 * the grid's inner condition) applied per angular eigenmode of the outermost
 * (innermost) shell.  For Phi from spp_solve, |r| is at rounding level of
 * |L||Phi| + |4 pi G rho| componentwise.
 *   rho_dev, phi_dev  device, [N_r][N_theta][N_phi] float64, read-only;
 *   r_dev             device, same shape, written (disjoint from both);
 *   workspace_dev     any FP64 workspace of the plan (256-byte aligned); the
 *                     call uses four shells of N_theta N_phi doubles after its
 *                     status record, which it leaves alone.
 * Errors (synchronous, nothing enqueued): SPP_EINVAL (NULL, misaligned,
 * overlap), SPP_ESTATE (plan not uploaded), SPP_ENOTSUP (N_theta > 3840),
 * SPP_EDEVICE (launch failure).
 */
spp_status spp_residual(spp_plan p, const double* rho_dev, const double* phi_dev, double G, double* r_dev,
                        void* workspace_dev, void* stream);

/*
 * spp_solve without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  The same kernels and result as spp_solve; the
 * workspace is the library's own device scratch of SPP_NOALLOC_SCRATCH_BYTES
 * (160 MiB), one copy per device, held by every device the library runs on
 * until the process ends.  The call allocates nothing (no hipMalloc, no
 * allocating library routine) and clears nothing: a solve writes its whole
 * workspace before reading it.  Every call on one device uses that device's
 * one scratch: calls that overlap on a device (several streams or threads)
 * race and must be serialised by the caller (one stream, or events).
 * Limit: the plan's current path must need at most SPP_NOALLOC_SCRATCH_BYTES
 * of workspace -- the fused path one field of N_r N_theta N_phi doubles plus
 * 6 KB (the 550 x 128 x 256 grid: 137.5 MiB), the staged path two fields.
 * Arguments as spp_solve.  Errors: as spp_solve; SPP_ENOTSUP when the plan
 * needs more scratch; SPP_EDEVICE when the scratch address cannot be found.
 */
#define SPP_NOALLOC_SCRATCH_BYTES ((size_t)160 << 20)
spp_status spp_solve_noalloc(spp_plan p, const double* rho_dev, double* phi_dev, double G, void* stream);

/*
 * Face fluxes of grad Phi through every cell face, enqueued on `stream`
 * (Sec. 3.1: the operator is a finite-volume divergence, (Delta Phi) delta V =
 * the sum over a cell's six faces of area x difference quotient; Sec. 3.2 for
 * the outer boundary face).  For Phi from spp_solve the six fluxes of every
 * cell add up to 4 pi G rho delta V to rounding (Gauss's law on the grid):
 * what a hydrodynamics code builds conservative gravity terms for its
 * momentum and energy equations from (Sec. 1, Sec. 3.1).  Each flux is signed along its
 * increasing coordinate:
 *   fr_dev[i][j][k]  face i+1/2:  r_{i+1/2}^2 dmu_j dphi (Phi_{i+1} - Phi_i)/(r_{i+1} - r_i);
 *                    i = N_r - 1 is the outer boundary face, dmu_j dphi times
 *                    the extrapolated derivative of the asymptotic condition,
 *                    applied per (l, m) mode of the outermost shell;
 *   ft_dev[i][j][k]  face j+1/2:  (r_{i+1/2}^2 - r_{i-1/2}^2)/2 sin th_{j+1/2} dphi
 *                    (Phi_{j+1} - Phi_j)/(r_i (th_{j+1} - th_j)); 0 at j = N_theta - 1 (pole);
 *   fp_dev[i][j][k]  face k+1/2:  (r_{i+1/2}^2 - r_{i-1/2}^2)/2 (th_{j+1/2} - th_{j-1/2})
 *                    (Phi_{k+1} - Phi_k)/(r_i sin th_j dphi); k + 1 wraps to 0;
 * with dmu_j = cos th_{j-1/2} - cos th_{j+1/2}, dphi = 2 pi / N_phi and cell
 * centres at interface midpoints.  The faces r = 0 and theta = 0 have zero
 * area and are not stored.
 *   phi_dev        device, [N_r][N_theta][N_phi] float64, read-only;
 *   fr/ft/fp_dev   device, same shape each, written;
 *   workspace_dev  device scratch of the plan's workspace_bytes (256-byte aligned).
 * All four fields 16-byte aligned, pairwise disjoint and disjoint from the
 * workspace.  The call reads the plan's uploaded tables and allocates nothing.
 * Errors (synchronous, nothing enqueued): SPP_EINVAL (NULL, misaligned,
 * overlap), SPP_ESTATE (plan not uploaded), SPP_ENOTSUP (N_theta > 3840),
 * SPP_EDEVICE (launch failure).
 */
spp_status spp_face_fluxes(spp_plan p, const double* phi_dev, double* fr_dev, double* ft_dev, double* fp_dev,
                           void* workspace_dev, void* stream);

/*
 * Momentum-conserving gravitational source term from Phi, enqueued on
 * `stream`: the force on every cell, -integral of rho grad Phi over it, as the
 * surface integral of the gravitational stress tensor
 *   T = (grad Phi grad Phi - |grad Phi|^2 I / 2) / (4 pi G),  div T = rho grad Phi
 * (a textbook identity, valid where Laplacian Phi = 4 pi G rho, which the
 * solver's Phi satisfies in the flux form of Sec. 3.1 to rounding; the paper
 * points to conservative source terms in Sec. 1 and Sec. 6 without giving
 * one).  On each face the normal gradient is the flux form's difference
 * quotient (outer face: the extrapolated derivative of Sec. 3.2), each
 * tangential component the mean of the two adjacent cells' centred ones; the
 * stress vector uses the exact integrals of the local unit vectors over the
 * curved face.  Every face's vector is the same in both cells that share it,
 * so interior faces cancel exactly: the grid's total momentum changes only
 * through its outer boundary, and a spherically symmetric Phi gives zero net
 * force (both to rounding).
 *   phi_dev        device, [N_r][N_theta][N_phi] float64, read-only;
 *   G              the gravitational constant (finite, non-zero);
 *   fx/fy/fz_dev   device, same shape each, written: the Cartesian components
 *                  (x along phi = 0 at theta = pi/2, z along theta = 0) of
 *                  the force on the cell; divide by the cell volume for a
 *                  force density;
 *   workspace_dev  any FP64 workspace of the plan (two shells after its status
 *                  record are used).
 * Fields pairwise disjoint and disjoint from the workspace.  Errors
 * (synchronous, nothing enqueued): SPP_EINVAL (NULL, misaligned, overlap,
 * G), SPP_ESTATE (plan not uploaded), SPP_ENOTSUP (N_theta > 3840, or the
 * regular inner condition with r_{1/2} > 0), SPP_EDEVICE (launch failure).
 */
spp_status spp_momentum_source(spp_plan p, const double* phi_dev, double G, double* fx_dev, double* fy_dev,
                               double* fz_dev, void* workspace_dev, void* stream);

/*
 * Workspace bytes of one solve in flight for a given precision (SPP_FP64: as
 * spp_plan_device_bytes; SPP_MIXED_FP32: the status record, four fields, two
 * shells and the residual maxima, at least the FP64 fallback's workspace).
 * Errors: SPP_EINVAL (NULL), SPP_ENOTSUP (precision not built).
 */
spp_status spp_plan_workspace_bytes(spp_plan p, spp_precision prec, size_t* bytes);

/*
 * Mixed-precision solve with iterative refinement (the production
 * form; the operator and its exact solution are those of spp_solve).
 *   s~ = FFT(4 pi G rho) in FP64, once;
 *   g  = H F^-1 H^-1 s~ with the theta projections (Sec. 3.2) as FP32 MFMA
 *        products (FP32-rounded eigenvector matrices, FP32 accumulation) and
 *        the radial solves in FP64;
 *   n_refine times: r = s~ - L g with L the FP64 discrete Laplacian of each
 *        Fourier component (local flux stencil of Sec. 3.1 plus the outer
 *        boundary term of Sec. 3.2), then g += H F^-1 H^-1 r as above;
 *   Phi = inverse FFT of g in FP64;
 * then a contraction check on the device: every refinement step must have
 * max|r_k| <= max|r_k-1| / 2 (r_0 = s~).  If one does not and fallback_fp64 is
 * non-zero, the FP64 solve (spp_solve's kernels, enqueued behind and gated on
 * the device) replaces Phi; spp_solve_status reports which happened.
 * Each FP32 pass has a relative error near 1e-7; one refinement brings the
 * result to the FP64 solution within ~1e-12 on the workloads tested.
 *   prec           SPP_MIXED_FP32 (SPP_FP64 runs spp_solve);
 *   n_refine       0..16 refinement steps;
 *   fallback_fp64  non-zero: the FP64 solve replaces a result whose
 *                  refinement did not contract;
 *   workspace_dev  spp_plan_workspace_bytes(p, prec) bytes, 256-byte aligned;
 * other arguments as spp_solve.  Needs N_theta <= 128 (SPP_ENOTSUP otherwise).
 * Errors: as spp_solve, plus SPP_EINVAL for n_refine out of range and
 * SPP_ENOTSUP for an unsupported precision.
 */
spp_status spp_solve_mixed(spp_plan p, spp_precision prec, int n_refine, int fallback_fp64, const double* rho_dev,
                           double* phi_dev, double G, void* workspace_dev, void* stream);

/*
 * For tests of the refinement's failure handling: multiply the host copies of
 * the low-precision eigenvector images the mixed form uses by `factor` (the
 * FP64 tables are untouched); takes effect at the next spp_plan_upload.  A
 * factor c makes each low-precision pass return about c^2 times its
 * correction, so that the refinement diverges for c^2 > 2.
 * Errors: SPP_EINVAL (NULL plan, non-finite factor).
 */
spp_status spp_plan_scale_lowprec_basis(spp_plan p, double factor);

/*
 * spp_solve with per-stage timing, for benchmarks and profiling.  Records
 * HIP events on `stream` before the first and after each of the five stages
 *   0 forward real FFT along phi (with s = 4 pi G rho)
 *   1 forward theta projection (MFMA GEMM per Fourier component)
 *   2 radial tridiagonal solves with the outer boundary condition
 *   3 inverse theta projection (MFMA GEMM)
 *   4 inverse real FFT along phi
 * then waits for the last event and writes the stage durations in
 * milliseconds to stage_ms (host, 5 doubles).  On the fused path stage 1
 * is the per-mode kernel (both projections and the radial solves) and
 * stages 2 and 3 are empty.  Blocks the calling thread.
 * Errors: as spp_solve, plus SPP_EINVAL for stage_ms == NULL.
 */
spp_status spp_solve_profiled(spp_plan p, const double* rho_dev, double* phi_dev, double G,
                              void* workspace_dev, void* stream, double* stage_ms);

/*
 * Projection tile autotuner.  Times each candidate row tile of the FP64
 * projection kernel on this plan's shape (N_theta, N_r), using workspace_dev
 * (spp_plan_device_bytes) as scratch, and records the fastest; later solves
 * of any plan with the same (N_theta, N_r) in this process use it.
 * Synchronises `stream`.  *chosen_rows (may be NULL) receives the rows per
 * wave tile.  Errors: SPP_EINVAL, SPP_ESTATE (not uploaded), SPP_EDEVICE.
 */
spp_status spp_autotune_projection(spp_plan p, void* workspace_dev, void* stream, int* chosen_rows);

/*
 * Batched solves: many right-hand sides on grids of uneven size (plans may be
 * shared between entries).  Solve r is exactly spp_solve(plans[r], rho_dev[r],
 * phi_dev[r], G[r], ...) -- or spp_solve_mixed with n_refine and the FP64
 * fallback for prec = SPP_MIXED_FP32 -- in arithmetic, so each result is
 * bitwise the one of a lone solve.  For FP64 the right-hand sides of a grid
 * class on the fused path run batched: each kernel of the solve (folded
 * forward FFT, per-mode kernel, folded inverse FFT) is one launch over all of
 * them (or over each half, as the tuner chooses), so that small grids fill
 * the device; other classes run one solve per right-hand side.  Everything is
 * captured once into one HIP graph with up to 8 concurrent branches.
 *   spp_batch_workspace_bytes: bytes of the one workspace the batch needs;
 *   spp_batch_create: validates every entry, uploads the per-RHS pointer
 *     tables into the workspace (synchronising `stream`), with autotune != 0
 *     times each fused class's launch variants (the per-mode kernel's unit
 *     order: XCD-paired or plain; one launch group or two concurrent halves)
 *     on the real inputs, writing phi, and keeps the fastest; then captures
 *     the graph.  Device pointers are fixed at creation; the host arrays are
 *     copied; device buffers must outlive the batch;
 *   spp_batch_launch: replays the graph on `stream` (asynchronous);
 *   spp_batch_describe: the classes and the tuner's choices and timings, as
 *     text (buf of len bytes, NUL-terminated; *needed may be NULL);
 *   spp_batch_status: spp_solve_status of entry r (synchronises `stream`);
 *   spp_solve_batched: create (no tuning) + launch + synchronise + destroy.
 * Errors: SPP_EINVAL (bad sizes/pointers/alignment, overlapping rho/phi),
 * SPP_ENOTSUP (precision), SPP_ESTATE (plan not uploaded), SPP_EDEVICE
 * (stream/graph calls).
 */
spp_status spp_batch_workspace_bytes(int n, const spp_plan* plans, spp_precision prec, size_t* bytes);
spp_status spp_batch_create(int n, const spp_plan* plans, const double* const* rho_dev, double* const* phi_dev,
                            const double* G, spp_precision prec, int n_refine, int autotune, void* workspace_dev,
                            void* stream, spp_batch* out);
spp_status spp_batch_launch(spp_batch b, void* stream);
spp_status spp_batch_describe(spp_batch b, char* buf, size_t len, size_t* needed);
spp_status spp_batch_status(spp_batch b, int r, void* stream, spp_solve_info* info);
void spp_batch_destroy(spp_batch b);
spp_status spp_solve_batched(int n, const spp_plan* plans, const double* const* rho_dev, double* const* phi_dev,
                             const double* G, spp_precision prec, int n_refine, void* workspace_dev, void* stream);

/*
 * Serving loop with continuous batching (FP64 and mixed-precision solves).
 *   spp_server_create: plans[0..n_plans) are the resident grid classes
 *     (uploaded; their eigenbases stay on the device); pool_dev/pool_bytes is
 *     caller-owned device memory from which each admitted request takes its
 *     workspace (HBM-footprint admission); n_slots (1..64) streams run
 *     admitted solves concurrently.  Starts one scheduler thread.
 *   spp_server_submit: thread-safe; queues *req to arrive at max(now,
 *     not_before) (server clock, seconds; pass 0 for "now").  Requests are
 *     admitted in arrival order when a slot is free and their workspace fits
 *     in the pool.  SPP_ENOMEM if one request exceeds the whole pool.
 *   spp_server_poll: moves up to max_out completion records to out (host);
 *     *n_out receives the count.  Returns SPP_EDEVICE once a solve failed.
 *   spp_server_drain: waits until every submitted request has completed
 *     (SPP_ESTATE after timeout_s seconds).
 *   spp_server_now: current server clock.
 *   spp_server_destroy: drops queued requests, waits for running ones.
 * Each request runs exactly the kernels of spp_solve (or of spp_solve_mixed
 * for a mixed request, whose workspace is the larger one of
 * spp_plan_workspace_bytes), so its result is bitwise the same alone and in
 * any mix.  rho/phi buffers must stay valid
 * until the request's completion has been polled.  The slot streams do not
 * wait on the caller's streams: rho must be complete at submission, or the
 * request names a ready_event to wait for.
 */
spp_status spp_server_create(int n_plans, const spp_plan* plans, void* pool_dev, size_t pool_bytes, int n_slots,
                             spp_server* out);
spp_status spp_server_submit(spp_server s, const spp_request* req, double not_before);
spp_status spp_server_poll(spp_server s, spp_completion* out, int max_out, int* n_out);
spp_status spp_server_drain(spp_server s, double timeout_s);
spp_status spp_server_now(spp_server s, double* t);
void spp_server_destroy(spp_server s);

/*
 * Host copy of the theta eigensystem of mode m (0 <= m <= N_phi/2), for tests:
 *   H    host, N_theta*N_theta doubles, H[j*N_theta + l] = H_{l,m}(j);
 *   lam  host, N_theta doubles, lambda_{Omega,l,m}: in ascending order, or,
 *        on theta grids symmetric about the equator (even N_theta), the
 *        N_theta/2 even modes in ascending order followed by the odd ones.
 * Errors: SPP_EINVAL.
 */
spp_status spp_theta_eigensystem(spp_plan p, int m, double* H, double* lam);

/*
 * *on = 1 if the FP64 solves of this plan use the parity-split projection
 * (Sec. 4.2: theta grid symmetric about the equator, even N_theta <= 128;
 * two (N_theta/2)^2 products per Fourier component instead of one
 * N_theta^2 product), else 0.  Errors: SPP_EINVAL.
 */
spp_status spp_plan_parity_split(spp_plan p, int* on);

/*
 * Kernel path of the FP64 solves of a plan (spp_solve, spp_solve_profiled,
 * batches and servers created afterwards).  The fused path applies to
 * equator-symmetric theta grids (Sec. 4.2) with N_theta % 4 == 0,
 * N_theta <= 128 and N_r <= 576 whose radial systems keep the products of
 * pivots over the kernel's chunks of rows within 2^+-300 for every
 * eigenvalue (the plan checks this bound; only extreme grids fail it, e.g.
 * polar cells of 1e-6 rad): the forward FFT stores the even and odd
 * theta folds s_j +- s_{N-1-j}; one kernel per (Fourier component, parity)
 * then runs the forward projection, the radial solves of Sec. 3.2 and the
 * inverse projection with its N_r x N_theta/2 slab held on chip; the
 * inverse FFT unfolds.  Both paths solve the same discrete system (results
 * agree to rounding).  The default is SPP_PATH_AUTO.  Not to be changed
 * while solves of the plan are being enqueued on other threads.
 * Errors: SPP_EINVAL (NULL, unknown path), SPP_ENOTSUP (SPP_PATH_FUSED for a
 * grid it does not cover).
 *   spp_plan_get_path: the path solves take now (SPP_PATH_STAGED or
 *   SPP_PATH_FUSED).
 */
spp_status spp_plan_set_path(spp_plan p, spp_path path);
spp_status spp_plan_get_path(spp_plan p, spp_path* path);

/*
 * Names of the kernels one FP64 solve of this plan launches, in launch order,
 * separated by semicolons (e.g. "k_rfft_fwd<256,fold>;modal::k_modal<4,3>;..."), for
 * tests and diagnostics; they follow the current path (spp_plan_set_path).
 *   buf     host, len bytes; receives the NUL-terminated list, truncated to
 *           len - 1 characters (buf may be NULL when len == 0);
 *   needed  host, may be NULL; receives the length including the NUL.
 * Errors: SPP_EINVAL (NULL plan).
 */
spp_status spp_plan_kernels(spp_plan p, char* buf, size_t len, size_t* needed);

/* Grid sizes of a plan (any pointer may be NULL). */
spp_status spp_plan_shape(spp_plan p, int* nr, int* nth, int* nphi);

/* Message of the last non-OK status on this thread ("" if none). */
const char* spp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPHPOISSON_H */
