// Host side of the library: grid validation, the set-up of Sec. 3.2 (geometry,
// per-m theta eigensystems, radial and boundary tables) in float64, the device
// layout of the plan, and the C ABI entry points other than the solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>

#include "internal.h"
#include "modal_layout.h"
#include "proj_layout.h"

static thread_local std::string g_last_error;

spp_status spp_fail(spp_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

extern "C" const char* spp_last_error(void) { return g_last_error.c_str(); }

static bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// ---------------------------------------------------------------- grid
extern "C" spp_status spp_grid_create(int nr, const double* r_if, int nth, const double* th_if,
                                      int nphi, spp_inner_bc inner, spp_grid* out)
{
    if (!out || !r_if || !th_if) return spp_fail(SPP_EINVAL, "spp_grid_create: NULL pointer");
    *out = nullptr;
    if (inner != SPP_INNER_AUTO && inner != SPP_INNER_ZERO_FLUX && inner != SPP_INNER_REGULAR)
        return spp_fail(SPP_EINVAL, "spp_grid_create: unknown inner boundary condition");
    if (nr < 2 || nth < 2 || nphi < 2)
        return spp_fail(SPP_EINVAL, "spp_grid_create: need nr >= 2, nth >= 2, nphi >= 2");
    if (!(r_if[0] >= 0.0)) return spp_fail(SPP_EINVAL, "spp_grid_create: r_if[0] must be >= 0");
    for (int i = 0; i < nr; ++i)
        if (!(r_if[i + 1] > r_if[i]) || !std::isfinite(r_if[i + 1]))
            return spp_fail(SPP_EINVAL, "spp_grid_create: r interfaces must increase strictly");
    for (int j = 0; j < nth; ++j)
        if (!(th_if[j + 1] > th_if[j]))
            return spp_fail(SPP_EINVAL, "spp_grid_create: theta interfaces must increase strictly");
    if (std::fabs(th_if[0]) > 1e-12 || std::fabs(th_if[nth] - M_PI) > 1e-12)
        return spp_fail(SPP_EINVAL, "spp_grid_create: theta interfaces must span [0, pi]");
    auto* g = new (std::nothrow) spp_grid_s;
    if (!g) return spp_fail(SPP_ENOMEM, "spp_grid_create: out of host memory");
    g->nr = nr;
    g->nth = nth;
    g->nphi = nphi;
    g->inner = inner;
    g->r_if.assign(r_if, r_if + nr + 1);
    g->th_if.assign(th_if, th_if + nth + 1);
    g->th_if.front() = 0.0;
    g->th_if.back() = M_PI;
    *out = g;
    return SPP_OK;
}

extern "C" void spp_grid_destroy(spp_grid g) { delete g; }

// ---------------------------------------------------------------- plan
namespace {

struct Geometry {
    std::vector<double> r, V, VR, alpha;          // radial
    std::vector<double> th, dmu, dth, sigma;      // theta (sigma has nth+1 faces)
};

Geometry make_geometry(const spp_grid_s& g)
{
    Geometry G;
    const int nr = g.nr, nth = g.nth;
    G.r.resize(nr);
    G.V.resize(nr);
    G.VR.resize(nr);
    G.alpha.assign(nr, 0.0);
    for (int i = 0; i < nr; ++i) {
        const double a = g.r_if[i], b = g.r_if[i + 1];
        G.r[i] = 0.5 * (a + b);
        // (b^3 - a^3)/3 and (b^2 - a^2)/2 in factored form (no cancellation)
        G.V[i] = (b - a) * (b * b + a * b + a * a) / 3.0;
        // V_i R_i = (r_{i+1/2}^2 - r_{i-1/2}^2) / (2 r_i)   (Sec. 3.1, R_i)
        G.VR[i] = (b - a) * (b + a) / (2.0 * G.r[i]);
    }
    // interior radial faces: area / distance with the angular factor removed
    for (int i = 0; i + 1 < nr; ++i) {
        const double f = g.r_if[i + 1];
        G.alpha[i] = f * f / (G.r[i + 1] - G.r[i]);
    }
    G.th.resize(nth);
    G.dmu.resize(nth);
    G.dth.resize(nth);
    G.sigma.assign(nth + 1, 0.0);                 // pole faces have zero area
    for (int j = 0; j < nth; ++j) {
        const double a = g.th_if[j], b = g.th_if[j + 1];
        G.th[j] = 0.5 * (a + b);
        G.dth[j] = b - a;
        // cos a - cos b = 2 sin((a+b)/2) sin((b-a)/2)
        G.dmu[j] = 2.0 * std::sin(0.5 * (a + b)) * std::sin(0.5 * (b - a));
    }
    for (int j = 1; j < nth; ++j) G.sigma[j] = std::sin(g.th_if[j]) / (G.th[j] - G.th[j - 1]);
    return G;
}


// The fused kernel's pass 1 works with the continuants of each chunk's
// interior block (determinants of its leading and trailing principal
// submatrices, rows scaled by 2^-e_p) instead of normalised pivots; they are
// the products of the pivots and, unlike the pivots, not of unit size.  This
// bounds their magnitude for every eigenvalue of the plan: from above by
// Hadamard's bound (product of absolute row sums of the scaled block), from
// below by the products of the pivot bounds |w_k| >= a_k (resp. a_{k-1} for
// the trailing ones), which hold because every row has
// -d_k >= a_{k-1} + a_k (lambda <= 0, beta >= 0); on the outermost row, where
// a_k = 0, |w_k| >= beta + V R |lambda| instead.  The chunk geometry and the
// scale follow the kernel: chunks of CH = 4 ceil(N_r / 192) rows, 2^-e_p from
// the middle row's alpha_{i-1} + alpha_i.  Keeping every partial product
// within 2^+-300 leaves the right-hand sides, which the continuants multiply,
// about 2^700 of range.
// Scale 2^-e_p of the chunk of CH rows from s0: the power of two at or below
// alpha_{mid-1} + alpha_mid of its middle row (the diagonal without the
// lambda term), 1 for a chunk whose middle row is padding.
double chunk_scale(const std::vector<double>& alpha, int nr, int s0, int CH)
{
    const int mid = s0 + CH / 2;
    return mid < nr ? std::ldexp(1.0, -std::ilogb(alpha[mid - 1] + alpha[mid])) : 1.0;
}

bool modal_continuants_in_range(const std::vector<double>& alpha, const std::vector<double>& VR,
                                const std::vector<double>& lam, const std::vector<double>& beta, int nr)
{
    const int T = modalimg::t_for(nr), CH = 4 * T, P = 4 * modalimg::NW;
    double lmax = 0.0, bmax = 0.0, bmin = HUGE_VAL;
    for (size_t t = 0; t < lam.size(); ++t) {
        lmax = std::max(lmax, std::fabs(lam[t]));
        bmax = std::max(bmax, beta[t]);
        bmin = std::min(bmin, beta[t] + VR[nr - 1] * std::fabs(lam[t]));
    }
    const double LIM = 300.0;
    for (int p = 0; p < P; ++p) {
        const int s0 = p * CH;
        const double sc = chunk_scale(alpha, nr, s0, CH);
        const int n = CH - 1;
        std::vector<double> up(n + 1), lo_f(n + 1), lo_b(n + 1);
        for (int k = 1; k <= n; ++k) {
            const int i = s0 + k;
            if (i >= nr) {            // padding: identity rows, 2^-e_p on the diagonal
                up[k] = lo_f[k] = lo_b[k] = std::log2(sc);
                continue;
            }
            const double am = alpha[i - 1], a = alpha[i];
            const double din = (am + a) + VR[i] * lmax + (i == nr - 1 ? bmax : 0.0);
            const double rs = din + (k > 1 ? am : 0.0) + (k < n ? a : 0.0);
            up[k] = std::log2(rs * sc);
            lo_f[k] = std::log2(std::max(i == nr - 1 ? bmin : a, 1e-300) * sc);
            lo_b[k] = std::log2(std::max(am, 1e-300) * sc);
        }
        double su = 0.0, sf = 0.0, sb = 0.0, bu = 0.0;
        for (int k = 1; k <= n; ++k) {
            su += up[k];
            sf += lo_f[k];
            if (su > LIM || sf < -LIM) return false;
        }
        for (int k = n; k >= 1; --k) {
            bu += up[k];
            sb += lo_b[k];
            if (bu > LIM || sb < -LIM) return false;
        }
    }
    return true;
}

// The record image of modal_layout.h: per row the diagonal without the lambda
// term x = -(alpha_{i-1} + alpha_i), y = V_i R_i, the outer-row flag z, the
// coupling a = alpha_i to row i+1, a^2 and V_i (rows >= N_r: identity rows);
// every chunk's rows but its first (the separator) multiplied by its scale.
std::vector<double> modal_records(const std::vector<double>& alpha, const std::vector<double>& VR,
                                  const std::vector<double>& V, int nr)
{
    using namespace modalimg;
    const int T = t_for(nr), CH = 4 * T, ROWS = NW * 16 * T, P = 4 * NW;
    std::vector<double> rec(rec_elems(T), 0.0);
    for (int i = 0; i < ROWS; ++i) {
        const bool in = i < nr;
        const double a = in ? alpha[i] : 0.0;
        const double am = (in && i > 0) ? alpha[i - 1] : 0.0;
        const double sc = i % CH == 0 ? 1.0 : chunk_scale(alpha, nr, i - i % CH, CH);
        double* r = &rec[size_t(i + i / CH) * RECD];
        r[0] = (in ? -(am + a) : 1.0) * sc;
        r[1] = (in ? VR[i] : 0.0) * sc;
        r[2] = (i == nr - 1 ? 1.0 : 0.0) * sc;
        r[3] = a * sc;
        r[4] = (a * sc) * (a * sc);
        r[5] = (in ? V[i] : 0.0) * sc;
    }
    for (int p = 0; p < P; ++p) {
        const int s0 = p * CH;
        const double sc = chunk_scale(alpha, nr, s0, CH);
        const double oL = s0 < nr ? alpha[s0] : 0.0;
        const double oR = s0 + CH - 1 < nr ? alpha[s0 + CH - 1] : 0.0;
        double pa = 1.0;
        for (int k = 1; k < CH - 1; ++k) pa *= (s0 + k < nr ? alpha[s0 + k] : 0.0) * sc;
        double* r = &rec[size_t(s0 + p + CH) * RECD];
        r[0] = oL;
        r[1] = oR;
        r[2] = sc;
        r[3] = -oL * oR * pa * sc;
    }
    return rec;
}

}  // namespace

extern "C" spp_status spp_plan_create(spp_grid g, spp_plan* out)
{
    if (!g || !out) return spp_fail(SPP_EINVAL, "spp_plan_create: NULL pointer");
    *out = nullptr;
    if (!is_pow2(g->nphi) || g->nphi < 4 || g->nphi > 2048)
        return spp_fail(SPP_ENOTSUP, "spp_plan_create: the GPU path needs nphi a power of two in [4, 2048]");
    auto* p = new (std::nothrow) spp_plan_s;
    if (!p) return spp_fail(SPP_ENOMEM, "spp_plan_create: out of host memory");
    try {
        const int nr = g->nr, nth = g->nth, nphi = g->nphi, nm = nphi / 2 + 1;
        p->nr = nr;
        p->nth = nth;
        p->nphi = nphi;
        p->nm = nm;
        p->r_if = g->r_if;
        p->th_if = g->th_if;
        const Geometry G = make_geometry(*g);
        p->alpha = G.alpha;
        p->V = G.V;
        p->VR = G.VR;

        // twiddles exp(-2 pi i t / N_phi), evaluated in long double
        p->tw.resize(2 * size_t(nphi));
        const long double two_pi = 6.283185307179586476925286766559005768L;
        for (int t = 0; t < nphi; ++t) {
            const long double a = two_pi * (long double)t / (long double)nphi;
            p->tw[2 * t] = (double)cosl(a);
            p->tw[2 * t + 1] = (double)-sinl(a);
        }

        // per-m theta eigensystems (Sec. 3.2): K H = lambda D H with
        // K_jj = -(sigma_{j-1/2} + sigma_{j+1/2}) + dth_j lambda_phi / sin th_j,
        // K_{j,j+1} = sigma_{j+1/2}, D = diag(dmu), solved through the
        // symmetric matrix D^-1/2 K D^-1/2.
        p->W.assign(size_t(nm) * nth * nth, 0.0);
        p->H.assign(size_t(nm) * nth * nth, 0.0);
        p->lam.assign(size_t(nm) * nth, 0.0);
        p->beta.assign(size_t(nm) * nth, 0.0);
        p->gamma.assign(size_t(nm) * nth, 0.0);
        // regular inner condition (the paper leaves the inner face open; with
        // r_{1/2} = 0 the face has no area and needs no condition)
        const double ri = g->r_if[0], r1 = G.r[0];
        p->inner_regular = g->inner == SPP_INNER_REGULAR && ri > 0.0;
        const double log_in = p->inner_regular ? std::log(ri / r1) : 0.0;
        const double dphi = 2.0 * M_PI / nphi;
        const double ro = g->r_if[nr], rn = G.r[nr - 1];
        const double log_ratio = std::log(ro / rn);
        std::vector<double> isd(nth);
        for (int j = 0; j < nth; ++j) isd[j] = 1.0 / std::sqrt(G.dmu[j]);

        // Equator-symmetric theta grids (Sec. 4.2, parity split): the theta
        // operator commutes with j -> N_theta-1-j, so its eigenvectors are even
        // or odd.  They are computed from the half-size even and odd operators
        // directly (near-degenerate pairs of the full operator may otherwise
        // mix parities): on j < h = N_theta/2 the reflected neighbour of the
        // last cell is the cell itself (+sigma_h for even, -sigma_h for odd).
        // Modes are then ordered even first, then odd.
        bool symmetric = nth % 2 == 0 && nth >= 4;
        for (int j = 0; symmetric && j <= nth; ++j)
            symmetric = std::fabs(g->th_if[j] + g->th_if[nth - j] - M_PI) <= 1e-12 * M_PI;
        const int hh = nth / 2;
        p->parity = symmetric;
        if (symmetric) {
            p->Ue.assign(size_t(nm) * hh * hh, 0.0);
            p->Uo.assign(size_t(nm) * hh * hh, 0.0);
        }

        // No flux crosses the poles (Sec. 3.1), so for m = 0 the theta operator
        // (and the even half-operator of the parity split) has zero row sums:
        // the constant is an exact eigenvector with eigenvalue 0, the largest.
        // It is set exactly -- a computed one is off by about eps |K| / gap,
        // which the large radial response of this mode carries into Phi --
        // and the other eigenvectors are made exactly orthogonal to it.  Here
        // z = D^1/2 h are the eigenvectors of the symmetrised matrix (columns
        // of the row-major n x n array Z), so the null vector is sqrt(dmu_j).
        auto exact_null_pair = [&](int n, std::vector<double>& d, std::vector<double>& Z) {
            int top = 0;
            for (int l = 1; l < n; ++l)
                if (d[l] > d[top]) top = l;
            std::vector<double> c(n);
            double nc = 0.0;
            for (int j = 0; j < n; ++j) nc += G.dmu[j];
            for (int j = 0; j < n; ++j) c[j] = std::sqrt(G.dmu[j] / nc);
            for (int l = 0; l < n; ++l) {
                if (l == top) continue;
                double dot = 0.0, nn = 0.0;
                for (int j = 0; j < n; ++j) dot += c[j] * Z[size_t(j) * n + l];
                for (int j = 0; j < n; ++j) {
                    Z[size_t(j) * n + l] -= dot * c[j];
                    nn += Z[size_t(j) * n + l] * Z[size_t(j) * n + l];
                }
                const double s = 1.0 / std::sqrt(nn);
                for (int j = 0; j < n; ++j) Z[size_t(j) * n + l] *= s;
            }
            for (int j = 0; j < n; ++j) Z[size_t(j) * n + top] = c[j];
            d[top] = 0.0;
        };

        bool ok = true;
        auto set_lam = [&](int m, int l, double lam) {
            p->lam[size_t(m) * nth + l] = lam;
            // outer face: flux / (dmu dphi) = -beta f_N with
            // beta = p r_o (r_o / r_N)^-p, p = (1 + sqrt(1 - 4 lambda))/2
            const double pp = 0.5 * (1.0 + std::sqrt(std::max(0.0, 1.0 - 4.0 * lam)));
            p->beta[size_t(m) * nth + l] = pp * ro * std::exp(-pp * log_ratio);
            // inner face: flux / (dmu dphi) = gamma f_1 with gamma = p' r_i (r_i/r_1)^p',
            // p' = (-1 + sqrt(1 - 4 lambda))/2, the regular interior solution r^p'
            if (p->inner_regular) {
                const double pi = pp - 1.0;
                p->gamma[size_t(m) * nth + l] = pi * ri * std::exp(pi * log_in);
            }
        };
        auto work = [&](int m0, int stride) {
            std::vector<double> d(nth), e(nth > 1 ? nth - 1 : 0), Z;
            for (int m = m0; m < nm; m += stride) {
                const double sm = std::sin(0.5 * m * dphi) / (0.5 * dphi);
                const double lam_phi = -sm * sm;   // eigenvalue of the phi second difference
                double* Hm = &p->H[size_t(m) * nth * nth];
                double* Wm = &p->W[size_t(m) * nth * nth];
                if (symmetric) {
                    const double r2 = std::sqrt(0.5);
                    for (int par = 0; par < 2; ++par) {
                        std::vector<double> dh(hh), eh(hh - 1), Zh;
                        for (int j = 0; j < hh; ++j) {
                            double k = -(G.sigma[j] + G.sigma[j + 1]) + G.dth[j] * lam_phi / std::sin(G.th[j]);
                            if (j == hh - 1) k += par == 0 ? G.sigma[hh] : -G.sigma[hh];
                            dh[j] = k * isd[j] * isd[j];
                        }
                        for (int j = 0; j + 1 < hh; ++j) eh[j] = G.sigma[j + 1] * isd[j] * isd[j + 1];
                        if (!spp_tridiag_eigen(hh, dh, eh, Zh)) { ok = false; return; }
                        if (m == 0 && par == 0) exact_null_pair(hh, dh, Zh);
                        double* U = &(par == 0 ? p->Ue : p->Uo)[size_t(m) * hh * hh];
                        const double sgn = par == 0 ? 1.0 : -1.0;
                        for (int j = 0; j < hh; ++j)
                            for (int l = 0; l < hh; ++l) {
                                const double u = Zh[size_t(j) * hh + l] * isd[j];   // D_h-orthonormal half vector
                                U[size_t(j) * hh + l] = u;
                                const int col = par * hh + l;
                                Hm[size_t(j) * nth + col] = u * r2;
                                Hm[size_t(nth - 1 - j) * nth + col] = sgn * u * r2;
                            }
                        for (int l = 0; l < hh; ++l) set_lam(m, par * hh + l, dh[l]);
                    }
                    for (int j = 0; j < nth; ++j)
                        for (int l = 0; l < nth; ++l) Wm[size_t(l) * nth + j] = Hm[size_t(j) * nth + l] * G.dmu[j];
                    continue;
                }
                for (int j = 0; j < nth; ++j)
                    d[j] = (-(G.sigma[j] + G.sigma[j + 1]) + G.dth[j] * lam_phi / std::sin(G.th[j]))
                           * isd[j] * isd[j];
                for (int j = 0; j + 1 < nth; ++j) e[j] = G.sigma[j + 1] * isd[j] * isd[j + 1];
                if (!spp_tridiag_eigen(nth, d, e, Z)) { ok = false; return; }
                if (m == 0) exact_null_pair(nth, d, Z);
                for (int j = 0; j < nth; ++j)
                    for (int l = 0; l < nth; ++l) {
                        const double h = Z[size_t(j) * nth + l] * isd[j];   // H = D^-1/2 V
                        Hm[size_t(j) * nth + l] = h;
                        Wm[size_t(l) * nth + j] = h * G.dmu[j];            // H^-1 = H^T D
                    }
                for (int l = 0; l < nth; ++l) set_lam(m, l, d[l]);
            }
        };
        const int nthreads = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        for (int t = 1; t < nthreads; ++t) pool.emplace_back(work, t, nthreads);
        work(0, nthreads);
        for (auto& th : pool) th.join();
        if (!ok) {
            delete p;
            return spp_fail(SPP_EDEVICE, "spp_plan_create: theta eigen iteration did not converge");
        }

        // shell operators of the boundary terms (Sec. 3.2): per mode m the
        // outer-face term of a shell's Fourier component g is
        // H diag(beta) H^T D g, and with the regular inner condition the
        // inner-face term is the same with gamma.  Each is one N_theta x
        // N_theta matrix B = H diag(c) W with W = H^T D, stored transposed
        // (row j' holds B[.][j']) for the column kernel that applies it.
        {
            const size_t nn = size_t(nth) * nth;
            p->Bo.assign(size_t(nm) * nn, 0.0);
            if (p->inner_regular) p->Bi.assign(size_t(nm) * nn, 0.0);
            auto shell_ops = [&](int m0, int stride) {
                std::vector<double> Ht(nn);   // H^T, so that the inner loop runs along rows
                for (int m = m0; m < nm; m += stride) {
                    const double* Wm = &p->W[size_t(m) * nn];
                    for (int j = 0; j < nth; ++j)
                        for (int l = 0; l < nth; ++l) Ht[size_t(l) * nth + j] = p->H[size_t(m) * nn + size_t(j) * nth + l];
                    for (int pass = 0; pass < (p->inner_regular ? 2 : 1); ++pass) {
                        const double* c = &(pass == 0 ? p->beta : p->gamma)[size_t(m) * nth];
                        double* B = &(pass == 0 ? p->Bo : p->Bi)[size_t(m) * nn];
                        // B^T[j'][j] = sum_l W[l][j'] c_l H[j][l]
                        for (int jp = 0; jp < nth; ++jp) {
                            double* row = B + size_t(jp) * nth;
                            for (int l = 0; l < nth; ++l) {
                                const double t = Wm[size_t(l) * nth + jp] * c[l];
                                const double* hl = &Ht[size_t(l) * nth];
                                for (int j = 0; j < nth; ++j) row[j] += t * hl[j];
                            }
                        }
                    }
                }
            };
            std::vector<std::thread> ops;
            for (int t = 1; t < nthreads; ++t) ops.emplace_back(shell_ops, t, nthreads);
            shell_ops(0, nthreads);
            for (auto& th : ops) th.join();
        }

        // theta and phi tables of the spectral residual (mixed-precision refinement)
        p->sig = G.sigma;
        p->dmu = G.dmu;
        p->Sj.resize(nth);
        for (int j = 0; j < nth; ++j) p->Sj[j] = G.dth[j] / (std::sin(G.th[j]) * G.dmu[j]);
        p->lamphi.resize(nm);
        for (int m = 0; m < nm; ++m) {
            const double sm = std::sin(0.5 * m * dphi) / (0.5 * dphi);
            p->lamphi[m] = -sm * sm;
        }

        // momentum source: the factors of the exact face integrals of the
        // local unit vectors and of the face difference quotients
        {
            const spp_mom_layout M(nr, nth, nphi);
            p->mom.assign(M.total, 0.0);
            double* q = p->mom.data();
            for (int i = 0; i <= nr; ++i) q[M.R2 + i] = g->r_if[i] * g->r_if[i];
            for (int i = 0; i < nr; ++i) {
                q[M.ring + i] = 0.5 * (g->r_if[i + 1] * g->r_if[i + 1] - g->r_if[i] * g->r_if[i]);
                q[M.invr + i] = 1.0 / G.r[i];
            }
            for (int i = 1; i < nr; ++i) q[M.invdr + i] = 1.0 / (G.r[i] - G.r[i - 1]);
            for (int j = 0; j < nth; ++j) {
                const double a = g->th_if[j], b = g->th_if[j + 1];
                q[M.is2 + j] = 0.5 * (b - a) - 0.25 * (std::sin(2 * b) - std::sin(2 * a));
                q[M.isc + j] = 0.5 * (std::sin(b) * std::sin(b) - std::sin(a) * std::sin(a));
                q[M.is + j] = std::cos(a) - std::cos(b);
                q[M.ic + j] = std::sin(b) - std::sin(a);
                q[M.dth + j] = b - a;
                q[M.invsdp + j] = 1.0 / (std::sin(G.th[j]) * dphi);
            }
            for (int j = 1; j < nth; ++j) {
                q[M.invdthc + j] = 1.0 / (G.th[j] - G.th[j - 1]);
                q[M.fst + j] = std::sin(g->th_if[j]);
            }
            for (int j = 0; j <= nth; ++j) q[M.fct + j] = std::cos(g->th_if[j]);
            for (int k = 0; k < nphi; ++k) {
                const double c = 2.0 * M_PI * k / nphi, d = 2.0 * M_PI * (k + 1) / nphi;
                q[M.jc + k] = std::sin(d) - std::sin(c);
                q[M.js + k] = std::cos(c) - std::cos(d);
                q[M.cp1 + k] = std::cos(d);
                q[M.sp1 + k] = std::sin(d);
            }
        }

        // LDS images of W_m and H_m for the projection kernel (N_theta <= 128)
        if (nth <= 128) {
            const int rn = projimg::rn_for(nth);
            const size_t ie = projimg::elems(rn);
            const int NP = projimg::np(rn), KG = projimg::kpad(nth) / 4;
            p->proj_rn = rn;
            p->Wimg.assign(size_t(nm) * ie, 0.0);
            p->Himg.assign(size_t(nm) * ie, 0.0);
            for (int m = 0; m < nm; ++m)
                for (int n = 0; n < nth; ++n)
                    for (int k = 0; k < nth; ++k) {
                        const size_t dst = size_t(m) * ie + size_t(projimg::row_of(k, KG)) * NP + n;
                        p->Wimg[dst] = p->W[(size_t(m) * nth + n) * nth + k];
                        p->Himg[dst] = p->H[(size_t(m) * nth + n) * nth + k];
                    }
            p->Wimg32.assign(p->Wimg.begin(), p->Wimg.end());
            p->Himg32.assign(p->Himg.begin(), p->Himg.end());
        }

        // LDS images of the half-size even/odd matrices for the parity-split
        // projection kernel ([m][parity][KMAX][NP], K = h <= 64):
        //   forward  B_p[l][j] = U_p[j][l] dmu_j / sqrt 2   (applied to s_j +- s_{N-1-j})
        //   inverse  B_p[j][l] = U_p[j][l] / sqrt 2         (g_j, g_{N-1-j} = G_e +- G_o)
        if (symmetric && hh <= 64) {
            const int rn = projimg::rn_for(hh);
            const size_t ie = projimg::elems(rn);
            const int NP = projimg::np(rn), KG = projimg::kpad(hh) / 4;
            const double r2 = std::sqrt(0.5);
            p->par_rn = rn;
            p->Wpar.assign(size_t(nm) * 2 * ie, 0.0);
            p->Hpar.assign(size_t(nm) * 2 * ie, 0.0);
            for (int m = 0; m < nm; ++m)
                for (int par = 0; par < 2; ++par) {
                    const double* U = &(par == 0 ? p->Ue : p->Uo)[size_t(m) * hh * hh];
                    const size_t base = (size_t(m) * 2 + par) * ie;
                    for (int n = 0; n < hh; ++n)
                        for (int k = 0; k < hh; ++k) {
                            const size_t dst = base + size_t(projimg::row_of(k, KG)) * NP + n;
                            p->Wpar[dst] = U[size_t(k) * hh + n] * G.dmu[k] * r2;   // n = l, k = j
                            p->Hpar[dst] = U[size_t(n) * hh + k] * r2;              // n = j, k = l
                        }
                }
        }

        // LDS images of the fused per-mode kernel ([m][parity][KP][NP], rows in
        // the interleaved k order of modal_layout.h):
        //   forward  B_p[k = j][n = l] = U_p[j][l] dmu_j / sqrt 2
        //   inverse  B_p[k = l][n = j] = U_p[j][l] / sqrt 2
        // the fused kernel's row records have no inner-face term: grids with the
        // regular inner condition take the staged kernels
        p->fused_ok = symmetric && hh % 2 == 0 && hh <= 64 && nr <= modalimg::NRMAX && !p->inner_regular &&
                      modal_continuants_in_range(p->alpha, p->VR, p->lam, p->beta, nr);
        if (p->fused_ok) {
            const int rn = modalimg::rn_for(hh);
            const size_t ie = modalimg::elems(rn);
            const int NP = modalimg::np(rn);
            const double r2 = std::sqrt(0.5);
            p->Rimg = modal_records(p->alpha, p->VR, p->V, nr);
            p->Fimg.assign(size_t(nm) * 2 * ie, 0.0);
            p->Iimg.assign(size_t(nm) * 2 * ie, 0.0);
            for (int m = 0; m < nm; ++m)
                for (int par = 0; par < 2; ++par) {
                    const double* U = &(par == 0 ? p->Ue : p->Uo)[size_t(m) * hh * hh];
                    const size_t base = (size_t(m) * 2 + par) * ie;
                    for (int k = 0; k < hh; ++k)
                        for (int n = 0; n < hh; ++n) {
                            const size_t dst = base + size_t(modalimg::row_of(k)) * NP + n;
                            p->Fimg[dst] = U[size_t(k) * hh + n] * G.dmu[k] * r2;
                            p->Iimg[dst] = U[size_t(n) * hh + k] * r2;
                        }
                }
        }

        // device layout
        spp_plan_layout& L = p->lay;
        size_t off = 0;
        auto take = [&](size_t n_doubles) {
            const size_t o = off;
            off = spp_align256(off + n_doubles * sizeof(double));
            return o;
        };
        auto take_f = [&](size_t n_floats) {
            const size_t o = off;
            off = spp_align256(off + n_floats * sizeof(float));
            return o;
        };
        L.tw = take(p->tw.size());
        L.W = take(p->W.size());
        L.H = take(p->H.size());
        L.lam = take(p->lam.size());
        L.beta = take(p->beta.size());
        L.gamma = take(p->gamma.size());
        L.alpha = take(p->alpha.size());
        L.V = take(p->V.size());
        L.VR = take(p->VR.size());
        L.Wimg = take(p->Wimg.size());
        L.Himg = take(p->Himg.size());
        L.Wimg32 = take_f(p->Wimg32.size());
        L.Himg32 = take_f(p->Himg32.size());
        L.Wpar = take(p->Wpar.size());
        L.Hpar = take(p->Hpar.size());
        L.Fimg = take(p->Fimg.size());
        L.Iimg = take(p->Iimg.size());
        L.Rimg = take(p->Rimg.size());
        L.sig = take(p->sig.size());
        L.dmu = take(p->dmu.size());
        L.Sj = take(p->Sj.size());
        L.lamphi = take(p->lamphi.size());
        L.mom = take(p->mom.size());
        L.Bo = take(p->Bo.size());
        L.Bi = take(p->Bi.size());
        L.total = off;
        // the larger of what either path needs (spp_plan_set_path may switch
        // paths after the caller has sized its workspace)
        p->workspace_bytes = std::max(spp_path_workspace_bytes(p, true), spp_path_workspace_bytes(p, false));
    } catch (const std::bad_alloc&) {
        delete p;
        return spp_fail(SPP_ENOMEM, "spp_plan_create: out of host memory");
    }
    *out = p;
    return SPP_OK;
}

extern "C" void spp_plan_destroy(spp_plan p) { delete p; }

extern "C" spp_status spp_plan_device_bytes(spp_plan p, size_t* plan_bytes, size_t* workspace_bytes)
{
    if (!p) return spp_fail(SPP_EINVAL, "spp_plan_device_bytes: NULL plan");
    if (plan_bytes) *plan_bytes = p->lay.total;
    if (workspace_bytes) *workspace_bytes = p->workspace_bytes;
    return SPP_OK;
}

extern "C" spp_status spp_plan_shape(spp_plan p, int* nr, int* nth, int* nphi)
{
    if (!p) return spp_fail(SPP_EINVAL, "spp_plan_shape: NULL plan");
    if (nr) *nr = p->nr;
    if (nth) *nth = p->nth;
    if (nphi) *nphi = p->nphi;
    return SPP_OK;
}

extern "C" spp_status spp_plan_set_path(spp_plan p, spp_path path)
{
    if (!p) return spp_fail(SPP_EINVAL, "spp_plan_set_path: NULL plan");
    if (path != SPP_PATH_AUTO && path != SPP_PATH_STAGED && path != SPP_PATH_FUSED)
        return spp_fail(SPP_EINVAL, "spp_plan_set_path: unknown path");
    if (path == SPP_PATH_FUSED && !p->fused_ok)
        return spp_fail(SPP_ENOTSUP, "spp_plan_set_path: the fused per-mode path needs an equator-symmetric "
                                     "theta grid with N_theta % 4 == 0, N_theta <= 128, N_r <= " +
                                         std::to_string(modalimg::NRMAX) +
                                         " and radial pivot products within its range");
    p->path.store(path);
    return SPP_OK;
}

extern "C" spp_status spp_plan_get_path(spp_plan p, spp_path* path)
{
    if (!p || !path) return spp_fail(SPP_EINVAL, "spp_plan_get_path: NULL pointer");
    *path = spp_plan_fused(p) ? SPP_PATH_FUSED : SPP_PATH_STAGED;
    return SPP_OK;
}

extern "C" spp_status spp_plan_kernels(spp_plan p, char* buf, size_t len, size_t* needed)
{
    if (!p) return spp_fail(SPP_EINVAL, "spp_plan_kernels: NULL plan");
    const std::string d = spp_describe_solve(p);
    if (needed) *needed = d.size() + 1;
    if (buf && len > 0) {
        const size_t n = std::min(len - 1, d.size());
        std::memcpy(buf, d.data(), n);
        buf[n] = '\0';
    }
    return SPP_OK;
}

extern "C" spp_status spp_plan_parity_split(spp_plan p, int* on)
{
    if (!p || !on) return spp_fail(SPP_EINVAL, "spp_plan_parity_split: NULL pointer");
    *on = p->par_rn != 0 ? 1 : 0;
    return SPP_OK;
}

extern "C" spp_status spp_plan_upload(spp_plan p, void* plan_dev, void* stream)
{
    if (!p || !plan_dev) return spp_fail(SPP_EINVAL, "spp_plan_upload: NULL pointer");
    if (reinterpret_cast<uintptr_t>(plan_dev) & 255)
        return spp_fail(SPP_EINVAL, "spp_plan_upload: plan buffer must be 256-byte aligned");
    std::vector<unsigned char> img(p->lay.total, 0);
    auto put = [&](size_t off, const std::vector<double>& v) {
        std::memcpy(img.data() + off, v.data(), v.size() * sizeof(double));
    };
    put(p->lay.tw, p->tw);
    put(p->lay.W, p->W);
    put(p->lay.H, p->H);
    put(p->lay.lam, p->lam);
    put(p->lay.beta, p->beta);
    put(p->lay.gamma, p->gamma);
    put(p->lay.alpha, p->alpha);
    put(p->lay.V, p->V);
    put(p->lay.VR, p->VR);
    put(p->lay.Wimg, p->Wimg);
    put(p->lay.Himg, p->Himg);
    std::memcpy(img.data() + p->lay.Wimg32, p->Wimg32.data(), p->Wimg32.size() * sizeof(float));
    std::memcpy(img.data() + p->lay.Himg32, p->Himg32.data(), p->Himg32.size() * sizeof(float));
    put(p->lay.Wpar, p->Wpar);
    put(p->lay.Hpar, p->Hpar);
    put(p->lay.Fimg, p->Fimg);
    put(p->lay.Iimg, p->Iimg);
    put(p->lay.Rimg, p->Rimg);
    put(p->lay.sig, p->sig);
    put(p->lay.dmu, p->dmu);
    put(p->lay.Sj, p->Sj);
    put(p->lay.Bo, p->Bo);
    put(p->lay.Bi, p->Bi);
    put(p->lay.lamphi, p->lamphi);
    put(p->lay.mom, p->mom);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(plan_dev, img.data(), img.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return spp_fail(SPP_EDEVICE, std::string("spp_plan_upload: ") + hipGetErrorString(e));
    p->dev = plan_dev;
    spp_noalloc_prepare_current_device();
    return SPP_OK;
}

extern "C" spp_status spp_theta_eigensystem(spp_plan p, int m, double* H, double* lam)
{
    if (!p || !H || !lam) return spp_fail(SPP_EINVAL, "spp_theta_eigensystem: NULL pointer");
    if (m < 0 || m >= p->nm) return spp_fail(SPP_EINVAL, "spp_theta_eigensystem: m out of range");
    const size_t n = p->nth;
    std::memcpy(H, &p->H[m * n * n], n * n * sizeof(double));
    std::memcpy(lam, &p->lam[m * n], n * sizeof(double));
    return SPP_OK;
}

spp_status spp_validate_solve(const char* who, const spp_plan_s* p, const double* rho_dev, const double* phi_dev,
                              double G, const void* workspace_dev)
{
    const std::string w(who);
    if (!p || !rho_dev || !phi_dev || !workspace_dev) return spp_fail(SPP_EINVAL, w + ": NULL pointer");
    if (!p->dev) return spp_fail(SPP_ESTATE, w + ": plan not uploaded");
    if (reinterpret_cast<uintptr_t>(workspace_dev) & 255)
        return spp_fail(SPP_EINVAL, w + ": workspace must be 256-byte aligned");
    if (!std::isfinite(G)) return spp_fail(SPP_EINVAL, w + ": G must be finite");
    const size_t n = size_t(p->nr) * p->nth * p->nphi * sizeof(double);
    const char *a = reinterpret_cast<const char*>(rho_dev), *b = reinterpret_cast<const char*>(phi_dev);
    if (a < b + n && b < a + n) return spp_fail(SPP_EINVAL, w + ": rho and phi must not overlap");
    return SPP_OK;
}

extern "C" spp_status spp_solve(spp_plan p, const double* rho_dev, double* phi_dev, double G,
                                void* workspace_dev, void* stream)
{
    const spp_status st = spp_validate_solve("spp_solve", p, rho_dev, phi_dev, G, workspace_dev);
    if (st != SPP_OK) return st;
    return spp_launch_solve_f64(p, rho_dev, phi_dev, G, workspace_dev, stream);
}

extern "C" spp_status spp_plan_workspace_bytes(spp_plan p, spp_precision prec, size_t* bytes)
{
    if (!p || !bytes) return spp_fail(SPP_EINVAL, "spp_plan_workspace_bytes: NULL pointer");
    if (prec == SPP_FP64) *bytes = p->workspace_bytes;
    else if (prec == SPP_MIXED_FP32) *bytes = spp_mixed_workspace_bytes(p);
    else return spp_fail(SPP_ENOTSUP, "spp_plan_workspace_bytes: precision not supported");
    return SPP_OK;
}

extern "C" spp_status spp_solve_mixed(spp_plan p, spp_precision prec, int n_refine, int fallback_fp64,
                                      const double* rho_dev, double* phi_dev, double G, void* workspace_dev,
                                      void* stream)
{
    const spp_status st = spp_validate_solve("spp_solve_mixed", p, rho_dev, phi_dev, G, workspace_dev);
    if (st != SPP_OK) return st;
    if (prec == SPP_FP64) return spp_launch_solve_f64(p, rho_dev, phi_dev, G, workspace_dev, stream);
    if (prec != SPP_MIXED_FP32) return spp_fail(SPP_ENOTSUP, "spp_solve_mixed: precision not supported");
    if (n_refine < 0 || n_refine > SPP_MAX_REFINE)
        return spp_fail(SPP_EINVAL, "spp_solve_mixed: n_refine must be in [0, 16]");
    if (p->proj_rn == 0) return spp_fail(SPP_ENOTSUP, "spp_solve_mixed: needs N_theta <= 128");
    return spp_launch_solve_mixed(p, prec, n_refine, fallback_fp64, rho_dev, phi_dev, G, workspace_dev, stream);
}

extern "C" spp_status spp_plan_scale_lowprec_basis(spp_plan p, double factor)
{
    if (!p || !std::isfinite(factor)) return spp_fail(SPP_EINVAL, "spp_plan_scale_lowprec_basis: bad arguments");
    for (auto& v : p->Wimg32) v = float(v * factor);
    for (auto& v : p->Himg32) v = float(v * factor);
    return SPP_OK;
}

extern "C" spp_status spp_solve_status(spp_plan p, const void* workspace_dev, void* stream, spp_solve_info* info)
{
    if (!p) return spp_fail(SPP_EINVAL, "spp_solve_status: NULL plan");
    const void* rec_dev = workspace_dev;
    if (!rec_dev) {
        void* scratch = nullptr;
        const spp_status st = spp_noalloc_scratch_current(&scratch);
        if (st != SPP_OK) return st;
        rec_dev = scratch;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    spp_status_record rec{};
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(&rec, rec_dev, sizeof(rec), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("spp_solve_status: ") + hipGetErrorString(e));
    auto dbl = [](unsigned long long b) {
        double d;
        std::memcpy(&d, &b, sizeof(d));
        return d;
    };
    const int n = int(std::min<unsigned>(rec.refine_iters, SPP_MAX_REFINE));
    const double s0 = dbl(rec.rmax[0]);
    if (info) {
        info->refine_iters = n;
        info->first_residual_rel = n > 0 && s0 > 0.0 ? dbl(rec.rmax[1]) / s0 : 0.0;
        info->last_residual_rel = n > 0 && s0 > 0.0 ? dbl(rec.rmax[n]) / s0 : 0.0;
        info->not_contracted = rec.not_contracted ? 1 : 0;
        info->fell_back_fp64 = rec.fallback ? 1 : 0;
        info->nonfinite = rec.nonfinite ? 1 : 0;
    }
    if (rec.nonfinite) return spp_fail(SPP_ENONFINITE, "spp_solve_status: Phi holds a non-finite value");
    if (rec.not_contracted && !rec.fallback)
        return spp_fail(SPP_ENOCONV, "spp_solve_status: the refinement did not contract (FP64 fallback disabled)");
    return SPP_OK;
}

extern "C" spp_status spp_momentum_source(spp_plan p, const double* phi_dev, double G, double* fx_dev,
                                          double* fy_dev, double* fz_dev, void* workspace_dev, void* stream)
{
    if (!p || !phi_dev || !fx_dev || !fy_dev || !fz_dev || !workspace_dev)
        return spp_fail(SPP_EINVAL, "spp_momentum_source: NULL pointer");
    if (!p->dev) return spp_fail(SPP_ESTATE, "spp_momentum_source: plan not uploaded");
    if (reinterpret_cast<uintptr_t>(workspace_dev) & 255)
        return spp_fail(SPP_EINVAL, "spp_momentum_source: workspace must be 256-byte aligned");
    if (!std::isfinite(G) || G == 0.0) return spp_fail(SPP_EINVAL, "spp_momentum_source: G must be finite and non-zero");
    const size_t n = size_t(p->nr) * p->nth * p->nphi * sizeof(double);
    const size_t wsn = SPP_STATUS_BYTES + 2 * spp_align256(size_t(p->nth) * p->nphi * sizeof(double));
    const char* b[4] = {reinterpret_cast<const char*>(phi_dev), reinterpret_cast<const char*>(fx_dev),
                        reinterpret_cast<const char*>(fy_dev), reinterpret_cast<const char*>(fz_dev)};
    const char* wsb = static_cast<const char*>(workspace_dev);
    for (int x = 0; x < 4; ++x) {
        for (int y = x + 1; y < 4; ++y)
            if (b[x] < b[y] + n && b[y] < b[x] + n)
                return spp_fail(SPP_EINVAL, "spp_momentum_source: phi and the three force fields must not overlap");
        if (b[x] < wsb + wsn && wsb < b[x] + n)
            return spp_fail(SPP_EINVAL, "spp_momentum_source: the workspace must not overlap a field");
    }
    return spp_launch_momentum(p, phi_dev, G, fx_dev, fy_dev, fz_dev, workspace_dev, stream);
}

extern "C" spp_status spp_residual(spp_plan p, const double* rho_dev, const double* phi_dev, double G,
                                   double* r_dev, void* workspace_dev, void* stream)
{
    if (!p || !rho_dev || !phi_dev || !r_dev || !workspace_dev)
        return spp_fail(SPP_EINVAL, "spp_residual: NULL pointer");
    if (!p->dev) return spp_fail(SPP_ESTATE, "spp_residual: plan not uploaded");
    if (reinterpret_cast<uintptr_t>(workspace_dev) & 255)
        return spp_fail(SPP_EINVAL, "spp_residual: workspace must be 256-byte aligned");
    if (!std::isfinite(G)) return spp_fail(SPP_EINVAL, "spp_residual: G must be finite");
    const size_t n = size_t(p->nr) * p->nth * p->nphi * sizeof(double);
    const size_t wsn = SPP_STATUS_BYTES + 4 * spp_align256(size_t(p->nth) * p->nphi * sizeof(double));
    const char* r = reinterpret_cast<const char*>(r_dev);
    const char* in[2] = {reinterpret_cast<const char*>(rho_dev), reinterpret_cast<const char*>(phi_dev)};
    const char* w = static_cast<const char*>(workspace_dev);
    for (const char* x : in)
        if (r < x + n && x < r + n) return spp_fail(SPP_EINVAL, "spp_residual: r must not overlap rho or phi");
    for (const char* x : {in[0], in[1], r})
        if (x < w + wsn && w < x + n) return spp_fail(SPP_EINVAL, "spp_residual: the workspace overlaps a field");
    return spp_launch_residual(p, rho_dev, phi_dev, G, r_dev, workspace_dev, stream);
}

extern "C" spp_status spp_face_fluxes(spp_plan p, const double* phi_dev, double* fr_dev, double* ft_dev,
                                      double* fp_dev, void* workspace_dev, void* stream)
{
    if (!p || !phi_dev || !fr_dev || !ft_dev || !fp_dev || !workspace_dev)
        return spp_fail(SPP_EINVAL, "spp_face_fluxes: NULL pointer");
    if (!p->dev) return spp_fail(SPP_ESTATE, "spp_face_fluxes: plan not uploaded");
    if (reinterpret_cast<uintptr_t>(workspace_dev) & 255)
        return spp_fail(SPP_EINVAL, "spp_face_fluxes: workspace must be 256-byte aligned");
    const size_t n = size_t(p->nr) * p->nth * p->nphi * sizeof(double);
    const char* b[4] = {reinterpret_cast<const char*>(phi_dev), reinterpret_cast<const char*>(fr_dev),
                        reinterpret_cast<const char*>(ft_dev), reinterpret_cast<const char*>(fp_dev)};
    // the part of the workspace the call uses: the status record, then two
    // shells of N_theta N_phi doubles
    const size_t wsn = SPP_STATUS_BYTES + 2 * spp_align256(size_t(p->nth) * p->nphi * sizeof(double));
    const char* wsb = static_cast<const char*>(workspace_dev);
    for (int x = 0; x < 4; ++x) {
        if (reinterpret_cast<uintptr_t>(b[x]) & 15)
            return spp_fail(SPP_EINVAL, "spp_face_fluxes: field pointers must be 16-byte aligned");
        for (int y = x + 1; y < 4; ++y)
            if (b[x] < b[y] + n && b[y] < b[x] + n)
                return spp_fail(SPP_EINVAL, "spp_face_fluxes: phi and the three flux fields must not overlap");
        if (b[x] < wsb + wsn && wsb < b[x] + n)
            return spp_fail(SPP_EINVAL, "spp_face_fluxes: the workspace must not overlap phi or the flux fields");
    }
    return spp_launch_face_fluxes(p, phi_dev, fr_dev, ft_dev, fp_dev, workspace_dev, stream);
}

extern "C" spp_status spp_autotune_projection(spp_plan p, void* workspace_dev, void* stream, int* chosen_rows)
{
    if (!p || !workspace_dev) return spp_fail(SPP_EINVAL, "spp_autotune_projection: NULL pointer");
    if (!p->dev) return spp_fail(SPP_ESTATE, "spp_autotune_projection: plan not uploaded");
    int rm = 0;
    const spp_status st = spp_autotune_projection_impl(p, workspace_dev, stream, &rm);
    if (st == SPP_OK && chosen_rows) *chosen_rows = 16 * rm;
    return st;
}

extern "C" spp_status spp_solve_profiled(spp_plan p, const double* rho_dev, double* phi_dev, double G,
                                         void* workspace_dev, void* stream, double* stage_ms)
{
    if (!stage_ms) return spp_fail(SPP_EINVAL, "spp_solve_profiled: NULL stage_ms");
    spp_status st = spp_validate_solve("spp_solve_profiled", p, rho_dev, phi_dev, G, workspace_dev);
    if (st != SPP_OK) return st;
    hipEvent_t ev[SPP_NUM_STAGES + 1] = {};
    int made = 0;
    for (; made <= SPP_NUM_STAGES; ++made)
        if (hipEventCreate(&ev[made]) != hipSuccess) break;
    if (made <= SPP_NUM_STAGES) st = spp_fail(SPP_EDEVICE, "spp_solve_profiled: hipEventCreate failed");
    if (st == SPP_OK) st = spp_launch_solve_f64(p, rho_dev, phi_dev, G, workspace_dev, stream, ev);
    if (st == SPP_OK && hipEventSynchronize(ev[SPP_NUM_STAGES]) != hipSuccess)
        st = spp_fail(SPP_EDEVICE, "spp_solve_profiled: hipEventSynchronize failed");
    for (int k = 0; st == SPP_OK && k < SPP_NUM_STAGES; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess)
            st = spp_fail(SPP_EDEVICE, "spp_solve_profiled: hipEventElapsedTime failed");
        stage_ms[k] = ms;
    }
    for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
    return st;
}
