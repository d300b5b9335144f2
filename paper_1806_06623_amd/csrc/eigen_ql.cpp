// Symmetric tridiagonal eigensolver: QL iteration with implicit Wilkinson
// shifts (Dubrulle, Martin & Wilkinson, Numer. Math. 12 (1968) 377, "The
// implicit QL algorithm"; the explicit-shift form is Bowdler, Martin, Reinsch
// & Wilkinson, Numer. Math. 11 (1968) 293).  The rotations are
// accumulated into an identity matrix, so the eigenvectors come out
// orthonormal to rounding, which the projections rely on (H^-1 = H^T D).
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

bool spp_tridiag_eigen(int n, std::vector<double>& d, std::vector<double> e, std::vector<double>& Z)
{
    // Zt holds the eigenvectors transposed: row k of Zt is eigenvector k, so
    // each plane rotation touches two contiguous rows.
    std::vector<double> Zt(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Zt[size_t(i) * n + i] = 1.0;
    e.resize(n, 0.0);
    e[n - 1] = 0.0;

    for (int l = 0; l < n; ++l) {
        for (int sweeps = 0;; ++sweeps) {
            // find the first negligible off-diagonal element at or below l
            int m = l;
            for (; m < n - 1; ++m) {
                const double scale = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= DBL_EPSILON * scale) break;
            }
            if (m == l) break;                 // d[l] has converged
            if (sweeps >= 60) return false;

            // Wilkinson shift from the leading 2x2 block of the unreduced part
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));

            // chase the bulge from the bottom (row m) up to row l
            double s = 1.0, c = 1.0, p = 0.0;
            bool deflated = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {                // underflow: split the matrix here
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                double* zi = &Zt[size_t(i) * n];
                double* zj = &Zt[size_t(i + 1) * n];
                for (int k = 0; k < n; ++k) {
                    const double t = zj[k];
                    zj[k] = s * zi[k] + c * t;
                    zi[k] = c * zi[k] - s * t;
                }
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }

    // ascending order; Z[j*n + col] = component j of eigenvector col
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
    std::vector<double> ds(n);
    Z.assign(size_t(n) * n, 0.0);
    for (int col = 0; col < n; ++col) {
        const int src = order[col];
        ds[col] = d[src];
        for (int j = 0; j < n; ++j) Z[size_t(j) * n + col] = Zt[size_t(src) * n + j];
    }
    d.swap(ds);
    return true;
}
