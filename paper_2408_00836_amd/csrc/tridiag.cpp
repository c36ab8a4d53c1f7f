// tridiag.cpp -- lowest eigenpair of a real symmetric tridiagonal matrix, the
// projected problem of the Krylov (Lanczos) ground-state driver.
//
// Eigenvalue: bisection on the Sturm count.  For T - x I the LDL^T pivots
// q_0 = a_0 - x, q_i = (a_i - x) - b_{i-1}^2 / q_{i-1} have as many negative
// entries as T has eigenvalues below x (Sylvester's law of inertia), so
// bisection between Gershgorin bounds isolates the lowest eigenvalue to
// rounding.  Eigenvector: inverse iteration, i.e. solves of (T - lambda I) y =
// x by Gaussian elimination with partial pivoting on the band.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "hubvqe.hpp"

namespace hv {

namespace {

// Number of eigenvalues of T below x.
int sturm_below(const double *a, const double *b, int m, double x)
{
    const double tiny = std::numeric_limits<double>::min();
    int cnt = 0;
    double q = a[0] - x;
    for (int i = 0;; ++i) {
        if (q == 0.0)
            q = -tiny;   // a zero pivot: count x itself as just above the eigenvalue
        cnt += q < 0.0;
        if (i + 1 == m)
            break;
        q = (a[i + 1] - x) - b[i] * b[i] / q;
    }
    return cnt;
}

// Solve (T - s I) y = rhs in place (rhs -> y) by elimination with partial
// pivoting: row i holds (sub, diag, sup, sup2), sup2 being fill-in from a
// row swap.
void shifted_solve(const double *a, const double *b, int m, double s, double *rhs)
{
    std::vector<double> dl(m, 0.0), d(m), du(m, 0.0), du2(m, 0.0);
    for (int i = 0; i < m; ++i) {
        d[i] = a[i] - s;
        if (i + 1 < m) {
            du[i] = b[i];
            dl[i + 1] = b[i];
        }
    }
    const double eps = std::numeric_limits<double>::epsilon();
    double scale = 0.0;
    for (int i = 0; i < m; ++i)
        scale = std::max(scale, std::fabs(a[i]) + (i + 1 < m ? std::fabs(b[i]) : 0.0) +
                                    (i > 0 ? std::fabs(b[i - 1]) : 0.0));
    const double floor_piv = eps * std::max(scale, 1.0);
    for (int i = 0; i + 1 < m; ++i) {
        // pivot between row i (d, du, du2) and row i+1 (dl, d, du)
        if (std::fabs(dl[i + 1]) > std::fabs(d[i])) {
            std::swap(d[i], dl[i + 1]);
            std::swap(du[i], d[i + 1]);
            std::swap(du2[i], du[i + 1]);
            std::swap(rhs[i], rhs[i + 1]);
        }
        if (std::fabs(d[i]) < floor_piv)
            d[i] = d[i] < 0.0 ? -floor_piv : floor_piv;
        const double f = dl[i + 1] / d[i];
        d[i + 1] -= f * du[i];
        du[i + 1] -= f * du2[i];
        rhs[i + 1] -= f * rhs[i];
        dl[i + 1] = 0.0;
    }
    if (std::fabs(d[m - 1]) < floor_piv)
        d[m - 1] = d[m - 1] < 0.0 ? -floor_piv : floor_piv;
    for (int i = m - 1; i >= 0; --i) {
        double r = rhs[i];
        if (i + 1 < m)
            r -= du[i] * rhs[i + 1];
        if (i + 2 < m)
            r -= du2[i] * rhs[i + 2];
        rhs[i] = r / d[i];
    }
}

}  // namespace

double tridiag_lowest(const double *a, const double *b, int m, double *vec)
{
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    // invariant: no eigenvalue below lo, at least one below hi (or equal)
    hi += std::numeric_limits<double>::epsilon() * std::max(1.0, std::fabs(hi));
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi)
            break;
        if (sturm_below(a, b, m, mid) >= 1)
            hi = mid;
        else
            lo = mid;
    }
    const double lam = 0.5 * (lo + hi);
    if (vec) {
        // inverse iteration from a vector with every component nonzero
        for (int i = 0; i < m; ++i)
            vec[i] = 1.0 + 0.01 * (double)(i % 7);
        for (int it = 0; it < 4; ++it) {
            shifted_solve(a, b, m, lam, vec);
            double nrm = 0.0;
            for (int i = 0; i < m; ++i)
                nrm += vec[i] * vec[i];
            nrm = std::sqrt(nrm);
            for (int i = 0; i < m; ++i)
                vec[i] /= nrm;
        }
        int big = 0;
        for (int i = 1; i < m; ++i)
            if (std::fabs(vec[i]) > std::fabs(vec[big]))
                big = i;
        if (vec[big] < 0.0)
            for (int i = 0; i < m; ++i)
                vec[i] = -vec[i];
    }
    return lam;
}

}  // namespace hv
