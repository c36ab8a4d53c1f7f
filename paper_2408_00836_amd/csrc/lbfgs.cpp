// lbfgs.cpp -- the optimiser of the VQE driver (Sec. 2.1 minimises the energy
// with L-BFGS): limited-memory BFGS with a line search that enforces the
// strong Wolfe conditions, written as a reverse-communication state machine
// so that one host loop can advance many independent optimisations whose
// evaluations run together (one batched energy+gradient launch for all).
//
// Method (the textbook one): search direction d = -H g from the two-loop
// recursion over the last m pairs (s, y) with the initial scaling
// gamma = s.y / y.y; step length by bracketing then zooming (bisection
// safeguarded quadratic interpolation) until
//   f(x + a d) <= f(x) + c1 a g.d   and   |g(x + a d).d| <= c2 |g.d|.
// Stopping (Sec. 2.1): |E_k - E_{k-1}| < e_tol between consecutive
// iterates, ||g||_2 < g_tol, or max_steps iterations.
#include <algorithm>
#include <cmath>
#include <vector>

#include "hubvqe.hpp"

namespace hv {

namespace {
double dot(const std::vector<double> &a, const std::vector<double> &b)
{
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i)
        s += a[i] * b[i];
    return s;
}
constexpr double kC1 = 1e-4, kC2 = 0.9;
constexpr int kMaxLineEvals = 25;
}  // namespace

Lbfgs::Lbfgs(const double *x0, int n, const LbfgsOptions &o) : opt(o), n(n)
{
    x.assign(x0, x0 + n);
    trial = x;
}

void Lbfgs::direction()
{
    // two-loop recursion: d = -H_k g
    const int k = (int)S.size();
    std::vector<double> q = g, al(k);
    for (int i = k - 1; i >= 0; --i) {
        al[i] = rho[i] * dot(S[i], q);
        for (int j = 0; j < n; ++j)
            q[j] -= al[i] * Y[i][j];
    }
    double gamma = 1.0;
    if (k > 0)
        gamma = dot(S[k - 1], Y[k - 1]) / dot(Y[k - 1], Y[k - 1]);
    for (int j = 0; j < n; ++j)
        q[j] *= gamma;
    for (int i = 0; i < k; ++i) {
        const double b = rho[i] * dot(Y[i], q);
        for (int j = 0; j < n; ++j)
            q[j] += S[i][j] * (al[i] - b);
    }
    d.resize(n);
    for (int j = 0; j < n; ++j)
        d[j] = -q[j];
    dphi0 = dot(g, d);
    if (!(dphi0 < 0.0)) {   // not a descent direction: restart from steepest descent
        S.clear();
        Y.clear();
        rho.clear();
        for (int j = 0; j < n; ++j)
            d[j] = -g[j];
        dphi0 = -dot(g, g);
    }
}

void Lbfgs::request(double a)
{
    alpha = a;
    for (int j = 0; j < n; ++j)
        trial[j] = x[j] + a * d[j];
    ++line_evals;
}

void Lbfgs::start_line_search()
{
    line_evals = 0;
    zooming = false;
    a_prev = 0.0;
    f_prev = f;
    df_prev = dphi0;
    // first iteration: a unit-length step along -g; later ones: a = 1
    double a0 = 1.0;
    if (S.empty())
        a0 = std::min(1.0, 1.0 / std::sqrt(std::max(dot(d, d), 1e-300)));
    request(a0);
}

int Lbfgs::finish(int reason)
{
    status = reason;
    trial = x;
    return status;
}

// Accept the trial point (its value and gradient ft, gt): update the
// history, test the stopping rules, start the next iteration.
int Lbfgs::accept(double ft, const double *gt)
{
    std::vector<double> s(n), y(n);
    for (int j = 0; j < n; ++j) {
        s[j] = trial[j] - x[j];
        y[j] = gt[j] - g[j];
    }
    const double sy = dot(s, y);
    const double f_old = f;
    x = trial;
    f = ft;
    g.assign(gt, gt + n);
    ++steps;
    if (sy > 1e-300) {
        S.push_back(s);
        Y.push_back(y);
        rho.push_back(1.0 / sy);
        if ((int)S.size() > opt.history) {
            S.erase(S.begin());
            Y.erase(Y.begin());
            rho.erase(rho.begin());
        }
    }
    gnorm = std::sqrt(dot(g, g));
    if (std::fabs(f - f_old) < opt.e_tol)
        return finish(LBFGS_ENERGY_TOL);
    if (gnorm < opt.g_tol)
        return finish(LBFGS_GRAD_TOL);
    if (steps >= opt.max_steps)
        return finish(LBFGS_MAX_STEPS);
    direction();
    start_line_search();
    return LBFGS_EVALUATE;
}

int Lbfgs::tell(double ft, const double *gt)
{
    if (status != LBFGS_EVALUATE)
        return status;
    ++evals;
    if (first) {   // the start point
        first = false;
        f = ft;
        g.assign(gt, gt + n);
        gnorm = std::sqrt(dot(g, g));
        if (!std::isfinite(f) || !std::isfinite(gnorm))
            return finish(LBFGS_NOT_FINITE);
        if (gnorm < opt.g_tol)
            return finish(LBFGS_GRAD_TOL);
        if (opt.max_steps <= 0)
            return finish(LBFGS_MAX_STEPS);
        direction();
        start_line_search();
        return LBFGS_EVALUATE;
    }
    if (give_up) {   // the best point of a failed line search, evaluated again
        give_up = false;
        if (std::isfinite(ft) && ft < f)
            return accept(ft, gt);
        return finish(LBFGS_LINE_SEARCH);
    }
    double dft = 0.0;
    for (int j = 0; j < n; ++j)
        dft += gt[j] * d[j];
    const bool finite = std::isfinite(ft) && std::isfinite(dft);
    const bool armijo = finite && ft <= f + kC1 * alpha * dphi0;
    const bool curv = finite && std::fabs(dft) <= -kC2 * dphi0;
    if (!zooming) {
        if (!armijo || (line_evals > 1 && ft >= f_prev)) {
            zooming = true;
            a_lo = a_prev, f_lo = f_prev, df_lo = df_prev, a_hi = alpha;
        } else if (curv) {
            return accept(ft, gt);
        } else if (dft >= 0.0) {
            zooming = true;
            a_lo = alpha, f_lo = ft, df_lo = dft, a_hi = a_prev;
        } else {
            // still descending: extrapolate
            a_prev = alpha, f_prev = ft, df_prev = dft;
            if (line_evals >= kMaxLineEvals)
                return accept(ft, gt);   // a decrease, though not a Wolfe point
            request(alpha * 2.0);
            return LBFGS_EVALUATE;
        }
    } else {
        if (!armijo || ft >= f_lo) {
            a_hi = alpha;
        } else {
            if (curv)
                return accept(ft, gt);
            if (dft * (a_hi - a_lo) >= 0.0)
                a_hi = a_lo;
            a_lo = alpha, f_lo = ft, df_lo = dft;
        }
    }
    if (line_evals >= kMaxLineEvals) {
        // no Wolfe point found: take the best point seen if it decreased f
        // (its gradient is needed, so it is evaluated once more)
        if (a_lo > 0.0 && f_lo < f) {
            request(a_lo);
            give_up = true;
            return LBFGS_EVALUATE;
        }
        return finish(LBFGS_LINE_SEARCH);
    }
    // zoom: minimiser of the quadratic through (a_lo, f_lo, df_lo) and
    // (a_hi, f(a_hi)) is not tracked for f(a_hi); use the derivative at a_lo
    // and the value at alpha, kept inside the middle 80% of the bracket
    const double lo = std::min(a_lo, a_hi), hi = std::max(a_lo, a_hi);
    double a = 0.5 * (lo + hi);
    const double da = alpha - a_lo;
    const double den = 2.0 * (ft - f_lo - df_lo * da);
    if (alpha != a_lo && den > 0.0)
        a = a_lo - df_lo * da * da / den;
    a = std::min(std::max(a, lo + 0.1 * (hi - lo)), hi - 0.1 * (hi - lo));
    request(a);
    return LBFGS_EVALUATE;
}

}  // namespace hv
