// Piecewise-polynomial interpolation of the costly thermodynamic functions
// of each reaction (paper Sec. 2.5: the chemistry library interpolates
// costly thermodynamic functions with polynomials of optimal degree).
//
// The functions fitted are the two the rate and Jacobian passes need per
// reaction, both sums over its species of NASA-7 values:
//   F1(T) = -sum_k nu_k g_k/(R T)   (ln K_c without its pressure term)
//   F2(T) =  sum_k nu_k h_k/(R T)   (the reaction enthalpy over R T)
// with nu_k the net (product minus reactant) coefficient.  The variable is
// u = ln T on a uniform grid over [ln Tmin, ln Tmax]: every term of a NASA-7
// function is a power of e^u or linear in u, so its derivatives are spread
// evenly over the range (a grid uniform in T crowds the error at low T).  On
// each interval the polynomial of degree d in the local coordinate
// t in [-1, 1] interpolates the function at the d + 1 Chebyshev points.
// Each degree takes the fewest intervals that meet the target maximum
// absolute error on a check grid of every interval.  The optimal degree is
// the lowest (the cheapest evaluation: d + 1 coefficients read and d fused
// multiply-adds per function) whose table fits THERMO_FIT_TABLE_BYTES, so
// that the tables of all cells stay in one die's L2 cache.
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "mech.hpp"

namespace sc {

namespace {

// g/RT and h/RT of species k at T (single-range NASA-7)
void nasa_gh(const Mech &m, int k, double T, double &gRT, double &hRT)
{
    const double *a = &m.nasa[(size_t)k * 7];
    const double lnT = std::log(T), iT = 1.0 / T;
    hRT = a[0] + T * (a[1] / 2 + T * (a[2] / 3 + T * (a[3] / 4 + T * a[4] / 5))) + a[5] * iT;
    const double sR = a[0] * lnT + T * (a[1] + T * (a[2] / 2 + T * (a[3] / 3 + T * a[4] / 4))) + a[6];
    gRT = hRT - sR;
}

// net coefficients of each reaction: (species, nu) pairs
std::vector<std::vector<std::pair<int, double>>> net_nu(const Mech &m)
{
    std::vector<std::vector<std::pair<int, double>>> out(m.R);
    for (int j = 0; j < m.R; ++j) {
        std::vector<double> nu(m.N, 0.0);
        for (auto &s : m.rx[j].reac) nu[s.first] -= s.second;
        for (auto &s : m.rx[j].prod) nu[s.first] += s.second;
        for (int k = 0; k < m.N; ++k)
            if (nu[k] != 0.0) out[j].push_back({k, nu[k]});
    }
    return out;
}

// solve the (d+1) x (d+1) system V c = f (partial pivoting)
void solve_small(std::vector<double> &V, std::vector<double> &f, int n)
{
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(V[r * n + c]) > std::fabs(V[p * n + c])) p = r;
        if (p != c) {
            for (int q = 0; q < n; ++q) std::swap(V[c * n + q], V[p * n + q]);
            std::swap(f[c], f[p]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double l = V[r * n + c] / V[c * n + c];
            for (int q = c; q < n; ++q) V[r * n + q] -= l * V[c * n + q];
            f[r] -= l * f[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double s = f[c];
        for (int q = c + 1; q < n; ++q) s -= V[c * n + q] * f[q];
        f[c] = s / V[c * n + c];
    }
}

struct Grid {
    int d, nint;
    double u0, du;
};

// Fit every reaction on the grid; returns the largest error on the check
// points (and fills coef when given: [interval][reaction][2][d+1])
double fit_grid(const Mech &m, const std::vector<std::vector<std::pair<int, double>>> &nu, const Grid &g,
                std::vector<double> *coef)
{
    const int d = g.d, np = d + 1, R = m.R, N = m.N;
    std::vector<double> tn(np), V((size_t)np * np);
    for (int i = 0; i < np; ++i) tn[i] = std::cos(M_PI * (2 * i + 1) / (2.0 * np));
    for (int i = 0; i < np; ++i) {
        double p = 1.0;
        for (int q = 0; q < np; ++q, p *= tn[i]) V[i * np + q] = p;
    }
    const int nchk = 3 * np + 2;  // check points per interval, ends included
    std::vector<double> tc(nchk);
    for (int i = 0; i < nchk; ++i) tc[i] = -1.0 + 2.0 * i / (nchk - 1);
    if (coef) coef->assign((size_t)g.nint * R * 2 * np, 0.0);
    std::vector<double> gk((size_t)N * np), hk((size_t)N * np), gc((size_t)N * nchk), hc((size_t)N * nchk);
    double worst = 0.0;
    for (int iv = 0; iv < g.nint; ++iv) {
        const double ua = g.u0 + iv * g.du, half = 0.5 * g.du;
        for (int k = 0; k < N; ++k) {
            for (int i = 0; i < np; ++i) nasa_gh(m, k, std::exp(ua + half * (1.0 + tn[i])), gk[k * np + i], hk[k * np + i]);
            for (int i = 0; i < nchk; ++i)
                nasa_gh(m, k, std::exp(ua + half * (1.0 + tc[i])), gc[k * nchk + i], hc[k * nchk + i]);
        }
        for (int j = 0; j < R; ++j)
            for (int fn = 0; fn < 2; ++fn) {
                std::vector<double> f(np, 0.0), W = V;
                for (auto &s : nu[j])
                    for (int i = 0; i < np; ++i) f[i] += s.second * (fn == 0 ? -gk[s.first * np + i] : hk[s.first * np + i]);
                solve_small(W, f, np);
                for (int i = 0; i < nchk; ++i) {
                    double ex = 0.0;
                    for (auto &s : nu[j]) ex += s.second * (fn == 0 ? -gc[s.first * nchk + i] : hc[s.first * nchk + i]);
                    double p = f[d];
                    for (int q = d - 1; q >= 0; --q) p = p * tc[i] + f[q];
                    worst = std::max(worst, std::fabs(p - ex));
                }
                if (coef)
                    std::copy(f.begin(), f.end(), coef->begin() + (((size_t)iv * R + j) * 2 + fn) * np);
            }
    }
    return worst;
}

}  // namespace

ThermoFit fit_thermo(const Mech &m, double Tmin, double Tmax, double tol, int degree)
{
    if (!(Tmin > 0.0) || !(Tmax > Tmin) || !std::isfinite(Tmax)) throw std::invalid_argument("need 0 < Tmin < Tmax");
    if (!(tol > 0.0)) throw std::invalid_argument("tol must be positive");
    if (degree != 0 && (degree < 1 || degree > THERMO_FIT_MAX_DEGREE))
        throw std::invalid_argument("degree must be 0 (optimal) or 1.." + std::to_string(THERMO_FIT_MAX_DEGREE));
    const auto nu = net_nu(m);
    const double u0 = std::log(Tmin), span = std::log(Tmax) - u0;
    ThermoFit best;
    const int d0 = degree ? degree : 1, d1 = degree ? degree : THERMO_FIT_MAX_DEGREE;
    for (int d = d0; d <= d1 && best.nint == 0; ++d) {
        // intervals allowed: the table budget (a chosen degree: the interval limit)
        const size_t per_int = (size_t)m.R * 2 * (d + 1) * sizeof(double);
        const int cap = degree ? THERMO_FIT_MAX_INTERVALS
                               : (int)std::min<size_t>(THERMO_FIT_MAX_INTERVALS, THERMO_FIT_TABLE_BYTES / per_int);
        if (cap < 1) continue;
        auto err = [&](int nint) { return fit_grid(m, nu, Grid{d, nint, u0, span / nint}, nullptr); };
        // the fewest intervals that meet tol: doubling, then bisection
        int hi = 1;
        double e = err(hi);
        while (e > tol && hi < cap) {
            hi = std::min(2 * hi, cap);
            e = err(hi);
        }
        if (e > tol) continue;  // this degree cannot reach tol within the allowed intervals
        int lo = hi / 2;        // lo fails (or is 0), hi meets tol
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (err(mid) <= tol)
                hi = mid;
            else
                lo = mid;
        }
        best.degree = d;
        best.nint = hi;
    }
    if (best.nint == 0) throw std::invalid_argument("no degree reaches tol within the table limits");
    best.Tmin = Tmin;
    best.Tmax = Tmax;
    best.u0 = u0;
    best.du = span / best.nint;
    best.max_err = fit_grid(m, nu, Grid{best.degree, best.nint, u0, best.du}, &best.coef);
    return best;
}

}  // namespace sc
