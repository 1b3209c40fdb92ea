// Host-only ray geometry of liblrt (Sec. 2.2.3); see lrt_geom.h.
#include "lrt_geom.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <numeric>

#include "../../include/lrt.h"

namespace lrt {

namespace {
constexpr double kPiG = 3.14159265358979323846;
thread_local std::string g_host_error;

lrt_status geom_fail(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_host_error = buf;
    return LRT_E_ARG;
}

// Roots of A2 s^2 + 2 B s + C = 0 (A2 > 0), smaller and larger; false if none.
bool quad_roots(double A2, double B, double C, double &lo, double &hi)
{
    const double disc = B * B - A2 * C;
    if (disc < 0.0) return false;
    const double sq = std::sqrt(disc);
    const double q = (B >= 0.0) ? -(B + sq) : (-B + sq);
    if (q == 0.0) {
        lo = hi = 0.0;
        return true;
    }
    double r1 = q / A2, r2 = C / q;
    lo = std::min(r1, r2);
    hi = std::max(r1, r2);
    return true;
}

}  // namespace

std::string &host_error() { return g_host_error; }

// Gauss-Legendre nodes and weights on [0, 1] (Newton on P_n).
void gauss_legendre_01(int n, std::vector<double> &mu, std::vector<double> &w)
{
    mu.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double x = std::cos(kPiG * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = x; p0 = 1.0; }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = x; p0 = 1.0; }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        // node on [-1, 1] -> [0, 1]
        mu[i] = 0.5 * (x + 1.0);
        w[i] = 0.5 * 2.0 / ((1.0 - x * x) * dp * dp);
    }
    // ascending order
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return mu[a] < mu[b]; });
    std::vector<double> m2(n), w2(n);
    for (int i = 0; i < n; ++i) { m2[i] = mu[idx[i]]; w2[i] = w[idx[i]]; }
    mu.swap(m2);
    w.swap(w2);
}

// Cell-to-cell traversal of one ray from the wall point (0, rw, 0) along
// (mu, st cos phi, st sin phi) through the nx x nr grid.  Appends segments in
// wall -> far order.  Returns false if the traversal does not terminate.
bool traverse_axi(int nx, int nr, double Lx, double R, double rw, double mu, double phi,
                  std::vector<int32_t> &cell, std::vector<double> &ds)
{
    const double dx = Lx / nx, dr = R / nr;
    const double st = std::sqrt(std::max(0.0, 1.0 - mu * mu));
    const double a = st * std::cos(phi);
    const double A2 = st * st;          // rho^2(s) = rw^2 + 2 B s + A2 s^2
    const double B = rw * a;
    int ix = 0;
    // start cell from the same face products the crossings use:
    // ir dr <= rw < (ir + 1) dr (floor(rw / dr) can be one off when dr is
    // not a power of two and rw sits on a face)
    int ir = std::min((int)std::floor(rw / dr), nr - 1);
    while (ir > 0 && rw < ir * dr) --ir;
    while (ir < nr - 1 && rw >= (ir + 1) * dr) ++ir;
    double s = 0.0;
    const int max_steps = 4 * (nx + 2 * nr) + 16;
    for (int step = 0; step < max_steps; ++step) {
        const double s_x = (ix + 1) * dx / mu;
        double s_r = INFINITY;
        int dir = 0;
        if (A2 > 0.0) {
            double lo, hi;
            if (ir > 0) {
                // inward crossing of the inner face: ahead of s, or at s when the
                // ray starts on that face heading inward (d rho^2/ds < 0).  A
                // tangency (lo == hi) touches the face without entering.
                const double rj = ir * dr;
                const bool inward = B + A2 * s < 0.0;
                if (quad_roots(A2, B, (rw - rj) * (rw + rj), lo, hi) && lo < hi &&
                    (lo > s || (lo == s && inward))) {
                    s_r = lo;
                    dir = -1;
                }
            }
            if (dir == 0) {
                // outward crossing of the outer face: ahead of s, or at s when
                // the ray starts on it heading outward
                const double rj = (ir + 1) * dr;
                const bool outward = B + A2 * s > 0.0;
                if (quad_roots(A2, B, (rw - rj) * (rw + rj), lo, hi) && (hi > s || (hi == s && outward))) {
                    s_r = hi;
                    dir = +1;
                }
            }
        }
        const double s_next = std::min(s_x, s_r);
        if (s_next > s) {
            cell.push_back((int32_t)((int64_t)ix * nr + ir));
            ds.push_back(s_next - s);
        }
        s = s_next;
        // an x-plane and an r-face crossed at the same s are both taken, since
        // a root equal to s is not found again on the next step
        const bool cross_x = s_x <= s_r, cross_r = s_r <= s_x;
        if (cross_x && ++ix >= nx) return true;
        if (cross_r) {
            ir += dir;
            if (ir >= nr) return true;
            if (ir < 0) ir = 0;
        }
    }
    return false;
}


// Fibonacci-sphere LOS seen from a wall with normal along +x, and the flux
// weight of each (Sec. 2.2.3): direction i (1-based) of n has polar component
// w = 1 - 2(i-1)/(n-1) along the normal and azimuth a = (i-1)(sqrt 5 - 1) pi;
// those with w > 0 look into the gas.  The interpolated angular rule carries
// the LOS results to the nodes of a uniform (polar phi, azimuth theta) grid,
// each node taking its nearest LOS, and sums over the grid cells the mean of
// the four corners times the cell's int sin(phi) cos(phi) dphi dtheta.  The
// rule is linear in the LOS results, so it reduces to one weight per LOS.
void fibonacci_rule(int n_los, int n_polar, int n_azim, std::vector<double> &dir,
                           std::vector<double> &wt)
{
    dir.clear();
    wt.clear();
    for (int i = 0; i < n_los; ++i) {
        const double w = 1.0 - 2.0 * (double)i / (double)(n_los - 1);
        if (!(w > 0.0)) continue;
        const double r = std::sqrt(std::max(0.0, 1.0 - w * w));
        const double a = ((double)i * (std::sqrt(5.0) - 1.0)) * kPiG;
        dir.push_back(w);
        dir.push_back(r * std::cos(a));
        dir.push_back(r * std::sin(a));
    }
    const int m = (int)(dir.size() / 3);
    wt.assign(m, 0.0);
    std::vector<int> near((size_t)(n_polar + 1) * (n_azim + 1));
    const double dphi = 0.5 * kPiG / n_polar, dth = 2.0 * kPiG / n_azim;
    for (int p = 0; p <= n_polar; ++p) {
        const double ph = p * dphi;
        for (int t = 0; t <= n_azim; ++t) {
            const double th = t * dth;
            const double nx_ = std::cos(ph), ny_ = std::sin(ph) * std::cos(th), nz_ = std::sin(ph) * std::sin(th);
            int best = 0;
            double bd = -2.0;
            for (int q = 0; q < m; ++q) {
                const double dd = dir[3 * q] * nx_ + dir[3 * q + 1] * ny_ + dir[3 * q + 2] * nz_;
                if (dd > bd) {
                    bd = dd;
                    best = q;
                }
            }
            near[(size_t)p * (n_azim + 1) + t] = best;
        }
    }
    for (int p = 0; p < n_polar; ++p) {
        const double s0 = std::sin(p * dphi), s1 = std::sin((p + 1) * dphi);
        const double band = 0.5 * (s1 * s1 - s0 * s0);
        for (int t = 0; t < n_azim; ++t) {
            const double quarter = 0.25 * band * (((t + 1) * dth) - (t * dth));
            wt[near[(size_t)p * (n_azim + 1) + t]] += quarter;
            wt[near[(size_t)(p + 1) * (n_azim + 1) + t]] += quarter;
            wt[near[(size_t)p * (n_azim + 1) + t + 1]] += quarter;
            wt[near[(size_t)(p + 1) * (n_azim + 1) + t + 1]] += quarter;
        }
    }
}

}  // namespace lrt

using namespace lrt;

extern "C" {

lrt_status lrt_fibonacci_quadrature(int n_los, int n_polar, int n_azim, int64_t cap, double *dirs,
                                    double *weights, int64_t *n)
{
    if (n_los < 3 || n_polar < 1 || n_azim < 1 || !n || (cap > 0 && (!dirs || !weights)))
        return geom_fail("fibonacci: invalid sizes");
    std::vector<double> dir, wt;
    fibonacci_rule(n_los, n_polar, n_azim, dir, wt);
    *n = (int64_t)wt.size();
    if (cap < *n) return geom_fail("fibonacci: capacity %lld < %lld", (long long)cap, (long long)*n);
    std::copy(dir.begin(), dir.end(), dirs);
    std::copy(wt.begin(), wt.end(), weights);
    return LRT_OK;
}

lrt_status lrt_trace_axi_ray(int nx, int nr, double Lx, double R, double rw, double mu, double phi,
                             int64_t cap, int32_t *cell, double *ds, int64_t *n)
{
    if (nx < 1 || nr < 1 || !(Lx > 0.0) || !(R > 0.0) || !(rw >= 0.0) || !(rw < R) || !(mu > 0.0) ||
        !(mu <= 1.0) || !std::isfinite(phi) || !n || (cap > 0 && (!cell || !ds)))
        return geom_fail("trace: invalid geometry or direction");
    std::vector<int32_t> cv;
    std::vector<double> dv;
    if (!traverse_axi(nx, nr, Lx, R, rw, mu, phi, cv, dv))
        return geom_fail("trace: traversal did not terminate");
    const int64_t m = (int64_t)cv.size();
    *n = m;
    if (cap < m) return geom_fail("trace: capacity %lld < %lld", (long long)cap, (long long)m);
    for (int64_t i = 0; i < m; ++i) {   // far -> wall
        cell[i] = cv[m - 1 - i];
        ds[i] = dv[m - 1 - i];
    }
    return LRT_OK;
}

}  // extern "C"
