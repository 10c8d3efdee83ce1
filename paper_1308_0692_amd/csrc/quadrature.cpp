// Gauss-Hermite velocity quadratures for the discrete-velocity model.
//
// The weight function is omega(xi) = (2 pi)^(-1/2) exp(-xi^2/2) (Eq. 4).  A
// half-range rule is the n-point Gauss rule of that weight on [0, inf),
// mirrored onto (-inf, 0] (Table I); a full-range rule is the Gauss rule on
// the whole line (probabilists' Hermite roots).
//
// Construction (host, long double):
//   * half-range: recurrence coefficients by the discretised Stieltjes
//     procedure on a composite Gauss-Legendre discretisation of the weight
//     over [0, 24] (the tail beyond is below 1e-120 of the mass);
//     full-range: the known recurrence a_k = 0, b_k = k;
//   * nodes as the zeros of the n-th orthogonal polynomial (the eigenvalues of
//     the Jacobi matrix) by bisection on Sturm counts;
//   * one Newton polish of each node on the recurrence, and weights from the
//     Christoffel numbers 1 / sum_k p_k(x)^2 / ||p_k||^2.
#include <algorithm>
#include <cmath>
#include <limits>
#include <stdexcept>
#include <vector>

#include "fdlb_internal.h"

namespace fdlb {
namespace {

using ld = long double;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_m.
void gauss_legendre(int m, std::vector<ld>& x, std::vector<ld>& w) {
    x.assign(m, 0);
    w.assign(m, 0);
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < (m + 1) / 2; ++i) {
        ld z = std::cos(pi * (i + 0.75L) / (m + 0.5L));
        ld dp = 0;
        for (int it = 0; it < 100; ++it) {
            ld p0 = 1, p1 = 0;
            for (int k = 1; k <= m; ++k) {
                ld p2 = p1;
                p1 = p0;
                p0 = ((2 * k - 1) * z * p1 - (k - 1) * p2) / k;
            }
            dp = m * (z * p0 - p1) / (z * z - 1);
            ld dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-21L) break;
        }
        x[i] = -z;
        x[m - 1 - i] = z;
        w[i] = w[m - 1 - i] = 2 / ((1 - z * z) * dp * dp);
    }
}

// Recurrence of the monic polynomials orthogonal for the half-range weight.
void half_range_recurrence(int n, std::vector<ld>& a, std::vector<ld>& b) {
    const int m = 24;          // Legendre points per panel
    const int panels = 96;     // [0, 24] in panels of 0.25
    const ld h = 0.25L;
    std::vector<ld> gx, gw;
    gauss_legendre(m, gx, gw);
    const ld inv_sqrt_2pi = 0.398942280401432677939946059934381868L;
    std::vector<ld> t, wt;
    t.reserve(m * panels);
    wt.reserve(m * panels);
    for (int p = 0; p < panels; ++p) {
        for (int i = 0; i < m; ++i) {
            ld xi = h * (p + (gx[i] + 1) / 2);
            t.push_back(xi);
            wt.push_back(gw[i] * h / 2 * inv_sqrt_2pi * std::exp(-xi * xi / 2));
        }
    }
    const size_t N = t.size();
    std::vector<ld> pm(N, 0), pc(N, 1), pn(N);
    a.assign(n, 0);
    b.assign(n, 0);
    ld norm_prev = 1;
    for (int k = 0; k < n; ++k) {
        ld norm = 0, xnorm = 0;
        for (size_t i = 0; i < N; ++i) {
            ld q = wt[i] * pc[i] * pc[i];
            norm += q;
            xnorm += q * t[i];
        }
        a[k] = xnorm / norm;
        b[k] = (k == 0) ? norm : norm / norm_prev;
        for (size_t i = 0; i < N; ++i) pn[i] = (t[i] - a[k]) * pc[i] - (k == 0 ? 0 : b[k] * pm[i]);
        std::swap(pm, pc);
        std::swap(pc, pn);
        norm_prev = norm;
    }
    b[0] = 0.5L;  // exact mass of the half-line
}

// Zeros of p_n, the n-th monic orthogonal polynomial of the recurrence
//   p_{k+1}(t) = (t - a_k) p_k(t) - b_k p_{k-1}(t),
// which are the eigenvalues of the Jacobi matrix, by bisection on Sturm counts (the
// eigenvalue-counting method of Givens; see Wilkinson, The Algebraic Eigenvalue Problem,
// 1965, ch. 5): the ratios q_k = p_{k+1}(t) / p_k(t) = (t - a_k) - b_k / q_{k-1} change sign
// once for every zero below t, so the number of negative ratios counts the zeros of p_n below
// t.  Each zero is isolated in its own interval of the Gershgorin bound and halved to the
// resolution of long double.  Ascending.
int zeros_below(const std::vector<ld>& a, const std::vector<ld>& b, ld t) {
    int count = 0;
    ld q = 1;
    for (size_t k = 0; k < a.size(); ++k) {
        q = (a[k] - t) - (k ? b[k] / q : 0);
        // (a ratio that vanishes is nudged by one rounding unit: a zero exactly at t counts
        // on one side consistently)
        if (q == 0) q = -std::numeric_limits<ld>::epsilon() * (std::fabs(a[k]) + std::fabs(t) + 1);
        if (q < 0) ++count;
    }
    return count;
}

std::vector<ld> recurrence_zeros(const std::vector<ld>& a, const std::vector<ld>& b) {
    const int n = (int)a.size();
    ld lo = 0, hi = 0;  // Gershgorin interval of the Jacobi matrix
    for (int k = 0; k < n; ++k) {
        const ld r = (k ? std::sqrt(b[k]) : 0) + (k + 1 < n ? std::sqrt(b[k + 1]) : 0);
        lo = (k == 0) ? a[k] - r : std::min(lo, a[k] - r);
        hi = (k == 0) ? a[k] + r : std::max(hi, a[k] + r);
    }
    std::vector<ld> z(n);
    for (int j = 0; j < n; ++j) {  // zero j: the smallest t with at least j + 1 zeros below it
        ld l = lo, h = hi;
        for (int it = 0; it < 200 && l < h; ++it) {
            const ld m = l + (h - l) / 2;
            if (m <= l || m >= h) break;
            if (zeros_below(a, b, m) > j) h = m;
            else l = m;
        }
        z[j] = l + (h - l) / 2;
    }
    return z;
}

// Gauss rule from a recurrence: nodes ascending and weights (total mass b[0]).
void gauss_from_recurrence(const std::vector<ld>& a, const std::vector<ld>& b, std::vector<ld>& x,
                  std::vector<ld>& w) {
    const int n = (int)a.size();
    const std::vector<ld> d = recurrence_zeros(a, b);
    x.resize(n);
    w.resize(n);
    for (int k = 0; k < n; ++k) {
        // Newton polish on p_n, then Christoffel weight.
        ld t = d[k];
        for (int it = 0; it < 3; ++it) {
            ld pm = 0, pc = 1, dm = 0, dc = 0;
            for (int j = 0; j < n; ++j) {
                ld pn = (t - a[j]) * pc - (j ? b[j] * pm : 0);
                ld dn = pc + (t - a[j]) * dc - (j ? b[j] * dm : 0);
                pm = pc;
                pc = pn;
                dm = dc;
                dc = dn;
            }
            if (dc == 0) break;
            t -= pc / dc;
        }
        ld pm = 0, pc = 1, norm = b[0], s = 1 / norm;
        for (int j = 0; j + 1 < n; ++j) {
            ld pn = (t - a[j]) * pc - (j ? b[j] * pm : 0);
            pm = pc;
            pc = pn;
            norm *= b[j + 1];
            s += pc * pc / norm;
        }
        x[k] = t;
        w[k] = 1 / s;
    }
}

}  // namespace

void quad_half_range(int n, double* nodes, double* weights) {
    if (n < 1 || n > 16) throw Error(FDLB_EINVAL, "half-range order must be 1..16 nodes per half");
    std::vector<ld> a, b, x, w;
    half_range_recurrence(n, a, b);
    gauss_from_recurrence(a, b, x, w);
    for (int i = 0; i < n; ++i) {
        nodes[n - 1 - i] = -(double)x[i];
        nodes[n + i] = (double)x[i];
        weights[n - 1 - i] = weights[n + i] = (double)w[i];
    }
}

void quad_full_range(int n, double* nodes, double* weights) {
    if (n < 1 || n > 32) throw Error(FDLB_EINVAL, "full-range order must be 1..32 nodes");
    std::vector<ld> a(n, 0), b(n), x, w;
    b[0] = 1;
    for (int k = 1; k < n; ++k) b[k] = k;
    gauss_from_recurrence(a, b, x, w);
    // The rule is symmetric: impose it exactly (an odd n has the node 0).
    for (int i = 0; i < n; ++i) {
        ld xs = (x[i] - x[n - 1 - i]) / 2, ws = (w[i] + w[n - 1 - i]) / 2;
        nodes[i] = (double)xs;
        weights[i] = (double)ws;
    }
}

}  // namespace fdlb
