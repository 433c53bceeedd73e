// Run-constant theta-grid data, computed once per solver on the host:
//   gamma = -W_{-1}(-1/t_max)           (eq. theta)
//   theta_i, 1 - theta_i                (eq. theta at alpha = 0)
//   nu_i                                (Sec. 3.4: integral of the global quintic spline)
//   barycentric stencil coefficients    (Sec. 3.3: the alternative theta-stencils)
#include "dmfe_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace dmfe {

// gamma > 1 solving gamma - ln(gamma) = ln(t_max); Newton from the asymptotic guess.
double lambert_gamma(double tmax) {
    const double lt = std::log(tmax);
    double g = lt + std::log(lt) + 1.0;
    for (int it = 0; it < 64; ++it) {
        const double step = (g - std::log(g) - lt) / (1.0 - 1.0 / g);
        g -= step;
        if (std::fabs(step) <= 4e-16 * g) break;
    }
    return g;
}

// theta(y) = [atan(e^g) - atan(e^{-g y})] / [atan(e^g) - atan(e^{-g})] with
// y = (2i + 1 - L)/(L - 1) (0-based i).  Using
// atan(e^a) - atan(e^b) = atan(sinh((a-b)/2) / cosh((a+b)/2)) the numerator is
// atan(sinh(g(1+y)/2) / cosh(g(1-y)/2)) and the denominator atan(sinh g); both
// keep full relative precision.  The lower half is evaluated, the upper half
// follows from theta(-y) = 1 - theta(y), so thc holds the small complements
// exactly as computed.
void theta_grid(int L, double g, double* th, double* thc) {
    const double den = std::atan(std::sinh(g));
    const int half = (L + 1) / 2;  // indices 0..half-1 have y <= 0
    for (int i = 0; i < half; ++i) {
        const double y = double(2 * i + 1 - L) / double(L - 1);
        th[i] = std::atan(std::sinh(0.5 * g * (1.0 + y)) / std::cosh(0.5 * g * (1.0 - y))) / den;
    }
    for (int i = 0; i < half; ++i) thc[i] = 1.0 - th[i];
    for (int i = half; i < L; ++i) {
        thc[i] = th[L - 1 - i];
        th[i] = 1.0 - thc[i];
    }
    th[0] = 0.0;
    thc[0] = 1.0;
    th[L - 1] = 1.0;
    thc[L - 1] = 0.0;
}

// Cox-de Boor: the k+1 = 6 non-zero quintic B-splines at x in span mu
// (knots[mu] <= x < knots[mu+1]), returned as N[0..5] = B_{mu-5..mu}(x).
static void bspline_basis5(const std::vector<double>& kn, int mu, double x, double N[6]) {
    double left[6], right[6];
    N[0] = 1.0;
    for (int j = 1; j <= 5; ++j) {
        left[j] = x - kn[mu + 1 - j];
        right[j] = kn[mu + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            const double tmp = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
}

// nu = A^{-T} b where A_{im} = B_m(theta_i) is the collocation matrix of the
// not-a-knot quintic spline (knots: theta_0 x6, theta_3..theta_{L-4}, theta_{L-1} x6)
// and b_m = int_0^1 B_m = (knot_{m+6} - knot_m)/6.  A is banded (at most 6
// non-zeros per row within 5 of the diagonal) and totally positive, so A^T is
// factored by banded Gaussian elimination without pivoting.
int quintic_weights(int L, const double* th, double* nu) {
    if (L < 6) return -1;
    std::vector<double> kn;
    kn.reserve(L + 6);
    for (int q = 0; q < 6; ++q) kn.push_back(th[0]);
    for (int i = 3; i <= L - 4; ++i) kn.push_back(th[i]);
    for (int q = 0; q < 6; ++q) kn.push_back(th[L - 1]);
    // A^T stored densely in a band: row m (basis index), columns i in [m-KW, m+KW]
    const int KW = 5, W = 2 * KW + 1;
    std::vector<double> AT((size_t)L * W, 0.0);
    auto at = [&](int r, int c) -> double& { return AT[(size_t)r * W + (c - r + KW)]; };
    int mu = 5;  // theta is increasing, so the span index only moves forward
    for (int i = 0; i < L; ++i) {
        const double x = th[i];
        if (i == L - 1) {
            mu = L - 1;  // last span, evaluated at its right end
        } else {
            while (mu + 1 < L && kn[mu + 1] <= x) ++mu;
        }
        double N[6];
        bspline_basis5(kn, mu, x, N);
        if (i == L - 1) {  // right end of the last span: only B_{L-1} is 1
            for (int q = 0; q < 6; ++q) N[q] = (q == 5) ? 1.0 : 0.0;
        }
        for (int q = 0; q < 6; ++q) {
            const int m = mu - 5 + q;  // basis index (column of A = row of A^T)
            if (std::abs(i - m) > KW) return -2;
            at(m, i) = N[q];
        }
    }
    std::vector<double> rhs(L);
    for (int m = 0; m < L; ++m) rhs[m] = (kn[m + 6] - kn[m]) / 6.0;
    // forward elimination on the band, no pivoting
    for (int k = 0; k < L; ++k) {
        const double piv = at(k, k);
        if (piv == 0.0) return -3;
        const int rmax = std::min(L - 1, k + KW);
        for (int r = k + 1; r <= rmax; ++r) {
            const double f = at(r, k) / piv;
            if (f == 0.0) continue;
            const int cmax = std::min(L - 1, k + KW);
            for (int c = k; c <= cmax; ++c) at(r, c) -= f * at(k, c);
            rhs[r] -= f * rhs[k];
        }
    }
    for (int k = L - 1; k >= 0; --k) {
        double acc = rhs[k];
        const int cmax = std::min(L - 1, k + KW);
        for (int c = k + 1; c <= cmax; ++c) acc -= at(k, c) * nu[c];
        nu[k] = acc / at(k, k);
    }
    return 0;
}

// Coefficients of the barycentric form of the theta-stencils (Sec. 3.3), one
// row per stencil base b = 0..L-s: c_0..c_{s-1} and, last, the inverse of the
// stencil's coordinate span (1 on the index coordinate).  A target z is given
// the weights w_k = c_k P_k / sum_m c_m P_m with P_k = prod_{m != k} dz_m and
// dz_m = (z - z_m) * inverse span, for
//   Lagrange:          c_k = 1 / prod_{m != k} (z_k - z_m)
//   Floater-Hormann d: c_k = sum over the windows i..i+d holding k (0 <= i <= s-1-d)
//                      of (-1)^i prod_{j = i..i+d, j != k} 1 / (z_k - z_j)
// (Floater and Hormann 2007).  Node differences are scaled by the inverse span
// and each row by its largest |c_k|; the form is invariant under both.  On
// theta, differences are taken from theta where both nodes sum to at most 1 and
// from 1 - theta otherwise, which keeps the clustered end nodes apart.
void stencil_coefficients(int L, int s, int scheme, int d, const double* th, const double* thc, double* out) {
    const bool on_theta = scheme == DMFE_INTERP_THETA_LAGRANGE || scheme == DMFE_INTERP_THETA_FH;
    const bool fh = scheme == DMFE_INTERP_INDEX_FH || scheme == DMFE_INTERP_THETA_FH;
    if (!fh) d = s - 1;  // one window: the Lagrange weights
    std::vector<double> z(s);
    for (int b = 0; b + s <= L; ++b) {
        auto diff = [&](int k, int m) {  // z_k - z_m, scaled below
            if (!on_theta) return double(k - m);
            const int n1 = b + k, n2 = b + m;
            return th[n1] + th[n2] <= 1.0 ? th[n1] - th[n2] : thc[n2] - thc[n1];
        };
        const double span = diff(s - 1, 0);
        const double inv = 1.0 / span;
        double* row = out + size_t(b) * (s + 1);
        double big = 0.0;
        for (int k = 0; k < s; ++k) {
            double c = 0.0;
            const int i_lo = std::max(0, k - d), i_hi = std::min(k, s - 1 - d);
            for (int i = i_lo; i <= i_hi; ++i) {
                double prod = (i & 1) ? -1.0 : 1.0;
                for (int j = i; j <= i + d; ++j)
                    if (j != k) prod /= diff(k, j) * inv;
                c += prod;
            }
            row[k] = c;
            big = std::max(big, std::fabs(c));
        }
        for (int k = 0; k < s; ++k) row[k] /= big;
        row[s] = on_theta ? inv : 1.0;
    }
}

}  // namespace dmfe
