/*
 * dmfe_oracle.c -- plain FP64 CPU oracle for the two-time DMFE of the mixed
 * spherical p-spin model (DYNAMITE, arXiv 2604.06309).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * What it computes (each function cites the passage it follows):
 *   - the model: f(q) = sum_p a_p^2 q^p / 2 and its derivatives (Sec. 2.1,
 *     covariance equation);
 *   - a uniform-grid solver: classical RK4 in t with trapezoid history
 *     integrals over the stored causal triangle (the direct O(N^3) baseline of
 *     Sec. 2.3; the scheme itself is not printed in the paper, see the
 *     readings list in the design notes);
 *   - the theta-grid of eq. (theta) at alpha = 0 and its inverse index map;
 *   - one evaluation of the right-hand side on the theta-grid: interpolation
 *     in theta by one of the schemes of Sec. 3.3 (Lagrange on the index
 *     coordinate -- the default -- or on theta, Floater-Hormann on either),
 *     optionally on log R (Appendix A), cubic Hermite interpolation
 *     in t (Sec. 3.3), the change of variables phi1 = theta_i theta_j and
 *     phi2 = theta_j + (1 - theta_j) theta_i and the quadrature sums of
 *     eq. (int) (Sec. 3.4), mu(t) and E(t) (Sec. 2.1);
 *   - the sparsification residual and greedy selection (Sec. 3.6);
 *   - the adaptive driver: Dormand-Prince then SSPRK(10,4), the 1-norm error
 *     and the step-size rules of Sec. 3.5.
 *
 * Everything is double precision, written as loops in the order of the
 * definitions, without blocking or fusion.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_TERMS 8

typedef struct {
    int n_terms;
    int p[OR_MAX_TERMS];
    double a2[OR_MAX_TERMS]; /* the a_p^2 */
    double T;
    double beta0;
} or_model;

/* ------------------------------------------------------------------ model */
/* f(q) = sum a_p^2 q^p / 2  (Sec. 2.1, covariance function). */
double or_f(const or_model *m, double q) {
    double s = 0.0;
    for (int k = 0; k < m->n_terms; ++k) s += 0.5 * m->a2[k] * pow(q, m->p[k]);
    return s;
}
/* f'(q) = sum a_p^2 p q^(p-1) / 2 */
double or_f1(const or_model *m, double q) {
    double s = 0.0;
    for (int k = 0; k < m->n_terms; ++k)
        s += 0.5 * m->a2[k] * m->p[k] * pow(q, m->p[k] - 1);
    return s;
}
/* f''(q) = sum a_p^2 p (p-1) q^(p-2) / 2 */
double or_f2(const or_model *m, double q) {
    double s = 0.0;
    for (int k = 0; k < m->n_terms; ++k)
        if (m->p[k] >= 2) s += 0.5 * m->a2[k] * m->p[k] * (m->p[k] - 1) * pow(q, m->p[k] - 2);
    return s;
}

/* ======================================================================
 * Uniform-grid solver.
 * Storage: packed lower triangle, row n holds X[n][0..n] at offset n(n+1)/2.
 * ====================================================================== */
static inline size_t tri(int n, int k) { return (size_t)n * (n + 1) / 2 + k; }

/* Trapezoid weight of node m on the nodes lo..hi with spacing h (zero if lo == hi). */
static double trap_w(int m, int lo, int hi, double h) {
    if (hi <= lo) return 0.0;
    if (m == lo || m == hi) return 0.5 * h;
    return h;
}

/*
 * Right-hand side of the DMFE (eq. genericDMFE with the -mu terms, kernels
 * K = f''(C)R, D = f'(C), forcing F_C = beta0 f'(C(t,0)) C(t',0) and mu of
 * Sec. 2.1) for the row C(t, t_k), R(t, t_k), k = 0..n, at t = t_n + delta.
 * The integrals over s are trapezoid sums on the stored nodes t_0..t_n plus
 * the partial panel [t_n, t] whose right end is the diagonal s = t, where
 * C(t,t) = R(t,t^-) = 1.
 */
static void uni_rhs(const or_model *m, int n, double h, double delta,
                    const double *Ct, const double *Rt,
                    const double *c, const double *r, double *dc, double *dr) {
    double *W = (double *)malloc(sizeof(double) * (n + 1));
    double *g1 = (double *)malloc(sizeof(double) * (n + 1)); /* f'(c_q)  */
    double *g2 = (double *)malloc(sizeof(double) * (n + 1)); /* f''(c_q) */
    for (int q = 0; q <= n; ++q) {
        W[q] = trap_w(q, 0, n, h);
        g1[q] = or_f1(m, c[q]);
        g2[q] = or_f2(m, c[q]);
    }
    W[n] += 0.5 * delta;
    const double Ws = 0.5 * delta;
    const double f1one = or_f1(m, 1.0), f2one = or_f2(m, 1.0);

    /* mu(t) = T + int_0^t [K C + D R](t,s) ds + F_C(t,t) */
    double mu = m->T;
    for (int q = 0; q <= n; ++q) mu += W[q] * (g2[q] * r[q] * c[q] + g1[q] * r[q]);
    mu += Ws * (f2one + f1one);
    mu += m->beta0 * g1[0] * c[0];

#pragma omp parallel for schedule(dynamic, 8)
    for (int k = 0; k <= n; ++k) {
        /* int_0^t K(t,s) C(s,t_k) ds, C symmetric */
        double A = 0.0;
        for (int q = 0; q <= n; ++q) {
            double Cqk = (q >= k) ? Ct[tri(q, k)] : Ct[tri(k, q)];
            A += W[q] * g2[q] * r[q] * Cqk;
        }
        A += Ws * f2one * c[k];
        /* int_0^{t_k} D(t,s) R(t_k,s) ds */
        double B = 0.0;
        for (int q = 0; q <= k; ++q) B += trap_w(q, 0, k, h) * g1[q] * Rt[tri(k, q)];
        /* int_{t_k}^t K(t,s) R(s,t_k) ds */
        double Q = 0.0;
        for (int q = k; q <= n; ++q) {
            double w = trap_w(q, k, n, h) + (q == n ? 0.5 * delta : 0.0);
            Q += w * g2[q] * r[q] * Rt[tri(q, k)];
        }
        Q += Ws * f2one * r[k];
        dc[k] = -mu * c[k] + A + B + m->beta0 * g1[0] * Ct[tri(k, 0)];
        dr[k] = -mu * r[k] + Q;
    }
    free(W);
    free(g1);
    free(g2);
}

/* E(t_n) = -int_0^{t_n} f'(C(t_n,s)) R(t_n,s) ds - beta0 f(C(t_n,0))  (Sec. 2.1) */
static double uni_energy(const or_model *m, int n, double h, const double *Ct, const double *Rt) {
    double e = 0.0;
    for (int q = 0; q <= n; ++q) e += trap_w(q, 0, n, h) * or_f1(m, Ct[tri(n, q)]) * Rt[tri(n, q)];
    return -e - m->beta0 * or_f(m, Ct[tri(n, 0)]);
}

/*
 * Classical RK4 over N steps of size h from C(0,0) = R(0,0^-) = 1.
 * C, R: packed triangles with room for N+1 rows.  E: N+1 energies.
 * Returns 0.
 */
int or_uniform_solve(const or_model *m, double h, int N, double *C, double *R, double *E) {
    C[0] = 1.0;
    R[0] = 1.0;
    E[0] = uni_energy(m, 0, h, C, R);
    int cap = N + 2;
    double *y = malloc(sizeof(double) * 2 * cap), *ys = malloc(sizeof(double) * 2 * cap);
    double *k1 = malloc(sizeof(double) * 2 * cap), *k2 = malloc(sizeof(double) * 2 * cap);
    double *k3 = malloc(sizeof(double) * 2 * cap), *k4 = malloc(sizeof(double) * 2 * cap);
    for (int n = 0; n < N; ++n) {
        int w = n + 1; /* unknowns k = 0..n for each field */
        for (int k = 0; k <= n; ++k) {
            y[k] = C[tri(n, k)];
            y[cap + k] = R[tri(n, k)];
        }
        uni_rhs(m, n, h, 0.0, C, R, y, y + cap, k1, k1 + cap);
        for (int k = 0; k < w; ++k) {
            ys[k] = y[k] + 0.5 * h * k1[k];
            ys[cap + k] = y[cap + k] + 0.5 * h * k1[cap + k];
        }
        uni_rhs(m, n, h, 0.5 * h, C, R, ys, ys + cap, k2, k2 + cap);
        for (int k = 0; k < w; ++k) {
            ys[k] = y[k] + 0.5 * h * k2[k];
            ys[cap + k] = y[cap + k] + 0.5 * h * k2[cap + k];
        }
        uni_rhs(m, n, h, 0.5 * h, C, R, ys, ys + cap, k3, k3 + cap);
        for (int k = 0; k < w; ++k) {
            ys[k] = y[k] + h * k3[k];
            ys[cap + k] = y[cap + k] + h * k3[cap + k];
        }
        uni_rhs(m, n, h, h, C, R, ys, ys + cap, k4, k4 + cap);
        for (int k = 0; k < w; ++k) {
            C[tri(n + 1, k)] = y[k] + h / 6.0 * (k1[k] + 2.0 * k2[k] + 2.0 * k3[k] + k4[k]);
            R[tri(n + 1, k)] = y[cap + k] +
                               h / 6.0 * (k1[cap + k] + 2.0 * k2[cap + k] + 2.0 * k3[cap + k] + k4[cap + k]);
        }
        C[tri(n + 1, n + 1)] = 1.0;
        R[tri(n + 1, n + 1)] = 1.0;
        E[n + 1] = uni_energy(m, n + 1, h, C, R);
    }
    free(y); free(ys); free(k1); free(k2); free(k3); free(k4);
    return 0;
}

/* One right-hand-side evaluation of the uniform scheme (exported for tests). */
void or_uniform_rhs(const or_model *m, int n, double h, double delta, const double *C,
                    const double *R, const double *c, const double *r, double *dc, double *dr) {
    uni_rhs(m, n, h, delta, C, R, c, r, dc, dr);
}

/* ======================================================================
 * theta-grid (eq. theta at alpha = 0).
 * ====================================================================== */

/* gamma = -W_{-1}(-1/t_max), i.e. the root gamma > 1 of gamma - ln(gamma) = ln(t_max). */
double or_gamma(double tmax) {
    double lt = log(tmax);
    double g = lt + log(lt) + 1.0;
    for (int it = 0; it < 100; ++it) {
        double F = g - log(g) - lt;
        double dF = 1.0 - 1.0 / g;
        double gn = g - F / dF;
        if (fabs(gn - g) <= 1e-16 * gn) { g = gn; break; }
        g = gn;
    }
    return g;
}

/*
 * theta_i for i = 0..L-1 (paper index i+1) and the complements 1 - theta_i.
 * The numerator atan(e^g) - atan(e^{-g y}) is evaluated through
 * atan(a) - atan(b) = atan((a - b)/(1 + ab)) (a, b > 0) with
 * a - b = -e^g expm1(-g (1 + y)), which keeps full relative precision near
 * theta = 0.  Points with theta > 1/2 are taken from the symmetry
 * theta(-y) = 1 - theta(y) of eq. (theta) at alpha = 0.
 */
void or_theta_grid(int L, double gamma, double *th, double *thc) {
    double D = atan(exp(gamma)) - atan(exp(-gamma));
    for (int i = 0; i < L; ++i) {
        if (2 * i + 1 - L > 0) continue; /* upper half below */
        double y = (double)(2 * i + 1 - L) / (double)(L - 1);
        double num = -exp(gamma) * expm1(-gamma * (1.0 + y)) / (1.0 + exp(gamma * (1.0 - y)));
        th[i] = atan(num) / D;
        thc[i] = 1.0 - th[i];
    }
    for (int i = 0; i < L; ++i) {
        if (2 * i + 1 - L <= 0) continue;
        thc[i] = th[L - 1 - i];
        th[i] = 1.0 - thc[i];
    }
}

/* theta-interpolation schemes of Sec. 3.3 */
#define OR_INDEX_LAGRANGE 0 /* Lagrange on the equidistant index coordinate (default) */
#define OR_THETA_LAGRANGE 1 /* Lagrange on theta itself */
#define OR_INDEX_FH 2       /* Floater-Hormann rational interpolation on the index coordinate */
#define OR_THETA_FH 3       /* Floater-Hormann on theta */

typedef struct {
    int L, s;
    double gamma, D;
    const double *th, *thc, *nu;
    int interp; /* OR_* scheme */
    int fh_d;   /* Floater-Hormann blending degree d, 0 <= d <= s-1 */
    int log_r;  /* interpolate log R instead of R (Appendix A) */
    int pad;
} or_grid;

/*
 * Continuous 0-based index x(theta) of the grid, the inverse of eq. (theta):
 * with T = tan(theta D), 1 + y = [ln(1 + e^g T) - ln(1 - e^{-g} T)] / g and
 * x = (L - 1)(1 + y)/2.  Used for theta <= 1/2; above, x = L-1 - x(1-theta)
 * with the complement supplied by the caller.
 */
static double or_xhalf(const or_grid *g, double th) {
    double T = tan(th * g->D);
    return 0.5 * (g->L - 1) * (log1p(exp(g->gamma) * T) - log1p(-exp(-g->gamma) * T)) / g->gamma;
}
static double or_xmap(const or_grid *g, double th, double thc) {
    if (th <= 0.5) return or_xhalf(g, th);
    return (double)(g->L - 1) - or_xhalf(g, thc);
}
double or_index_of(int L, double gamma, double th, double thc) {
    or_grid g = {L, 10, gamma, atan(exp(gamma)) - atan(exp(-gamma)), 0, 0, 0, 0, 0, 0, 0};
    return or_xmap(&g, th, thc);
}

/*
 * A theta-coordinate to interpolate at: the grid node `node` (node >= 0, no
 * interpolation), or the point with continuous index x, theta = th and
 * 1 - theta = thc (both supplied, so that either is exact where it is small).
 */
typedef struct {
    int node;
    double x, th, thc;
} or_pt;

/*
 * The s-point stencil of a target (Sec. 3.3): nodes base..base+s-1 with
 * base = floor(x) - (s-1)/2 clamped to [0, L-s], for every scheme.
 */
static int stencil_base(const or_grid *g, double x) {
    int base = (int)floor(x) - (g->s - 1) / 2;
    if (base < 0) base = 0;
    if (base > g->L - g->s) base = g->L - g->s;
    return base;
}

static int on_theta(const or_grid *g) { return g->interp == OR_THETA_LAGRANGE || g->interp == OR_THETA_FH; }

/*
 * Coordinate differences of the scheme.  Index schemes: x - n and n1 - n2.
 * Theta schemes: theta differences taken from whichever of theta and 1 - theta
 * is exact near the points involved (theta below 1/2, the complement above), so
 * that the clustered nodes at both ends keep their relative spacing.
 */
static double dq(const or_grid *g, const or_pt *q, int n) {
    if (!on_theta(g)) return q->x - (double)n;
    return q->th <= 0.5 ? q->th - g->th[n] : g->thc[n] - q->thc;
}
static double dn(const or_grid *g, int n1, int n2) {
    if (!on_theta(g)) return (double)(n1 - n2);
    return g->th[n1] + g->th[n2] <= 1.0 ? g->th[n1] - g->th[n2] : g->thc[n2] - g->thc[n1];
}

/* The polynomial through (node base+k, v[k]), k < n, at q: Lagrange's product form. */
static double poly_at(const or_grid *g, const or_pt *q, int base, int n, const double *v) {
    double val = 0.0;
    for (int k = 0; k < n; ++k) {
        double w = 1.0;
        for (int l = 0; l < n; ++l)
            if (l != k) w *= dq(g, q, base + l) / dn(g, base + k, base + l);
        val += w * v[k];
    }
    return val;
}

/*
 * Floater-Hormann rational interpolant of degree d on the s stencil nodes
 * (Floater and Hormann 2007, cited in Sec. 3.3), from its definition: the blend
 * r = sum_i lam_i p_i / sum_i lam_i over the s-d windows i..i+d, p_i the
 * polynomial through the window, lam_i = (-1)^i / prod_{j=i}^{i+d} (z - z_j).
 * At a node r takes the node's value.
 */
static double fh_at(const or_grid *g, const or_pt *q, int base, const double *v) {
    int s = g->s, d = g->fh_d;
    for (int k = 0; k < s; ++k)
        if (dq(g, q, base + k) == 0.0) return v[k];
    double num = 0.0, den = 0.0;
    for (int i = 0; i + d < s; ++i) {
        double lam = (i & 1) ? -1.0 : 1.0;
        for (int j = i; j <= i + d; ++j) lam /= dq(g, q, base + j);
        num += lam * poly_at(g, q, base + i, d + 1, v + i);
        den += lam;
    }
    return num / den;
}

/* The scheme's interpolant through the stencil values v[0..s-1] at q. */
static double stencil_at(const or_grid *g, const or_pt *q, int base, const double *v) {
    if (g->interp == OR_INDEX_FH || g->interp == OR_THETA_FH) return fh_at(g, q, base, v);
    return poly_at(g, q, base, g->s, v);
}

/* Values of a row at the stencil of q (one value at a node); returns their count. */
static int gather(const or_grid *g, const double *row, const or_pt *q, int *base, double *v) {
    if (q->node >= 0) {
        *base = q->node;
        v[0] = row[q->node];
        return 1;
    }
    *base = stencil_base(g, q->x);
    for (int k = 0; k < g->s; ++k) v[k] = row[*base + k];
    return g->s;
}
static double interp_vals(const or_grid *g, const or_pt *q, int base, int n, const double *v) {
    return n == 1 ? v[0] : stencil_at(g, q, base, v);
}
static int all_positive(const double *v, int n) {
    for (int k = 0; k < n; ++k)
        if (!(v[k] > 0.0)) return 0;
    return 1;
}

#define OR_MAX_S 16

/*
 * A row interpolated at q.  With as_log (the R field under the log option of
 * Appendix A) the interpolant of log R is exponentiated, unless a stencil value
 * is not positive: then R itself is interpolated.
 */
static double row_at(const or_grid *g, const double *row, const or_pt *q, int as_log) {
    double v[OR_MAX_S];
    int base, n = gather(g, row, q, &base, v);
    if (as_log && all_positive(v, n)) {
        for (int k = 0; k < n; ++k) v[k] = log(v[k]);
        return exp(interp_vals(g, q, base, n, v));
    }
    return interp_vals(g, q, base, n, v);
}

/* Stored history in the oracle's own layout: four [M][L] arrays. */
typedef struct {
    int M;           /* slices 0..M-1 */
    int nb;          /* slices 0..nb-1 carry a stored d/dt (nb = M-1 at stage 1, M later) */
    const double *t; /* t_n */
    const double *C, *R, *dC, *dR;
    double tcur;                /* current stage time t */
    const double *yC, *yR;      /* current stage slice C(t, theta_i t), R(t, theta_i t) */
} or_hist;

/*
 * (C, R)(tau, q) for 0 <= tau <= t: a rule in t over at most two slices, each
 * slice theta-interpolated at q first (Sec. 3.3, the 2-D stencil of I_2).
 *  - tau inside the stored slices with known d/dt: cubic Hermite in t between
 *    the bracketing slices m, m+1 from value and d/dt on each;
 *  - tau above the last slice b with known d/dt (inside the current step): the
 *    quadratic in t through value and d/dt at b and the value of the current
 *    stage slice at t;
 *  - only t_0 stored: slice 0 (or the stage slice before any slice has d/dt).
 * Under the log option, R follows the same rule applied to log R with the
 * scaled derivative (dR/dt)/R, whenever every R value the rule reads is
 * positive; otherwise R itself.
 */
static void or_hist_at(const or_grid *g, const or_hist *H, double tau, const or_pt *q, double out[2]) {
    int L = g->L;
    /* slice a (and b when nb_used == 2); -1 stands for the stage slice; weights on
     * value and d/dt of each */
    int sa = -1, sb = -1, two = 0;
    double wa = 1.0, wda = 0.0, wb = 0.0, wdb = 0.0;
    if (H->nb >= 1) {
        int b = H->nb - 1;
        double tb = H->t[b];
        if (tau <= tb) {
            if (b == 0) {
                sa = 0;
            } else {
                int m = 0;
                while (m + 1 < b && H->t[m + 1] <= tau) ++m;
                double h = H->t[m + 1] - H->t[m];
                double u = (tau - H->t[m]) / h;
                sa = m;
                sb = m + 1;
                two = 1;
                wa = 2 * u * u * u - 3 * u * u + 1;
                wda = (u * u * u - 2 * u * u + u) * h;
                wb = -2 * u * u * u + 3 * u * u;
                wdb = (u * u * u - u * u) * h;
            }
        } else {
            double h = H->tcur - tb;
            double u = (tau - tb) / h;
            sa = b;
            sb = -1;
            two = 1;
            wa = 1.0 - u * u;
            wda = h * (u - u * u);
            wb = u * u;
        }
    }
    const double *val[2] = {H->C, H->R}, *der[2] = {H->dC, H->dR}, *cur[2] = {H->yC, H->yR};
    for (int f = 0; f < 2; ++f) {
        const double *va = sa < 0 ? cur[f] : val[f] + (size_t)sa * L;
        const double *da = sa < 0 ? NULL : der[f] + (size_t)sa * L;
        const double *vb = sb < 0 ? cur[f] : val[f] + (size_t)sb * L;
        const double *db = sb < 0 ? NULL : der[f] + (size_t)sb * L;
        double Va[OR_MAX_S], Da[OR_MAX_S], Vb[OR_MAX_S], Db[OR_MAX_S];
        int base, n = gather(g, va, q, &base, Va);
        if (da) gather(g, da, q, &base, Da);
        if (two) gather(g, vb, q, &base, Vb);
        if (two && db) gather(g, db, q, &base, Db);
        int use_log = f == 1 && g->log_r && all_positive(Va, n) && (!two || all_positive(Vb, n));
        if (use_log) {
            for (int k = 0; k < n; ++k) {
                if (da) Da[k] = Da[k] / Va[k];
                Va[k] = log(Va[k]);
                if (two) {
                    if (db) Db[k] = Db[k] / Vb[k];
                    Vb[k] = log(Vb[k]);
                }
            }
        }
        double r = wa * interp_vals(g, q, base, n, Va);
        if (da) r += wda * interp_vals(g, q, base, n, Da);
        if (two) r += wb * interp_vals(g, q, base, n, Vb);
        if (two && db) r += wdb * interp_vals(g, q, base, n, Db);
        out[f] = use_log ? exp(r) : r;
    }
}

/* mu(t) and E(t) of a slice (Sec. 2.1): s = theta t, ds = t dtheta, quadrature nu. */
void or_mu_energy(const or_model *m, int L, const double *nu, double t, const double *yC,
                  const double *yR, double *mu, double *E) {
    double sk = 0.0, se = 0.0;
    for (int i = 0; i < L; ++i) {
        sk += nu[i] * (or_f2(m, yC[i]) * yR[i] * yC[i] + or_f1(m, yC[i]) * yR[i]);
        se += nu[i] * or_f1(m, yC[i]) * yR[i];
    }
    *mu = m->T + t * sk + m->beta0 * or_f1(m, yC[0]) * yC[0];
    *E = -t * se - m->beta0 * or_f(m, yC[0]);
}

/*
 * Right-hand side on the theta-grid: d/dt of C(t, theta_j t) and
 * R(t, theta_j t) for the rows listed in `rows` (all rows if rows == NULL).
 *
 * For row j (t' = theta_j t) and quadrature node i, with the readings of
 * Sec. 3.3-3.4 (Jacobians theta_j and 1 - theta_j restored):
 *   a = (C,R)(t, theta_i theta_j t)     phi1 = theta_i theta_j
 *   b = (C,R)(t, phi t)                 phi  = theta_j + (1-theta_j) theta_i
 *   c = (C,R)(t', theta_i t')           row Hermite in t
 *   d = (C,R)(phi t, psi phi t)         psi  = theta_j / phi, 2-D stencil
 * and the DMFE at (t, t') and at the swapped arguments (t', t):
 *   d1C = -mu C + t[th S1 + th S2 + (1-th) S3] + beta0 f'(C(t,0)) C(t',0)
 *   d1R = -mu R + t (1-th) S4
 *   mu' = T + t th S9 + beta0 f'(C(t',0)) C(t',0)
 *   d2C = -mu' C + t[th S5 + th S6 + (1-th) S7] + 2T R + beta0 f'(C(t',0)) C(t,0)
 *   d2R =  mu' R - t (1-th) S8            (left-resolvent form of the R equation)
 *   dC/dt|_theta = d1C + th d2C,  dR/dt|_theta = d1R + th d2R.
 * Output rows not listed are left untouched.  sums9 (optional) receives the
 * nine sums per listed row as [row][9].  The diagonal row j = L-1 is returned
 * as computed (callers pin it).
 */
int or_theta_rhs(const or_model *m, const or_grid *g, const or_hist *H, double mu,
                 const int *rows, int nrows, double *outC, double *outR, double *sums9) {
    int L = g->L;
    int nr = rows ? nrows : L;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < nr; ++r) {
        int j = rows ? rows[r] : r;
        double thj = g->th[j], thcj = g->thc[j], t = H->tcur, tp = thj * t;
        double S[9] = {0};
        for (int i = 0; i < L; ++i) {
            double thi = g->th[i], thci = g->thc[i], w = g->nu[i];
            double tha = thi * thj, thca = thci + thi * thcj;
            or_pt qa = {-1, or_xmap(g, tha, thca), tha, thca};
            double aC = row_at(g, H->yC, &qa, 0), aR = row_at(g, H->yR, &qa, g->log_r);
            double phi = thj + thcj * thi, phic = thcj * thci;
            or_pt qb = {-1, or_xmap(g, phi, phic), phi, phic};
            double bC = row_at(g, H->yC, &qb, 0), bR = row_at(g, H->yR, &qb, g->log_r);
            double cv[2];
            or_pt qc = {i, 0.0, thi, thci};
            or_hist_at(g, H, tp, &qc, cv);
            double psi = 0.0, psic = 1.0; /* psi = 0/0 := 0 at i = j = 0 */
            if (phi > 0.0) { psi = thj / phi; psic = thcj * thi / phi; }
            or_pt qd = {-1, or_xmap(g, psi, psic), psi, psic};
            double dv[2];
            or_hist_at(g, H, phi * t, &qd, dv);
            double cC = cv[0], cR = cv[1], dC = dv[0], dR = dv[1];
            S[0] += w * or_f2(m, aC) * aR * cC;
            S[1] += w * or_f1(m, aC) * cR;
            S[2] += w * or_f2(m, bC) * bR * dC;
            S[3] += w * or_f2(m, bC) * bR * dR;
            S[4] += w * or_f2(m, cC) * cR * aC;
            S[5] += w * or_f1(m, cC) * aR;
            S[6] += w * or_f1(m, dC) * bR;
            S[7] += w * bR * or_f2(m, dC) * dR;
            S[8] += w * (or_f2(m, cC) * cR * cC + or_f1(m, cC) * cR);
        }
        double c0[2];
        or_pt q0 = {0, 0.0, 0.0, 1.0};
        or_hist_at(g, H, tp, &q0, c0); /* C(t', 0) */
        double Ct0 = H->yC[0];            /* C(t, 0) */
        double Cj = H->yC[j], Rj = H->yR[j];
        double d1C = -mu * Cj + t * (thj * S[0] + thj * S[1] + thcj * S[2]) + m->beta0 * or_f1(m, Ct0) * c0[0];
        double d1R = -mu * Rj + t * thcj * S[3];
        double mup = m->T + t * thj * S[8] + m->beta0 * or_f1(m, c0[0]) * c0[0];
        double d2C = -mup * Cj + t * (thj * S[4] + thj * S[5] + thcj * S[6]) + 2.0 * m->T * Rj +
                     m->beta0 * or_f1(m, c0[0]) * Ct0;
        double d2R = mup * Rj - t * thcj * S[7];
        outC[j] = d1C + thj * d2C;
        outR[j] = d1R + thj * d2R;
        if (sums9)
            for (int q = 0; q < 9; ++q) sums9[(size_t)r * 9 + q] = S[q];
    }
    return 0;
}

/* Interpolated history value (C, R) at tau and the node, or at the point with
 * index x and theta th, 1 - theta = thc -- exported for tests. */
void or_hist_value(const or_grid *g, const or_hist *H, double tau, int node, double x, double th, double thc,
                   double *out2) {
    or_pt q = {node, x, th, thc};
    or_hist_at(g, H, tau, &q, out2);
}

/* ======================================================================
 * Sparsification (Sec. 3.6).
 * ====================================================================== */

/* Integral over [ta, tb] of the cubic Hermite interpolant through (ya, da), (yb, db). */
static double herm_int(double ta, double tb, double ya, double da, double yb, double db) {
    double h = tb - ta;
    return h * (ya + yb) / 2.0 + h * h * (da - db) / 12.0;
}

/*
 * eps_n = sum_i |Delta_n^C(theta_i)| + |Delta_n^R(theta_i)|, where Delta_n is
 * the integral over [t_{n-1}, t_{n+1}] of the Hermite interpolant with slice n
 * minus the one without it.  Computed for n = 1..M-2; eps[0] = eps[M-1] = -1.
 */
void or_sparsify_residuals(int M, int L, const double *t, const double *C, const double *R,
                           const double *dC, const double *dR, double *eps) {
    eps[0] = -1.0;
    if (M >= 1) eps[M - 1] = -1.0;
    for (int n = 1; n + 1 < M; ++n) {
        double e = 0.0;
        const double *vals[2] = {C, R}, *ders[2] = {dC, dR};
        for (int f = 0; f < 2; ++f) {
            const double *Y = vals[f], *Dd = ders[f];
            for (int i = 0; i < L; ++i) {
                size_t a = (size_t)(n - 1) * L + i, c = (size_t)n * L + i, b = (size_t)(n + 1) * L + i;
                double with = herm_int(t[n - 1], t[n], Y[a], Dd[a], Y[c], Dd[c]) +
                              herm_int(t[n], t[n + 1], Y[c], Dd[c], Y[b], Dd[b]);
                double without = herm_int(t[n - 1], t[n + 1], Y[a], Dd[a], Y[b], Dd[b]);
                e += fabs(with - without);
            }
        }
        eps[n] = e;
    }
}

/*
 * One greedy pass over candidates n = 1..last: drop n when eps[n] < thr and
 * continue at n+2, otherwise continue at n+1.  drop[n] = 1 for dropped slices.
 * Returns the number dropped.
 */
int or_sparsify_select(int M, int last, const double *eps, double thr, int *drop) {
    int cnt = 0;
    for (int n = 0; n < M; ++n) drop[n] = 0;
    int n = 1;
    while (n <= last) {
        if (eps[n] < thr) {
            drop[n] = 1;
            ++cnt;
            n += 2;
        } else {
            n += 1;
        }
    }
    return cnt;
}

/* ======================================================================
 * Adaptive driver (Sec. 3.5): DP5 until its stability boundary, then
 * SSPRK(10,4); 1-norm error; accept / x0.9 / x1.01 / revert-10-and-halve.
 * ====================================================================== */

typedef struct {
    int S;                 /* stages */
    double A[10][10], b[10], e[10], c[10]; /* e = b - bhat */
} or_tableau;

typedef struct {
    double eps, dt0, dt_min;
    double rho;            /* 4 sqrt(f''(1)) */
    double dp5_limit, ssp_limit;
    int M_cap;
    int auto_passes;
    const or_tableau *dp5, *ssp;
} or_adapt;

typedef struct {
    /* history: slots in logical order, capacity M_cap */
    double *t, *C, *R, *dC, *dR;
    int M, nb_last_valid; /* nb_last_valid unused in the oracle: stage 1 always recomputes */
    double dt;
    int scheme;           /* 0 = DP5, 1 = SSPRK(10,4) */
    int64_t accepted, rejected, reverts, removed, n_sparsify;
    double last_eps;
} or_state;

static void drop_slices(or_state *s, int L, const int *drop) {
    int w = 0;
    for (int n = 0; n < s->M; ++n) {
        if (drop[n]) continue;
        if (w != n) {
            s->t[w] = s->t[n];
            memcpy(s->C + (size_t)w * L, s->C + (size_t)n * L, sizeof(double) * L);
            memcpy(s->R + (size_t)w * L, s->R + (size_t)n * L, sizeof(double) * L);
            memcpy(s->dC + (size_t)w * L, s->dC + (size_t)n * L, sizeof(double) * L);
            memcpy(s->dR + (size_t)w * L, s->dR + (size_t)n * L, sizeof(double) * L);
        }
        ++w;
    }
    s->M = w;
}

/* One sparsification pass over the protected candidate range n = 1..M-12. */
int or_sparsify_pass(or_state *s, int L, double eps_tol) {
    int M = s->M;
    if (M < 13) return 0;
    double *eps = malloc(sizeof(double) * M);
    int *drop = malloc(sizeof(int) * M);
    or_sparsify_residuals(M, L, s->t, s->C, s->R, s->dC, s->dR, eps);
    int cnt = or_sparsify_select(M, M - 12, eps, eps_tol / 10.0, drop);
    drop_slices(s, L, drop);
    free(eps);
    free(drop);
    s->removed += cnt;
    s->n_sparsify += 1;
    return cnt;
}

/* status codes (same meaning as the product's, defined independently) */
#define OR_OK 0
#define OR_DONE 1
#define OR_CAPACITY (-3)
#define OR_UNDERFLOW (-4)
#define OR_NONFINITE (-5)

/*
 * Advance until t >= t_target or max_steps steps (accepted + rejected) have
 * been taken.  On entry s holds M >= 1 slices; slice M-1 is the state.
 */
int or_adaptive_run(const or_model *m, const or_grid *g, const or_adapt *ad, or_state *s,
                    double t_target, int64_t max_steps) {
    int L = g->L;
    double *y0 = malloc(sizeof(double) * 2 * L), *ys = malloc(sizeof(double) * 2 * L);
    double *k = malloc(sizeof(double) * 2 * L * 10);
    int status = OR_OK;
    for (int64_t step = 0; step < max_steps; ++step) {
        int M = s->M;
        double tn = s->t[M - 1];
        if (tn >= t_target) break;
        if (M >= ad->M_cap) {
            int got = 0;
            for (int p = 0; p < ad->auto_passes; ++p) got += or_sparsify_pass(s, L, ad->eps);
            if (got == 0) { status = OR_CAPACITY; break; }
            M = s->M;
        }
        const or_tableau *tb = s->scheme == 0 ? ad->dp5 : ad->ssp;
        double dt = s->dt;
        memcpy(y0, s->C + (size_t)(M - 1) * L, sizeof(double) * L);
        memcpy(y0 + L, s->R + (size_t)(M - 1) * L, sizeof(double) * L);
        for (int st = 0; st < tb->S; ++st) {
            for (int q = 0; q < 2 * L; ++q) {
                double acc = y0[q];
                for (int l = 0; l < st; ++l) acc += dt * tb->A[st][l] * k[(size_t)l * 2 * L + q];
                ys[q] = acc;
            }
            ys[L - 1] = 1.0;
            ys[2 * L - 1] = 1.0;
            double tst = tn + tb->c[st] * dt;
            or_hist H = {M, st == 0 ? M - 1 : M, s->t, s->C, s->R, s->dC, s->dR, tst, ys, ys + L};
            double mu, E;
            or_mu_energy(m, L, g->nu, tst, ys, ys + L, &mu, &E);
            double *kc = k + (size_t)st * 2 * L;
            or_theta_rhs(m, g, &H, mu, NULL, 0, kc, kc + L, NULL);
            kc[L - 1] = 0.0;
            kc[2 * L - 1] = 0.0;
            if (st == 0) { /* the stage-1 derivative is the stored d/dt of slice M-1 */
                memcpy(s->dC + (size_t)(M - 1) * L, kc, sizeof(double) * L);
                memcpy(s->dR + (size_t)(M - 1) * L, kc + L, sizeof(double) * L);
            }
        }
        double err = 0.0;
        for (int q = 0; q < 2 * L; ++q) {
            double acc = 0.0;
            for (int l = 0; l < tb->S; ++l) acc += tb->e[l] * k[(size_t)l * 2 * L + q];
            err += fabs(dt * acc);
        }
        s->last_eps = err;
        if (!isfinite(err)) { status = OR_NONFINITE; break; }
        if (err > 2.0 * ad->eps) {
            int nrev = M - 1 < 10 ? M - 1 : 10;
            s->M -= nrev;
            s->rejected += 1;
            s->reverts += 1;
            s->dt = 0.5 * dt;
        } else {
            for (int q = 0; q < 2 * L; ++q) {
                double acc = y0[q];
                for (int l = 0; l < tb->S; ++l) acc += dt * tb->b[l] * k[(size_t)l * 2 * L + q];
                ys[q] = acc;
            }
            ys[L - 1] = 1.0;
            ys[2 * L - 1] = 1.0;
            int n = s->M;
            s->t[n] = tn + dt;
            memcpy(s->C + (size_t)n * L, ys, sizeof(double) * L);
            memcpy(s->R + (size_t)n * L, ys + L, sizeof(double) * L);
            memset(s->dC + (size_t)n * L, 0, sizeof(double) * L);
            memset(s->dR + (size_t)n * L, 0, sizeof(double) * L);
            s->M = n + 1;
            s->accepted += 1;
            if (err > ad->eps) s->dt = 0.9 * dt;
            else if (err < 0.5 * ad->eps) s->dt = 1.01 * dt;
            if (s->scheme == 0 && s->dt * ad->rho >= ad->dp5_limit) {
                s->scheme = 1;
                s->dt *= 0.5;
            }
            if (s->scheme == 1 && s->dt * ad->rho > ad->ssp_limit) s->dt = ad->ssp_limit / ad->rho;
        }
        if (s->dt < ad->dt_min) { status = OR_UNDERFLOW; break; }
    }
    free(y0); free(ys); free(k);
    if (status == OR_OK && s->t[s->M - 1] >= t_target) status = OR_DONE;
    return status;
}

/* threads the OpenMP loops of this file use */
int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* struct sizes, so the Python side can check its ctypes mirrors */
int or_sizeof(int which) {
    switch (which) {
    case 0: return (int)sizeof(or_model);
    case 1: return (int)sizeof(or_grid);
    case 2: return (int)sizeof(or_hist);
    case 3: return (int)sizeof(or_tableau);
    case 4: return (int)sizeof(or_adapt);
    case 5: return (int)sizeof(or_state);
    }
    return -1;
}
