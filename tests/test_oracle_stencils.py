"""Pins of the oracle's alternative theta-stencils (Sec. 3.3) and of the log-R
option (Appendix A), against facts fixed independently of the oracle:
scipy's barycentric polynomial interpolator, the closed-form Floater-Hormann
weights on equispaced nodes, exact reproduction of the function classes each
scheme is exact on, and the fallback rule.

The oracle evaluates Floater-Hormann interpolation from its definition (a blend
of local polynomials) and Lagrange interpolation from the product formula; the
checks below use the barycentric form or a library routine instead.
"""
import numpy as np
import pytest

import oracle
import p2_exact as px

from scipy.interpolate import BarycentricInterpolator

KINDS = [oracle.INDEX_LAGRANGE, oracle.THETA_LAGRANGE, oracle.INDEX_FH, oracle.THETA_FH]


def _base(x, s, L):
    return int(min(max(int(np.floor(x)) - (s - 1) // 2, 0), L - s))


def _at(ts, row_c, row_r, x, th=None, thc=None):
    """theta-interpolation of a slice alone (the stage slice, nb = 0)."""
    L = ts.L
    z = np.zeros((1, L))
    return oracle.hist_value(ts, np.zeros(1), z, z, z, z, 0, 0.0, row_c, row_r, 0.0, -1, x, th, thc)


def _targets(rng, L, n):
    xs = list(rng.uniform(0.0, L - 1.0, n)) + [0.25, 1.5, L - 1.75, L / 2 - 0.5]
    return [x for x in xs if abs(x - round(x)) > 1e-6]


# ----------------------------------------------------------------------------- Lagrange on theta
@pytest.mark.parametrize("s", [6, 10])
def test_theta_lagrange_matches_scipy_barycentric(s):
    L = 64
    ts = oracle.ThetaSetup(L, 50.0, s=s, interp=oracle.THETA_LAGRANGE)
    rng = np.random.default_rng(11 + s)
    vc = np.sin(7 * ts.th) + rng.normal(scale=0.1, size=L)
    vr = np.cos(5 * ts.th) + rng.normal(scale=0.1, size=L)
    for x in _targets(rng, L, 25):
        th, thc = oracle.theta_at_index(ts, x)
        b = _base(x, s, L)
        nodes = ts.th[b:b + s]
        got = _at(ts, vc, vr, x, th, thc)
        for k, v in enumerate((vc, vr)):
            ref = BarycentricInterpolator(nodes, v[b:b + s])(th)
            assert abs(got[k] - ref) <= 1e-11 * (1 + np.abs(v[b:b + s]).max()), (x, k)


def _scaled_poly_rows(ts, x, s, deg, rng):
    """Data that varies on the scale of the stencil of x: q(z/z0) with z = theta
    (lower half) or 1 - theta (upper half) and z0 its largest value on the
    stencil, q a random polynomial of degree deg; also the exact value at x."""
    b = _base(x, s, ts.L)
    coef = rng.normal(size=deg + 1)
    th, thc = oracle.theta_at_index(ts, x)
    if th <= 0.5:
        z, zt = ts.th, th
    else:
        z, zt = ts.thc, thc
    z0 = np.abs(z[b:b + s]).max()
    row = np.polyval(coef, z / z0)
    return row, np.polyval(coef, zt / z0), th, thc


@pytest.mark.parametrize("interp,deg", [(oracle.THETA_LAGRANGE, 9), (oracle.THETA_FH, 3)])
def test_theta_schemes_reproduce_polynomials_at_clustered_ends(interp, deg):
    """At t_max = 1e7 the nodes next to theta = 0 and theta = 1 are ~1e-10 apart.
    Polynomials in theta of degree s-1 (Lagrange) or d (Floater-Hormann) are
    reproduced to rounding when the data vary on the stencil's scale; a theta
    difference formed from the rounded theta near 1, instead of from 1 - theta,
    loses ~7 digits and fails this."""
    L, s = 256, 10
    ts = oracle.ThetaSetup(L, 1e7, s=s, interp=interp, fh_d=3)
    rng = np.random.default_rng(5 + interp)
    for x in (0.3, 2.6, 4.5, 7.2, 60.4, L - 8.3, L - 4.5, L - 2.6, L - 1.3):
        row, exact, th, thc = _scaled_poly_rows(ts, x, s, deg, rng)
        got = _at(ts, row, row, x, th, thc)
        scale = 1 + np.abs(row[_base(x, s, L):_base(x, s, L) + s]).max()
        assert abs(got[0] - exact) <= 1e-10 * scale, (x, got[0], exact)


# ----------------------------------------------------------------------------- Floater-Hormann
# |w_k| of the barycentric form on 8 equispaced nodes (n = 7) for d = 0..3; the
# signs alternate.  (Sum over the windows containing k of binomial(d, k - i).)
_FH_EQUI_8 = {
    0: [1, 1, 1, 1, 1, 1, 1, 1],
    1: [1, 2, 2, 2, 2, 2, 2, 1],
    2: [1, 3, 4, 4, 4, 4, 3, 1],
    3: [1, 4, 7, 8, 8, 7, 4, 1],
}


@pytest.mark.parametrize("d", [0, 1, 2, 3])
def test_index_fh_equals_barycentric_form_with_equispaced_weights(d):
    L, s = 48, 8
    ts = oracle.ThetaSetup(L, 1e3, s=s, interp=oracle.INDEX_FH, fh_d=d)
    rng = np.random.default_rng(20 + d)
    vc = rng.normal(size=L)
    vr = np.exp(rng.normal(size=L))
    w = np.array(_FH_EQUI_8[d], dtype=float) * (-1.0) ** np.arange(s)
    for x in _targets(rng, L, 30):
        b = _base(x, s, L)
        u = x - b
        c = w / (u - np.arange(s))
        got = _at(ts, vc, vr, x)
        for k, v in enumerate((vc, vr)):
            ref = np.dot(c, v[b:b + s]) / c.sum()
            assert abs(got[k] - ref) <= 1e-12 * (1 + np.abs(v[b:b + s]).max()), (d, x, k)


@pytest.mark.parametrize("interp", [oracle.INDEX_FH, oracle.THETA_FH])
def test_fh_of_full_degree_is_the_polynomial_interpolant(interp):
    """d = s-1 leaves one window: the blend is the interpolating polynomial."""
    L, s = 64, 8
    ts = oracle.ThetaSetup(L, 50.0, s=s, interp=interp, fh_d=s - 1)
    rng = np.random.default_rng(31 + interp)
    v = rng.normal(size=L)
    for x in _targets(rng, L, 20):
        b = _base(x, s, L)
        th, thc = oracle.theta_at_index(ts, x)
        nodes, tgt = (np.arange(b, b + s, dtype=float), x) if interp == oracle.INDEX_FH else (ts.th[b:b + s], th)
        ref = BarycentricInterpolator(nodes, v[b:b + s])(tgt)
        got = _at(ts, v, v, x, th, thc)
        assert abs(got[0] - ref) <= 1e-11 * (1 + np.abs(v[b:b + s]).max())


@pytest.mark.parametrize("d", [1, 3, 5])
def test_index_fh_reproduces_degree_d_and_converges_at_order_d_plus_1(d):
    L, s = 400, 10
    ts = oracle.ThetaSetup(L, 1e3, s=s, interp=oracle.INDEX_FH, fh_d=d)
    rng = np.random.default_rng(40 + d)
    coef = rng.normal(size=d + 1)
    idx = np.arange(L, dtype=float)
    row = np.polyval(coef, idx / 7.0)
    for x in _targets(rng, L, 15):
        got = _at(ts, row, row, x)
        assert abs(got[0] - np.polyval(coef, x / 7.0)) <= 1e-11 * (1 + np.abs(row).max() / 1e3)
    # a smooth non-polynomial sampled at spacing h: the error falls like h^(d+1)
    errs = []
    for h in (0.08, 0.04):
        f = np.sin(idx * h)
        xs = np.arange(100.3, 300.0, 7.1)
        errs.append(max(abs(_at(ts, f, f, x)[0] - np.sin(x * h)) for x in xs))
    rate = np.log2(errs[0] / errs[1])
    assert rate > d + 0.5, (errs, rate)


# ----------------------------------------------------------------------------- log R
def test_log_r_exact_on_exponentials_of_polynomials_in_theta():
    """log-R interpolation reproduces R = exp(q(index)) for q of degree s-1; plain
    interpolation of the same data does not.  C is untouched by the option."""
    L, s = 80, 10
    rng = np.random.default_rng(50)
    coef = rng.normal(size=s) * 0.5
    idx = np.arange(L) / L
    R = np.exp(3.0 * np.polyval(coef, idx) + 2.0 * idx)
    Cv = np.cos(9 * idx)
    lg = oracle.ThetaSetup(L, 1e3, s=s, log_r=True)
    pl = oracle.ThetaSetup(L, 1e3, s=s, log_r=False)
    worst_plain = 0.0
    for x in _targets(rng, L, 25):
        exact = np.exp(3.0 * np.polyval(coef, x / L) + 2.0 * x / L)
        a, b = _at(lg, Cv, R, x), _at(pl, Cv, R, x)
        assert abs(a[1] - exact) <= 1e-12 * exact
        assert a[0] == b[0]
        worst_plain = max(worst_plain, abs(b[1] - exact) / exact)
    assert worst_plain > 1e-9


def test_log_r_exact_on_exponential_cubics_in_t_and_quadratics_in_step():
    L = 24
    ts = oracle.ThetaSetup(L, 1e3, log_r=True)
    rng = np.random.default_rng(51)
    cf = rng.normal(size=(4, L)) * np.array([[1.0], [0.5], [0.2], [0.05]])
    lr = lambda t: cf[0] + cf[1] * t + cf[2] * t ** 2 + cf[3] * t ** 3
    dlr = lambda t: cf[1] + 2 * cf[2] * t + 3 * cf[3] * t ** 2
    times = np.array([0.0, 0.3, 0.7, 1.6, 2.0, 2.9])
    R = np.exp([lr(t) for t in times])
    dR = R * np.array([dlr(t) for t in times])
    C = np.ones_like(R)
    t = 3.4
    for tau in (0.0, 0.1, 0.7, 1.2, 2.0, 2.5, 2.9):
        for node in (0, 5, 23):
            v = oracle.hist_value(ts, times, C, R, C * 0, dR, times.size, t, np.ones(L), np.exp(lr(t)), tau, node)
            ex = np.exp(lr(tau)[node])
            assert abs(v[1] - ex) <= 1e-12 * ex, (tau, node)
    # inside the step: exp of the quadratic through (log R, (dR/dt)/R) at the last
    # slice and log R of the stage slice
    q = lambda t: cf[0] + cf[1] * t + cf[2] * t ** 2
    dq = lambda t: cf[1] + 2 * cf[2] * t
    Rq = np.exp([q(x) for x in times])
    dRq = Rq * np.array([dq(x) for x in times])
    for tau in (2.95, 3.1, 3.4):
        v = oracle.hist_value(ts, times, C, Rq, C * 0, dRq, times.size, t, np.ones(L), np.exp(q(t)), tau, 9)
        ex = np.exp(q(tau)[9])
        assert abs(v[1] - ex) <= 1e-12 * ex


def test_log_r_falls_back_to_plain_interpolation_on_non_positive_stencils():
    """One non-positive value in the values a target reads switches that target,
    and only that target, to plain interpolation of R."""
    L, s = 64, 10
    rng = np.random.default_rng(52)
    lg = oracle.ThetaSetup(L, 1e3, s=s, log_r=True)
    pl = oracle.ThetaSetup(L, 1e3, s=s, log_r=False)
    R = np.exp(rng.normal(size=L))
    R[30] = -0.2
    Cv = rng.normal(size=L)
    for x in (27.4, 30.0 + 0.3, 33.9, 36.2, 10.5, 50.5):
        a, b = _at(lg, Cv, R, x), _at(pl, Cv, R, x)
        touches = _base(x, s, L) <= 30 < _base(x, s, L) + s
        if touches:
            assert a[1] == b[1]
        else:
            assert a[1] != b[1]
    # in t: a non-positive R at one of the two bracketing slices
    times = np.array([0.0, 1.0, 2.0])
    Rh = np.exp(rng.normal(size=(3, L)))
    Rh[1, 7] = 0.0
    dRh = rng.normal(size=(3, L))
    Ch = rng.normal(size=(3, L))
    Rs = R + 3.0  # the stage slice, positive except at node 9
    Rs[9] = -1.0
    # (tau, node, falls back): slice 1 is the first of the bracket at tau = 1.4,
    # the second at tau = 0.6; tau = 2.3 is inside the step (slice 2 and the stage slice)
    for tau, node, same in ((1.4, 7, True), (0.6, 7, True), (1.4, 8, False), (0.6, 8, False),
                            (2.3, 9, True), (2.3, 8, False)):
        a = oracle.hist_value(lg, times, Ch, Rh, Ch, dRh, 3, 2.5, Cv, Rs, tau, node)
        b = oracle.hist_value(pl, times, Ch, Rh, Ch, dRh, 3, 2.5, Cv, Rs, tau, node)
        assert a[0] == b[0]
        assert (a[1] == b[1]) == same, (tau, node)


# ----------------------------------------------------------------------------- the right-hand side
def _along_theta(partials, th):
    """d/dt at fixed theta from the two partial derivatives."""
    d1, d2 = partials
    return d1 + th * d2


@pytest.mark.parametrize("interp,log_r", [(k, False) for k in KINDS] + [(oracle.INDEX_LAGRANGE, True)])
def test_theta_rhs_schemes_converge_to_p2_exact_derivative(interp, log_r):
    """On the exact p = 2 history every scheme's right-hand side converges to the
    exact d/dt C(t, theta t), d/dt R(t, theta t) as L grows (R > 0 here, so the
    log option interpolates log R everywhere)."""
    m = oracle.make_model({2: 1.0}, T=0.0)
    t = 8.0
    errs = []
    for L in (48, 96):
        ts = oracle.ThetaSetup(L, 1e3, s=10, interp=interp, fh_d=5, log_r=log_r)
        times = np.concatenate([[0.0], np.geomspace(1e-3, t - 0.0125, 799)])
        th = ts.th
        C = np.array([px.C0(x, th * x) for x in times])
        R = np.array([px.R0(x, th * x) for x in times])
        dC = np.array([_along_theta(px.dC0(x, th * x), th) for x in times])
        dR = np.array([_along_theta(px.dR0(x, th * x), th) for x in times])
        C[:, -1] = R[:, -1] = 1.0
        yC, yR = px.C0(t, th * t), px.R0(t, th * t)
        yC[-1] = yR[-1] = 1.0
        oc, orr, _, _ = oracle.theta_rhs(m, ts, times, C, R, dC, dR, times.size, t, yC, yR)
        a, b = px.dC0(t, th * t)
        exC = a + th * b
        a, b = px.dR0(t, th * t)
        exR = a + th * b
        errs.append(max(np.abs(oc - exC)[:-1].max(), np.abs(orr - exR)[:-1].max()))
    assert errs[1] < errs[0] / 3, errs
    assert errs[1] < 1e-4, errs
