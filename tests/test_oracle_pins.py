"""Pins of the oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the exact
p = 2 solution, closed-form identities of the DMFE, the equilibrium solution,
exactness properties of the interpolation and quadrature rules, convergence
orders of the Runge-Kutta tableaux, and tiny brute-force cases.
"""
import numpy as np
import pytest

import oracle
import p2_exact as px


# ----------------------------------------------------------------------------- uniform solver
def _grid_err(h, T, tend=5.0, step=0.5):
    m = oracle.make_model({2: 1.0}, T=T)
    N = int(round(tend / h))
    Ct, Rt, E = oracle.uniform_solve(m, h, N)
    C = oracle.tri_to_dense(Ct, N)
    R = oracle.tri_to_dense(Rt, N)
    ex = px.WarmP2(T, tend) if T > 0 else None
    errs = []
    for a in np.arange(1, int(tend / step) + 1) * step:
        for b in np.arange(0, int(a / step) + 1) * step:
            n, k = int(round(a / h)), int(round(b / h))
            if T == 0:
                ce, re_ = px.C0(a, b), px.R0(a, b)
            else:
                ce, re_ = ex.C(a, b), ex.R(a, b)
            errs += [abs(C[n, k] - ce), abs(R[n, k] - re_)]
        n = int(round(a / h))
        errs.append(abs(E[n] - (px.E0(a) if T == 0 else ex.E(a))))
    return max(errs)


@pytest.mark.parametrize("T", [0.0, 0.5])
def test_uniform_second_order_against_p2_exact(T):
    """Uniform scheme vs the exact p = 2 solution: O(h^2), ratio ~4 per halving."""
    e1 = _grid_err(0.05, T)
    e2 = _grid_err(0.025, T)
    assert e2 < 1e-4
    assert 3.5 < e1 / e2 < 4.6


def test_uniform_diagonal_identities():
    """C(t,t) = R(t,t^-) = 1 are stored, and d_1 C(t, t^-) = -T at the first stage."""
    m = oracle.make_model({3: 1.0}, T=0.5)
    h, N = 0.05, 60
    Ct, Rt, E = oracle.uniform_solve(m, h, N)
    C = oracle.tri_to_dense(Ct, N)
    R = oracle.tri_to_dense(Rt, N)
    assert np.all(np.diag(C) == 1.0) and np.all(np.diag(R) == 1.0)
    for n in (1, 17, 60):
        c, r = C[n, : n + 1], R[n, : n + 1]
        dc, dr = oracle.uniform_rhs(m, n, h, 0.0, Ct, Rt, c, r)
        assert abs(dc[n] + 0.5) < 1e-12
    # causality / R jump: (R(t_{n+1}, t_n) - 1)/h ~ -mu(t_n), mu from its definition
    assert np.all(R[1:, :] [np.tril_indices(N, -1)] < 1.0 + 1e-12)


def test_uniform_equilibrium_start():
    """beta0 = 1/T above T_d: E = -f(1)/T, C depends on t - t' only, R = -dC/dtau / T,
    each to O(h^2)."""
    T = 1.0
    m = oracle.make_model({3: 1.0}, T=T, beta0=1.0 / T)
    out = []
    for h in (0.05, 0.025):
        N = int(round(5.0 / h))
        Ct, Rt, E = oracle.uniform_solve(m, h, N)
        C = oracle.tri_to_dense(Ct, N)
        R = oracle.tri_to_dense(Rt, N)
        eE = np.max(np.abs(E - (-oracle.f(m, 1.0) / T)))
        d = int(round(1.0 / h))
        eS = max(abs(C[N, k] - C[N - d, k - d]) for k in range(d, N, d // 2))
        # FDT: R(tau) ~ -(C(tau + h) - C(tau - h)) / (2 h T) (second-order difference)
        eF = max(abs(R[N, k] + (C[N, k - 1] - C[N, k + 1]) / (2 * h) / T) for k in range(N // 2, N - 1, 3))
        out.append((eE, eS, eF))
    for a, b in zip(out[0], out[1]):
        assert 3.3 < a / b < 4.8
    assert out[1][0] < 3e-4 and out[1][1] < 6e-5 and out[1][2] < 3e-3


# ----------------------------------------------------------------------------- theta grid
@pytest.mark.parametrize("tmax,gam", [(50.0, 5.642), (1e2, 6.473), (1e4, 11.667), (1e6, 16.627), (1e7, 19.066)])
def test_gamma_lambert(tmax, gam):
    g = oracle.gamma_of(tmax)
    assert abs(g * np.exp(-g) * tmax - 1.0) < 1e-13
    assert abs(g - gam) < 1e-3


def _theta_naive_ld(L, g, i):
    """eq. (theta) at alpha = 0 evaluated literally in extended precision."""
    ld = np.longdouble
    y = ld(2 * (i + 1) - 1 - L) / ld(L - 1)
    G = ld(g)
    num = np.arctan(np.exp(G)) - np.arctan(np.exp(-G * y))
    den = np.arctan(np.exp(G)) - np.arctan(np.exp(-G))
    return num / den


@pytest.mark.parametrize("L,tmax", [(64, 1e4), (512, 1e2), (4096, 1e7)])
def test_theta_grid_matches_definition(L, tmax):
    th, thc = oracle.theta_grid(L, tmax)
    g = oracle.gamma_of(tmax)
    assert th[0] == 0.0 and th[-1] == 1.0
    assert np.all(np.diff(th) > 0)
    idx = np.unique(np.r_[np.arange(0, L, max(1, L // 97)), L - 1, 1, 2])
    for i in idx:
        ref = _theta_naive_ld(L, g, int(i))
        # relative agreement where the literal form is well conditioned
        assert abs(th[i] - float(ref)) <= 5e-15 * abs(float(ref)) + 4e-18
        assert abs(th[i] + thc[i] - 1.0) <= 2.3e-16
    # the grid condition: min spacing * t_max ~ 4 / (pi (L - 1))
    md = np.min(np.diff(th)) * tmax
    assert 0.5 < md / (4.0 / (np.pi * (L - 1))) < 1.5


@pytest.mark.parametrize("L,tmax", [(64, 1e4), (4096, 1e7)])
def test_index_map_inverts_grid(L, tmax):
    th, thc = oracle.theta_grid(L, tmax)
    for i in range(0, L, max(1, L // 211)):
        x = oracle.index_of(L, tmax, th[i], thc[i])
        assert abs(x - i) < 1e-11 * L
    # random points: forward definition (extended precision) of x(theta) returns theta
    rng = np.random.default_rng(1)
    g = oracle.gamma_of(tmax)
    for th_t in rng.uniform(0, 1, 20):
        x = oracle.index_of(L, tmax, th_t, 1.0 - th_t)
        ld = np.longdouble
        y = (2 * ld(x) + 1 - L) / ld(L - 1)
        G = ld(g)
        back = (np.arctan(np.exp(G)) - np.arctan(np.exp(-G * y))) / (np.arctan(np.exp(G)) - np.arctan(np.exp(-G)))
        assert abs(float(back) - th_t) < 1e-13


@pytest.mark.parametrize("L,tmax", [(64, 1e4), (300, 1e2), (2048, 1e4)])
def test_quadrature_weights_exact_on_quintics(L, tmax):
    th, _ = oracle.theta_grid(L, tmax)
    nu = oracle.quad_weights(th)
    assert abs(nu.sum() - 1.0) < 1e-13
    for k in range(1, 6):
        assert abs(nu @ th ** k - 1.0 / (k + 1)) < 1e-13
    if L == 64:
        assert abs(nu @ th ** 6 - 1.0 / 7) > 1e-12  # quintic, not sextic


def test_quadrature_converges_on_smooth_function():
    from scipy.integrate import quad
    ref = quad(lambda x: np.exp(np.sin(3 * x)), 0.0, 1.0, epsabs=1e-15, epsrel=1e-15)[0]
    errs = []
    for L in (64, 128, 256):
        th, _ = oracle.theta_grid(L, 1e2)
        nu = oracle.quad_weights(th)
        errs.append(abs(nu @ np.exp(np.sin(3 * th)) - ref))
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 1e-8


# ----------------------------------------------------------------------------- interpolation
def _empty_hist(L):
    return np.zeros(1), np.ones((1, L)), np.ones((1, L)), np.zeros((1, L)), np.zeros((1, L))


def test_index_lagrange_reproduces_polynomials():
    """s-point index Lagrange is exact on polynomials of degree s-1 in the index."""
    L, s = 64, 10
    ts = oracle.ThetaSetup(L, 1e4, s=s)
    rng = np.random.default_rng(2)
    coef = rng.normal(size=s)
    idx = np.arange(L) / L
    yC = np.polyval(coef, idx)
    yR = np.polyval(coef[::-1], idx)
    t_h, C, R, dC, dR = _empty_hist(L)
    for x in np.r_[rng.uniform(0, L - 1, 30), 0.0, L - 1.0, 3.5, L - 1.5]:
        v = oracle.hist_value(ts, t_h, C, R, dC, dR, 0, 0.0, yC, yR, 0.0, -1, x)
        assert abs(v[0] - np.polyval(coef, x / L)) < 1e-11
        assert abs(v[1] - np.polyval(coef[::-1], x / L)) < 1e-11
    # degree s is not reproduced
    yC = (idx - 0.5) ** s * L ** 2
    v = oracle.hist_value(ts, t_h, C, R, dC, dR, 0, 0.0, yC, yC, 0.0, -1, 30.5)
    assert abs(v[0] - (30.5 / L - 0.5) ** s * L ** 2) > 1e-12


def test_hermite_in_t_exact_on_cubics_and_quadratic_in_step():
    L = 40
    ts = oracle.ThetaSetup(L, 1e3)
    rng = np.random.default_rng(3)
    cf = rng.normal(size=(4, L))  # per-node cubic in t
    p = lambda t: cf[0] + cf[1] * t + cf[2] * t ** 2 + cf[3] * t ** 3
    dp = lambda t: cf[1] + 2 * cf[2] * t + 3 * cf[3] * t ** 2
    times = np.array([0.0, 0.3, 0.7, 1.6, 2.0, 2.9])
    C = np.array([p(t) for t in times])
    dC = np.array([dp(t) for t in times])
    R, dR = 2 * C, 2 * dC
    t = 3.4
    for tau in (0.0, 0.1, 0.7, 1.2, 2.0, 2.5, 2.9):
        for node in (0, 7, 39):
            v = oracle.hist_value(ts, times, C, R, dC, dR, times.size, t, p(t), 2 * p(t), tau, node)
            assert abs(v[0] - p(tau)[node]) < 1e-12 * (1 + abs(p(tau)[node]))
            assert abs(v[1] - 2 * p(tau)[node]) < 1e-12 * (1 + abs(p(tau)[node]))
    # inside the step: the quadratic through (y, y') at the last slice and y at t
    q = lambda t: cf[0] + cf[1] * t + cf[2] * t ** 2
    dq = lambda t: cf[1] + 2 * cf[2] * t
    Cq = np.array([q(x) for x in times])
    dCq = np.array([dq(x) for x in times])
    for tau in (2.95, 3.1, 3.4):
        v = oracle.hist_value(ts, times, Cq, Cq, dCq, dCq, times.size, t, q(t), q(t), tau, 11)
        assert abs(v[0] - q(tau)[11]) < 1e-12 * (1 + abs(q(tau)[11]))


# ----------------------------------------------------------------------------- theta-grid RHS
def _p2_history(ts, times):
    th = ts.th
    C = np.array([px.C0(t, th * t) for t in times])
    R = np.array([px.R0(t, th * t) for t in times])
    dC, dR = [], []
    for t in times:
        a, b = px.dC0(t, th * t)
        dC.append(a + th * b)
        a, b = px.dR0(t, th * t)
        dR.append(a + th * b)
    C[:, -1] = 1.0
    R[:, -1] = 1.0
    return C, R, np.array(dC), np.array(dR)


def test_theta_rhs_converges_to_p2_exact_derivative():
    """E5-style diagnostic: on an exact p = 2 history the RHS along fixed theta
    converges to the exact d/dt C(t, theta t), d/dt R(t, theta t) as L grows."""
    m = oracle.make_model({2: 1.0}, T=0.0)
    t = 8.0
    errs = []
    for L in (32, 64, 128):
        ts = oracle.ThetaSetup(L, 1e3)
        times = np.concatenate([[0.0], np.geomspace(1e-3, t - 0.0125, 799)])
        C, R, dC, dR = _p2_history(ts, times)
        yC = px.C0(t, ts.th * t)
        yR = px.R0(t, ts.th * t)
        yC[-1] = yR[-1] = 1.0
        oc, orr, mu, _ = oracle.theta_rhs(m, ts, times, C, R, dC, dR, times.size, t, yC, yR)
        a, b = px.dC0(t, ts.th * t)
        exC = a + ts.th * b
        a, b = px.dR0(t, ts.th * t)
        exR = a + ts.th * b
        errs.append(max(np.abs(oc - exC)[:-1].max(), np.abs(orr - exR)[:-1].max()))
        # diagonal identities: d/dt C(t,t) = d/dt R(t,t^-) = 0
        assert abs(oc[-1]) < 1e-13 and abs(orr[-1]) < 1e-13
        assert abs(mu - px.mu0(t)) < 1e-4
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 5
    assert errs[2] < 2e-7


@pytest.mark.parametrize("beta0", [0.0, 0.7])
def test_theta_rhs_at_t0(beta0):
    """At t = 0 every integral vanishes: dC/dt = -T(1-theta), dR/dt = -mu(0)(1-theta),
    mu(0) = T + beta0 f'(1)."""
    m = oracle.make_model({3: 0.5, 4: 0.5}, T=0.6, beta0=beta0)
    L = 48
    ts = oracle.ThetaSetup(L, 1e4)
    one = np.ones(L)
    oc, orr, mu, _ = oracle.theta_rhs(m, ts, np.zeros(1), one[None], one[None], 0 * one[None], 0 * one[None],
                                      0, 0.0, one, one)
    mu0 = 0.6 + beta0 * oracle.f1(m, 1.0)
    assert abs(mu - mu0) < 1e-15
    assert np.max(np.abs(oc - (-0.6 * ts.thc))) < 1e-14
    assert np.max(np.abs(orr - (-mu0 * ts.thc))) < 1e-14


def test_theta_rhs_first_stage_d1C_is_minus_T():
    """On any smooth history, d_1 C(t, t^-) = -T: row L-1 gives d1C + d2C = 0 and
    the sums of that row reproduce mu(t) - T."""
    m = oracle.make_model({2: 0.3, 4: 0.7}, T=0.45)
    L = 64
    ts = oracle.ThetaSetup(L, 1e4)
    times = np.array([0.0, 0.5, 1.1, 1.8, 2.6])
    rng = np.random.default_rng(5)
    base = np.exp(-np.outer(times, ts.thc))  # C ~ exp(-(t - t'))
    C = base.copy()
    R = base * (1 + 0.05 * rng.uniform(size=base.shape))
    C[:, -1] = R[:, -1] = 1.0
    dC = -ts.thc * base
    dR = -ts.thc * base
    t = 3.0
    yC = np.exp(-t * ts.thc)
    yR = yC.copy()
    oc, orr, mu, S = oracle.theta_rhs(m, ts, times, C, R, dC, dR, times.size, t, yC, yR,
                                      rows=[L - 1], want_sums=True)
    assert abs(oc[-1]) < 1e-13 and abs(orr[-1]) < 1e-13
    # row L-1: t (S1 + S2) = t S9 = mu - T
    assert abs(t * (S[0, 0] + S[0, 1]) - (mu - 0.45)) < 1e-13
    assert abs(t * S[0, 8] - (mu - 0.45)) < 1e-13


# ----------------------------------------------------------------------------- sparsification
def test_sparsify_cubic_history_has_zero_residual():
    L = 16
    rng = np.random.default_rng(6)
    cf = rng.normal(size=(4, L))
    times = np.cumsum(rng.uniform(0.1, 0.5, 30))
    C = np.array([cf[0] + cf[1] * t + cf[2] * t ** 2 + cf[3] * t ** 3 for t in times])
    dC = np.array([cf[1] + 2 * cf[2] * t + 3 * cf[3] * t ** 2 for t in times])
    eps = oracle.sparsify_residuals(times, C, 2 * C, dC, 2 * dC)
    assert np.all(np.abs(eps[1:-1]) < 1e-11)
    n, drop = oracle.sparsify_select(eps, 30 - 12, 1e-9)
    assert list(np.flatnonzero(drop)) == list(range(1, 19, 2))
    # a quartic is not reproduced: residual = h^5/... nonzero
    C4 = np.array([t ** 4 * np.ones(L) for t in times])
    dC4 = np.array([4 * t ** 3 * np.ones(L) for t in times])
    eps4 = oracle.sparsify_residuals(times, C4, C4, dC4, dC4)
    # exact: with/without differ by the quartic error of Hermite integrals
    n1 = 5
    a, b, c = times[n1 - 1], times[n1], times[n1 + 1]
    hi = lambda x, y: (y - x) * (x ** 4 + y ** 4) / 2 + (y - x) ** 2 * (4 * x ** 3 - 4 * y ** 3) / 12
    ex = abs(hi(a, b) + hi(b, c) - hi(a, c))
    assert abs(eps4[n1] - 2 * L * ex) < 1e-9 * max(1.0, eps4[n1])
    assert eps4[n1] > 1e-6


def test_sparsify_greedy_rule_brute_force():
    # candidates 1..last; drop when below threshold, then skip the next one
    eps = np.array([-1, 0.1, 0.1, 0.1, 5.0, 0.1, 0.1, 5.0, 0.1, -1])
    n, drop = oracle.sparsify_select(eps, 8, 1.0)
    assert list(np.flatnonzero(drop)) == [1, 3, 5, 8]
    n, drop = oracle.sparsify_select(eps, 6, 1.0)
    assert list(np.flatnonzero(drop)) == [1, 3, 5]
    n, drop = oracle.sparsify_select(np.full(10, 3.0), 8, 1.0)
    assert n == 0


# ----------------------------------------------------------------------------- RK tableaux
def _local_orders(A, b, hs=(0.1, 0.05, 0.025)):
    """log2 ratios of one-step errors on a nonlinear non-autonomous 2-D system;
    a method of order p has local error ~ h^(p+1)."""
    import warnings
    from scipy.integrate import solve_ivp
    f = lambda t, y: np.array([-y[0] * y[1] + np.sin(3 * t), y[0] - 0.5 * y[1] ** 2 + np.cos(t)])
    y0 = np.array([0.3, 0.7])

    def one(h):
        k = []
        for i in range(b.size):
            yi = y0 + h * sum(A[i, j] * k[j] for j in range(i))
            k.append(f(h * A[i].sum(), yi))
        return y0 + h * sum(bj * kj for bj, kj in zip(b, k))

    errs = []
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        for h in hs:
            ref = solve_ivp(f, (0, h), y0, rtol=1e-14, atol=1e-16, method="DOP853").y[:, -1]
            errs.append(np.abs(one(h) - ref).max())
    return [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_rk_tableau_orders():
    A, b, bh, c = oracle.dp5_tableau()
    assert min(_local_orders(A, b)) > 5.8          # 5th order (local h^6)
    assert 4.8 < _local_orders(A, bh)[-1] < 5.6    # 4th order embedded
    A, b, bh, c = oracle.ssprk104_tableau()
    assert 4.8 < _local_orders(A, b)[-1] < 5.2     # 4th order
    assert 3.8 < _local_orders(A, bh)[-1] < 4.2    # 3rd order embedded
    assert np.all(bh >= 0) and bh[-1] == 0.0
    assert np.allclose(c, [0, 1 / 6, 2 / 6, 3 / 6, 4 / 6, 2 / 6, 3 / 6, 4 / 6, 5 / 6, 1])
    assert np.allclose(bh, [3 / 20, 1 / 12, 7 / 120, 3 / 40, 2 / 15, 7 / 120, 3 / 40, 2 / 15, 7 / 30, 0])


def test_stability_limits():
    A, b, _, _ = oracle.dp5_tableau()
    dp = oracle.stability_limit(A, b)
    A, b, _, _ = oracle.ssprk104_tableau()
    sp = oracle.stability_limit(A, b)
    assert 3.3065 <= dp < 3.3066 and oracle.DP5_LIMIT <= dp
    assert 13.917 <= sp < 13.918 and oracle.SSP_LIMIT <= sp


# ----------------------------------------------------------------------------- adaptive driver
def test_adaptive_grow_rule_and_switch():
    """With a loose tolerance every step is accepted and dt grows by 1.01 until the
    DP5 boundary, where it halves and SSPRK(10,4) takes over."""
    m = oracle.make_model({2: 1.0}, T=0.0)
    ts = oracle.ThetaSetup(64, 1e3)
    run = oracle.AdaptiveRun(m, ts, eps=1e3, dt0=0.3, dt_min=1e-12, M_cap=200)
    st = run.run(1e9, 40)
    assert run.st.rejected == 0 and run.st.accepted == 40
    rho = 4.0
    # dt0 * 1.01^k crosses 3.3065/4 = 0.8266 at k = 103, so still DP5 after 40 steps
    assert run.st.scheme == 0
    assert abs(run.st.dt - 0.3 * 1.01 ** 40) < 1e-12
    run2 = oracle.AdaptiveRun(m, ts, eps=1e3, dt0=0.82, dt_min=1e-12, M_cap=200)
    run2.run(1e9, 1)
    assert run2.st.scheme == 1 and abs(run2.st.dt - 0.5 * 0.82 * 1.01) < 1e-15


def test_adaptive_p2_energy_against_exact():
    m = oracle.make_model({2: 1.0}, T=0.0)
    ts = oracle.ThetaSetup(64, 1e3)
    run = oracle.AdaptiveRun(m, ts, eps=1e-8, dt0=1e-3, dt_min=1e-10, M_cap=4000)
    st = run.run(6.0, 100000)
    assert st == 1
    t, C, R, dC, dR = run.history()
    E = np.array([oracle.mu_energy(m, ts, tt, C[i], R[i])[1] for i, tt in enumerate(t)])
    err = np.abs(E - px.E0(t))
    assert err.max() < 2e-6
    # the diagonal stays pinned and the state is finite
    assert np.all(C[:, -1] == 1.0) and np.all(np.isfinite(C))


# ----------------------------------------------------------------------------- theta grid: equilibrium start
def _equilibrium_run(L):
    """Pure p = 3 (f = q^3/2) at T = 1 > T_d = 0.6124 started in equilibrium
    (beta0 = 1/T, Sec. 2.1 forcing term), solved on the theta grid to t = 6."""
    T = 1.0
    m = oracle.make_model({3: 1.0}, T=T, beta0=1.0 / T)
    ts = oracle.ThetaSetup(L, 1e4)
    run = oracle.AdaptiveRun(m, ts, eps=1e-8, dt0=1e-3, dt_min=1e-12, M_cap=4000)
    assert run.run(6.0, 100000) == 1
    return m, ts, run


def test_theta_equilibrium_start_is_stationary():
    """An equilibrium start stays in equilibrium (derived from Sec. 2.1 with
    beta0 = 1/T): E(t) = -f(1)/T and mu(t) = T + f'(1)/T at every stored slice,
    C(t, t - tau) independent of t, and the FDT R(tau) = -C'(tau)/T.  All four
    hold up to the discretisation error, which falls as L grows.  The forcing
    term F_C = beta0 f'(C(t,0)) C(t',0) enters only at t > 0, so this is the pin
    that tells C(t,0) from C(t',0)."""
    errs = []
    for L in (48, 96):
        m, ts, run = _equilibrium_run(L)
        t, C, R, dC, dR = run.history()
        mE = np.array([oracle.mu_energy(m, ts, tt, C[i], R[i]) for i, tt in enumerate(t)])
        eE = np.abs(mE[:, 1] + oracle.f(m, 1.0) / m.T).max()
        eM = np.abs(mE[:, 0] - m.T - oracle.f1(m, 1.0) / m.T).max()
        # stationarity: C and R at fixed tau = t - t' on every slice with t >= tau + 1/4
        eS = 0.0
        for tau in (0.5, 1.0, 2.0):
            vals = []
            for n in range(run.M):
                if t[n] < tau + 0.25:
                    continue
                thc = tau / t[n]
                x = oracle.index_of(L, 1e4, 1.0 - thc, thc)
                vals.append(oracle.hist_value(ts, t, C, R, dC, dR, run.M, t[-1], C[-1], R[-1], t[n], -1, x,
                                              1.0 - thc, thc))
            vals = np.array(vals)
            eS = max(eS, np.ptp(vals[:, 0]), np.ptp(vals[:, 1]))
        # FDT on the slice before the last (its stored d/dt along fixed theta is
        # C'(tau) (1 - theta) in equilibrium): R = -dC / ((1 - theta) T)
        n = run.M - 2
        tau = ts.thc * t[n]
        sel = (tau > 0.2) & (tau < 4.0)
        eF = np.abs(R[n, sel] + dC[n, sel] / (ts.thc[sel] * m.T)).max()
        errs.append((eE, eM, eS, eF))
    (e48, e96) = errs
    assert e96[0] < 3e-7 and e96[1] < 1e-6 and e96[2] < 3e-6 and e96[3] < 3e-5
    for a, b in zip(e48, e96):
        assert b < a / 8


# ----------------------------------------------------------------------------- sparsification pass
def _load_history(run, t, C, R, dC, dR):
    M = t.size
    run.t[:M], run.C[:M], run.R[:M], run.dC[:M], run.dR[:M] = t, C, R, dC, dR
    run.st.M = M


def test_sparsify_pass_range_threshold_and_compaction():
    """One pass of Sec. 3.6 through the oracle's driver state: candidates are
    n = 1..M-12 (the first slice and the revert window of the last eleven are
    kept), a slice goes when its residual is below eps/10 and the next candidate
    is then skipped, and the kept slices are compacted in order.

    History quartic in t on a uniform grid: every residual equals the closed
    form 1.5 L |H[a,b] + H[b,c] - H[a,c]| of the Hermite integrals of t^4 (C
    = t^4 and R = C/2 at each of the L nodes), so a threshold 1% above it drops exactly 1, 3, ..., 17 of
    M = 30 slices and one 1% below drops none; a cubic history drops the same
    slices at any tolerance."""
    L, M = 16, 30
    m = oracle.make_model({2: 1.0}, T=0.0)
    ts = oracle.ThetaSetup(L, 1e3)
    times = 0.3 * np.arange(M)
    one = np.ones(L)
    C = np.array([tt ** 4 * one for tt in times])
    dC = np.array([4 * tt ** 3 * one for tt in times])
    hi = lambda x, y: (y - x) * (x ** 4 + y ** 4) / 2 + (y - x) ** 2 * (4 * x ** 3 - 4 * y ** 3) / 12
    res = 1.5 * L * abs(hi(times[0], times[1]) + hi(times[1], times[2]) - hi(times[0], times[2]))
    assert res > 0
    kept = [n for n in range(M) if not (n % 2 == 1 and n <= 17)]
    for factor, expect in ((1.01, kept), (0.99, list(range(M)))):
        run = oracle.AdaptiveRun(m, ts, eps=10.0 * res * factor, dt0=1e-3, dt_min=1e-12, M_cap=64)
        _load_history(run, times, C, 0.5 * C, dC, 0.5 * dC)
        removed = run.sparsify(1)
        assert removed == M - len(expect)
        assert run.M == len(expect) and run.st.removed == removed and run.st.n_sparsify == 1
        t2, C2, R2, dC2, dR2 = run.history()
        assert np.array_equal(t2, times[expect])
        assert np.array_equal(C2, C[expect]) and np.array_equal(dR2, 0.5 * dC[expect])
    # cubic history: zero residual everywhere, the same greedy selection
    rng = np.random.default_rng(11)
    cf = rng.normal(size=(4, L))
    tt = np.cumsum(rng.uniform(0.1, 0.4, M))
    C3 = np.array([cf[0] + cf[1] * x + cf[2] * x ** 2 + cf[3] * x ** 3 for x in tt])
    dC3 = np.array([cf[1] + 2 * cf[2] * x + 3 * cf[3] * x ** 2 for x in tt])
    run = oracle.AdaptiveRun(m, ts, eps=1e-9, dt0=1e-3, dt_min=1e-12, M_cap=64)
    _load_history(run, tt, C3, C3, dC3, dC3)
    assert run.sparsify(1) == 9
    assert np.array_equal(run.history()[0], tt[kept])
    # a short history has no candidates
    run = oracle.AdaptiveRun(m, ts, eps=1.0, dt0=1e-3, dt_min=1e-12, M_cap=64)
    _load_history(run, tt[:12], C3[:12], C3[:12], dC3[:12], dC3[:12])
    assert run.sparsify(1) == 0 and run.M == 12


# ----------------------------------------------------------------------------- controller: reject and revert
def _scripted_state(M):
    """A p = 2 history of M slices from the oracle's own driver (loose tolerance,
    every step accepted), then a step of dt = 0.5 from it."""
    m = oracle.make_model({2: 1.0}, T=0.0)
    ts = oracle.ThetaSetup(32, 1e3)
    run = oracle.AdaptiveRun(m, ts, eps=1e3, dt0=0.05, dt_min=1e-12, M_cap=64)
    run.run(1e9, M - 1)
    assert run.M == M and run.st.rejected == 0
    return m, ts, run.history()


def _step_once(m, ts, hist, eps, dt):
    t, C, R, dC, dR = hist
    run = oracle.AdaptiveRun(m, ts, eps=eps, dt0=dt, dt_min=1e-12, M_cap=64)
    _load_history(run, t, C, R, dC, dR)
    run.st.dt = dt
    run.run(1e9, 1)
    return run


@pytest.mark.parametrize("M", [15, 5])
def test_controller_bands_and_revert(M):
    """Sec. 3.5 on one scripted step whose error estimate eps_RK is fixed by the
    state and dt alone (not by the tolerance): eps_RK > 2 eps rejects, drops the
    last min(10, M-1) slices, halves dt and leaves the kept slices untouched;
    eps < eps_RK <= 2 eps accepts with dt x 0.9; eps/2 <= eps_RK <= eps accepts
    with dt unchanged; eps_RK < eps/2 accepts with dt x 1.01."""
    m, ts, hist = _scripted_state(M)
    dt = 0.5  # DP5 boundary at dt 4 = 3.3065 is not reached by 1.01 dt
    probe = _step_once(m, ts, hist, 1e3, dt)
    e_rk = probe.st.last_eps
    assert e_rk > 0 and probe.st.accepted == 1 and probe.M == M + 1
    nrev = min(10, M - 1)
    run = _step_once(m, ts, hist, e_rk / 3.0, dt)
    assert run.st.last_eps == e_rk
    assert run.st.rejected == 1 and run.M == M - nrev and run.st.dt == 0.5 * dt
    t2, C2, R2, dC2, dR2 = run.history()
    k = M - nrev
    assert np.array_equal(t2, hist[0][:k]) and np.array_equal(C2, hist[1][:k]) and np.array_equal(R2, hist[2][:k])
    assert np.array_equal(dC2[: k - 1], hist[3][: k - 1]) and np.array_equal(dR2[: k - 1], hist[4][: k - 1])
    for eps, factor in ((e_rk / 1.5, 0.9), (e_rk / 0.8, 1.0), (e_rk * 3.0, 1.01)):
        run = _step_once(m, ts, hist, eps, dt)
        assert run.st.rejected == 0 and run.M == M + 1 and run.st.scheme == 0
        assert run.st.dt == factor * dt if factor != 1.0 else run.st.dt == dt
        assert run.t[M] == hist[0][-1] + dt
    # the band edge 2 eps itself is accepted
    run = _step_once(m, ts, hist, e_rk / 2.0, dt)
    assert run.st.rejected == 0 and run.st.dt == 0.9 * dt
