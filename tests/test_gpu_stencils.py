"""Parity of the alternative theta-stencils (Sec. 3.3) and of the log-R option
(Appendix A) on the HIP path with the oracle, element by element, through the
C-ABI.  The oracle forms Floater-Hormann values from their definition as a
blend of local polynomials and Lagrange values from the product formula; the
kernels use the barycentric form with host-built coefficients.

Bars as for the default stencil: one right-hand-side evaluation within 1e-12
(FP64) or 2e-6 (FP32-comp) of |mu| + T + max|output|; adaptive runs with the
same accept/reject decisions and time grid, states within 1e-10 relative.
Histories are the smooth family of the default tests, or one whose R changes
sign, so that the log option meets stencils that fall back to plain R.
"""
import sys

import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
import paper_2604_06309_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu

# (scheme, fh_d, log_r)
SCHEMES = [
    (pk.INTERP_THETA_LAGRANGE, 3, False),
    (pk.INTERP_INDEX_FH, 3, False),
    (pk.INTERP_THETA_FH, 3, False),
    (pk.INTERP_INDEX_LAGRANGE, 3, True),
    (pk.INTERP_THETA_FH, 5, True),
]
IDS = ["theta-lagrange", "index-fh3", "theta-fh3", "index-lagrange-logR", "theta-fh5-logR"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pk.lib()
    yield
    torch.cuda.synchronize()


def _rhs(L, M, nb, t, seed, interp, fh_d, log_r, s=10, precision=pk.FP64, hist="smooth", tmax=1e4, rows=None,
         terms=None, T=0.6):
    terms = terms or {3: 0.5, 4: 0.5}
    p = pk.make_params(terms, T, t_max=tmax, L=L, M_cap=max(M + 4, 16), s=s, precision=precision,
                       theta_interp=interp, fh_d=fh_d, log_r=log_r)
    solver = pk.Solver(p)
    ts = oracle.ThetaSetup(L, tmax, s=s, interp=interp, fh_d=fh_d, log_r=log_r)
    m = oracle.make_model(terms, T=T)
    times = inputs.geometric_times(M, t * 0.97 if nb == M else t) if M > 1 else np.zeros(1)
    if hist == "sign":
        C, R, dC, dR = inputs.sign_changing_history(ts.th, times, seed)
        yC, yR = inputs.sign_changing_stage(ts.th, t, seed)
    else:
        C, R, dC, dR = inputs.smooth_history(ts.th, times, seed)
        yC, yR = inputs.smooth_stage(ts.th, t, seed)
    if nb == M - 1:
        dC[-1] = 0.0
        dR[-1] = 0.0
    solver.set_history(times, C, R, dC, dR, nb=max(nb, M - 1))
    gC, gR, gmu, gdiag = solver.rhs(t, torch.tensor(yC, device="cuda"), torch.tensor(yR, device="cuda"), nb)
    solver.close()
    oC, oR, omu, _ = oracle.theta_rhs(m, ts, times, C, R, dC, dR, nb, t, yC, yR, rows=rows)
    return gC.cpu().numpy(), gR.cpu().numpy(), gmu, gdiag, oC, oR, omu


def _check(gC, gR, gdiag, oC, oR, gmu, omu, bar, T=0.6, rows=None, mu_bar=1e-13):
    L = gC.size
    rows = np.arange(L) if rows is None else np.asarray(rows)
    reg = rows[rows < L - 1]
    for g, o, d in ((gC, oC, gdiag[0]), (gR, oR, gdiag[1])):
        scale = abs(omu) + T + np.max(np.abs(o[rows]))
        err = np.max(np.abs(g[reg] - o[reg]))
        say(f"  max error {err:.2e} (scale {scale:.3g}); diagonal {abs(d - o[L - 1]):.2e}")
        assert err <= bar * scale, (err, scale)
        assert abs(d - o[L - 1]) <= bar * scale
        assert g[L - 1] == 0.0
    assert abs(gmu - omu) <= mu_bar * max(1.0, abs(omu))


@pytest.mark.parametrize("scheme", SCHEMES, ids=IDS)
@pytest.mark.parametrize("L,M,nb,t,seed,hist", [
    (203, 45, 45, 11.0, 3, "smooth"),   # L ragged against rows per block and nodes per iteration
    (203, 45, 44, 11.0, 4, "sign"),     # first stage; R of both signs
    (96, 2, 1, 0.3, 5, "smooth"),       # one stored interval
    (96, 1, 1, 0.2, 6, "sign"),         # only t = 0 stored
    (64, 1, 0, 0.0, 7, "smooth"),       # t = 0
])
def test_scheme_rhs_parity(scheme, L, M, nb, t, seed, hist):
    interp, d, log_r = scheme
    say(f"scheme rhs parity interp={interp} d={d} log_r={log_r} L={L} M={M} nb={nb} t={t} hist={hist}")
    gC, gR, gmu, gdiag, oC, oR, omu = _rhs(L, M, nb, t, seed, interp, d, log_r, hist=hist)
    _check(gC, gR, gdiag, oC, oR, gmu, omu, 1e-12)


@pytest.mark.parametrize("scheme", SCHEMES, ids=IDS)
@pytest.mark.parametrize("nb_off,precision,bar", [(0, pk.FP64, 1e-12), (1, pk.FP64, 1e-12),
                                                  (0, pk.FP32_COMP, 2e-6)])
def test_scheme_more_slices_than_lds_holds_times_for(scheme, nb_off, precision, bar):
    """20000 stored slices: beyond the ~19K slice times that LDS holds, the history-integral kernel
    of every scheme reads them from global memory.  R changes sign, so the log-R schemes take both
    the log branch and the fallback.  Every row against the oracle."""
    interp, d, log_r = scheme
    L, M = 64, 20000
    say(f"scheme rhs with M={M} slices (times in global memory) interp={interp} d={d} log_r={log_r} "
        f"nb=M-{nb_off} precision={precision}")
    gC, gR, gmu, gdiag, oC, oR, omu = _rhs(L, M, M - nb_off, 50.0, 21, interp, d, log_r, precision=precision,
                                           hist="sign")
    _check(gC, gR, gdiag, oC, oR, gmu, omu, bar)


@pytest.mark.parametrize("interp,s,d,log_r", [
    (pk.INTERP_INDEX_LAGRANGE, 16, 0, False),   # the default scheme on the largest stencil
    (pk.INTERP_THETA_FH, 14, 9, False),         # a wider Floater-Hormann stencil of degree 9
    (pk.INTERP_INDEX_FH, 16, 9, True),
    (pk.INTERP_THETA_LAGRANGE, 4, 0, True),
])
def test_scheme_stencil_sizes(interp, s, d, log_r):
    say(f"scheme stencil sizes interp={interp} s={s} d={d} log_r={log_r}")
    gC, gR, gmu, gdiag, oC, oR, omu = _rhs(160, 40, 40, 9.0, 8, interp, d, log_r, s=s, hist="sign")
    _check(gC, gR, gdiag, oC, oR, gmu, omu, 1e-12)


@pytest.mark.parametrize("scheme", [SCHEMES[2], SCHEMES[4]], ids=[IDS[2], IDS[4]])
def test_scheme_fp32_history(scheme):
    interp, d, log_r = scheme
    say(f"scheme fp32 interp={interp} d={d} log_r={log_r}")
    gC, gR, gmu, gdiag, oC, oR, omu = _rhs(203, 45, 45, 11.0, 9, interp, d, log_r, precision=pk.FP32_COMP,
                                           hist="sign")
    _check(gC, gR, gdiag, oC, oR, gmu, omu, 2e-6)


@pytest.mark.parametrize("interp,s,d,log_r", [
    (pk.INTERP_THETA_FH, 14, 9, False),
    (pk.INTERP_INDEX_LAGRANGE, 10, 0, True),
])
def test_scheme_full_size_sampled_rows(interp, s, d, log_r):
    """The L = 4096 workload's steady state (M = 2500, t = 200.08) on sampled rows."""
    L, M = 4096, 2500
    rng = np.random.default_rng(L + M + interp)
    fixed = [0, 1, 7, 8, 63, 64, 65, L // 2 - 1, L // 2, L - 65, L - 2, L - 1]
    rows = np.unique(np.concatenate([fixed, rng.choice(np.arange(2, L - 2), 8, replace=False)])).astype(np.int32)
    say(f"scheme full size interp={interp} s={s} d={d} log_r={log_r} rows={rows.size}")
    terms, T, tmax, t = {3: 0.5, 4: 0.5}, 0.55, 1e7, 200.08
    p = pk.make_params(terms, T, t_max=tmax, L=L, M_cap=M, eps=1e-8, s=s, theta_interp=interp, fh_d=d, log_r=log_r)
    solver = pk.Solver(p)
    ts = oracle.ThetaSetup(L, tmax, s=s, interp=interp, fh_d=d, log_r=log_r)
    times = inputs.geometric_times(M, 200.0, t_first=0.01)
    C, R, dC, dR = inputs.smooth_history(ts.th, times, 44)
    yC, yR = inputs.smooth_stage(ts.th, t, 44)
    solver.set_history(times, C, R, dC, dR, nb=M)
    gC, gR, gmu, gdiag = solver.rhs(t, torch.tensor(yC, device="cuda"), torch.tensor(yR, device="cuda"), M)
    solver.close()
    oC, oR, omu, _ = oracle.theta_rhs(oracle.make_model(terms, T=T), ts, times, C, R, dC, dR, M, t, yC, yR,
                                      rows=rows)
    _check(gC.cpu().numpy(), gR.cpu().numpy(), gdiag, oC, oR, gmu, omu, 1e-12, T=T, rows=rows)


@pytest.mark.parametrize("scheme", [SCHEMES[2], SCHEMES[4]], ids=[IDS[2], IDS[4]])
def test_scheme_adaptive_parity(scheme):
    """A run through DP5 and the switch to SSPRK(10,4), with each scheme."""
    interp, d, log_r = scheme
    terms, T, L, M_cap, eps, t_end = {3: 0.5, 4: 0.5}, 0.6, 64, 400, 1e-8, 8.0
    say(f"scheme adaptive parity interp={interp} d={d} log_r={log_r}")
    ts = oracle.ThetaSetup(L, 1e4, interp=interp, fh_d=d, log_r=log_r)
    run = oracle.AdaptiveRun(oracle.make_model(terms, T=T), ts, eps=eps, dt0=1e-3, dt_min=1e-10, M_cap=M_cap)
    run.run(t_end, 100000)
    s = pk.Solver(pk.make_params(terms, T, t_max=1e4, L=L, M_cap=M_cap, eps=eps, dt0=1e-3, dt_min=1e-10,
                                 theta_interp=interp, fh_d=d, log_r=log_r))
    _, info = s.step(t_end)
    say(f"  oracle: M={run.M} acc={run.st.accepted} rej={run.st.rejected}; "
        f"gpu: M={info.M} acc={info.accepted} rej={info.rejected}")
    assert (info.accepted, info.rejected, info.M) == (run.st.accepted, run.st.rejected, run.M)
    t, C, R, _, _ = run.history()
    np.testing.assert_array_equal(s.read(pk.F_T_GRID), t)
    for name, f, ref in (("C", pk.F_C, C), ("R", pk.F_R, R)):
        g = s.read(f)
        err = np.max(np.abs(g - ref) / (np.abs(ref) + 1e-4))
        say(f"  {name}: worst scaled error {err:.2e}")
        assert np.all(np.abs(g - ref) <= 1e-10 * np.abs(ref) + 1e-14), name
    s.close()


def test_pool_admits_the_default_stencil_only():
    """The batched kernel serves the default stencil with at most 16384 stored slices."""
    say("pool: non-default stencils and larger histories refused")
    base = dict(t_max=1e4, L=64, M_cap=100, eps=1e-8)
    pool = pk.Pool(4 * pk.dmfe_footprint(pk.make_params({3: 1.0}, 0.5, **base)), max_instances=4)
    for kw in (dict(theta_interp=pk.INTERP_THETA_FH), dict(log_r=True), dict(s=12), dict(M_cap=20000)):
        with pytest.raises(pk.DmfeError) as e:
            pool.submit(pk.make_params({3: 1.0}, 0.5, **{**base, **kw}))
        assert e.value.status == pk.ERR_UNSUPPORTED, kw
    pool.submit(pk.make_params({3: 1.0}, 0.5, **base))
    pool.close()


def _lebesgue_max(ts, on_theta, n_samples=120, seed=3):
    """Largest Lebesgue function sum_k |l_k(z)| of the s-node polynomial stencils
    over sampled targets, in exact rational arithmetic on the FP64 nodes."""
    from fractions import Fraction
    L, s = ts.L, ts.s
    rng = np.random.default_rng(seed)
    worst = 1.0
    for x in np.concatenate([rng.uniform(0.0, L - 1.0, n_samples), [0.3, L - 1.3]]):
        base = int(min(max(int(np.floor(x)) - (s - 1) // 2, 0), L - s))
        if on_theta:
            z, nodes = oracle.theta_at_index(ts, x)[0], ts.th[base:base + s]
        else:
            z, nodes = x, np.arange(base, base + s, dtype=float)
        N = [Fraction(float(v)) for v in nodes]
        Z = Fraction(float(z))
        tot = Fraction(0)
        for k in range(s):
            w = Fraction(1)
            for l in range(s):
                if l != k:
                    w *= (Z - N[l]) / (N[k] - N[l])
            tot += abs(w)
        worst = max(worst, float(tot))
    return worst


@pytest.mark.parametrize("interp,d,log_r", [(pk.INTERP_THETA_FH, 7, True), (pk.INTERP_INDEX_FH, 15, False),
                                            (pk.INTERP_THETA_LAGRANGE, 0, False)])
def test_scheme_smallest_grid(interp, d, log_r):
    """L = 2s with s = 16: every stencil is clamped at one end of the grid or the
    other.  Degree-15 interpolation on such stencils is ill-conditioned: on theta
    one stencil spans node spacings from 1e-5 to 0.2 and the Lebesgue constant of
    the polynomial stencils reaches ~1e8 (about 400 on the index coordinate).  Two
    correct evaluations (the kernels' barycentric form, the oracle's product and
    blend forms) then differ by rounding times that constant, so the bar here is
    4e-14 Lambda (u Lambda with a margin for the quadrature sums), not 1e-12.
    The quadrature weights of a 32-point grid oscillate (sum |nu| ~ 200 against 1
    from L = 64 on), and the library's and the oracle's independent spline solves
    agree to ~1e-11 there, so mu is held to 1e-13 sum|nu| rather than 1e-13."""
    L, s = 32, 16
    ts = oracle.ThetaSetup(L, 1e4, s=s)
    on_theta = interp in (pk.INTERP_THETA_LAGRANGE, pk.INTERP_THETA_FH)
    lam = _lebesgue_max(ts, on_theta)
    bar = max(1e-12, 4e-14 * lam)
    mu_bar = 1e-13 * max(1.0, float(np.abs(ts.nu).sum()))
    say(f"scheme smallest grid interp={interp} d={d} log_r={log_r}: Lebesgue constant {lam:.3g}, bar {bar:.2g}, "
        f"mu bar {mu_bar:.2g}")
    gC, gR, gmu, gdiag, oC, oR, omu = _rhs(L, 20, 20, 5.0, 12, interp, d, log_r, s=s, hist="sign")
    _check(gC, gR, gdiag, oC, oR, gmu, omu, bar, mu_bar=mu_bar)
