"""The FP32-compensated form (history stored in FP32 and widened to FP64 as it
is read; every sum, mu, RK, control and sparsification in FP64) against the
FP64 oracle and the FP64 solver.

Bars: one right-hand-side evaluation within 2e-6 of the term scale
(|mu| + T + max|out|): the stored values carry FP32 rounding (6e-8 relative)
and the quadrature sums of up to 4096 such values keep it below 1e-6.  Runs:
energy and mu of the FP32-comp solver against the FP64 solver's at common
times (splines through each run's stored times), per test below.
"""
import sys

import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
import paper_2604_06309_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("L,M,nb,t,seed", [(128, 40, 40, 9.0, 21), (1000, 80, 79, 40.0, 22), (64, 1, 0, 0.0, 23)])
def test_fp32_rhs_against_fp64_oracle(L, M, nb, t, seed):
    say(f"fp32 rhs L={L} M={M} nb={nb} t={t}")
    terms, T = {3: 0.5, 4: 0.5}, 0.6
    ts = oracle.ThetaSetup(L, 1e4)
    m = oracle.make_model(terms, T=T)
    times = np.zeros(1) if M == 1 else inputs.geometric_times(M, t * 0.97 if nb == M else t)
    C, R, dC, dR = inputs.smooth_history(ts.th, times, seed)
    yC, yR = inputs.smooth_stage(ts.th, t, seed)
    if nb == M - 1:
        dC[-1] = dR[-1] = 0.0
    s = pk.Solver(pk.make_params(terms, T, t_max=1e4, L=L, M_cap=max(M + 4, 16), precision=pk.FP32_COMP))
    s.set_history(times, C, R, dC, dR, nb=max(nb, M - 1))
    gC, gR, gmu, _ = s.rhs(t, torch.tensor(yC, device="cuda"), torch.tensor(yR, device="cuda"), nb)
    oC, oR, omu, _ = oracle.theta_rhs(m, ts, times, C, R, dC, dR, nb, t, yC, yR)
    oC[-1] = oR[-1] = 0.0
    for a, b in ((gC.cpu().numpy(), oC), (gR.cpu().numpy(), oR)):
        scale = abs(omu) + T + np.max(np.abs(b))
        err = np.max(np.abs(a - b))
        say(f"  max error {err:.2e} (scale {scale:.3g})")
        assert err <= 2e-6 * scale
    assert abs(gmu - omu) <= 1e-13 * max(1.0, abs(omu))  # mu(t) is FP64 on the FP64 stage slice
    s.close()


def test_fp32_run_against_fp64_run():
    """Same problem, same controller: FP32-comp vs FP64, observables at common stored times."""
    say("fp32 run vs fp64 run")
    terms, T, L = {3: 0.5, 4: 0.5}, 0.6, 256
    runs = {}
    for prec in (pk.FP64, pk.FP32_COMP):
        s = pk.Solver(pk.make_params(terms, T, t_max=1e4, L=L, M_cap=2000, eps=1e-6, dt0=1e-3, dt_min=1e-10,
                                     precision=prec))
        st, info = s.step(20.0)
        runs[prec] = (s.read(pk.F_T_GRID), s.read(pk.F_ENERGY), s.read(pk.F_MU), s.read(pk.F_C), info)
        say(f"  precision={prec}: steps={info.accepted} rejected={info.rejected} M={info.M} t={info.t:.4g}")
        s.close()
    from scipy.interpolate import CubicSpline
    t64, E64, mu64, C64, _ = runs[pk.FP64]
    t32, E32, mu32, C32, _ = runs[pk.FP32_COMP]
    tq = np.linspace(1.0, 19.0, 73)  # the time grids may differ: compare splines through each run
    eE = np.max(np.abs(CubicSpline(t32, E32)(tq) - CubicSpline(t64, E64)(tq)))
    emu = np.max(np.abs(CubicSpline(t32, mu32)(tq) - CubicSpline(t64, mu64)(tq)))
    # C(t, t_w) at t_w = 2 (theta = t_w / t on each slice, interpolated linearly in theta)
    th = oracle.theta_grid(L, 1e4)[0]
    cw32 = np.array([np.interp(2.0 / tt, th, c) for tt, c in zip(t32, C32) if tt > 2.5])
    cw64 = np.array([np.interp(2.0 / tt, th, c) for tt, c in zip(t64, C64) if tt > 2.5])
    tq2 = np.linspace(3.0, 19.0, 41)
    eC = np.max(np.abs(CubicSpline(t32[t32 > 2.5], cw32)(tq2) - CubicSpline(t64[t64 > 2.5], cw64)(tq2)))
    say(f"  |dE| {eE:.2e}  |dmu| {emu:.2e}  |dC(t, 2)| {eC:.2e}")
    assert eE <= 1e-6 and emu <= 1e-5 and eC <= 1e-5


def test_fp32_run_with_sparsification_against_fp64_run():
    """A low-temperature solve whose history must be sparsified to fit (cap 512
    slices): the FP32-comp residual, less its rounding allowance, still lets
    sparsification free slices, the solve reaches t_max, and its energy stays
    within 1e-6 of the FP64 solve's."""
    say("fp32 run with sparsification vs fp64 run")
    terms, T, L = {2: 0.499, 3: 0.184, 4: 0.317}, 0.477, 512
    runs = {}
    for prec in (pk.FP64, pk.FP32_COMP):
        s = pk.Solver(pk.make_params(terms, T, t_max=36.0, L=L, M_cap=512, eps=1e-6, dt0=1e-3, dt_min=1e-12,
                                     precision=prec))
        st, info = s.step(float("inf"))
        assert st == pk.DONE
        runs[prec] = (s.read(pk.F_T_GRID), s.read(pk.F_ENERGY), s.read(pk.F_MU), info)
        say(f"  precision={prec}: steps={info.accepted} rejected={info.rejected} M={info.M} "
            f"removed={info.removed} t={info.t:.4g}")
        s.close()
    from scipy.interpolate import CubicSpline
    t64, E64, mu64, i64 = runs[pk.FP64]
    t32, E32, mu32, i32 = runs[pk.FP32_COMP]
    assert i32.removed > 0
    tq = np.linspace(1.0, 35.0, 69)
    eE = np.max(np.abs(CubicSpline(t32, E32)(tq) - CubicSpline(t64, E64)(tq)))
    emu = np.max(np.abs(CubicSpline(t32, mu32)(tq) - CubicSpline(t64, mu64)(tq)))
    say(f"  |dE| {eE:.2e}  |dmu| {emu:.2e}")
    assert eE <= 1e-6 and emu <= 1e-5


def test_fp32_controller_not_limited_by_rounding():
    """At the workload's tolerance (1e-8) and a grid of 1024 points, the embedded
    error estimate of the FP32-comp solver must see the solution's error, not
    rounding: it takes the same number of steps as the FP64 solver to t = 30
    (within 2%), with the energy within 1e-7 of the FP64 solve's."""
    say("fp32 controller at eps=1e-8")
    terms, T, L = {3: 0.5, 4: 0.5}, 0.55, 1024
    runs = {}
    for prec in (pk.FP64, pk.FP32_COMP):
        s = pk.Solver(pk.make_params(terms, T, t_max=1e7, L=L, M_cap=4096, eps=1e-8, dt0=1e-3, dt_min=1e-12,
                                     precision=prec))
        st, info = s.step(30.0)
        runs[prec] = (s.read(pk.F_T_GRID), s.read(pk.F_ENERGY), info)
        say(f"  precision={prec}: steps={info.accepted} rejected={info.rejected} t={info.t:.4g} dt={info.dt:.3g}")
        s.close()
    from scipy.interpolate import CubicSpline
    t64, E64, i64 = runs[pk.FP64]
    t32, E32, i32 = runs[pk.FP32_COMP]
    assert abs(i32.accepted - i64.accepted) <= 0.02 * i64.accepted
    assert i32.rejected <= i64.rejected + 2
    tq = np.linspace(1.0, 29.0, 57)
    eE = np.max(np.abs(CubicSpline(t32, E32)(tq) - CubicSpline(t64, E64)(tq)))
    say(f"  |dE| {eE:.2e}")
    assert eE <= 1e-7
