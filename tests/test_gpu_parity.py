"""Parity of the HIP path (through the C-ABI) with the oracle, element by element.

Tolerances:
  * uniform solver, C(t,t'), R(t,t'), E: |x - ref| <= 1e-10 |ref| + 1e-14;
  * one right-hand-side evaluation on the theta grid: every output within
    1e-12 of the reference relative to the size of the terms it is formed
    from.  Each output is d1 + theta d2 where d1 and d2 each contain -mu C,
    mu' R and integrals of size O(mu); they cancel to values that can be
    1e-6 of mu, so the scale is |mu| + T + max|output|, not |output|;
  * multi-step adaptive runs: identical accept/reject decisions and time grid,
    states within 1e-10 relative (+1e-14).
"""
import sys

import numpy as np
import pytest

import inputs
import oracle
import p2_exact as px

torch = pytest.importorskip("torch")
import paper_2604_06309_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pk.lib()  # raises if the library is missing: no fallback
    yield
    torch.cuda.synchronize()


def close(x, ref, rtol, atol):
    x, ref = np.asarray(x), np.asarray(ref)
    err = np.abs(x - ref)
    bad = err > rtol * np.abs(ref) + atol
    return not bad.any(), float(np.max(err / (np.abs(ref) + atol / rtol)))


# ----------------------------------------------------------------------------- uniform (C1)
@pytest.mark.parametrize("terms,T,beta0,h,N", [
    ({3: 1.0}, 0.5, 0.0, 0.05, 1000),       # the pure p=3 quench, t_max = 50
    ({2: 0.3, 4: 0.7}, 0.45, 0.0, 0.04, 77),
    ({3: 1.0}, 1.0, 1.0, 0.05, 65),          # equilibrium start
    ({2: 0.5, 5: 0.5}, 0.8, 0.0, 0.05, 40),  # p = 5: general polynomial path
])
def test_uniform_parity(terms, T, beta0, h, N):
    say(f"uniform parity terms={terms} T={T} beta0={beta0} h={h} N={N}")
    m = oracle.make_model(terms, T=T, beta0=beta0)
    Ct, Rt, E = oracle.uniform_solve(m, h, N)
    p = pk.make_params(terms, T, beta0=beta0, mode=pk.UNIFORM, h=h, N=N)
    s = pk.Solver(p)
    st, info = s.step(float("inf"))
    assert st == pk.DONE and info.M == N + 1
    gC = s.read(pk.F_C, 0, N + 1)
    gR = s.read(pk.F_R, 0, N + 1)
    gE = s.read(pk.F_ENERGY, 0, N + 1)
    for name, a, b in (("C", gC, Ct), ("R", gR, Rt), ("E", gE, E)):
        ok, worst = close(a, b, 1e-10, 1e-14)
        say(f"  {name}: worst scaled error {worst:.2e}")
        assert ok, name
    s.close()


# ----------------------------------------------------------------------------- one RHS evaluation
def _rhs_case(L, M, nb, t, seed, terms=None, T=0.6, beta0=0.0, tmax=1e4, s=10, hist="smooth"):
    terms = terms or {3: 0.5, 4: 0.5}
    p = pk.make_params(terms, T, beta0=beta0, t_max=tmax, L=L, M_cap=max(M + 4, 16), s=s)
    solver = pk.Solver(p)
    ts = oracle.ThetaSetup(L, tmax, s=s)
    m = oracle.make_model(terms, T=T, beta0=beta0)
    if M == 1:
        times = np.zeros(1)
    elif hist == "p2":
        times = inputs.geometric_times(M, t - 0.0125)  # a short last step, as in a resolved run
    else:
        times = inputs.geometric_times(M, t * 0.97 if nb == M else t)
    if hist == "p2":
        C = np.array([px.C0(tt, ts.th * tt) for tt in times])
        R = np.array([px.R0(tt, ts.th * tt) for tt in times])
        dC = np.array([sum(a * w for a, w in zip(px.dC0(tt, ts.th * tt), (1, ts.th))) for tt in times])
        dR = np.array([sum(a * w for a, w in zip(px.dR0(tt, ts.th * tt), (1, ts.th))) for tt in times])
        C[:, -1] = R[:, -1] = 1.0
        yC, yR = px.C0(t, ts.th * t), px.R0(t, ts.th * t)
        yC[-1] = yR[-1] = 1.0
    else:
        C, R, dC, dR = inputs.smooth_history(ts.th, times, seed)
        yC, yR = inputs.smooth_stage(ts.th, t, seed)
    if nb == M - 1:
        dC[-1] = 0.0
        dR[-1] = 0.0
    solver.set_history(times, C, R, dC, dR, nb=max(nb, M - 1))
    gC, gR, gmu, gdiag = solver.rhs(t, torch.tensor(yC, device="cuda"), torch.tensor(yR, device="cuda"), nb)
    oC, oR, omu, _ = oracle.theta_rhs(m, ts, times, C, R, dC, dR, nb, t, yC, yR)
    solver.close()
    return gC.cpu().numpy(), gR.cpu().numpy(), gmu, gdiag, oC, oR, omu


def _check_rhs(gC, gR, oC, oR, gmu, omu, T=0.6):
    oC, oR = oC.copy(), oR.copy()
    oC[-1] = oR[-1] = 0.0  # the product pins the diagonal row
    for a, b in ((gC, oC), (gR, oR)):
        scale = abs(omu) + T + np.max(np.abs(b))
        err = np.abs(a - b)
        say(f"  max error {np.max(err):.2e} (scale {scale:.3g})")
        assert np.max(err) <= 1e-12 * scale, (np.max(err), scale)
    assert abs(gmu - omu) <= 1e-13 * max(1.0, abs(omu))


@pytest.mark.parametrize("L,M,nb,t,seed", [
    (64, 30, 30, 6.0, 1),      # every target inside the stored slices or the last step
    (64, 30, 29, 6.0, 2),      # first stage: last slice without derivative
    (200, 45, 45, 11.0, 3),    # L not a multiple of the wave or block size
    (203, 45, 45, 11.0, 3),    # L odd: the last row groups of a wave are partly outside the grid
    (1000, 80, 80, 40.0, 4),   # many tiles per row
    (96, 2, 1, 0.3, 5),        # one stored interval
    (96, 1, 1, 0.2, 6),        # only t = 0 stored
    (64, 1, 0, 0.0, 7),        # t = 0
])
def test_rhs_parity_smooth(L, M, nb, t, seed):
    say(f"rhs parity L={L} M={M} nb={nb} t={t} seed={seed}")
    gC, gR, gmu, gdiag, oC, oR, omu = _rhs_case(L, M, nb, t, seed)
    _check_rhs(gC, gR, oC, oR, gmu, omu)
    # the diagonal row computed by the kernel agrees with the oracle's value
    assert abs(gdiag[0] - oC[-1]) <= 1e-12 * max(1.0, np.max(np.abs(oC)))
    assert abs(gdiag[1] - oR[-1]) <= 1e-12 * max(1.0, np.max(np.abs(oR)))


@pytest.mark.parametrize("s", [4, 6, 8, 12])
def test_rhs_parity_stencil_sizes(s):
    say(f"rhs parity stencil s={s}")
    gC, gR, gmu, gdiag, oC, oR, omu = _rhs_case(128, 40, 40, 9.0, 8, s=s)
    _check_rhs(gC, gR, oC, oR, gmu, omu)


def test_rhs_parity_forcing_and_high_p():
    say("rhs parity beta0 > 0, p up to 6")
    gC, gR, gmu, gdiag, oC, oR, omu = _rhs_case(96, 25, 25, 5.0, 9, terms={2: 0.2, 6: 0.8}, T=0.9, beta0=0.7)
    _check_rhs(gC, gR, oC, oR, gmu, omu, T=0.9)


def test_rhs_p2_exact_history():
    """On the exact p = 2 history the GPU right-hand side reproduces the exact
    derivative along fixed theta to the interpolation/quadrature error, and the
    diagonal identities hold to roundoff."""
    say("rhs p=2 exact history")
    L, t = 128, 8.0
    gC, gR, gmu, gdiag, oC, oR, omu = _rhs_case(L, 800, 800, t, 0, terms={2: 1.0}, T=0.0, tmax=1e3, hist="p2")
    _check_rhs(gC, gR, oC, oR, gmu, omu, T=0.0)
    th, _ = oracle.theta_grid(L, 1e3)
    a, b = px.dC0(t, th * t)
    exC = a + th * b
    a, b = px.dR0(t, th * t)
    exR = a + th * b
    assert np.max(np.abs(gC - exC)[:-1]) < 2e-7 and np.max(np.abs(gR - exR)[:-1]) < 2e-7
    assert abs(gdiag[0]) < 1e-13 and abs(gdiag[1]) < 1e-13


# ----------------------------------------------------------------------------- observables
def test_energy_and_mu_per_slice():
    say("observables per slice")
    L = 150
    ts = oracle.ThetaSetup(L, 1e4)
    times = inputs.geometric_times(20, 7.0)
    C, R, dC, dR = inputs.smooth_history(ts.th, times, 12)
    m = oracle.make_model({2: 0.3, 4: 0.7}, T=0.45, beta0=0.3)
    s = pk.Solver(pk.make_params({2: 0.3, 4: 0.7}, 0.45, beta0=0.3, t_max=1e4, L=L, M_cap=32))
    s.set_history(times, C, R, dC, dR)
    E = s.read(pk.F_ENERGY)
    mu = s.read(pk.F_MU)
    for n, tt in enumerate(times):
        omu, oE = oracle.mu_energy(m, ts, tt, C[n], R[n])
        assert abs(E[n] - oE) <= 1e-13 * max(1, abs(oE))
        assert abs(mu[n] - omu) <= 1e-13 * max(1, abs(omu))
    s.close()


# ----------------------------------------------------------------------------- sparsification
def test_sparsify_parity():
    say("sparsify parity")
    L, M = 80, 60
    ts = oracle.ThetaSetup(L, 1e4)
    times = inputs.geometric_times(M, 30.0, t_first=0.05)
    C, R, dC, dR = inputs.smooth_history(ts.th, times, 13)
    eps_n = oracle.sparsify_residuals(times, C, R, dC, dR)
    # a threshold between well separated residuals so the decision is robust to rounding
    cand = np.sort(eps_n[1:M - 11])
    gaps = np.diff(cand) / cand[1:]
    k = int(np.argmax(gaps[len(gaps) // 4: 3 * len(gaps) // 4])) + len(gaps) // 4
    eps = 10 * 0.5 * (cand[k] + cand[k + 1])
    run = oracle.AdaptiveRun(oracle.make_model({3: 1.0}, T=0.5), ts, eps=eps, dt0=0.1, dt_min=1e-9, M_cap=M + 4)
    run.t[:M], run.C[:M], run.R[:M], run.dC[:M], run.dR[:M] = times, C, R, dC, dR
    run.st.M = M
    n_or = run.sparsify(1)
    s = pk.Solver(pk.make_params({3: 1.0}, 0.5, t_max=1e4, L=L, M_cap=M + 4, eps=eps))
    s.set_history(times, C, R, dC, dR)
    n_gpu = s.sparsify(1)
    assert n_gpu == n_or and n_gpu > 0
    np.testing.assert_array_equal(s.read(pk.F_T_GRID), run.t[:run.M])
    np.testing.assert_array_equal(s.read(pk.F_C), run.C[:run.M])
    s.close()


# ----------------------------------------------------------------------------- adaptive runs
@pytest.mark.parametrize("terms,T,L,M_cap,eps,t_end,policy", [
    ({3: 0.5, 4: 0.5}, 0.6, 64, 400, 1e-8, 12.0, 0),   # DP5, then the switch to SSPRK(10,4)
    ({2: 1.0}, 0.0, 72, 150, 1e-7, 8.0, 0),            # history cap reached: auto sparsification
    ({3: 1.0}, 0.5, 64, 400, 1e-8, 6.0, 1),            # SSPRK(10,4) from the start
])
def test_adaptive_parity(terms, T, L, M_cap, eps, t_end, policy):
    say(f"adaptive parity terms={terms} L={L} M_cap={M_cap} eps={eps} t_end={t_end} policy={policy}")
    m = oracle.make_model(terms, T=T)
    ts = oracle.ThetaSetup(L, 1e4)
    run = oracle.AdaptiveRun(m, ts, eps=eps, dt0=1e-3, dt_min=1e-10, M_cap=M_cap)
    if policy == 1:
        run.st.scheme = 1
    st_o = run.run(t_end, 100000)
    s = pk.Solver(pk.make_params(terms, T, t_max=1e4, L=L, M_cap=M_cap, eps=eps, dt0=1e-3, dt_min=1e-10,
                                 scheme_policy=policy))
    st_g, info = s.step(t_end)
    say(f"  oracle: M={run.M} acc={run.st.accepted} rej={run.st.rejected} removed={run.st.removed}; "
        f"gpu: M={info.M} acc={info.accepted} rej={info.rejected} removed={info.removed} rhs={info.rhs_evals}")
    assert (info.accepted, info.rejected, info.M) == (run.st.accepted, run.st.rejected, run.M)
    assert info.removed == run.st.removed
    t, C, R, dC, dR = run.history()
    np.testing.assert_array_equal(s.read(pk.F_T_GRID), t)
    for name, f, ref in (("C", pk.F_C, C), ("R", pk.F_R, R), ("dC", pk.F_DC, dC[:-1]), ("dR", pk.F_DR, dR[:-1])):
        g = s.read(f)
        if name in ("dC", "dR"):
            g = g[:-1]  # the newest slice's derivative is written at the next first stage
        ok, worst = close(g, ref, 1e-10, 1e-14)
        say(f"  {name}: worst scaled error {worst:.2e}")
        assert ok, name
    assert abs(info.t - t[-1]) == 0.0 and abs(info.dt - run.st.dt) <= 1e-15 * run.st.dt
    s.close()


def test_workspace_and_stream():
    """Caller-owned workspace (a torch tensor) and a caller stream give the same result."""
    say("workspace + stream")
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=64, M_cap=400, eps=1e-8, dt0=1e-3)
    a = pk.Solver(p)
    a.step(2.0)
    stream = torch.cuda.Stream()
    b = pk.Solver(p, stream=stream, use_workspace=True)
    b.step(2.0)
    np.testing.assert_array_equal(a.read(pk.F_C), b.read(pk.F_C))
    a.close()
    b.close()


def test_timing_of_selected_kernels():
    """Per-launch timing counts launches of the selected kernels only (DP5: six
    history-integral launches per step, the first stage reused from the step
    before), and timing does not change the results."""
    say("timing selection")
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=64, M_cap=400, eps=1e-8, dt0=1e-3)
    a, b = pk.Solver(p), pk.Solver(p)
    a.step(1.0)
    b.step(1.0)
    e0 = a.info().rhs_evals
    a.timing(True, [pk.K_HIST_INTEGRAL])
    b.timing(True)
    _, ia = a.step(float("inf"), 10)
    b.step(float("inf"), 10)
    na, msa, _ = a.timing_read(pk.K_HIST_INTEGRAL)
    assert na == ia.rhs_evals - e0 and na > 0 and msa > 0.0
    assert a.timing_read(pk.K_RK)[0] == 0 and a.timing_read(pk.K_STAGE_PREP)[0] == 0
    assert b.timing_read(pk.K_RK)[0] > 0 and b.timing_read(pk.K_STAGE_PREP)[0] == b.timing_read(pk.K_HIST_INTEGRAL)[0]
    assert na == b.timing_read(pk.K_HIST_INTEGRAL)[0]
    np.testing.assert_array_equal(a.read(pk.F_C), b.read(pk.F_C))
    with pytest.raises(pk.DmfeError):
        pk.dmfe_timing_select(a.h, [pk.K_COUNT])
    a.close()
    b.close()


def test_errors_from_device_calls():
    say("error paths")
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=64, M_cap=16, eps=1e-30, dt0=1e-3)
    s = pk.Solver(p)
    with pytest.raises(pk.DmfeError) as e:
        s.step(5.0)
    assert e.value.status in (pk.ERR_CAPACITY, pk.ERR_STEP_UNDERFLOW)
    s.close()
    s = pk.Solver(pk.make_params({3: 1.0}, 0.5, t_max=1e4, L=64))
    with pytest.raises(pk.DmfeError):
        s.read(pk.F_C, 0, 5)  # only one slice stored
    s.close()


# ----------------------------------------------------------------------------- forced failures
def _reference_history(p, steps):
    s = pk.Solver(p)
    s.step(float("inf"), steps)
    info = s.info()
    h = [s.read(f) for f in (pk.F_T_GRID, pk.F_C, pk.F_R, pk.F_DC, pk.F_DR)]
    s.close()
    return info, h


def test_nan_in_the_state_is_reported_not_stepped():
    """A NaN in the state (forced from the host) makes the error estimate non-finite:
    the step ends with DMFE_ERR_NONFINITE."""
    say("forced NaN in the state")
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=64, M_cap=400, eps=1e-8, dt0=1e-3, dt_min=1e-12)
    info, (t, C, R, dC, dR) = _reference_history(p, 50)
    C = C.copy()
    C[-1, 20] = np.nan
    s = pk.Solver(p)
    s.set_history(t, C, R, dC, dR, nb=t.size - 1, dt=info.dt)
    with pytest.raises(pk.DmfeError) as e:
        s.step(float("inf"), 5)
    assert e.value.status == pk.ERR_NONFINITE
    s.close()


def test_forced_revert_keeps_the_earlier_slices_bitwise():
    """A step 20 times too large (forced through the controller's dt) has an error
    above 2 eps: it is rejected, the last 10 slices are dropped and dt halved, and
    the slices kept are bitwise those given before (Sec. 3.5)."""
    say("forced revert")
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.6, t_max=1e4, L=64, M_cap=400, eps=1e-8, dt0=1e-3, dt_min=1e-12)
    info, (t, C, R, dC, dR) = _reference_history(p, 100)
    M = t.size
    s = pk.Solver(p)
    s.set_history(t, C, R, dC, dR, nb=M - 1, dt=20 * info.dt)
    st, got = s.step(float("inf"), 1)
    assert (got.accepted, got.rejected, got.reverts) == (0, 1, 10)  # reverts counts the slices dropped
    assert got.M == M - 10 and got.dt == 10 * info.dt
    np.testing.assert_array_equal(s.read(pk.F_T_GRID), t[:M - 10])
    for f, ref in ((pk.F_C, C), (pk.F_R, R), (pk.F_DC, dC), (pk.F_DR, dR)):
        np.testing.assert_array_equal(s.read(f), ref[:M - 10])
    # and the solve goes on from there
    st, got = s.step(float("inf"), 20)
    assert got.accepted > 0 and np.all(np.isfinite(s.read(pk.F_C)))
    s.close()
