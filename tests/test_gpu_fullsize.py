"""Parity at the full workload sizes, in the launch configuration the solver
uses for its steps: grid lengths 2048, 4096 and 8192 with histories of
thousands of slices (up to 1 GB per field), checked against the oracle on
sampled rows (the oracle computes rows one by one).

The sample always holds the first rows, rows at wave and block boundaries, the
last regular row and the pinned diagonal row L-1, plus seeded random rows.
Bars as in the small parity tests: FP64 within 1e-12 of the term scale
|mu| + T + max|out|, FP32-comp within 2e-6 of it.
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


def _rows(L, seed, n_random=12):
    rng = np.random.default_rng(seed)
    fixed = [0, 1, 7, 8, 63, 64, 65, L // 2 - 1, L // 2, L - 65, L - 2, L - 1]
    extra = rng.choice(np.arange(2, L - 2), size=n_random, replace=False)
    return np.unique(np.concatenate([fixed, extra])).astype(np.int32)


@pytest.mark.parametrize("L,M,nb_off,precision,bar,t_last,t", [
    (4096, 4096, 0, pk.FP64, 1e-12, 500.0, 510.0),     # L=4096 history at its cap, wide last step
    (4096, 4096, 1, pk.FP64, 1e-12, 500.0, 510.0),     # first stage of a step: newest slice without derivative
    (4096, 2500, 0, pk.FP64, 1e-12, 200.0, 200.08),    # the L=4096 workload's steady state: M, t and dt
    (2048, 2048, 0, pk.FP64, 1e-12, 500.0, 510.0),     # the L=2048 workload at its cap
    (8192, 3000, 0, pk.FP64, 1e-12, 500.0, 510.0),     # L=8192: stage slice too large for LDS staging
    (4096, 4096, 0, pk.FP32_COMP, 2e-6, 500.0, 510.0),  # FP32-comp history at L=4096
    (4096, 2500, 0, pk.FP32_COMP, 2e-6, 200.0, 200.08),
])
def test_rhs_sampled_rows_full_size(L, M, nb_off, precision, bar, t_last, t):
    say(f"full-size rhs L={L} M={M} nb=M-{nb_off} precision={precision} t={t}")
    terms, T = {3: 0.5, 4: 0.5}, 0.55
    ts = oracle.ThetaSetup(L, 1e7)
    m = oracle.make_model(terms, T=T)
    times = inputs.geometric_times(M, t_last, t_first=0.01)
    C, R, dC, dR = inputs.smooth_history(ts.th, times, 40 + L // 1024)
    yC, yR = inputs.smooth_stage(ts.th, t, 40 + L // 1024)
    nb = M - nb_off
    if nb_off:
        dC[-1] = 0.0
        dR[-1] = 0.0
    s = pk.Solver(pk.make_params(terms, T, t_max=1e7, L=L, M_cap=M, eps=1e-8, precision=precision))
    s.set_history(times, C, R, dC, dR, nb=M - 1 if nb_off else M)
    gC, gR, gmu, gdiag = s.rhs(t, torch.tensor(yC, device="cuda"), torch.tensor(yR, device="cuda"), nb)
    gC, gR = gC.cpu().numpy(), gR.cpu().numpy()
    s.close()
    rows = _rows(L, L + M)
    oC, oR, omu, _ = oracle.theta_rhs(m, ts, times, C, R, dC, dR, nb, t, yC, yR, rows=rows)
    assert abs(gmu - omu) <= 1e-13 * max(1.0, abs(omu))
    reg = rows[rows < L - 1]
    for g, o, d in ((gC, oC, gdiag[0]), (gR, oR, gdiag[1])):
        scale = abs(omu) + T + np.max(np.abs(o[rows]))
        err = np.max(np.abs(g[reg] - o[reg]))
        say(f"  {rows.size} rows: max error {err:.2e} (scale {scale:.3g}); diagonal {abs(d - o[L - 1]):.2e}")
        assert err <= bar * scale
        assert abs(d - o[L - 1]) <= bar * scale
        assert g[L - 1] == 0.0  # the diagonal row is pinned in the product's output


@pytest.mark.parametrize("precision,bar,nb_off", [(pk.FP64, 1e-12, 0), (pk.FP64, 1e-12, 1), (pk.FP32_COMP, 2e-6, 0)])
def test_rhs_with_more_slices_than_lds_holds_times_for(precision, bar, nb_off):
    """20000 stored slices: their times no longer fit in LDS beside the kernel's other tables, and
    the history-integral kernel reads them from global memory.  Every row against the oracle.
    (t_max = 1e4 keeps the 64-point quadrature well conditioned: at t_max = 1e7 its weights
    oscillate and two independent spline solves differ by ~1e-6.)"""
    L, M, t_last, t = 64, 20000, 50.0, 50.01
    say(f"rhs with M={M} slices (times in global memory), precision={precision}, nb=M-{nb_off}")
    terms, T = {3: 0.5, 4: 0.5}, 0.55
    ts = oracle.ThetaSetup(L, 1e4)
    times = inputs.geometric_times(M, t_last, t_first=1e-4)
    C, R, dC, dR = inputs.smooth_history(ts.th, times, 77)
    yC, yR = inputs.smooth_stage(ts.th, t, 77)
    if nb_off:
        dC[-1] = 0.0
        dR[-1] = 0.0
    nb = M - nb_off
    s = pk.Solver(pk.make_params(terms, T, t_max=1e4, L=L, M_cap=M + 8, eps=1e-8, precision=precision))
    s.set_history(times, C, R, dC, dR, nb=M - 1 if nb_off else M)
    gC, gR, gmu, gdiag = s.rhs(t, torch.tensor(yC, device="cuda"), torch.tensor(yR, device="cuda"), nb)
    gC, gR = gC.cpu().numpy(), gR.cpu().numpy()
    s.close()
    oC, oR, omu, _ = oracle.theta_rhs(oracle.make_model(terms, T=T), ts, times, C, R, dC, dR, nb, t, yC, yR)
    assert abs(gmu - omu) <= 1e-13 * max(1.0, abs(omu))
    for g, o, d in ((gC, oC, gdiag[0]), (gR, oR, gdiag[1])):
        scale = abs(omu) + T + np.max(np.abs(o))
        err = np.max(np.abs(g[:-1] - o[:-1]))
        say(f"  max error {err:.2e} (scale {scale:.3g})")
        assert err <= bar * scale and abs(d - o[-1]) <= bar * scale
