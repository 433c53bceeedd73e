"""dmfe_rhs_noalloc against dmfe_rhs: the same right-hand side from the static
scratch array as from the handle's workspace, through the C-ABI, on two calls in
a row whose second has a smaller grid (so stale scratch contents from the first
would show), for FP64 and FP32 histories and for the log-R option."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2604_06309_amd as pk  # noqa: E402
import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def _case(L, M, precision, seed, **extra):
    p = pk.make_params({3: 0.5, 4: 0.5}, 0.55, t_max=1e7, L=L, M_cap=M, eps=1e-8, precision=precision, **extra)
    s = pk.Solver(p)
    th = s.read(pk.F_THETA)
    times = inputs.geometric_times(M, 200.0, t_first=0.01)
    C, R, dC, dR = inputs.smooth_history(th, times, seed)
    s.set_history(times, C, R, dC, dR)
    t = 200.08
    yC, yR = inputs.smooth_stage(th, t, seed)
    return s, t, torch.tensor(yC, device="cuda"), torch.tensor(yR, device="cuda"), M


@pytest.mark.parametrize("precision,extra", [(pk.FP64, {}), (pk.FP32_COMP, {}), (pk.FP64, {"log_r": True})])
def test_noalloc_rhs_equals_rhs(precision, extra):
    for L, M, seed in ((512, 300, 1), (256, 200, 2)):  # the second call has the smaller grid
        print(f"noalloc rhs L={L} M={M} precision={precision} {extra}", flush=True)
        sys.stdout.flush()
        s, t, yC, yR, nb = _case(L, M, precision, seed, **extra)
        gC, gR, mu, diag = s.rhs(t, yC, yR, nb)
        oC = torch.full_like(yC, float("nan"))
        oR = torch.full_like(yR, float("nan"))
        mu2, diag2 = pk.dmfe_rhs_noalloc(s.h, t, yC, yR, nb, oC, oR)
        torch.cuda.synchronize()
        s.close()
        np.testing.assert_array_equal(oC.cpu().numpy(), gC.cpu().numpy())
        np.testing.assert_array_equal(oR.cpu().numpy(), gR.cpu().numpy())
        assert mu2 == mu and np.array_equal(diag2, diag)


def test_noalloc_rhs_at_the_largest_grid():
    """L = 16384, the largest grid (the scratch array's limit), with a short history."""
    print("noalloc rhs L=16384 M=16", flush=True)
    s, t, yC, yR, nb = _case(16384, 16, pk.FP64, 3)
    gC, gR, mu, diag = s.rhs(t, yC, yR, nb)
    oC = torch.empty_like(yC)
    oR = torch.empty_like(yR)
    mu2, diag2 = pk.dmfe_rhs_noalloc(s.h, t, yC, yR, nb, oC, oR)
    torch.cuda.synchronize()
    s.close()
    np.testing.assert_array_equal(oC.cpu().numpy(), gC.cpu().numpy())
    np.testing.assert_array_equal(oR.cpu().numpy(), gR.cpu().numpy())
    assert mu2 == mu and np.array_equal(diag2, diag)
