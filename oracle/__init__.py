"""Plain FP64 CPU oracle for the DMFE history-integral solver (DYNAMITE, arXiv 2604.06309).

TEST INFRASTRUCTURE ONLY.  The product package never imports this module; only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
use it.  It shares no code with the HIP path.

The arithmetic lives in ``dmfe_oracle.c`` (plain C loops); this module holds the
ctypes mirror, the quadrature weights nu (Sec. 3.4: a global quintic spline on
the theta grid, evaluated with scipy's not-a-knot interpolating B-spline) and
the Runge-Kutta tableaux (Sec. 3.5: Dormand-Prince 5(4) and SSPRK(10,4)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dmfe_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAX_TERMS = 8


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (IEEE arithmetic, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Model(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int), ("p", ctypes.c_int * MAX_TERMS),
                ("a2", ctypes.c_double * MAX_TERMS), ("T", ctypes.c_double), ("beta0", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("s", ctypes.c_int), ("gamma", ctypes.c_double), ("D", ctypes.c_double),
                ("th", ctypes.c_void_p), ("thc", ctypes.c_void_p), ("nu", ctypes.c_void_p),
                ("interp", ctypes.c_int), ("fh_d", ctypes.c_int), ("log_r", ctypes.c_int), ("pad", ctypes.c_int)]


# theta-interpolation schemes (Sec. 3.3)
INDEX_LAGRANGE, THETA_LAGRANGE, INDEX_FH, THETA_FH = 0, 1, 2, 3


class Hist(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("nb", ctypes.c_int), ("t", ctypes.c_void_p),
                ("C", ctypes.c_void_p), ("R", ctypes.c_void_p), ("dC", ctypes.c_void_p), ("dR", ctypes.c_void_p),
                ("tcur", ctypes.c_double), ("yC", ctypes.c_void_p), ("yR", ctypes.c_void_p)]


class Tableau(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int), ("A", (ctypes.c_double * 10) * 10), ("b", ctypes.c_double * 10),
                ("e", ctypes.c_double * 10), ("c", ctypes.c_double * 10)]


class Adapt(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("dt0", ctypes.c_double), ("dt_min", ctypes.c_double),
                ("rho", ctypes.c_double), ("dp5_limit", ctypes.c_double), ("ssp_limit", ctypes.c_double),
                ("M_cap", ctypes.c_int), ("auto_passes", ctypes.c_int),
                ("dp5", ctypes.c_void_p), ("ssp", ctypes.c_void_p)]


class State(ctypes.Structure):
    _fields_ = [("t", ctypes.c_void_p), ("C", ctypes.c_void_p), ("R", ctypes.c_void_p),
                ("dC", ctypes.c_void_p), ("dR", ctypes.c_void_p),
                ("M", ctypes.c_int), ("nb_last_valid", ctypes.c_int), ("dt", ctypes.c_double),
                ("scheme", ctypes.c_int), ("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("reverts", ctypes.c_int64), ("removed", ctypes.c_int64), ("n_sparsify", ctypes.c_int64),
                ("last_eps", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        d, i, vp = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        for name in ("or_f", "or_f1", "or_f2"):
            getattr(_lib, name).restype = d
            getattr(_lib, name).argtypes = [ctypes.POINTER(Model), d]
        _lib.or_gamma.restype = d
        _lib.or_gamma.argtypes = [d]
        _lib.or_theta_grid.argtypes = [i, d, vp, vp]
        _lib.or_index_of.restype = d
        _lib.or_index_of.argtypes = [i, d, d, d]
        _lib.or_uniform_solve.argtypes = [ctypes.POINTER(Model), d, i, vp, vp, vp]
        _lib.or_uniform_rhs.argtypes = [ctypes.POINTER(Model), i, d, d, vp, vp, vp, vp, vp, vp]
        _lib.or_mu_energy.argtypes = [ctypes.POINTER(Model), i, vp, d, vp, vp, vp, vp]
        _lib.or_theta_rhs.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Grid), ctypes.POINTER(Hist), d,
                                      vp, i, vp, vp, vp]
        _lib.or_hist_value.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Hist), d, i, d, d, d, vp]
        _lib.or_sparsify_residuals.argtypes = [i, i, vp, vp, vp, vp, vp, vp]
        _lib.or_sparsify_select.restype = i
        _lib.or_sparsify_select.argtypes = [i, i, vp, d, vp]
        _lib.or_sparsify_pass.restype = i
        _lib.or_sparsify_pass.argtypes = [ctypes.POINTER(State), i, d]
        _lib.or_adaptive_run.restype = i
        _lib.or_adaptive_run.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Grid), ctypes.POINTER(Adapt),
                                         ctypes.POINTER(State), d, ctypes.c_int64]
        _lib.or_num_threads.restype = i
        _lib.or_num_threads.argtypes = []
        _lib.or_sizeof.restype = i
        _lib.or_sizeof.argtypes = [i]
        for k, cls in enumerate([Model, Grid, Hist, Tableau, Adapt, State]):
            assert _lib.or_sizeof(k) == ctypes.sizeof(cls), cls.__name__
    return _lib


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return lib().or_num_threads()


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------- model
def make_model(terms: dict[int, float], T: float, beta0: float = 0.0) -> Model:
    """terms maps p -> a_p^2 (Sec. 2.1: f(q) = sum_p a_p^2 q^p / 2)."""
    m = Model()
    m.n_terms = len(terms)
    for k, (p, a2) in enumerate(sorted(terms.items())):
        m.p[k] = int(p)
        m.a2[k] = float(a2)
    m.T = float(T)
    m.beta0 = float(beta0)
    return m


def f(m: Model, q: float) -> float:
    return lib().or_f(ctypes.byref(m), q)


def f1(m: Model, q: float) -> float:
    return lib().or_f1(ctypes.byref(m), q)


def f2(m: Model, q: float) -> float:
    return lib().or_f2(ctypes.byref(m), q)


# ----------------------------------------------------------------------------- uniform
def uniform_solve(m: Model, h: float, N: int):
    """RK4 + trapezoid uniform solver.  Returns (C, R, E) with C, R dense (N+1)x(N+1)
    lower-triangular arrays (upper triangle NaN) and E[N+1]."""
    ntri = (N + 1) * (N + 2) // 2
    Ct = np.zeros(ntri)
    Rt = np.zeros(ntri)
    E = np.zeros(N + 1)
    lib().or_uniform_solve(ctypes.byref(m), h, N, _p(Ct), _p(Rt), _p(E))
    return Ct, Rt, E


def tri_to_dense(X: np.ndarray, N: int) -> np.ndarray:
    out = np.full((N + 1, N + 1), np.nan)
    rows, cols = np.tril_indices(N + 1)
    out[rows, cols] = X
    return out


def uniform_rhs(m: Model, n: int, h: float, delta: float, Ct: np.ndarray, Rt: np.ndarray,
                c: np.ndarray, r: np.ndarray):
    dc = np.zeros(n + 1)
    dr = np.zeros(n + 1)
    lib().or_uniform_rhs(ctypes.byref(m), n, h, delta, _p(Ct), _p(Rt), _p(np.ascontiguousarray(c)),
                         _p(np.ascontiguousarray(r)), _p(dc), _p(dr))
    return dc, dr


# ----------------------------------------------------------------------------- theta grid
def gamma_of(tmax: float) -> float:
    """gamma = -W_{-1}(-1/t_max) (eq. theta)."""
    return lib().or_gamma(tmax)


def theta_grid(L: int, tmax: float):
    g = gamma_of(tmax)
    th = np.zeros(L)
    thc = np.zeros(L)
    lib().or_theta_grid(L, g, _p(th), _p(thc))
    return th, thc


def index_of(L: int, tmax: float, th: float, thc: float) -> float:
    return lib().or_index_of(L, gamma_of(tmax), th, thc)


def quad_weights(th: np.ndarray) -> np.ndarray:
    """nu_i with int_0^1 g(theta) dtheta ~ sum_i nu_i g(theta_i): the integral of the
    not-a-knot quintic interpolating spline on the grid (Sec. 3.4).  Spline i
    interpolates the i-th unit vector; scipy's make_interp_spline (default
    not-a-knot) builds all L splines from one collocation matrix."""
    from scipy.interpolate import make_interp_spline
    L = th.size
    spl = make_interp_spline(th, np.eye(L), k=5)
    return np.asarray(spl.integrate(th[0], th[-1]), dtype=np.float64)


class ThetaSetup:
    """The run-constant theta-grid data of the oracle: theta, 1-theta, nu, gamma,
    and the theta-interpolation scheme: `interp` (INDEX_LAGRANGE, THETA_LAGRANGE,
    INDEX_FH, THETA_FH) on s-point stencils, the Floater-Hormann degree `fh_d`,
    and `log_r` (interpolate log R, Appendix A)."""

    def __init__(self, L: int, tmax: float, s: int = 10, interp: int = INDEX_LAGRANGE, fh_d: int = 3,
                 log_r: bool = False):
        assert 2 <= s <= 16 and 0 <= fh_d <= s - 1
        self.L, self.s, self.tmax = L, s, tmax
        self.interp, self.fh_d, self.log_r = interp, fh_d, bool(log_r)
        self.gamma = gamma_of(tmax)
        self.th, self.thc = theta_grid(L, tmax)
        self.nu = quad_weights(self.th)
        self.grid = Grid()
        self.grid.L, self.grid.s, self.grid.gamma = L, s, self.gamma
        self.grid.D = float(np.arctan(np.exp(self.gamma)) - np.arctan(np.exp(-self.gamma)))
        self.grid.th, self.grid.thc, self.grid.nu = _p(self.th), _p(self.thc), _p(self.nu)
        self.grid.interp, self.grid.fh_d, self.grid.log_r = int(interp), int(fh_d), int(bool(log_r))


def mu_energy(m: Model, ts: ThetaSetup, t: float, yC: np.ndarray, yR: np.ndarray):
    mu = ctypes.c_double()
    E = ctypes.c_double()
    lib().or_mu_energy(ctypes.byref(m), ts.L, _p(ts.nu), t, _p(yC), _p(yR), ctypes.byref(mu), ctypes.byref(E))
    return mu.value, E.value


def _hist(t_hist, C, R, dC, dR, nb, t, yC, yR, keep):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (t_hist, C, R, dC, dR, yC, yR)]
    keep.extend(arrs)
    H = Hist()
    H.M = int(arrs[0].size)
    H.nb = int(nb)
    H.t, H.C, H.R, H.dC, H.dR = (_p(a) for a in arrs[:5])
    H.tcur = float(t)
    H.yC, H.yR = _p(arrs[5]), _p(arrs[6])
    return H


def theta_rhs(m: Model, ts: ThetaSetup, t_hist, C, R, dC, dR, nb: int, t: float, yC, yR,
              rows=None, want_sums: bool = False):
    """Right-hand side dC/dt, dR/dt along fixed theta for the listed rows.

    t_hist[M]; C, R, dC, dR are [M, L]; slices 0..nb-1 carry valid d/dt.
    Returns (outC, outR, mu, sums) with outC/outR of length L (NaN for rows not
    computed) and sums [nrows, 9] if requested."""
    keep: list = []
    H = _hist(t_hist, C, R, dC, dR, nb, t, yC, yR, keep)
    mu, _ = mu_energy(m, ts, t, keep[5], keep[6])
    outC = np.full(ts.L, np.nan)
    outR = np.full(ts.L, np.nan)
    if rows is None:
        rp, nr = None, ts.L
    else:
        rarr = np.ascontiguousarray(rows, dtype=np.int32)
        keep.append(rarr)
        rp, nr = _p(rarr), rarr.size
    sums = np.zeros((nr, 9)) if want_sums else None
    lib().or_theta_rhs(ctypes.byref(m), ctypes.byref(ts.grid), ctypes.byref(H), mu, rp, nr if rows is not None else 0,
                       _p(outC), _p(outR), _p(sums) if want_sums else None)
    return outC, outR, mu, sums


def hist_value(ts: ThetaSetup, t_hist, C, R, dC, dR, nb, t, yC, yR, tau, node=-1, x=0.0, th=None, thc=None):
    """(C, R) at time tau and the grid node `node`, or (node < 0) at the point of
    continuous index x; the theta schemes also need its theta and 1 - theta
    (default: from x through the grid map)."""
    keep: list = []
    H = _hist(t_hist, C, R, dC, dR, nb, t, yC, yR, keep)
    if node < 0 and th is None:
        th, thc = theta_at_index(ts, x)
    if th is None:
        th, thc = 0.0, 1.0
    if thc is None:
        thc = 1.0 - th
    out = np.zeros(2)
    lib().or_hist_value(ctypes.byref(ts.grid), ctypes.byref(H), tau, node, x, float(th), float(thc), _p(out))
    return out


def theta_at_index(ts: ThetaSetup, x: float):
    """theta and 1 - theta at continuous index x (eq. theta at alpha = 0, the
    0-based index i taken as continuous)."""
    L, g = ts.L, ts.gamma
    y = (2.0 * x + 1.0 - L) / (L - 1)
    y = min(max(y, -1.0), 1.0)
    def lower(yy):  # theta(yy) for yy <= 0, full relative precision
        return np.arctan(np.sinh(0.5 * g * (1.0 + yy)) / np.cosh(0.5 * g * (1.0 - yy))) / np.arctan(np.sinh(g))
    if y <= 0.0:
        th = float(lower(y))
        return th, 1.0 - th
    thc = float(lower(-y))
    return 1.0 - thc, thc


# ----------------------------------------------------------------------------- sparsify
def sparsify_residuals(t, C, R, dC, dR):
    M, L = C.shape
    eps = np.zeros(M)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (t, C, R, dC, dR)]
    lib().or_sparsify_residuals(M, L, *(_p(a) for a in arrs), _p(eps))
    return eps


def sparsify_select(eps: np.ndarray, last: int, thr: float):
    drop = np.zeros(eps.size, dtype=np.int32)
    e = np.ascontiguousarray(eps, dtype=np.float64)
    n = lib().or_sparsify_select(e.size, last, _p(e), thr, _p(drop))
    return n, drop.astype(bool)


# ----------------------------------------------------------------------------- RK tableaux
def dp5_tableau():
    """Dormand-Prince 5(4) (Sec. 3.5): A, b (5th order), bhat (4th order), c."""
    A = np.zeros((7, 7))
    A[1, 0] = 1 / 5
    A[2, :2] = [3 / 40, 9 / 40]
    A[3, :3] = [44 / 45, -56 / 15, 32 / 9]
    A[4, :4] = [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729]
    A[5, :5] = [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656]
    A[6, :6] = [35 / 384, 0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84]
    b = A[6].copy()
    bhat = np.array([5179 / 57600, 0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100, 1 / 40])
    return A, b, bhat, A.sum(axis=1)


def ssprk104_tableau():
    """SSPRK(10,4) (Sec. 3.5) in Butcher form, from its two-register form:
    five Euler stages of dt/6, the combination q1 <- (3/5) u + (2/5) q1, four
    more Euler stages and a final weight 1/10 on every stage.  The embedded
    third-order weights are the minimum-norm solution of the four third-order
    conditions over stages 1..9 (last weight zero)."""
    A = np.zeros((10, 10))
    for k in range(1, 5):
        A[k, :k] = 1 / 6
    A[5, :5] = 1 / 15
    for k in range(6, 10):
        A[k, :5] = 1 / 15
        A[k, 5:k] = 1 / 6
    b = np.full(10, 0.1)
    c = A.sum(axis=1)
    cond = np.vstack([np.ones(10), c, c ** 2, A @ c])[:, :9]
    rhs = np.array([1.0, 0.5, 1 / 3, 1 / 6])
    bh9 = np.linalg.lstsq(cond, rhs, rcond=None)[0]
    bhat = np.zeros(10)
    bhat[:9] = bh9
    return A, b, bhat, c


def stability_limit(A: np.ndarray, b: np.ndarray, step: float = 1e-3) -> float:
    """Largest r with |R(-x)| <= 1 on [0, r], R(z) = 1 + z b^T (I - zA)^{-1} 1."""
    n = b.size
    one = np.ones(n)
    eye = np.eye(n)

    def Rz(z):
        return 1.0 + z * b @ np.linalg.solve(eye - z * A, one)

    x = 0.0
    while abs(Rz(-(x + step))) <= 1.0 + 1e-13:
        x += step
    lo, hi = x, x + step
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if abs(Rz(-mid)) <= 1.0 + 1e-13:
            lo = mid
        else:
            hi = mid
    return lo


def _tab(A, b, bhat, c) -> Tableau:
    T = Tableau()
    T.S = b.size
    for i in range(b.size):
        for j in range(b.size):
            T.A[i][j] = A[i, j]
        T.b[i] = b[i]
        T.e[i] = b[i] - bhat[i]
        T.c[i] = c[i]
    return T


# Real-axis stability limits used for the scheme switch and the step cap.  The
# values are those of stability_limit() for the two tableaux, truncated.
DP5_LIMIT = 3.3065
SSP_LIMIT = 13.917


class AdaptiveRun:
    """The oracle's adaptive solve on the theta grid (history in four [M_cap, L] arrays)."""

    def __init__(self, m: Model, ts: ThetaSetup, eps: float, dt0: float, dt_min: float, M_cap: int,
                 auto_passes: int = 1):
        self.m, self.ts = m, ts
        L = ts.L
        self.M_cap = M_cap
        self.t = np.zeros(M_cap + 1)
        self.C = np.zeros((M_cap + 1, L))
        self.R = np.zeros((M_cap + 1, L))
        self.dC = np.zeros((M_cap + 1, L))
        self.dR = np.zeros((M_cap + 1, L))
        self.C[0] = 1.0
        self.R[0] = 1.0
        self._dp5 = _tab(*dp5_tableau())
        self._ssp = _tab(*ssprk104_tableau())
        self.ad = Adapt()
        self.ad.eps, self.ad.dt0, self.ad.dt_min = eps, dt0, dt_min
        self.ad.rho = 4.0 * np.sqrt(f2(m, 1.0))
        self.ad.dp5_limit, self.ad.ssp_limit = DP5_LIMIT, SSP_LIMIT
        self.ad.M_cap, self.ad.auto_passes = M_cap, auto_passes
        self.ad.dp5 = ctypes.cast(ctypes.pointer(self._dp5), ctypes.c_void_p)
        self.ad.ssp = ctypes.cast(ctypes.pointer(self._ssp), ctypes.c_void_p)
        self.st = State()
        self.st.t, self.st.C, self.st.R = _p(self.t), _p(self.C), _p(self.R)
        self.st.dC, self.st.dR = _p(self.dC), _p(self.dR)
        self.st.M = 1
        self.st.dt = dt0
        self.st.scheme = 0

    def run(self, t_target: float, max_steps: int) -> int:
        return lib().or_adaptive_run(ctypes.byref(self.m), ctypes.byref(self.ts.grid), ctypes.byref(self.ad),
                                     ctypes.byref(self.st), t_target, max_steps)

    def sparsify(self, passes: int = 1) -> int:
        n = 0
        for _ in range(passes):
            n += lib().or_sparsify_pass(ctypes.byref(self.st), self.ts.L, self.ad.eps)
        return n

    @property
    def M(self) -> int:
        return self.st.M

    def history(self):
        M = self.st.M
        return self.t[:M].copy(), self.C[:M].copy(), self.R[:M].copy(), self.dC[:M].copy(), self.dR[:M].copy()
