"""Exact solution of the pure p = 2 spherical model, f(q) = q^2/2 (Sec. 2.1).

For p = 2 the Langevin dynamics of Sec. 2.1 is linear in the eigenbasis of the
coupling matrix, whose spectrum is the semicircle on [-2, 2].  With
G(x) = int rho(l) e^{l x} dl = I_1(2x)/x and Gamma(t) = exp(2 int_0^t mu):

  Gamma(t)  = G(2t) + 2T int_0^t G(2(t-s)) Gamma(s) ds        (C(t,t) = 1)
  R(t,t')   = G(t-t') sqrt(Gamma(t')/Gamma(t))
  C(t,t')   = [G(t+t') + 2T int_0^{t'} G(t+t'-2s) Gamma(s) ds] / sqrt(Gamma(t) Gamma(t'))
  mu(t)     = Gamma'(t) / (2 Gamma(t))
  E(t)      = -1/2 [G'(2t) + 2T int_0^t G'(2(t-s)) Gamma(s) ds] / Gamma(t)

At T = 0 everything is in closed form; at T > 0 the Volterra equation is solved
on a fine uniform grid with the trapezoid rule and Richardson extrapolation.
This module is a pin for the oracle (it shares nothing with it).
"""
from __future__ import annotations

import numpy as np
from scipy.special import i0e, i1e


def G(x):
    """I_1(2x)/x, with G(0) = 1."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    small = np.abs(x) < 1e-4
    xs = x[small]
    out[small] = 1.0 + xs ** 2 / 2.0 + xs ** 4 / 12.0
    xl = x[~small]
    out[~small] = np.exp(2 * np.abs(xl)) * i1e(2 * xl) / xl
    return out


def Gp(x):
    """G'(x) = 2 (I_0(2x) - G(x)) / x."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    small = np.abs(x) < 1e-4
    xs = x[small]
    out[small] = xs + xs ** 3 / 3.0
    xl = x[~small]
    out[~small] = 2.0 * (np.exp(2 * np.abs(xl)) * i0e(2 * xl) - G(xl)) / xl
    return out


def logG(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x < 1e-4, np.log(G(np.minimum(x, 1e-4))), 2 * x + np.log(i1e(2 * np.maximum(x, 1e-4)) / np.maximum(x, 1e-4)))


# --------------------------------------------------------------------------- T = 0
def C0(t, tp):
    t, tp = np.broadcast_arrays(np.asarray(t, float), np.asarray(tp, float))
    return np.exp(logG(t + tp) - 0.5 * (logG(2 * t) + logG(2 * tp)))


def R0(t, tp):
    t, tp = np.broadcast_arrays(np.asarray(t, float), np.asarray(tp, float))
    return G(t - tp) * np.exp(0.5 * (logG(2 * tp) - logG(2 * t)))


def E0(t):
    t = np.asarray(t, float)
    return -0.5 * Gp(2 * t) / G(2 * t)


def mu0(t):
    t = np.asarray(t, float)
    return Gp(2 * t) / G(2 * t)


def dC0(t, tp):
    """(d/dt C, d/dt' C) at T = 0."""
    c = C0(t, tp)
    g = Gp(t + tp) / G(t + tp)
    return c * (g - Gp(2 * t) / G(2 * t)), c * (g - Gp(2 * tp) / G(2 * tp))


def dR0(t, tp):
    """(d/dt R, d/dt' R) at T = 0."""
    t, tp = np.broadcast_arrays(np.asarray(t, float), np.asarray(tp, float))
    sq = np.exp(0.5 * (logG(2 * tp) - logG(2 * t)))
    gp = Gp(t - tp)
    r = G(t - tp) * sq
    return gp * sq - r * Gp(2 * t) / G(2 * t), -gp * sq + r * Gp(2 * tp) / G(2 * tp)


# --------------------------------------------------------------------------- T > 0
class WarmP2:
    """Exact p = 2 solution at temperature T > 0 on [0, tmax], tabulated on a fine grid."""

    def __init__(self, T: float, tmax: float, delta: float = 2e-3):
        self.T, self.tmax = T, tmax
        n = int(round(tmax / delta))
        self.delta = tmax / n
        g1 = self._gamma(n)
        g2 = self._gamma(2 * n)
        self.s = np.linspace(0.0, tmax, n + 1)
        # Richardson on the common nodes
        self.gam = (4.0 * g2[::2] - g1) / 3.0
        self._g_fine = (g1, g2)

    def _gamma(self, n):
        T, d = self.T, self.tmax / n
        s = np.linspace(0.0, self.tmax, n + 1)
        Gv = G(2 * s)  # G(2 (t_n - t_k)) = Gv[n - k]
        gam = np.zeros(n + 1)
        gam[0] = 1.0
        for k in range(1, n + 1):
            acc = 0.5 * Gv[k] * gam[0] + np.dot(Gv[k - 1:0:-1], gam[1:k])
            gam[k] = (Gv[k] + 2 * T * d * acc) / (1.0 - T * d * Gv[0])
        return gam

    def _trap(self, n, idx_t, idx_tp, deriv=False):
        """int_0^{t'} G(t+t'-2s) Gamma(s) ds on the grid with n panels over [0, tmax]."""
        gam = self._g_fine[0] if n == self.s.size - 1 else self._g_fine[1]
        d = self.tmax / n
        sc = n // (self.s.size - 1)
        it, ip = idx_t * sc, idx_tp * sc
        s = np.arange(ip + 1) * d
        arg = (it + ip) * d - 2 * s
        gv = Gp(arg) if deriv else G(arg)
        w = np.full(ip + 1, d)
        if ip == 0:
            return 0.0
        w[0] = w[-1] = 0.5 * d
        return float(np.sum(w * gv * gam[: ip + 1]))

    def idx(self, t):
        return int(round(t / self.delta))

    def gamma_at(self, t):
        return self.gam[self.idx(t)]

    def C(self, t, tp):
        it, ip = self.idx(t), self.idx(tp)
        n1 = self.s.size - 1
        vals = []
        for n in (n1, 2 * n1):
            gam = self._g_fine[0] if n == n1 else self._g_fine[1]
            sc = n // n1
            num = G(np.array([(it + ip) * self.delta]))[0] + 2 * self.T * self._trap(n, it, ip)
            vals.append(num / np.sqrt(gam[it * sc] * gam[ip * sc]))
        return (4 * vals[1] - vals[0]) / 3

    def R(self, t, tp):
        return G(np.array([t - tp]))[0] * np.sqrt(self.gamma_at(tp) / self.gamma_at(t))

    def E(self, t):
        it = self.idx(t)
        n1 = self.s.size - 1
        vals = []
        for n in (n1, 2 * n1):
            gam = self._g_fine[0] if n == n1 else self._g_fine[1]
            sc = n // n1
            num = Gp(np.array([2 * it * self.delta]))[0] + 2 * self.T * self._trap(n, it, it, deriv=True)
            vals.append(-0.5 * num / gam[it * sc])
        return (4 * vals[1] - vals[0]) / 3
