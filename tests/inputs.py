"""Seeded synthetic inputs shared by the oracle and the HIP path.

Nothing here computes any step of the method: these are smooth test functions
sampled on given grids, and time grids.  Both sides receive the same arrays.
"""
from __future__ import annotations

import numpy as np


def geometric_times(M: int, t_last: float, t_first: float = 1e-3) -> np.ndarray:
    """t_0 = 0 followed by M-1 geometrically spaced times ending at t_last."""
    if M == 1:
        return np.zeros(1)
    return np.concatenate([[0.0], np.geomspace(t_first, t_last, M - 1)])


def smooth_history(th: np.ndarray, times: np.ndarray, seed: int):
    """A smooth two-time field pair sampled at (t_n, theta_i t_n), with its exact
    derivative along fixed theta.  C = exp(-k (1-theta) t) (1 + a sin(w theta + v t)),
    R = exp(-k2 (1-theta) t) (1 + b cos(w2 theta)), pinned to 1 at theta = 1."""
    rng = np.random.default_rng(seed)
    k, k2 = rng.uniform(0.3, 0.8, 2)
    a, b = rng.uniform(0.02, 0.08, 2)
    w, w2, v = rng.uniform(1.0, 4.0, 3)
    one = 1.0 - th
    C, R, dC, dR = [], [], [], []
    for t in times:
        e1 = np.exp(-k * one * t)
        s1 = 1 + a * np.sin(w * th + v * t) - a * np.sin(w + v * t)  # = 1 at theta = 1
        ds1 = a * v * (np.cos(w * th + v * t) - np.cos(w + v * t))
        C.append(e1 * s1)
        dC.append(-k * one * e1 * s1 + e1 * ds1)
        e2 = np.exp(-k2 * one * t)
        s2 = 1 + b * (np.cos(w2 * th) - np.cos(w2))
        R.append(e2 * s2)
        dR.append(-k2 * one * e2 * s2)
    C, R, dC, dR = (np.array(x) for x in (C, R, dC, dR))
    C[:, -1] = 1.0
    R[:, -1] = 1.0
    dC[:, -1] = 0.0
    dR[:, -1] = 0.0
    return C, R, dC, dR


def smooth_stage(th: np.ndarray, t: float, seed: int):
    """Stage slice (C, R) at time t from the same family as smooth_history."""
    C, R, _, _ = smooth_history(th, np.array([t]), seed)
    return C[0], R[0]


def sign_changing_history(th: np.ndarray, times: np.ndarray, seed: int):
    """As smooth_history, but R = exp(-k2 (1-theta) t) cos(w3 (1-theta) t) changes
    sign where (1-theta) t passes pi/(2 w3): stencils there hold values of both
    signs.  R = 1 at theta = 1."""
    rng = np.random.default_rng(seed)
    k2, w3 = rng.uniform(0.1, 0.3), rng.uniform(0.6, 1.2)
    C, _, dC, _ = smooth_history(th, times, seed)
    one = 1.0 - th
    R, dR = [], []
    for t in times:
        e2 = np.exp(-k2 * one * t)
        R.append(e2 * np.cos(w3 * one * t))
        dR.append(-one * e2 * (k2 * np.cos(w3 * one * t) + w3 * np.sin(w3 * one * t)))
    R, dR = np.array(R), np.array(dR)
    R[:, -1] = 1.0
    dR[:, -1] = 0.0
    return C, R, dC, dR


def sign_changing_stage(th: np.ndarray, t: float, seed: int):
    C, R, _, _ = sign_changing_history(th, np.array([t]), seed)
    return C[0], R[0]
