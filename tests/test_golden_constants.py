"""The oracle's model functions against constants printed in the paper."""
import json
import os

import numpy as np

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_threshold_energy_identity():
    for p in GOLD["E_th_identity"]["pure_p"]:
        m = oracle.make_model({p: 1.0}, T=0.0)
        f, f1, f2 = oracle.f(m, 1.0), oracle.f1(m, 1.0), oracle.f2(m, 1.0)
        eth = (f - f1) / np.sqrt(f2) - f * np.sqrt(f2) / f1
        assert abs(eth + np.sqrt(2 * (p - 1) / p)) < 1e-14


def test_x_th_identity():
    for p in GOLD["x_th_T0_identity"]["pure_p"]:
        m = oracle.make_model({p: 1.0}, T=0.0)
        f1, f2 = oracle.f1(m, 1.0), oracle.f2(m, 1.0)
        assert abs(np.sqrt(f2) / f1 - 1 / np.sqrt(f2) - np.sqrt(2 / (p * (p - 1))) * (p - 2)) < 1e-14


def test_pure3_marginal_pair():
    g = GOLD["pure3_T_half"]
    m = oracle.make_model({3: g["a_p_squared"]}, T=g["T"])
    q = g["q_EA"]
    # marginal stability of the threshold states: f''(q) (1-q)^2 = T^2
    assert abs(oracle.f2(m, q) * (1 - q) ** 2 - g["T"] ** 2) < 2e-6
    # slope of chi vs C below q_EA: x/T with x = (p-2)(1-q)/q for a pure model
    assert abs((3 - 2) * (1 - q) / q / g["T"] - g["slope"]) < 2e-6
