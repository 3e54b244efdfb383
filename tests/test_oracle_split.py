"""Pins for the oracle's short-range split factor (sec. 3.1, Eq. equ:split).

g(x) = erfc(x) + (2x/sqrt(pi)) exp(-x^2) with x = s / (2 r_s) is pinned by
  * an independent 50-digit evaluation (mpmath),
  * g(0) = 1 and the hand-derived derivative g'(x) = -(4/sqrt(pi)) x^2 e^{-x^2},
  * the split identity: the PM side keeps the potential of a point mass
    smoothed by the Gaussian filter exp(-k^2 r_s^2), phi_long(s) = -erf(s/2r_s)/s
    (per G m); its force factor -s^2 d(phi_long)/ds, differentiated
    numerically at 50 digits, plus g must be exactly 1 (short + long =
    Newtonian 1/s^2).
"""
import math

import mpmath as mp
import numpy as np
import pytest


def g_ref(x):
    mp.mp.dps = 50
    x = mp.mpf(x)
    return mp.erfc(x) + 2 * x / mp.sqrt(mp.pi) * mp.exp(-x * x)


def test_split_factor_vs_mpmath(oracle_mod):
    xs = np.concatenate([np.linspace(0.0, 4.0, 161), [1e-8, 0.0078125, 2.25, 2.2500001, 5.5]])
    got = oracle_mod.split_factor(xs)
    for x, v in zip(xs, got):
        ref = float(g_ref(x))
        assert abs(v - ref) <= 4e-15 * abs(ref) + 1e-300, (x, v, ref)


def test_split_factor_at_zero_and_cut(oracle_mod):
    assert oracle_mod.split_factor(0.0)[0] == 1.0
    # at r_cut = 4.5 r_s, x = 2.25: about 1.75 % of the Newtonian force remains
    v = oracle_mod.split_factor(2.25)[0]
    assert abs(v - float(g_ref(2.25))) < 1e-16
    assert 0.0175 < v < 0.0176


def test_split_factor_derivative(oracle_mod):
    h = 1e-5
    for x in np.linspace(0.05, 3.5, 40):
        num = (oracle_mod.split_factor(x + h)[0] - oracle_mod.split_factor(x - h)[0]) / (2 * h)
        ana = -(4.0 / math.sqrt(math.pi)) * x * x * math.exp(-x * x)
        assert abs(num - ana) < 1e-9, (x, num, ana)


@pytest.mark.parametrize("rs", [0.7, 1.953125, 3.90625])
def test_split_identity_short_plus_long_is_newton(oracle_mod, rs):
    mp.mp.dps = 50
    rs_m = mp.mpf(rs)
    for s in np.linspace(0.01, 4.5 * rs, 37):
        phi_long = lambda r: -mp.erf(r / (2 * rs_m)) / r
        # attraction magnitude is dphi/ds; in units of the Newtonian 1/s^2:
        long_factor = mp.mpf(s) ** 2 * mp.diff(phi_long, mp.mpf(s))
        short = oracle_mod.split_factor(s / (2 * rs))[0]
        assert abs(short + float(long_factor) - 1.0) < 2e-15, (s, short, float(long_factor))
