"""Pins of the oracle's smoothing kernel (cubic spline, support 2h; Sec. 4.1).

The cubic spline is the unique piecewise cubic with compact support 2h that is
C2-continuous, even, and normalised; these checks fix each of those properties
on the oracle's own W and dW/dr, so a wrong coefficient, knot or normalisation
fails one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate

H = 0.012


def test_normalisation(orc):
    # integral of W over R^3 is 1
    v, _ = integrate.quad(lambda r: 4 * math.pi * r * r * orc.W(r, H), 0, 2 * H, points=[H],
                          epsabs=1e-15, epsrel=1e-14, limit=200)
    assert abs(v - 1.0) < 1e-12


def test_compact_support_and_continuity(orc):
    e = 1e-9 * H
    assert orc.W(2 * H, H) == 0.0 and orc.dWdr(2 * H, H) == 0.0
    assert orc.W(3 * H, H) == 0.0
    for knot in (H, 2 * H):
        assert abs(orc.W(knot - e, H) - orc.W(knot + e, H)) < 1e-6 * orc.W(0, H)
        assert abs(orc.dWdr(knot - e, H) - orc.dWdr(knot + e, H)) < 1e-6 * abs(orc.dWdr(H, H))
    # second derivative continuous at q = 1 (C2 spline)
    d = 1e-6 * H
    left = (orc.dWdr(H - d, H) - orc.dWdr(H - 2 * d, H)) / d
    right = (orc.dWdr(H + 2 * d, H) - orc.dWdr(H + d, H)) / d
    assert abs(left - right) < 1e-3 * abs(left)


def test_derivative_matches_finite_difference(orc):
    for q in (0.05, 0.3, 0.77, 0.99, 1.01, 1.4, 1.9):
        r = q * H
        d = 1e-7 * H
        fd = (orc.W(r + d, H) - orc.W(r - d, H)) / (2 * d)
        assert abs(fd - orc.dWdr(r, H)) < 1e-6 * abs(orc.dWdr(r, H)) + 1e-6


def test_peak_and_flat_top(orc):
    # maximum at the origin, zero slope there, monotone decreasing
    assert orc.dWdr(0.0, H) == 0.0
    r = np.linspace(0, 2 * H, 200)
    w = np.array([orc.W(x, H) for x in r])
    assert np.all(np.diff(w) <= 0)
    # value at the origin of a normalised M4 spline: 1/(pi h^3)
    assert abs(orc.W(0.0, H) * math.pi * H ** 3 - 1.0) < 1e-14


def test_lattice_partition_of_unity(orc):
    # sum_j dx^3 W_ij on an interior point of a cubic lattice with h = 1.2 dx:
    # 57 lattice points lie within 2h, and the sum is 1 up to O((dx/h)^2) terms.
    dx = H / 1.2
    rng = np.arange(-3, 4)
    tot, cnt = 0.0, 0
    for i in rng:
        for j in rng:
            for k in rng:
                r = dx * math.sqrt(i * i + j * j + k * k)
                if r < 2 * H:
                    cnt += 1
                    tot += dx ** 3 * orc.W(r, H)
    assert cnt == 57
    assert abs(tot - 1.0) < 2e-3


# --- quintic Wendland C2 kernel (the second kernel the paper's solver offers,
# Sec. 4.1): W = a (1 - q/2)^4 (2q + 1), a = 21 / (16 pi h^3), support 2h.

def test_wendland_normalisation(orc):
    v, _ = integrate.quad(lambda r: 4 * math.pi * r * r * orc.W(r, H, kernel=1), 0, 2 * H,
                          epsabs=1e-15, epsrel=1e-14, limit=200)
    assert abs(v - 1.0) < 1e-12


def test_wendland_support_smoothness_and_peak(orc):
    W = lambda r: orc.W(r, H, kernel=1)
    dW = lambda r: orc.dWdr(r, H, kernel=1)
    assert W(2 * H) == 0.0 and dW(2 * H) == 0.0 and W(2.5 * H) == 0.0
    assert dW(0.0) == 0.0
    assert abs(W(0.0) * 16 * math.pi * H ** 3 / 21 - 1.0) < 1e-14
    # C2 at the support edge: W'' -> 0 as q -> 2 (it is (1 - q/2)^2 times bounded terms)
    d = 1e-4 * H
    w2 = (dW(2 * H - d) - dW(2 * H - 2 * d)) / d
    w2_mid = (dW(H + d) - dW(H - d)) / (2 * d)
    assert abs(w2) < 1e-6 * abs(w2_mid)
    r = np.linspace(0, 2 * H, 200)
    w = np.array([W(x) for x in r])
    assert np.all(w >= 0) and np.all(np.diff(w) <= 0)


def test_wendland_derivative_matches_finite_difference(orc):
    for q in (0.05, 0.3, 0.77, 1.0, 1.4, 1.9):
        r = q * H
        d = 1e-7 * H
        fd = (orc.W(r + d, H, kernel=1) - orc.W(r - d, H, kernel=1)) / (2 * d)
        assert abs(fd - orc.dWdr(r, H, kernel=1)) < 1e-6 * abs(orc.dWdr(r, H, kernel=1)) + 1e-6
