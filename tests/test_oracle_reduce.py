"""Pins for the oracle's FP64 global diagnostics (mass, kinetic energy,
sum lnrho, max |u|, non-finite count).

Closed forms: the periodic trapezoid sum of a smooth periodic function is
spectrally exact, so lnrho = eps sin x gives mass (2 pi)^3 I0(eps), and
u = u0 sin(y) e_x with lnrho = 0 gives kinetic energy u0^2 (2 pi)^3 / 4.
"""
import math

import numpy as np
import pytest
from scipy.special import i0


def grid(n):
    return np.meshgrid(*(np.arange(m) * 2 * np.pi / m for m in n), indexing="ij")


def test_mass_closed_form(orc):
    n = (12, 10, 16)
    z, y, x = grid(n)
    eps = 0.4
    f = [eps * np.sin(x), np.zeros(n), np.zeros(n), np.zeros(n)]
    h = [2 * np.pi / m for m in n]
    r = orc.reduce(f, h[2], h[1], h[0])
    assert r["mass"] == pytest.approx((2 * np.pi) ** 3 * i0(eps), rel=1e-14)
    assert abs(r["sum_lnrho"]) < 1e-13
    assert r["kinetic_energy"] == 0.0
    assert r["nonfinite"] == 0


def test_kinetic_energy_closed_form(orc):
    n = (8, 14, 6)
    z, y, x = grid(n)
    u0 = 0.7
    f = [np.zeros(n), u0 * np.sin(y), np.zeros(n), np.zeros(n)]
    h = [2 * np.pi / m for m in n]
    r = orc.reduce(f, h[2], h[1], h[0])
    assert r["kinetic_energy"] == pytest.approx(u0 ** 2 * (2 * np.pi) ** 3 / 4, rel=1e-14)
    assert r["umax"] == pytest.approx(u0 * np.max(np.abs(np.sin(y))), rel=1e-15)


def test_sums_match_exact_summation(orc):
    rng = np.random.default_rng(0)
    n = (9, 10, 11)
    f = [rng.normal(0, 0.5, n), rng.normal(0, 1, n), rng.normal(0, 1, n), rng.normal(0, 1, n)]
    r = orc.reduce(f, 0.1, 0.2, 0.3)
    dv = 0.1 * 0.2 * 0.3
    rho = np.exp(f[0])
    mass = dv * math.fsum(rho.ravel())
    ke = dv * math.fsum((0.5 * rho * (f[1] ** 2 + f[2] ** 2 + f[3] ** 2)).ravel())
    assert r["mass"] == pytest.approx(mass, rel=1e-15)
    assert r["kinetic_energy"] == pytest.approx(ke, rel=1e-15)
    assert r["sum_lnrho"] == pytest.approx(math.fsum(f[0].ravel()), rel=1e-13, abs=1e-13)
    assert r["umax"] == np.sqrt(np.max(f[1] ** 2 + f[2] ** 2 + f[3] ** 2))


def test_nonfinite_count(orc):
    n = (6, 6, 6)
    f = [np.zeros(n) for _ in range(4)]
    f[0][1, 2, 3] = np.nan
    f[2][0, 0, 0] = np.inf
    f[3][0, 0, 0] = -np.inf  # same point as above: counted once
    f[1][5, 5, 5] = np.nan
    r = orc.reduce(f, 1, 1, 1)
    assert r["nonfinite"] == 3
