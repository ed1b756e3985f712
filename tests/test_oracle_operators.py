"""Pins for the oracle's finite-difference operators (Sec. 2.3 of the paper).

* the impulse response of every operator reproduces the weights printed in
  equations first_derivatives / second_derivatives / mixed_derivatives
  (tests/golden/paper_stencils.json);
* polynomial exactness with integer coordinates and unit spacing (exact FP64
  equality), and the exact first-failure constants;
* Fourier symbols on periodic grids and sixth-order convergence;
* the 19- and 55-point footprints of Sec. 2.3;
* the periodic ghost fill reproduces every periodic image bit for bit.
"""
import json
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")

AX = {"x": 2, "y": 1, "z": 0}  # direction -> array axis of a [z][y][x] array


def ghosted_from_function(fun, n=(9, 8, 7)):
    """Ghosted array (nz+6, ny+6, nx+6) with values fun(x, y, z) at integer
    coordinates x = i (i = -3 .. nx+2), NOT periodic."""
    nz, ny, nx = n
    z, y, x = np.meshgrid(np.arange(-3, nz + 3), np.arange(-3, ny + 3), np.arange(-3, nx + 3),
                          indexing="ij")
    return fun(x.astype(np.float64), y.astype(np.float64), z.astype(np.float64))


def test_impulse_response_matches_printed_stencils(orc):
    gold = json.load(open(os.path.join(GOLD, "paper_stencils.json")))
    n = 9
    h = 0.37
    # one-point impulse at the centre of a periodic 9^3 box
    f = np.zeros((n, n, n))
    c = n // 2
    f[c, c, c] = 1.0
    g = np.zeros((n + 6,) * 3)
    g[3:-3, 3:-3, 3:-3] = f
    g = orc.fill_ghosts(g)
    for axis in "xyz":
        ax = AX[axis]
        # operator applied to an impulse at offset 0 gives, at offset -o, the weight of tap +o
        d1 = orc.apply_op_ghosted(g, "d1" + axis, h, h, h)
        d2 = orc.apply_op_ghosted(g, "d2" + axis, h, h, h)
        for o in range(-3, 4):
            idx = [c, c, c]
            idx[ax] = c - o
            w1 = gold["d1"]["weights"][o + 3] / (60 * h)
            w2 = gold["d2"]["weights"][o + 3] / (180 * h * h)
            assert d1[tuple(idx)] == pytest.approx(w1, rel=1e-14, abs=1e-14)
            assert d2[tuple(idx)] == pytest.approx(w2, rel=1e-14, abs=1e-14)
        # no other point is touched by the axis stencils
        assert np.count_nonzero(d1) == 6
        assert np.count_nonzero(d2) == 7
    hx, hy, hz = 0.3, 0.5, 0.7
    for pair in ("xy", "xz", "yz"):
        hs = {"x": hx, "y": hy, "z": hz}
        dm = orc.apply_op_ghosted(g, "d" + pair, hx, hy, hz)
        a, b = pair
        den = 720 * hs[a] * hs[b]
        seen = 0
        for k, wk in zip((1, 2, 3), gold["mixed"]["diagonal_weights"]):
            # tap at (+k, +k) has weight +w, (-k, +k) -w, (-k, -k) +w, (+k, -k) -w
            for sa, sb, sign in ((1, 1, 1), (-1, 1, -1), (-1, -1, 1), (1, -1, -1)):
                idx = [c, c, c]
                idx[AX[a]] = c - sa * k
                idx[AX[b]] = c - sb * k
                assert dm[tuple(idx)] == pytest.approx(sign * wk / den, rel=1e-14)
                seen += 1
        assert np.count_nonzero(dm) == seen == 12


def test_footprints_are_19_and_55_points(orc):
    """Union of the taps the right-hand side reads: 19 (axis-aligned) or 55."""
    gold = json.load(open(os.path.join(GOLD, "paper_physics.json")))["stencil_sizes"]
    n = 9
    c = n // 2
    f = np.zeros((n, n, n))
    f[c, c, c] = 1.0
    g = orc.fill_ghosts(np.pad(f, 3))
    axis_ops = ["d1x", "d1y", "d1z", "d2x", "d2y", "d2z"]
    fp19 = sum(np.abs(orc.apply_op_ghosted(g, o)) for o in axis_ops)
    fp55 = fp19 + sum(np.abs(orc.apply_op_ghosted(g, o)) for o in ("dxy", "dxz", "dyz"))
    assert np.count_nonzero(fp19) == gold["axis_aligned"]
    assert np.count_nonzero(fp55) == gold["with_mixed"]


@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_d1_d2_polynomial_exactness(orc, axis):
    for deg in range(0, 9):
        g = ghosted_from_function(lambda x, y, z: {"x": x, "y": y, "z": z}[axis] ** deg)
        d1 = orc.apply_op_ghosted(g, "d1" + axis)
        d2 = orc.apply_op_ghosted(g, "d2" + axis)
        nz, ny, nx = d1.shape
        zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        s = {"x": xx, "y": yy, "z": zz}[axis].astype(np.float64)
        exact1 = deg * s ** (deg - 1) if deg >= 1 else np.zeros_like(s)
        exact2 = deg * (deg - 1) * s ** (deg - 2) if deg >= 2 else np.zeros_like(s)
        if deg <= 6:
            assert np.array_equal(d1, exact1), (axis, deg)
        if deg <= 7:
            assert np.array_equal(d2, exact2), (axis, deg)
    # first failures at the origin: D1(s^7)(0) = 36 h^6, D2(s^8)(0) = 72 h^6 (h = 1)
    g7 = ghosted_from_function(lambda x, y, z: {"x": x, "y": y, "z": z}[axis] ** 7)
    g8 = ghosted_from_function(lambda x, y, z: {"x": x, "y": y, "z": z}[axis] ** 8)
    assert orc.apply_op_ghosted(g7, "d1" + axis)[0, 0, 0] == 36.0
    assert orc.apply_op_ghosted(g8, "d2" + axis)[0, 0, 0] == 72.0


@pytest.mark.parametrize("pair", ["xy", "xz", "yz"])
def test_mixed_polynomial_exactness(orc, pair):
    a, b = pair
    for da in range(0, 8):
        for db in range(0, 8 - da):
            def fun(x, y, z):
                v = {"x": x, "y": y, "z": z}
                return v[a] ** da * v[b] ** db
            g = ghosted_from_function(fun)
            dm = orc.apply_op_ghosted(g, "d" + pair)
            nz, ny, nx = dm.shape
            zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
            v = {"x": xx, "y": yy, "z": zz}
            va, vb = v[a].astype(float), v[b].astype(float)
            ea = da * va ** (da - 1) if da >= 1 else 0 * va
            eb = db * vb ** (db - 1) if db >= 1 else 0 * vb
            assert np.array_equal(dm, ea * eb), (pair, da, db)
    # degree 8: a^1 b^7 and a^3 b^5 give 4 sum_k w_k k^8 / 720 = 36 at the origin
    for da, db in ((1, 7), (3, 5)):
        g = ghosted_from_function(lambda x, y, z: {"x": x, "y": y, "z": z}[a] ** da
                                  * {"x": x, "y": y, "z": z}[b] ** db)
        assert orc.apply_op_ghosted(g, "d" + pair)[0, 0, 0] == 36.0


def _periodic_ghosted(f, orc):
    return orc.fill_ghosts(np.pad(f, 3))


def _grid(n):
    x = np.arange(n) * 2 * np.pi / n
    return x


@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_fourier_symbols_and_sixth_order(orc, axis):
    """D1 sin(kx) = k1 cos(kx), D2 sin(kx) = -k2^2 sin(kx) with
    k1 h = (45 sin t - 9 sin 2t + sin 3t)/30 and
    k2^2 h^2 = (490 - 540 cos t + 54 cos 2t - 4 cos 3t)/180, t = k h;
    the errors against k and k^2 shrink as h^6."""
    k = 3
    errs1, errs2 = [], []
    for n in (24, 48, 96):
        shape = [8, 8, 8]
        shape[AX[axis]] = n
        h = 2 * np.pi / n
        s = _grid(n)
        bshape = [1, 1, 1]
        bshape[AX[axis]] = n
        f = np.broadcast_to(np.sin(k * s).reshape(bshape), shape).copy()
        cosf = np.broadcast_to(np.cos(k * s).reshape(bshape), shape)
        g = _periodic_ghosted(f, orc)
        hs = [1.0, 1.0, 1.0]
        hs["xyz".index(axis)] = h
        d1 = orc.apply_op_ghosted(g, "d1" + axis, *hs)
        d2 = orc.apply_op_ghosted(g, "d2" + axis, *hs)
        t = k * h
        k1 = (45 * math.sin(t) - 9 * math.sin(2 * t) + math.sin(3 * t)) / (30 * h)
        k2sq = (490 - 540 * math.cos(t) + 54 * math.cos(2 * t) - 4 * math.cos(3 * t)) / (180 * h * h)
        np.testing.assert_allclose(d1, k1 * cosf, atol=1e-12 * k)
        np.testing.assert_allclose(d2, -k2sq * f, atol=1e-11 * k * k)
        errs1.append(abs(k1 - k) / k)
        errs2.append(abs(k2sq - k * k) / k ** 2)
        # leading truncation terms: k1 = k (1 - t^6/140 + ...), k2^2 = k^2 (1 - t^6/560 + ...)
        assert errs1[-1] == pytest.approx(t ** 6 / 140, rel=0.15)
        assert errs2[-1] == pytest.approx(t ** 6 / 560, rel=0.15)
    for e in (errs1, errs2):
        for a, b in zip(e, e[1:]):
            assert 5.8 < math.log2(a / b) < 6.2


@pytest.mark.parametrize("pair", ["xy", "xz", "yz"])
def test_mixed_fourier_symbol(orc, pair):
    """D_ab cos(p a + q b) = -sigma cos(p a + q b) with
    sigma = sum_k w_k sin(k p ha) sin(k q hb) / (180 ha hb), w = (270, -27, 2);
    sigma -> p q as h -> 0."""
    n = (40, 48, 56)  # (nz, ny, nx)
    hs = {"x": 2 * np.pi / n[2], "y": 2 * np.pi / n[1], "z": 2 * np.pi / n[0]}
    z, y, x = np.meshgrid(*(np.arange(m) * 2 * np.pi / m for m in n), indexing="ij")
    v = {"x": x, "y": y, "z": z}
    a, b = pair
    p, q = 2, 3
    f = np.cos(p * v[a] + q * v[b])
    g = _periodic_ghosted(f, orc)
    dm = orc.apply_op_ghosted(g, "d" + pair, hs["x"], hs["y"], hs["z"])
    ha, hb = hs[a], hs[b]
    sigma = sum(w * math.sin(k * p * ha) * math.sin(k * q * hb)
                for k, w in ((1, 270), (2, -27), (3, 2))) / (180 * ha * hb)
    np.testing.assert_allclose(dm, -sigma * f, atol=1e-11)
    assert sigma == pytest.approx(p * q, rel=1e-2)


def test_periodic_sums_vanish(orc):
    """sum_i (D f)_i = 0 on a periodic grid (telescoping), to round-off."""
    rng = np.random.default_rng(3)
    f = rng.normal(size=(10, 11, 12))
    g = _periodic_ghosted(f, orc)
    for op in ("d1x", "d1y", "d1z", "d2x", "d2y", "d2z", "dxy", "dxz", "dyz"):
        d = orc.apply_op_ghosted(g, op, 0.1, 0.2, 0.3)
        assert abs(d.sum()) < 1e-11 * np.abs(d).sum(), op


def test_ghost_fill_is_periodic_image(orc):
    rng = np.random.default_rng(1)
    nz, ny, nx = 7, 9, 8
    f = rng.normal(size=(nz, ny, nx))
    g = np.full((nz + 6, ny + 6, nx + 6), np.nan)
    g[3:-3, 3:-3, 3:-3] = f
    g = orc.fill_ghosts(g)
    iz = (np.arange(-3, nz + 3) % nz)[:, None, None]
    iy = (np.arange(-3, ny + 3) % ny)[None, :, None]
    ix = (np.arange(-3, nx + 3) % nx)[None, None, :]
    assert np.array_equal(g, f[iz, iy, ix])
