"""Pins for the oracle's right-hand side and time integrator.

Closed forms (exact up to round-off):
* shear wave u_b = u0 sin(k s_a): every nonlinear, pressure and grad-div term
  vanishes, so one RK3 step multiplies the amplitude by the cubic Taylor
  polynomial R(z) = 1 + z + z^2/2 + z^3/6 at z = -nu k2^2 dt (Sec. 6 shear-wave
  test, eq. dissipation; Sec. 2.4 eq. 2N-RK_scheme with a three-stage
  third-order scheme);
* linear sound wave lnrho = L sin(k s), u_s = U cos(k s): [L, U] advances by
  the matrix polynomial R(dt M), M = [[0, k1], [-cs^2 k1, -nu_eff]], with
  nu_eff = 4/3 nu k2^2 (55 points) or nu (k2^2 + k1^2/3) (19 points, whose
  grad-div is D1 of D1, Sec. 4.2 / Appendix A).

Properties of the continuum equations of Sec. 2.1 that the discrete
right-hand side must reproduce up to O(h^6):
* mass: d/dt int rho = 0;
* momentum: d/dt int rho u = 0 (needs every term of eq. navierstokes with the
  right sign and weight, including 2 S . grad lnrho and (1/3) grad div u);
* energy: d/dt int (rho u^2/2 + cs^2 rho ln rho) = -2 nu int rho S:S (needs
  the pressure term to match eq. continuity).

Exact to round-off on the periodic grid: the continuity right-hand side sums
to -sum u . D lnrho (the divergence telescopes), and to zero when lnrho is
uniform.

Exact symmetries: translation by whole cells (bitwise), axis permutation and
reflection (round-off), rest state (bitwise).
"""
import json
import math
import os

import numpy as np
import pytest

import synthetic_inputs as si
from oracle import numpy_ref

GOLD = os.path.join(os.path.dirname(__file__), "golden")
AX = {"x": 2, "y": 1, "z": 0}


def taylor3(z):
    return 1 + z + z * z / 2 + z ** 3 / 6


def k1_of(k, h):
    t = k * h
    return (45 * math.sin(t) - 9 * math.sin(2 * t) + math.sin(3 * t)) / (30 * h)


def k2sq_of(k, h):
    t = k * h
    return (490 - 540 * math.cos(t) + 54 * math.cos(2 * t) - 4 * math.cos(3 * t)) / (180 * h * h)


def line_field(shape, axis, values):
    b = [1, 1, 1]
    b[AX[axis]] = len(values)
    return np.broadcast_to(np.asarray(values).reshape(b), shape).copy()


def spacings(shape):
    nz, ny, nx = shape
    return 2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / nz


# --------------------------------------------------------------------------
# shear wave
# --------------------------------------------------------------------------

@pytest.mark.parametrize("variant", ["55p", "19p"])
@pytest.mark.parametrize("a,b", [("x", "y"), ("y", "z"), ("z", "x"), ("x", "z")])
def test_shear_wave_fully_discrete_closed_form(orc, variant, a, b):
    shape = [6, 6, 6]
    n = 16
    shape[AX[a]] = n
    shape = tuple(shape)
    h = spacings(shape)["xyz".index(a)]
    k, u0, nu, dt, nsteps = 3, 1e-3, 0.05, 0.03, 7
    s = np.arange(n) * 2 * np.pi / n
    f = [np.zeros(shape) for _ in range(4)]
    f[1 + "xyz".index(b)] = line_field(shape, a, u0 * np.sin(k * s))
    out = orc.rk3(f, nu, 1.0, *spacings(shape), dt, variant, nsteps)
    z = -nu * k2sq_of(k, h) * dt
    expect = line_field(shape, a, u0 * taylor3(z) ** nsteps * np.sin(k * s))
    np.testing.assert_allclose(out[1 + "xyz".index(b)], expect, rtol=0, atol=1e-15)
    for q in range(4):
        if q != 1 + "xyz".index(b):
            assert np.max(np.abs(out[q])) < 1e-18


def test_shear_wave_rk3_is_third_order_in_time(orc):
    """Against the semi-discrete solution exp(-nu k2^2 t), the error of the
    time integration falls by 2^3 per halving of dt."""
    shape = (6, 6, 16)
    h = 2 * np.pi / 16
    k, u0, nu, t_end = 3, 1.0, 0.4, 1.2
    s = np.arange(16) * h
    errs = []
    for nsteps in (20, 40, 80):
        dt = t_end / nsteps
        f = [np.zeros(shape) for _ in range(4)]
        f[2] = line_field(shape, "x", u0 * np.sin(k * s))
        out = orc.rk3(f, nu, 1.0, *spacings(shape), dt, "55p", nsteps)
        exact = u0 * math.exp(-nu * k2sq_of(k, h) * t_end)
        errs.append(abs(out[2][0, 0, 1] / math.sin(k * s[1]) - exact))
    for e0, e1 in zip(errs, errs[1:]):
        assert 2.85 < math.log2(e0 / e1) < 3.15


def test_shear_wave_convergence_against_continuum(orc):
    """Paper's test (Sec. 6): u = u0 sin(13 x) e_y decays as exp(-nu k^2 t);
    the deviation drops by about 2^5.7 per halving of dx."""
    gold = json.load(open(os.path.join(GOLD, "paper_physics.json")))["shear_wave"]
    k = gold["k"]
    u0, nu, t_end = 1e-3, 5e-3, 1.5
    errs = []
    for n in (96, 192, 384):
        shape = (6, 6, n)
        h = 2 * np.pi / n
        nsteps = int(round(t_end / (0.1 * h)))
        dt = t_end / nsteps
        s = np.arange(n) * h
        f = [np.zeros(shape) for _ in range(4)]
        f[2] = line_field(shape, "x", u0 * np.sin(k * s))
        out = orc.rk3(f, nu, 1.0, *spacings(shape), dt, "55p", nsteps)
        exact = u0 * math.exp(-nu * k * k * t_end) * np.sin(k * s)
        errs.append(np.sqrt(np.mean((out[2][0, 0, :] - exact) ** 2)))
    slopes = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    mean_slope = sum(slopes) / len(slopes)
    # the sixth-order operators give 6 asymptotically; the paper reports 5.7
    assert abs(mean_slope - gold["log2_error_ratio_per_halving"]) < 0.5, slopes


# --------------------------------------------------------------------------
# sound wave
# --------------------------------------------------------------------------

def sound_prediction(k, h, cs, nu, dt, nsteps, L0, variant):
    k1, k2sq = k1_of(k, h), k2sq_of(k, h)
    nu_eff = nu * (4.0 / 3.0) * k2sq if variant == "55p" else nu * (k2sq + k1 * k1 / 3.0)
    M = np.array([[0.0, k1], [-cs * cs * k1, -nu_eff]]) * dt
    P = np.eye(2) + M + M @ M / 2 + M @ M @ M / 6
    v = np.array([L0, 0.0])
    for _ in range(nsteps):
        v = P @ v
    return v


@pytest.mark.parametrize("variant", ["55p", "19p"])
@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_sound_wave_fully_discrete_closed_form(orc, variant, axis):
    n, k, cs, nu, dt, nsteps, A = 16, 3, 1.3, 0.05, 0.05, 20, 1e-9
    shape = [6, 6, 6]
    shape[AX[axis]] = n
    shape = tuple(shape)
    h = 2 * np.pi / n
    s = np.arange(n) * h
    f = [np.zeros(shape) for _ in range(4)]
    f[0] = line_field(shape, axis, A * np.sin(k * s))
    out = orc.rk3(f, nu, cs, *spacings(shape), dt, variant, nsteps)
    L, U = sound_prediction(k, h, cs, nu, dt, nsteps, A, variant)
    q = 1 + "xyz".index(axis)
    np.testing.assert_allclose(out[0], line_field(shape, axis, L * np.sin(k * s)), atol=1e-8 * A)
    np.testing.assert_allclose(out[q], line_field(shape, axis, U * np.cos(k * s)), atol=1e-8 * A)
    # the other discretisation's prediction is far away: the test tells them apart
    other = "19p" if variant == "55p" else "55p"
    L2, U2 = sound_prediction(k, h, cs, nu, dt, nsteps, A, other)
    assert abs(U2 - U) > 1e-3 * A


# --------------------------------------------------------------------------
# conservation laws of the continuum equations
# --------------------------------------------------------------------------

def smooth_fields(n, seed=5, amp=0.3, kmax=2.0, nmodes=4):
    """Fields as explicit Fourier sums together with their exact gradients."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*(np.arange(n) * 2 * np.pi / n,) * 3, indexing="ij")
    X = (x, y, z)
    vals, grads = [], []
    for _ in range(4):
        ks, ph = si.draw_modes(rng, nmodes, kmax)
        f = np.zeros((n, n, n))
        g = [np.zeros((n, n, n)) for _ in range(3)]
        for kv, p in zip(ks, ph):
            arg = kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2] + p
            f += amp * np.cos(arg)
            for j in range(3):
                g[j] += -amp * kv[j] * np.sin(arg)
        vals.append(f)
        grads.append(g)
    return vals, grads


@pytest.mark.parametrize("variant", ["55p", "19p"])
def test_mass_momentum_energy_balance(orc, variant):
    nu, cs = 0.05, 0.9
    residuals = []
    for n in (16, 32):
        f, grads = smooth_fields(n)
        h = 2 * np.pi / n
        r = orc.rhs(f, nu, cs, h, h, h, variant)
        rho = np.exp(f[0])
        u = f[1:]
        dv = h ** 3
        dmass = np.sum(rho * r[0]) * dv
        mscale = np.sum(np.abs(rho * r[0])) * dv
        res = [abs(dmass) / mscale]
        for i in range(3):
            dp = np.sum(rho * (r[1 + i] + u[i] * r[0])) * dv
            pscale = np.sum(np.abs(rho * r[1 + i]) + np.abs(rho * u[i] * r[0])) * dv
            res.append(abs(dp) / pscale)
        J = [[grads[1 + i][j] for j in range(3)] for i in range(3)]
        div = J[0][0] + J[1][1] + J[2][2]
        SS = 0
        for i in range(3):
            for j in range(3):
                sij = 0.5 * (J[i][j] + J[j][i]) - (div / 3 if i == j else 0)
                SS = SS + sij * sij
        u2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
        dE = np.sum(rho * (u[0] * r[1] + u[1] * r[2] + u[2] * r[3]
                           + (0.5 * u2 + cs * cs * (f[0] + 1)) * r[0])) * dv
        diss = -2 * nu * np.sum(rho * SS) * dv
        escale = np.sum(np.abs(rho * (u[0] * r[1] + u[1] * r[2] + u[2] * r[3]))) * dv
        res.append(abs(dE - diss) / escale)
        residuals.append(res)
    coarse, fine = residuals
    for c_, f_ in zip(coarse, fine):
        # the continuum balance holds up to the O(h^6) truncation error
        assert f_ < 2e-5, residuals
        assert c_ / f_ > 16 or f_ < 1e-12, residuals


@pytest.mark.parametrize("variant", ["55p", "19p"])
def test_continuity_sum_identities_to_round_off(orc, variant):
    """The exact discrete counterpart of mass conservation.  The continuity
    right-hand side is -u . D lnrho - D . u (eq. continuity), and every
    first-derivative stencil of Sec. 2.3 sums to zero over a periodic grid
    (it telescopes).  So, to round-off:
    * with uniform lnrho, sum_i r_lnrho = 0 for any velocity field (Sigma
      lnrho is constant to first order in dt);
    * in general, sum_i r_lnrho = -sum_i u . D lnrho, with D taken from the
      independent np.roll formulation.
    Mass itself, sum exp(lnrho), is not a discrete invariant of the ln rho
    form: it holds to the O(h^6) truncation error
    (test_mass_momentum_energy_balance)."""
    rng = np.random.default_rng(11)
    shape = (12, 10, 14)
    h = (0.3, 0.4, 0.5)  # dx, dy, dz
    u = [rng.normal(scale=0.1, size=shape) for _ in range(3)]
    r = orc.rhs([np.full(shape, 0.3)] + u, 0.02, 1.0, *h, variant)
    assert abs(r[0].sum()) < 1e-13 * np.abs(r[0]).sum()
    lnrho = rng.normal(scale=0.05, size=shape)
    r = orc.rhs([lnrho] + u, 0.02, 1.0, *h, variant)
    adv = sum(u[j] * numpy_ref.d1(lnrho, j, h[j]) for j in range(3))
    tol = 1e-13 * np.abs(r[0]).sum()
    assert abs(r[0].sum() + adv.sum()) < tol
    # not satisfied trivially: a planted sign error in the advection term
    # misses the identity by about 10^9 times the tolerance
    assert abs(r[0].sum() - adv.sum()) > 1e6 * tol


def test_balance_detects_a_planted_sign_error(orc):
    """A plausible mistake (flipped sign of 2 S.grad lnrho) breaks the
    momentum balance by orders of magnitude: the balance test has teeth."""
    n, nu, cs = 32, 0.05, 0.9
    f, _ = smooth_fields(n)
    h = 2 * np.pi / n
    r = numpy_ref.rhs(f, nu, cs, (h, h, h))
    # rebuild the viscous S.grad lnrho term and subtract it twice
    g = [numpy_ref.d1(f[0], j, h) for j in range(3)]
    J = [[numpy_ref.d1(f[1 + i], j, h) for j in range(3)] for i in range(3)]
    div = J[0][0] + J[1][1] + J[2][2]
    rho = np.exp(f[0])
    bad = []
    for i in range(3):
        sg = sum((0.5 * (J[i][j] + J[j][i]) - (div / 3 if i == j else 0)) * g[j] for j in range(3))
        bad.append(r[1 + i] - 2 * nu * 2 * sg)
    worst = max(abs(np.sum(rho * (bad[i] + f[1 + i] * r[0]))) /
                np.sum(np.abs(rho * bad[i]) + np.abs(rho * f[1 + i] * r[0])) for i in range(3))
    assert worst > 1e-3


# --------------------------------------------------------------------------
# symmetries and special states
# --------------------------------------------------------------------------

def test_rest_state_is_bitwise_fixed(orc):
    shape = (7, 8, 9)
    f = [np.full(shape, 0.3), np.zeros(shape), np.zeros(shape), np.zeros(shape)]
    for variant in ("55p", "19p"):
        out = orc.rk3(f, 0.01, 1.0, *spacings(shape), 0.05, variant, 2)
        for a, b in zip(out, f):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", ["55p", "19p"])
def test_translation_equivariance_bitwise(orc, variant):
    w = si.noise_box((10, 11, 12), seed=2)
    shift = (2, -3, 5)
    out = orc.rk3(w.fields, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, 1)
    rolled = [np.roll(f, shift, axis=(0, 1, 2)) for f in w.fields]
    out2 = orc.rk3(rolled, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, 1)
    for a, b in zip(out2, out):
        assert np.array_equal(a, np.roll(b, shift, axis=(0, 1, 2)))


@pytest.mark.parametrize("variant", ["55p", "19p"])
def test_axis_permutation_and_reflection(orc, variant):
    w = si.noise_box((10, 10, 10), seed=4)
    h = w.dx
    out = orc.rk3(w.fields, w.nu, w.cs, h, h, h, w.dt, variant, 1)
    # swap x and y: array axes 2 and 1, components ux <-> uy
    sw = lambda a: np.ascontiguousarray(np.swapaxes(a, 1, 2))
    f = w.fields
    fs = [sw(f[0]), sw(f[2]), sw(f[1]), sw(f[3])]
    o = orc.rk3(fs, w.nu, w.cs, h, h, h, w.dt, variant, 1)
    for a, b in zip(o, [sw(out[0]), sw(out[2]), sw(out[1]), sw(out[3])]):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)
    # reflect x: index i -> -i mod n, ux -> -ux
    rf = lambda a: np.ascontiguousarray(np.roll(a[:, :, ::-1], 1, axis=2))
    fr = [rf(f[0]), -rf(f[1]), rf(f[2]), rf(f[3])]
    o = orc.rk3(fr, w.nu, w.cs, h, h, h, w.dt, variant, 1)
    for a, b in zip(o, [rf(out[0]), -rf(out[1]), rf(out[2]), rf(out[3])]):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# implementation cross-checks
# --------------------------------------------------------------------------

@pytest.mark.parametrize("variant", ["55p", "19p"])
@pytest.mark.parametrize("shape", [(7, 9, 8), (6, 6, 13)])
def test_c_oracle_matches_numpy_formulation(orc, variant, shape):
    w = si.noise_box(shape, seed=7)
    h = (w.dx, w.dy, w.dz)
    a = orc.rk3(w.fields, w.nu, w.cs, *h, w.dt, variant, 2)
    b = numpy_ref.rk3(w.fields, w.nu, w.cs, h, w.dt, variant, 2)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-14 * np.abs(y).max())
    ra = orc.rhs(w.fields, w.nu, w.cs, *h, variant)
    rb = numpy_ref.rhs(w.fields, w.nu, w.cs, h, variant)
    for x, y in zip(ra, rb):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-13 * np.abs(y).max())


@pytest.mark.parametrize("variant,nsteps", [("55p", 1), ("55p", 2), ("19p", 1)])
def test_patch_update_equals_periodic_run(orc, variant, nsteps):
    """A point's value after n steps depends only on its neighbourhood of
    half-width 9n (55p) or 18n (19p); the patch evaluation is bitwise the
    periodic run."""
    w = si.noise_box((12, 11, 13), seed=9)
    out = orc.rk3(w.fields, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, nsteps)
    for c in [(0, 0, 0), (5, 10, 12), (11, 3, 7)]:
        v = orc.rk3_point(w.fields, c, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, nsteps)
        assert np.array_equal(v, np.array([o[c] for o in out]))


def test_19p_two_pass_equals_single_pass_with_d1d1_graddiv(orc):
    """Appendix A: the two passes of Algorithm 3 -- pass 1 with the
    right-hand side lacking (nu/3) grad div u and the divergence stored, pass
    2 adding dt (nu/3) D1_i(div) to w and beta times it to the output -- add
    up to the oracle's single 2N-RK3 update with the full 19-point
    right-hand side (grad div term D1_i of D1 . u)."""
    w = si.noise_box((8, 9, 10), seed=11)
    h = (w.dx, w.dy, w.dz)
    f = [np.array(a) for a in w.fields]
    wr = [np.zeros_like(a) for a in f]
    for s in range(3):
        rp = numpy_ref.rhs(f, w.nu, w.cs, h, "no_graddiv")
        div = sum(numpy_ref.d1(f[1 + j], j, h[j]) for j in range(3))
        wr = [numpy_ref.ALPHA[s] * a + w.dt * b for a, b in zip(wr, rp)]
        out = [a + numpy_ref.BETA[s] * b for a, b in zip(f, wr)]
        for i in range(3):
            t = w.dt * (w.nu / 3.0) * numpy_ref.d1(div, i, h[i])
            wr[1 + i] = wr[1 + i] + t
            out[1 + i] = out[1 + i] + numpy_ref.BETA[s] * t
        f = out
    one = orc.rk3(w.fields, w.nu, w.cs, *h, w.dt, "19p", 1)
    for a, b in zip(f, one):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-15 * max(1, np.abs(b).max()))
    # and it is a different discretisation from the 55-point one
    d55 = orc.rk3(w.fields, w.nu, w.cs, *h, w.dt, "55p", 1)
    assert max(np.abs(a - b).max() for a, b in zip(one[1:], d55[1:])) > 1e-9
