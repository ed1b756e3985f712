"""Pins of the oracle's external force (Sec. 6, eq. forcing): one Fourier mode
f(x) = Re{N f_k exp(i k.x + i phi)} added to the momentum equation, constant
over a full step and seen by every substep.

* the right-hand side of a rest state is exactly the force: a single Fourier
  mode at +-k (numpy FFT) with the drawn phase, whose amplitude vector is
  perpendicular to k (solenoidal) and to e, oriented along k x e, and scales
  like f0, dt^(-1/2) and |k|^(1/2) (white noise in time);
* a mode with k along z and f along x stays a linear shear wave (every
  nonlinear and pressure term vanishes): the fully discrete RK3 closed form
  U <- R(z) U + dt (1 + z/2 + z^2/6) a with z = -nu k2^2 dt holds to
  round-off for both methods (a force applied once per step, in one substep
  only, with a wrong sign or phase breaks it);
* the local patch update with the force equals the periodic run.
"""
import math

import numpy as np
import pytest

import synthetic_inputs as si

FORCE = {"k": (1.0, -2.0, 1.0), "e": (0.0, 0.0, 0.0), "f0": 0.02, "phase": 0.7}


@pytest.fixture(autouse=True)
def _no_force_after(orc):
    yield
    orc.set_forcing(None)


def unit_perp(k, seed=0):
    k = np.asarray(k, float)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=3)
    v -= (v @ k) / (k @ k) * k
    return tuple(v / np.linalg.norm(v))


def rest_state(n):
    shape = (n, n, n)
    return [np.full(shape, 0.25), np.zeros(shape), np.zeros(shape), np.zeros(shape)]


def test_rest_state_rhs_is_the_force_mode(orc):
    n = 16
    h = 2 * math.pi / n
    force = dict(FORCE, e=unit_perp(FORCE["k"]))
    a = orc.set_forcing(force, cs=1.0, dt=0.01)
    r = orc.rhs(rest_state(n), 1e-2, 1.0, h, h, h, "55p")
    assert np.all(r[0] == 0.0)
    k = np.array(force["k"])
    # amplitude vector: solenoidal, perpendicular to e, along k x e
    assert abs(a @ k) <= 1e-15 * np.linalg.norm(a)
    assert abs(a @ np.array(force["e"])) <= 1e-15 * np.linalg.norm(a)
    assert a @ np.cross(k, force["e"]) > 0
    for i in range(3):
        F = np.fft.fftn(r[1 + i])  # axes (z, y, x)
        kz, ky, kx = (int(v) % n for v in (k[2], k[1], k[0]))
        mkz, mky, mkx = (int(-v) % n for v in (k[2], k[1], k[0]))
        peak = F[kz, ky, kx]
        # every other coefficient vanishes
        rest = F.copy()
        rest[kz, ky, kx] = 0
        rest[mkz, mky, mkx] = 0
        assert np.max(np.abs(rest)) <= 1e-12 * n ** 3 * max(abs(a[i]), 1e-300)
        # cos(k.x + phi) = (e^{i(k.x+phi)} + c.c.) / 2: coefficient n^3 a e^{i phi} / 2
        expect = n ** 3 * a[i] * np.exp(1j * force["phase"]) / 2
        assert abs(peak - expect) <= 1e-12 * n ** 3 * max(abs(a[i]), 1e-300)


def test_force_scales_as_white_noise(orc):
    base = dict(FORCE, e=unit_perp(FORCE["k"], 1))
    a0 = np.linalg.norm(orc.set_forcing(base, cs=1.0, dt=0.01))
    assert np.linalg.norm(orc.set_forcing(dict(base, f0=2 * base["f0"]), 1.0, 0.01)) == \
        pytest.approx(2 * a0, rel=1e-14)
    assert np.linalg.norm(orc.set_forcing(base, 1.0, 0.04)) == pytest.approx(a0 / 2, rel=1e-14)
    k2 = tuple(2 * v for v in base["k"])
    assert np.linalg.norm(orc.set_forcing(dict(base, k=k2), 1.0, 0.01)) == \
        pytest.approx(math.sqrt(2) * a0, rel=1e-14)
    with pytest.raises(ValueError):
        orc.set_forcing(dict(base, e=tuple(np.array(base["k"]) / 6 ** 0.5)), 1.0, 0.01)


@pytest.mark.parametrize("variant", ["55p", "19p"])
def test_forced_shear_closed_form(orc, variant):
    n, nsteps, nu, dt = 32, 6, 2e-2, 0.01
    h = 2 * math.pi / n
    kz = 2
    force = {"k": (0.0, 0.0, float(kz)), "e": (0.0, 1.0, 0.0), "f0": 0.05, "phase": 0.4}
    a = orc.set_forcing(force, cs=1.0, dt=dt)
    assert a[1] == 0.0 and a[2] == 0.0 and a[0] < 0.0  # k x e = -2 x_hat
    out = orc.rk3(rest_state(n), nu, 1.0, h, h, h, dt, variant, nsteps)
    th = kz * h
    k2 = (490 - 540 * math.cos(th) + 54 * math.cos(2 * th) - 4 * math.cos(3 * th)) / (180 * h * h)
    z = -nu * k2 * dt
    R = 1 + z + z * z / 2 + z ** 3 / 6
    P = 1 + z / 2 + z * z / 6
    U = 0.0
    for _ in range(nsteps):
        U = R * U + dt * P * a[0]
    zc = np.arange(n) * h
    prof = U * np.cos(kz * zc + force["phase"])
    assert np.all(out[0] == 0.25)
    # the second differences of a field that is constant along an axis cancel
    # only to round-off, so the other components are zero to round-off
    assert np.max(np.abs(out[2])) <= 1e-15 * abs(U) and np.max(np.abs(out[3])) <= 1e-15 * abs(U)
    err = np.max(np.abs(out[1] - prof[:, None, None]))
    assert err <= 1e-13 * abs(U)
    # the damping makes U differ from the undamped n dt a by far more than the
    # tolerance, so the check resolves how the force enters the substeps
    assert abs(U - nsteps * dt * a[0]) > 1e-6 * abs(U)


@pytest.mark.parametrize("variant", ["55p", "19p"])
def test_patch_update_with_force_equals_periodic_run(orc, variant):
    w = si.noise_box((14, 16, 18), seed=31)
    force = {"k": (1.0, 2.0, -1.0), "e": unit_perp((1.0, 2.0, -1.0), 2), "f0": 0.03,
             "phase": 2.1}
    orc.set_forcing(force, cs=w.cs, dt=w.dt)
    full = orc.rk3(w.fields, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, 1)
    for c in [(0, 0, 0), (13, 15, 17), (7, 3, 11)]:
        pt = orc.rk3_point(w.fields, c, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, 1)
        for q in range(4):
            assert pt[q] == full[q][c]


def test_forcing_draws_are_valid(orc):
    draws = si.forcing_draws(50, 1.0, 2.0, 0.02, seed=4)
    ks = si.forcing_wavevectors(1.0, 2.0)
    kk = np.linalg.norm(ks, axis=1)
    assert kk.min() >= 1.0 and kk.max() <= 2.0 and len(ks) == 32  # 6 + 12 + 8 + 6
    for d in draws:
        k, e = np.array(d["k"]), np.array(d["e"])
        assert abs(np.linalg.norm(e) - 1) < 1e-14 and abs(k @ e) < 1e-14
        assert 0 <= d["phase"] < 2 * np.pi
