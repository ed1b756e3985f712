"""Seeded synthetic inputs for the isothermal compressible-flow substep.

This module is shared by the oracle side (tests, CPU baseline) and the GPU side
(tests, benchmark).  It holds only input synthesis -- random fields, Fourier
sums, the time-step rule -- and none of the method's arithmetic.

Conventions
-----------
* Arrays are float64, C-ordered ``[z][y][x]`` with shape ``(nz, ny, nx)``.
* The periodic box is ``[0, 2 pi)^3`` with ``x_i = i * 2 pi / n``.
* Random draws use ``numpy.random.default_rng(seed)`` (PCG64) in the fixed
  order lnrho, ux, uy, uz.
* A "random-phase Fourier field" of amplitude A with M modes is
  ``A / sqrt(M) * sum_m cos(k_m . x + phi_m)`` with distinct integer wave
  vectors ``1 <= |k_m| <= kmax`` and ``phi_m ~ U[0, 2 pi)``; its RMS is
  ``A / sqrt(2)``, the RMS of a single mode of amplitude A.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

TWO_PI = 2.0 * math.pi


def spacing(n: int) -> float:
    return TWO_PI / n


def cfl_dt(fields, dx, dy, dz, cs: float = 1.0, courant: float = 0.4) -> float:
    """dt = courant * min(dx, dy, dz) / (cs + max |u|), from the initial state."""
    _, ux, uy, uz = fields
    umax = float(np.sqrt(np.max(ux * ux + uy * uy + uz * uz)))
    return courant * min(dx, dy, dz) / (cs + umax)


# --------------------------------------------------------------------------
# Fourier sums
# --------------------------------------------------------------------------

def draw_modes(rng: np.random.Generator, nmodes: int, kmax: float) -> Tuple[np.ndarray, np.ndarray]:
    """Distinct integer wave vectors with 1 <= |k| <= kmax, and phases."""
    kint = int(math.floor(kmax))
    ks: List[Tuple[int, int, int]] = []
    seen = set()
    while len(ks) < nmodes:
        k = tuple(int(v) for v in rng.integers(-kint, kint + 1, size=3))
        n2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2]
        if n2 == 0 or n2 > kmax * kmax or k in seen:
            continue
        seen.add(k)
        ks.append(k)
    phases = rng.uniform(0.0, TWO_PI, size=nmodes)
    return np.array(ks, dtype=np.int64), phases


def _expo(kcomp: np.ndarray, n: int) -> np.ndarray:
    """exp(i k x_j) for x_j = 2 pi j / n, with the angle reduced exactly."""
    j = np.arange(n, dtype=np.int64)
    m = np.mod(np.outer(kcomp, j), n).astype(np.float64)
    ang = TWO_PI * m / n
    return np.cos(ang) + 1j * np.sin(ang)


def fourier_field(shape, ks: np.ndarray, phases: np.ndarray, amplitude: float) -> np.ndarray:
    """A / sqrt(M) * sum_m cos(k_m . x + phi_m) on a (nz, ny, nx) periodic grid."""
    nz, ny, nx = shape
    M = len(ks)
    ex = _expo(ks[:, 0], nx)                      # (M, nx)
    ey = _expo(ks[:, 1], ny)                      # (M, ny)
    ez = _expo(ks[:, 2], nz) * np.exp(1j * phases)[:, None]  # (M, nz)
    c = (ez[:, :, None] * ey[:, None, :]).reshape(M, nz * ny).T  # (nz*ny, M)
    a = np.concatenate([c.real, -c.imag], axis=1)            # (nz*ny, 2M)
    b = np.concatenate([ex.real, ex.imag], axis=0)            # (2M, nx)
    out = (a @ b).reshape(nz, ny, nx)
    out *= amplitude / math.sqrt(M)
    return np.ascontiguousarray(out)


def fourier_fields(shape, seed: int, amplitude: float, kmax: float, nmodes: int = 16):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(4):  # lnrho, ux, uy, uz
        ks, ph = draw_modes(rng, nmodes, kmax)
        out.append(fourier_field(shape, ks, ph, amplitude))
    return out


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    shape: Tuple[int, int, int]         # (nz, ny, nx)
    fields: list
    nu: float
    cs: float
    dx: float
    dy: float
    dz: float
    dt: float
    meta: dict = field(default_factory=dict)


def _make(name, shape, fields, nu, cs=1.0, meta=None, dt=None):
    nz, ny, nx = shape
    dx, dy, dz = spacing(nx), spacing(ny), spacing(nz)
    if dt is None:
        dt = cfl_dt(fields, dx, dy, dz, cs)
    return Workload(name, shape, fields, nu, cs, dx, dy, dz, dt, meta or {})


def noise_box(shape=(32, 32, 32), seed: int = 0, nu: float = 5e-3) -> Workload:
    """lnrho ~ U(-1e-3, 1e-3), u_i ~ Normal(0, 1e-2), on any (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    lnrho = rng.uniform(-1e-3, 1e-3, size=shape)
    u = [rng.normal(0.0, 1e-2, size=shape) for _ in range(3)]
    return _make(f"noise{shape}", tuple(shape), [lnrho] + u, nu,
                 meta={"recipe": "lnrho U(-1e-3,1e-3); u N(0,1e-2)", "seed": seed})


def small_parity_box(seed: int = 0) -> Workload:
    """32^3 periodic box, noise fields, nu = 5e-3, dt = 0.4 CFL, seed 0."""
    w = noise_box((32, 32, 32), seed=seed, nu=5e-3)
    w.name = "32^3 noise box"
    return w


def fourier_box(n: int, seed: int = 0, amplitude: float = 1e-2, kmax: float = 8.0,
                nu: float = 2e-3, shape=None) -> Workload:
    shape = tuple(shape) if shape is not None else (n, n, n)
    f = fourier_fields(shape, seed, amplitude, kmax)
    return _make(f"{shape[2]}x{shape[1]}x{shape[0]} random-phase |k|<={kmax:g} A={amplitude:g}",
                 shape, f, nu,
                 meta={"recipe": "16 random-phase modes per field", "seed": seed,
                       "amplitude": amplitude, "kmax": kmax})


def mid_box(n: int = 128, seed: int = 0) -> Workload:
    """128^3: 16 random-phase modes, |k| <= 8, A = 1e-2, nu = 2e-3."""
    return fourier_box(n, seed, amplitude=1e-2, kmax=8.0, nu=2e-3)


def large_box(n: int = 512, seed: int = 0) -> Workload:
    """256^3 / 512^3: 16 random-phase modes, |k| <= 16, A = 0.1, nu = 1e-3."""
    return fourier_box(n, seed, amplitude=0.1, kmax=16.0, nu=1e-3)


def sound_wave_box(n: int = 768, amplitude: float = 1e-4, k: int = 4, nu: float = 1e-4,
                   shape=None) -> Workload:
    """lnrho = A sin(k x), u = 0; dt = 0.4 dx (cs = 1, u = 0)."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    nz, ny, nx = shape
    x = np.arange(nx) * spacing(nx)
    lnrho = np.broadcast_to(amplitude * np.sin(k * x), shape).copy()
    z = np.zeros(shape)
    return _make(f"sound wave {nx}x{ny}x{nz} k={k}", shape, [lnrho, z, z.copy(), z.copy()], nu,
                 meta={"amplitude": amplitude, "k": k})


@dataclass
class EnsembleMember:
    seed: int
    n: int
    workload: Workload


def ensemble(nboxes: int = 64, sizes=(32, 48, 64, 96), nmodes: int = 16) -> List[EnsembleMember]:
    """Independent periodic boxes: box b draws, from default_rng(b), its edge n_b
    from ``sizes``, nu_b ~ U[1e-3, 1e-2], A_b ~ U[1e-3, 1e-1], then its four
    fields (16 modes, |k| <= n_b / 8)."""
    out = []
    for b in range(nboxes):
        rng = np.random.default_rng(b)
        n = int(rng.choice(np.array(sizes)))
        nu = float(rng.uniform(1e-3, 1e-2))
        amp = float(rng.uniform(1e-3, 1e-1))
        f = []
        for _ in range(4):
            ks, ph = draw_modes(rng, nmodes, n / 8.0)
            f.append(fourier_field((n, n, n), ks, ph, amp))
        w = _make(f"box{b} n={n}", (n, n, n), f, nu, meta={"seed": b, "amplitude": amp})
        out.append(EnsembleMember(b, n, w))
    return out


def as_float32_exact(fields):
    """The FP32 values a float32 store of these fields holds, as float64 (round
    to nearest even, done on the host by numpy)."""
    return [np.asarray(f, dtype=np.float32).astype(np.float64) for f in fields]


# ---------------------------------------------------------------------------
# Random draws of the forcing (Sec. 6): the method picks, at every time step,
# a wave vector from an isotropic set, a unit vector e perpendicular to it and
# a phase.  These draws are inputs to both the library and the oracle; the
# force itself (its normalisation and direction) is computed by each of them.
# ---------------------------------------------------------------------------
def forcing_wavevectors(kmin: float, kmax: float) -> np.ndarray:
    """All integer wave vectors of a 2 pi periodic box with kmin <= |k| <= kmax."""
    m = int(np.floor(kmax))
    r = np.arange(-m, m + 1)
    k = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    kk = np.linalg.norm(k, axis=1)
    return k[(kk >= kmin) & (kk <= kmax) & (kk > 0)].astype(np.float64)


def forcing_draws(nsteps: int, kmin: float, kmax: float, f0: float, seed: int = 0) -> List[dict]:
    """Per time step: k uniformly from the isotropic set, e a uniformly random
    unit vector perpendicular to k, phase uniform in [0, 2 pi)."""
    ks = forcing_wavevectors(kmin, kmax)
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nsteps):
        k = ks[rng.integers(len(ks))]
        khat = k / np.linalg.norm(k)
        t = np.array([1.0, 0.0, 0.0]) if abs(khat[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        b1 = t - (t @ khat) * khat
        b1 /= np.linalg.norm(b1)
        b2 = np.cross(khat, b1)
        th = rng.uniform(0.0, 2.0 * np.pi)
        e = np.cos(th) * b1 + np.sin(th) * b2
        out.append({"k": tuple(k), "e": tuple(e), "f0": f0,
                    "phase": float(rng.uniform(0.0, 2.0 * np.pi))})
    return out


def explosion_box(n: int = 64, nu: float = 5e-3, u_ampl: float = 1.0, d_shell: float = 0.2,
                  r_shell: float = 0.8) -> Workload:
    """Radial kinetic explosion of Sec. 6: rho = 1 (lnrho = 0) and
    u = u_ampl exp(-(r - r_shell)^2 / (2 d_shell^2)) e_r about the domain
    centre (pi, pi, pi), which is grid point n / 2 for even n.  (The printed
    exponent lacks its minus sign; the Gaussian shell decays away from
    r_shell.)"""
    h = spacing(n)
    c = np.arange(n) * h - math.pi
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    prof = u_ampl * np.exp(-((r - r_shell) ** 2) / (2.0 * d_shell ** 2))
    with np.errstate(invalid="ignore", divide="ignore"):
        inv = np.where(r > 0, 1.0 / r, 0.0)
    fields = [np.zeros((n, n, n)), prof * x * inv, prof * y * inv, prof * z * inv]
    return _make(f"explosion {n}^3", (n, n, n), fields, nu,
                 meta={"u_ampl": u_ampl, "d_shell": d_shell, "r_shell": r_shell})


def axis_line_integrals(field: np.ndarray) -> np.ndarray:
    """Line integrals of a field along the 7 axes through the centre of an
    even-sized cubic 2 pi box (x, y, z and the 4 body diagonals), over
    r <= pi on every axis, by the trapezoid rule with the point spacing of
    the axis (delta on the coordinate axes, sqrt(3) delta on the diagonals).
    The grid cannot give every axis the same extent, so fields with a
    background should have it subtracted first."""
    n = field.shape[0]
    c = n // 2
    h = spacing(n)
    m = np.arange(-c, c + 1)
    out = []
    for step, dirs in ((h, ((0, 0, 1), (0, 1, 0), (1, 0, 0))),
                       (math.sqrt(3.0) * h, ((1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1)))):
        mm = m[np.abs(m) * step <= math.pi + 1e-12]
        for dz, dy, dx in dirs:
            vals = field[(c + dz * mm) % n, (c + dy * mm) % n, (c + dx * mm) % n]
            out.append(step * float(np.sum(vals) - 0.5 * (vals[0] + vals[-1])))
    return np.array(out)
