"""FP64 CPU oracle for the sixth-order finite-difference RK3 substep.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product package never imports
this module and shares no code with it.

The arithmetic lives in ``fd6_oracle.c`` (plain loops, FP64, no FMA), which
follows Sec. 2.1 (equations continuity, navierstokes, tensor), Sec. 2.3
(equations first_derivatives, second_derivatives, mixed_derivatives), Sec. 2.4
(equation 2N-RK_scheme, Algorithm 1) and Sec. 4.2 (Algorithm 3, Appendix A) of
Pekkila et al. (2017).  This module only marshals numpy arrays into it.

Field arrays are compact, C-ordered ``[z][y][x]`` float64 arrays of shape
``(nz, ny, nx)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fd6_oracle.c")
_LIB = os.path.join(_HERE, "libfd6_oracle.so")

VARIANTS = {"55p": 0, "19p": 1}
OPS = {"d1x": 0, "d1y": 1, "d1z": 2, "d2x": 3, "d2y": 4, "d2z": 5, "dxy": 6, "dxz": 7, "dyz": 8}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, -O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        lib.orc_version.restype = i
        lib.orc_fill_ghosts.argtypes = [i, i, i, dp]
        lib.orc_apply_op_ghosted.argtypes = [i, i, i, dp, i, d, d, d, dp]
        lib.orc_apply_op_ghosted.restype = i
        lib.orc_rk3.argtypes = [i, i, i, dp, dp, dp, dp, d, d, d, d, d, d, i, i, i]
        lib.orc_rk3.restype = i
        lib.orc_rhs.argtypes = [i, i, i, dp, dp, dp, dp, d, d, d, d, d, i, dp, dp, dp, dp, i]
        lib.orc_rhs.restype = i
        lib.orc_rk3_patch.argtypes = [i, dp, dp, dp, dp, d, d, d, d, d, d, i, i, dp, dp, dp, dp]
        lib.orc_rk3_patch.restype = i
        lib.orc_reduce.argtypes = [i, i, i, dp, dp, dp, dp, d, d, d, dp]
        lib.orc_reduce.restype = i
        lib.orc_set_forcing.argtypes = [dp]
        lib.orc_set_forcing.restype = i
        lib.orc_get_forcing_amplitude.argtypes = [dp]
        lib.orc_get_forcing_amplitude.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fields(fields: Sequence[np.ndarray]):
    out = [np.ascontiguousarray(f, dtype=np.float64).copy() for f in fields]
    shape = out[0].shape
    assert len(out) == 4 and all(f.shape == shape for f in out) and len(shape) == 3
    return out, shape


def set_forcing(forcing=None, cs=1.0, dt=1.0):
    """External force of the momentum equation for every later call: one mode
    of eq. (forcing) with wave vector k, unit vector e, magnitude f0 and phase,
    given as ``{"k": (kx, ky, kz), "e": (ex, ey, ez), "f0": f0, "phase": phi}``
    (cs and dt enter its normalisation); None: no force.  Returns the force
    amplitude vector N f_k the oracle uses."""
    lib = _load()
    if forcing is None:
        lib.orc_set_forcing(None)
        return None
    v = np.array(list(forcing["k"]) + list(forcing["e"]) +
                 [forcing["f0"], forcing["phase"], cs, dt], dtype=np.float64)
    if lib.orc_set_forcing(_ptr(v)) != 0:
        raise ValueError("forcing: |k| = 0 or e parallel to k")
    a = np.zeros(3)
    lib.orc_get_forcing_amplitude(_ptr(a))
    return a


def rk3(fields, nu, cs, dx, dy, dz, dt, variant="55p", nsteps=1, threads=0):
    """Advance (lnrho, ux, uy, uz) by ``nsteps`` full RK3 steps; returns new arrays."""
    f, (nz, ny, nx) = _fields(fields)
    rc = _load().orc_rk3(nx, ny, nz, *[_ptr(a) for a in f], nu, cs, dx, dy, dz, dt,
                         VARIANTS[variant], nsteps, threads)
    if rc != 0:
        raise ValueError(f"orc_rk3 failed ({rc})")
    return f


def rhs(fields, nu, cs, dx, dy, dz, variant="55p", threads=0):
    """Time derivative of (lnrho, ux, uy, uz) of the given periodic state."""
    f, (nz, ny, nx) = _fields(fields)
    out = [np.empty((nz, ny, nx)) for _ in range(4)]
    rc = _load().orc_rhs(nx, ny, nz, *[_ptr(a) for a in f], nu, cs, dx, dy, dz,
                         VARIANTS[variant], *[_ptr(a) for a in out], threads)
    if rc != 0:
        raise ValueError(f"orc_rhs failed ({rc})")
    return out


def fill_ghosts(ghosted: np.ndarray) -> np.ndarray:
    """Periodic ghost fill of one ghosted array of shape (nz+6, ny+6, nx+6)."""
    g = np.ascontiguousarray(ghosted, dtype=np.float64).copy()
    nz, ny, nx = (s - 6 for s in g.shape)
    _load().orc_fill_ghosts(nx, ny, nz, _ptr(g))
    return g


def apply_op_ghosted(ghosted: np.ndarray, op: str, hx=1.0, hy=1.0, hz=1.0) -> np.ndarray:
    """One derivative operator at every interior point of a ghosted array whose
    ghost cells are already set (periodic or not)."""
    g = np.ascontiguousarray(ghosted, dtype=np.float64)
    nz, ny, nx = (s - 6 for s in g.shape)
    out = np.empty((nz, ny, nx))
    rc = _load().orc_apply_op_ghosted(nx, ny, nz, _ptr(g), OPS[op], hx, hy, hz, _ptr(out))
    if rc != 0:
        raise ValueError(op)
    return out


def patch_halfwidth(variant="55p", nsteps=1) -> int:
    """Half-width of the cube that determines one point after ``nsteps`` steps."""
    return nsteps * 3 * (3 if variant == "55p" else 6)


def rk3_point(fields, center, nu, cs, dx, dy, dz, dt, variant="55p", nsteps=1):
    """Value of (lnrho, ux, uy, uz) at grid point ``center`` = (k, j, i) after
    ``nsteps`` steps of the periodic box, computed from a local patch only."""
    m = patch_halfwidth(variant, nsteps)
    nz, ny, nx = fields[0].shape
    k, j, i = center
    iz = (np.arange(k - m, k + m + 1) % nz)[:, None, None]
    iy = (np.arange(j - m, j + m + 1) % ny)[None, :, None]
    ix = (np.arange(i - m, i + m + 1) % nx)[None, None, :]
    patch = [np.ascontiguousarray(f[iz, iy, ix], dtype=np.float64) for f in fields]
    # coordinates of the patch points, wrapped as in the periodic box
    coords = [np.ascontiguousarray(idx.ravel() * h, dtype=np.float64)
              for idx, h in ((ix, dx), (iy, dy), (iz, dz))]
    out = np.zeros(4)
    rc = _load().orc_rk3_patch(m, *[_ptr(a) for a in patch], nu, cs, dx, dy, dz, dt,
                               VARIANTS[variant], nsteps, *[_ptr(c) for c in coords], _ptr(out))
    if rc != 0:
        raise ValueError(f"orc_rk3_patch failed ({rc})")
    return out


def reduce(fields, dx, dy, dz):
    """(mass, kinetic energy, sum lnrho, max |u|, non-finite count) in FP64."""
    f, (nz, ny, nx) = _fields(fields)
    out = np.zeros(5)
    rc = _load().orc_reduce(nx, ny, nz, *[_ptr(a) for a in f], dx, dy, dz, _ptr(out))
    if rc != 0:
        raise MemoryError("orc_reduce")
    return {"mass": out[0], "kinetic_energy": out[1], "sum_lnrho": out[2], "umax": out[3],
            "nonfinite": int(out[4])}
