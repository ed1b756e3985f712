"""Second, independent FP64 formulation of the same scheme with whole-array
``np.roll`` shifts on periodic arrays (no ghost zone).  TEST INFRASTRUCTURE
ONLY; meant for tiny grids, where it cross-checks ``fd6_oracle.c``.

It follows the same passages of Pekkila et al. (2017): Sec. 2.3 for the three
operators, Sec. 2.1 for the right-hand side, Sec. 2.4 and Algorithm 1 for the
2N-RK3 substeps, Algorithm 3 for the 19-point variant.  Arrays are indexed
``[z, y, x]``; axis 2 is x.
"""
from __future__ import annotations

import numpy as np

ALPHA = (0.0, -5.0 / 9.0, -153.0 / 128.0)
BETA = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)
_AXIS = {0: 2, 1: 1, 2: 0}  # spatial direction (x, y, z) -> array axis


def _sh(f, d, k):
    """f at offset +k along direction d (x=0, y=1, z=2), periodic."""
    return np.roll(f, -k, axis=_AXIS[d])


def d1(f, d, h):
    """First derivative, eq. first_derivatives."""
    return (-_sh(f, d, -3) + 9 * _sh(f, d, -2) - 45 * _sh(f, d, -1)
            + 45 * _sh(f, d, 1) - 9 * _sh(f, d, 2) + _sh(f, d, 3)) / (60 * h)


def d2(f, d, h):
    """Second derivative, eq. second_derivatives with the 1/(180 h^2) prefactor."""
    return (2 * _sh(f, d, -3) - 27 * _sh(f, d, -2) + 270 * _sh(f, d, -1) - 490 * f
            + 270 * _sh(f, d, 1) - 27 * _sh(f, d, 2) + 2 * _sh(f, d, 3)) / (180 * h * h)


def dmix(f, a, b, ha, hb):
    """Bidiagonal mixed derivative, eq. mixed_derivatives."""
    def at(i, j):
        return _sh(_sh(f, a, i), b, j)
    tot = 0
    for k, w in ((1, 270), (2, -27), (3, 2)):
        tot = tot + w * (at(k, k) - at(-k, k) + at(-k, -k) - at(k, -k))
    return tot / (720 * ha * hb)


def rhs(fields, nu, cs, h, variant="55p"):
    """(d lnrho/dt, d u/dt) from eqs. continuity, navierstokes (f = 0), tensor;
    variant "55p" or "19p" (grad div u as D1 of D1 . u), or "no_graddiv"
    (without the (nu/3) grad div u term)."""
    lnrho, *u = fields
    g = [d1(lnrho, j, h[j]) for j in range(3)]
    J = [[d1(u[i], j, h[j]) for j in range(3)] for i in range(3)]
    div = J[0][0] + J[1][1] + J[2][2]
    r_lnrho = -sum(u[j] * g[j] for j in range(3)) - div
    if variant == "19p":
        dfield = div
        gdiv = [d1(dfield, i, h[i]) for i in range(3)]
    elif variant == "no_graddiv":  # the right-hand side of pass 1 of Algorithm 3
        gdiv = [0.0, 0.0, 0.0]
    out = [r_lnrho]
    for i in range(3):
        adv = sum(u[j] * J[i][j] for j in range(3))
        lap = sum(d2(u[i], j, h[j]) for j in range(3))
        S = [0.5 * (J[i][j] + J[j][i]) - (div / 3 if i == j else 0) for j in range(3)]
        sg = sum(S[j] * g[j] for j in range(3))
        if variant == "55p":
            gd = sum(d2(u[i], i, h[i]) if j == i else dmix(u[j], i, j, h[i], h[j])
                     for j in range(3))
        else:
            gd = gdiv[i]
        out.append(-adv - cs * cs * g[i] + nu * (lap + gd / 3 + 2 * sg))
    return out


def rk3(fields, nu, cs, h, dt, variant="55p", nsteps=1):
    """Algorithm 1 (a single fused pass per substep is the same arithmetic)."""
    f = [np.array(a, dtype=np.float64) for a in fields]
    w = [np.zeros_like(a) for a in f]
    for _ in range(nsteps):
        for s in range(3):
            r = rhs(f, nu, cs, h, variant)
            w = [ALPHA[s] * wq + dt * rq for wq, rq in zip(w, r)]
            f = [fq + BETA[s] * wq for fq, wq in zip(f, w)]
    return f
