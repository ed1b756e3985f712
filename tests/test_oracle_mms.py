"""Manufactured-solution pin of the oracle's right-hand side (CPU).

Smooth periodic fields with several Fourier modes in every field and every
direction are differentiated exactly by sympy in the continuum equations of
Sec. 2.1 -- continuity D lnrho/Dt = -div u and momentum
D u/Dt = -cs^2 grad lnrho + nu (lap u + (1/3) grad div u + 2 S . grad lnrho)
with the traceless rate-of-strain tensor S, D/Dt = d/dt + u . grad -- and the
oracle's discrete right-hand side (both the 55-point and the 19-point
discretisation) must converge to that exact value at the sixth order of the
Sec. 2.3 operators: the error falls by about 2^6 per halving of the spacing.
Every term (advection, pressure, Laplacian, grad div, S . grad lnrho) is
non-zero here, and a dropped term, a wrong sign or a wrong factor leaves an
O(1) error that does not converge."""
import math

import numpy as np
import pytest

sp = pytest.importorskip("sympy")

NU, CS = 0.07, 0.9


def continuum_rhs():
    """The exact right-hand side as numpy functions of (x, y, z)."""
    x, y, z = sp.symbols("x y z", real=True)
    X = (x, y, z)
    lnrho = sp.Rational(1, 10) * sp.sin(x + 2 * y) + sp.Rational(1, 20) * sp.cos(3 * z - y)
    u = [sp.Rational(1, 5) * sp.sin(y) * sp.cos(z) + sp.Rational(1, 10) * sp.cos(2 * x),
         sp.Rational(3, 20) * sp.sin(z + x) + sp.Rational(1, 20) * sp.sin(2 * y - z),
         sp.Rational(1, 10) * sp.cos(x - y) + sp.Rational(1, 10) * sp.sin(3 * z)]
    div = sum(sp.diff(u[j], X[j]) for j in range(3))
    grad_l = [sp.diff(lnrho, X[j]) for j in range(3)]
    r = [-sum(u[j] * grad_l[j] for j in range(3)) - div]
    for i in range(3):
        adv = sum(u[j] * sp.diff(u[i], X[j]) for j in range(3))
        lap = sum(sp.diff(u[i], X[j], 2) for j in range(3))
        S = [sp.Rational(1, 2) * (sp.diff(u[i], X[j]) + sp.diff(u[j], X[i])) -
             (sp.Rational(1, 3) * div if i == j else 0) for j in range(3)]
        sgl = sum(S[j] * grad_l[j] for j in range(3))
        visc = lap + sp.Rational(1, 3) * sp.diff(div, X[i]) + 2 * sgl
        r.append(-adv - CS ** 2 * grad_l[i] + NU * visc)
    fields = [lnrho] + u
    mk = lambda e: sp.lambdify(X, e, "numpy")  # noqa: E731
    return [mk(f) for f in fields], [mk(e) for e in r]


@pytest.fixture(scope="module")
def exact():
    return continuum_rhs()


def errors(orc, exact, n, variant):
    fields_fn, rhs_fn = exact
    h = 2 * math.pi / n
    g = np.arange(n) * h
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")  # arrays are [z][y][x]
    fields = [np.broadcast_to(f(X, Y, Z), (n, n, n)).astype(np.float64) for f in fields_fn]
    want = [np.broadcast_to(r(X, Y, Z), (n, n, n)) for r in rhs_fn]
    got = orc.rhs(fields, NU, CS, h, h, h, variant)
    return [float(np.max(np.abs(a - b))) for a, b in zip(got, want)]


@pytest.mark.parametrize("variant", ["55p", "19p"])
def test_rhs_converges_at_sixth_order(orc, exact, variant):
    e = {n: errors(orc, exact, n, variant) for n in (24, 48, 96)}
    for q in range(4):
        order = math.log2(e[48][q] / e[96][q])
        print(f"{variant} field {q}: errors {e[24][q]:.3e} {e[48][q]:.3e} {e[96][q]:.3e}, "
              f"order {order:.2f}")
        assert e[96][q] < e[48][q] < e[24][q]
        assert 5.6 <= order <= 6.6, (variant, q, order)
        assert e[96][q] < 1e-6


def test_55p_and_19p_converge_to_the_same_limit(orc, exact):
    """The two discretisations differ only in the grad div u term, whose
    difference also vanishes at sixth order."""
    fields_fn, _ = exact
    d = {}
    for n in (48, 96):
        h = 2 * math.pi / n
        g = np.arange(n) * h
        Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
        fields = [np.broadcast_to(f(X, Y, Z), (n, n, n)).astype(np.float64) for f in fields_fn]
        a = orc.rhs(fields, NU, CS, h, h, h, "55p")
        b = orc.rhs(fields, NU, CS, h, h, h, "19p")
        assert np.array_equal(a[0], b[0])  # continuity has no grad div term
        d[n] = max(float(np.max(np.abs(x - y))) for x, y in zip(a[1:], b[1:]))
    assert 5.6 <= math.log2(d[48] / d[96]) <= 6.6
