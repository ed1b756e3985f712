"""GPU: the degenerate states of the method stay exactly fixed.

A uniform state (constant ln rho, constant velocity) has a right-hand side of
exactly zero: every first-derivative stencil of Sec. 2.3 is a sum of mirrored
differences, and the second and mixed stencils have weights that sum to zero,
so with values that are dyadic rationals (exact in FP32 and FP64, and so are
their products with the stencils' small integer weights) every derivative is
exactly 0.  Then eqs. continuity and navierstokes give zero tendencies, the
2N-RK3 register stays zero, and each substep adds exactly nothing
(Sec. 2.4): the state must come back bit for bit.  Checked for the rest state
(u = 0) and a uniform flow, in every kernel shape, both methods, all three
precision forms and both layouts, through the C ABI.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPE = (13, 22, 70)  # ragged: partial tiles in x and y, odd z
LNRHO = 0.375
FLOWS = {"rest": (0.0, 0.0, 0.0), "uniform": (0.125, -0.25, 0.0625)}


@pytest.fixture(scope="module")
def fd6():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible ROCm GPU")
    import paper_1707_08900_amd as p
    return p


def shapes_for(fd6, variant, layout):
    if layout == "aos":  # the register-loader z-sweeps
        return [t for t in range(1, fd6.tile_count()) if t != 9]
    return list(range(fd6.tile_count()))


@pytest.mark.parametrize("flow", ["rest", "uniform"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_acc64"])
@pytest.mark.parametrize("variant,layout", [("55p", "soa"), ("55p", "aos"), ("19p", "soa")])
def test_uniform_state_is_fixed_bitwise(fd6, flow, precision, variant, layout):
    nz, ny, nx = SHAPE
    h = 2 * np.pi / 64
    init = [np.full(SHAPE, LNRHO)] + [np.full(SHAPE, v) for v in FLOWS[flow]]
    for tile in shapes_for(fd6, variant, layout):
        box = fd6.Box(SHAPE, precision, variant, layout=layout)
        box.set_tile(tile)
        box.set_params(2e-3, 1.0, h, h, h, 0.01)
        box.init_fields(init)
        box.step(3)
        out = box.get_fields()
        red = box.reduce()
        box.close()
        for q in range(4):
            assert np.array_equal(out[q], init[q]), (tile, q)
        # the FP64 diagnostics of the unchanged state
        n = nx * ny * nz
        assert red["nonfinite"] == 0
        assert red["sum_lnrho"] == pytest.approx(n * LNRHO, rel=1e-15)
        assert red["mass"] == pytest.approx(n * np.exp(LNRHO) * h ** 3, rel=1e-14)
        u2 = sum(v * v for v in FLOWS[flow])
        assert red["umax"] == pytest.approx(np.sqrt(u2), rel=1e-15, abs=0.0)
