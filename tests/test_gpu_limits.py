"""GPU: the size limits and degenerate cases of the boundary.

* the longest axis the ABI accepts (4096) with the other two at the minimum
  (6, twice the stencil radius, so every periodic image is a single wrap):
  one FP64 step against the full oracle, both methods and both layouts;
* the largest plane (4096 x 4096, six planes) in FP64 with the array-of-
  structures layout, where a plane spans 0.54 GB and the kernels' 32-bit
  in-plane byte offsets are largest: sampled points against the oracle's
  patch update, including the corners and the periodic seams;
* zero steps leave the state bit for bit unchanged.
"""
import numpy as np
import pytest

import synthetic_inputs as si

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fd6():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible ROCm GPU")
    import paper_1707_08900_amd as p
    return p


def rel_err(a, b):
    return max(float(np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300)) for x, y in zip(a, b))


@pytest.mark.parametrize("shape", [(6, 6, 4096), (6, 4096, 6), (4096, 6, 6)])
@pytest.mark.parametrize("variant,layout", [("55p", "soa"), ("55p", "aos"), ("19p", "soa")])
def test_longest_axis(fd6, orc, shape, variant, layout):
    w = si.noise_box(shape, seed=sum(shape) % 97)
    box = fd6.Box(w.shape, "fp64", variant, layout=layout)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    box.step(1)
    out = box.get_fields()
    box.close()
    ref = orc.rk3(w.fields, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, 1)
    err = rel_err(out, ref)
    print(f"{shape} {variant} {layout}: rel err {err:.3e}", flush=True)
    assert err <= 1e-12


def test_largest_plane_fp64_aos(fd6, orc):
    import torch
    n, nz = 4096, 6
    rng = np.random.default_rng(11)
    fields = [rng.uniform(-1e-3, 1e-3, (nz, n, n))] + \
        [rng.normal(0.0, 1e-2, (nz, n, n)) for _ in range(3)]
    h = 2 * np.pi / n
    hz = 2 * np.pi / nz
    nu, cs = 5e-3, 1.0
    dt = si.cfl_dt(fields, h, h, hz, cs)
    box = fd6.Box((nz, n, n), "fp64", "55p", layout="aos")
    box.set_params(nu, cs, h, h, hz, dt)
    box.init_fields(fields)
    box.step(1)
    out = box.get_fields_device()
    box.close()
    pts = [(0, 0, 0), (nz - 1, n - 1, n - 1), (0, n - 1, 0), (nz - 1, 0, n - 1),
           (2, n // 2, n - 2), (3, 1, 2)]
    pts += [tuple(int(v) for v in (rng.integers(nz), rng.integers(n), rng.integers(n)))
            for _ in range(6)]
    scale = [float(np.max(np.abs(f))) for f in fields]
    worst = 0.0
    for c in pts:
        ref = orc.rk3_point(fields, c, nu, cs, h, h, hz, dt, "55p", 1)
        for q in range(4):
            worst = max(worst, abs(float(out[q][c].item()) - ref[q]) / scale[q])
    print(f"4096^2 x 6 fp64 aos: sampled rel err {worst:.3e}", flush=True)
    assert worst <= 1e-12
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_zero_steps_is_a_no_op(fd6, layout):
    w = si.noise_box((9, 14, 33), seed=2)
    box = fd6.Box(w.shape, "fp32", "55p", layout=layout)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    before = box.get_fields()
    box.step(0)
    after = box.get_fields()
    box.close()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
