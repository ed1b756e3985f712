"""The entry point for callers that cannot allocate (fd6_reduce_fields_static):
its FP64 diagnostics of caller-owned compact device arrays equal those of
fd6_reduce_device on a box holding the same values (same kernels, same fixed
summation order), over two calls in a row whose second input is smaller, in
both storage precisions, and with a non-finite value planted."""
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


def box_diagnostics(fd6, w, precision, fields):
    import torch
    box = fd6.Box(w.shape, precision)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(fields)
    out = torch.full((8,), -1.0, dtype=torch.float64, device="cuda")
    box.reduce_device(out)
    torch.cuda.synchronize()
    box.close()
    return out[:5].cpu().numpy()


def static_diagnostics(fd6, w, precision, fields):
    import torch
    dt = torch.float64 if precision == "fp64" else torch.float32
    dev = [torch.from_numpy(np.ascontiguousarray(f)).to("cuda", dt) for f in fields]
    out = torch.full((8,), -1.0, dtype=torch.float64, device="cuda")
    fd6.reduce_fields_static(dev, w.dx, w.dy, w.dz, out)
    torch.cuda.synchronize()
    return out[:5].cpu().numpy()


def check_equal(a, b, what):
    # the same partition and order of the FP64 sums: equal to the last bit is
    # expected; the bar asserted is the FP64 parity tolerance
    print(f"{what}: static {a.tolist()} box {b.tolist()} bitwise {np.array_equal(a, b)}",
          flush=True)
    for q in (0, 1, 2):
        assert abs(a[q] - b[q]) <= 1e-13 * max(abs(b[q]), 1e-300), (what, q, a[q], b[q])
    assert a[3] == b[3] and a[4] == b[4], what


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_reduce_equals_box_reduce_two_calls(fd6, orc, precision):
    # second call smaller than the first: the shared scratch keeps the first
    # call's partials, none of which may leak into the second result
    for shape, seed in (((40, 36, 33), 3), ((11, 7, 9), 4)):
        w = si.noise_box(shape, seed=seed, nu=1e-3)
        fields = si.as_float32_exact(w.fields) if precision == "fp32" else w.fields
        a = static_diagnostics(fd6, w, precision, fields)
        b = box_diagnostics(fd6, w, precision, w.fields)
        check_equal(a, b, f"{precision} {shape}")
        ref = orc.reduce(fields, w.dx, w.dy, w.dz)
        assert a[0] == pytest.approx(ref["mass"], rel=1e-12)
        assert a[1] == pytest.approx(ref["kinetic_energy"], rel=1e-12)
        assert a[3] == ref["umax"] and a[4] == 0


def test_static_reduce_counts_nonfinite(fd6):
    w = si.noise_box((16, 12, 10), seed=5, nu=1e-3)
    fields = [f.copy() for f in w.fields]
    fields[2][3, 4, 5] = np.nan
    fields[0][7, 1, 2] = np.inf
    a = static_diagnostics(fd6, w, "fp64", fields)
    b = box_diagnostics(fd6, w, "fp64", fields)
    assert a[4] == 2 and b[4] == 2
    small = si.noise_box((6, 6, 7), seed=6, nu=1e-3)
    c = static_diagnostics(fd6, small, "fp64", small.fields)
    assert c[4] == 0 and np.isfinite(c[:4]).all()
