"""GPU parity of the external force (Sec. 6, eq. forcing): the library and the
oracle receive the same per-step draws (k, e, phase) and compute the force
each on its own.

* every kernel shape, both methods, FP64 (<= 1e-12) and FP32 (<= 1e-5): three
  steps with a fresh draw each step;
* the axis-aligned forced shear wave on the GPU follows the fully discrete
  RK3 closed form;
* graph replay with a new force every step equals the launch-by-launch path
  bit for bit; switching the force off restores the unforced kernels;
* the fused diagnostics of a forced run match the oracle;
* 256^3 FP32 box, one forced step: sampled points against the oracle's local
  patch update (checks the force's coordinates across tiles and chunks).
"""
import math

import numpy as np
import pytest

import synthetic_inputs as si

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def fd6():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible ROCm GPU")
    import paper_1707_08900_amd as p
    return p


@pytest.fixture(autouse=True)
def _oracle_force_off(orc):
    yield
    orc.set_forcing(None)


def rel_err(a, b):
    return max(float(np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300)) for x, y in zip(a, b))


def oracle_forced(orc, w, fields, draws, variant):
    f = [np.array(x) for x in fields]
    for d in draws:
        orc.set_forcing(d, cs=w.cs, dt=w.dt)
        f = orc.rk3(f, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, 1)
    orc.set_forcing(None)
    return f


def gpu_forced(fd6, w, precision, variant, draws, tile, graph=False):
    box = fd6.Box(w.shape, precision, variant)
    box.set_tile(tile)
    box.set_graph(graph)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    for d in draws:
        box.set_forcing(d)
        box.step(1)
    out = box.get_fields()
    box.close()
    return out


@pytest.mark.parametrize("variant", ["55p", "19p"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_forced_steps_all_kernels(fd6, orc, variant, precision):
    w = si.noise_box((20, 21, 22), seed=33)
    draws = si.forcing_draws(3, 1.0, 3.0, 0.05, seed=5)
    inp = w.fields if precision == "fp64" else si.as_float32_exact(w.fields)
    ref = oracle_forced(orc, w, inp, draws, variant)
    # the force is a visible part of the result
    unforced = orc.rk3(inp, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, 3)
    assert rel_err(unforced, ref) > 1e-3
    errs = {}
    for tile in range(fd6.tile_count()):
        errs[tile] = rel_err(gpu_forced(fd6, w, precision, variant, draws, tile), ref)
        print(f"forced {variant} {precision} tile {tile}: {errs[tile]:.3e}", flush=True)
    assert max(errs.values()) <= TOL[precision], errs


@pytest.mark.parametrize("tile", [0, 6])
def test_forced_shear_closed_form_gpu(fd6, tile):
    n, nsteps, nu, dt = 32, 6, 2e-2, 0.01
    h = 2 * math.pi / n
    kz = 2
    force = {"k": (0.0, 0.0, float(kz)), "e": (0.0, 1.0, 0.0), "f0": 0.05, "phase": 0.4}
    shape = (n, n, n)
    f = [np.full(shape, 0.25), np.zeros(shape), np.zeros(shape), np.zeros(shape)]
    box = fd6.Box(shape, "fp64")
    box.set_tile(tile)
    box.set_params(nu, 1.0, h, h, h, dt)
    box.init_fields(f)
    box.set_forcing(force)
    box.step(nsteps)
    out = box.get_fields()
    a = -0.05 * math.sqrt(kz / dt)  # N f_k for k x e = -kz x_hat, |k| = kz
    th = kz * h
    k2 = (490 - 540 * math.cos(th) + 54 * math.cos(2 * th) - 4 * math.cos(3 * th)) / (180 * h * h)
    z = -nu * k2 * dt
    U = 0.0
    for _ in range(nsteps):
        U = (1 + z + z * z / 2 + z ** 3 / 6) * U + dt * (1 + z / 2 + z * z / 6) * a
    prof = U * np.cos(kz * np.arange(n) * h + force["phase"])
    assert np.all(out[0] == 0.25)
    assert np.max(np.abs(out[1] - prof[:, None, None])) <= 1e-13 * abs(U)
    assert np.max(np.abs(out[2])) <= 1e-15 * abs(U) and np.max(np.abs(out[3])) <= 1e-15 * abs(U)


@pytest.mark.parametrize("variant,tile", [("55p", 6), ("19p", 2), ("55p", 0)])
def test_forced_graph_replay_matches_eager(fd6, variant, tile):
    w = si.noise_box((16, 18, 20), seed=34)
    draws = si.forcing_draws(5, 1.0, 2.5, 0.05, seed=6)
    a = gpu_forced(fd6, w, "fp64", variant, draws, tile, graph=False)
    b = gpu_forced(fd6, w, "fp64", variant, draws, tile, graph=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_force_off_restores_unforced_run(fd6):
    w = si.noise_box((16, 16, 16), seed=35)
    draws = si.forcing_draws(1, 1.0, 2.0, 0.05, seed=7)
    plain = fd6.Box(w.shape, "fp64")
    plain.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    plain.init_fields(w.fields)
    plain.step(2)
    toggled = fd6.Box(w.shape, "fp64")
    toggled.set_graph(True)
    toggled.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    toggled.set_forcing(draws[0])
    toggled.set_forcing(None)
    toggled.init_fields(w.fields)
    toggled.step(2)
    for x, y in zip(plain.get_fields(), toggled.get_fields()):
        assert np.array_equal(x, y)


def test_forced_step_reduce_matches_oracle(fd6, orc):
    import torch
    w = si.fourier_box(40, seed=3, amplitude=0.05, kmax=6.0)
    draws = si.forcing_draws(2, 1.0, 2.0, 0.1, seed=8)
    box = fd6.Box(w.shape, "fp64")
    box.set_tile(6)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    red = torch.zeros(8, dtype=torch.float64, device="cuda")
    for d in draws:
        box.set_forcing(d)
        box.step_reduce(1, red)
    got = red.cpu().numpy()
    ref_state = oracle_forced(orc, w, w.fields, draws, "55p")
    ref = orc.reduce(ref_state, w.dx, w.dy, w.dz)
    assert got[0] == pytest.approx(ref["mass"], rel=1e-12)
    assert got[1] == pytest.approx(ref["kinetic_energy"], rel=1e-11)
    assert got[3] == pytest.approx(ref["umax"], rel=1e-11)
    assert rel_err(box.get_fields(), ref_state) <= 1e-12


def test_forced_256_sampled_points(fd6, orc):
    import torch
    n = 256
    w = si.large_box(n)
    d = si.forcing_draws(1, 2.0, 4.0, 0.1, seed=9)[0]
    box = fd6.Box(w.shape, "fp32")
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields([torch.from_numpy(f).cuda() for f in w.fields])
    box.set_forcing(d)
    box.step(1)
    out = box.get_fields_device()
    inp = si.as_float32_exact(w.fields)
    orc.set_forcing(d, cs=w.cs, dt=w.dt)
    rng = np.random.default_rng(11)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (n // 2, 63, 64)]
    pts += [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(7)]
    scale = [float(np.max(np.abs(f))) for f in inp]
    worst = 0.0
    for c in pts:
        ref = orc.rk3_point(inp, c, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, "55p", 1)
        for q in range(4):
            worst = max(worst, abs(float(out[q][c].item()) - ref[q]) / scale[q])
    print(f"forced 256^3 fp32 sampled rel err {worst:.3e}", flush=True)
    assert worst <= 1e-5
