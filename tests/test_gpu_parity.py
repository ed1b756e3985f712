"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Tolerances (per field, ||gpu - oracle||_inf / ||oracle||_inf):
  FP64            1e-12 after one full step (3 substeps)
  FP32            1e-5 after one step
  FP32 + FP64 w   1e-5, and after one step no worse than FP32 (max norm
                  within 5%, RMS)
FP32 inputs are the FP64 generator values rounded to float32 on the host by
numpy; the oracle receives the same rounded values.
"""
import numpy as np
import pytest

import synthetic_inputs as si

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp32_acc64": 1e-5}


@pytest.fixture(scope="module")
def fd6():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible ROCm GPU")
    import paper_1707_08900_amd as p
    return p


def rel_err(a, b):
    return max(float(np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300)) for x, y in zip(a, b))


def oracle_inputs(fields, precision):
    return si.as_float32_exact(fields) if precision != "fp64" else [np.array(f) for f in fields]


def run_gpu(fd6, w, precision, variant="55p", nsteps=1, tile=None):
    box = fd6.Box(w.shape, precision, variant)
    if tile is not None:
        box.set_tile(tile)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    box.step(nsteps)
    out = box.get_fields()
    box.close()
    return out


def run_oracle(orc, w, precision, variant="55p", nsteps=1):
    return orc.rk3(oracle_inputs(w.fields, precision), w.nu, w.cs, w.dx, w.dy, w.dz, w.dt,
                   variant, nsteps)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_acc64"])
def test_small_box_one_step_all_kernels(fd6, orc, precision):
    w = si.small_parity_box()
    ref = run_oracle(orc, w, precision)
    errs = {}
    for tile in range(fd6.tile_count()):
        out = run_gpu(fd6, w, precision, tile=tile)
        errs[tile] = rel_err(out, ref)
        print(f"32^3 {precision} tile {tile}: rel err {errs[tile]:.3e}", flush=True)
    assert max(errs.values()) <= TOL[precision], errs


@pytest.mark.parametrize("box", ["noise32", "fourier64"])
def test_acc64_no_worse_than_fp32_one_step(fd6, orc, box):
    """FP32 state with the FP64 RK3 register and FP64 RK3 arithmetic against
    plain FP32, both against the oracle on the same FP32-rounded inputs,
    after one step: no worse in the max norm (5% allowed for the scatter of
    two rounding-noise maxima) and in the RMS."""
    w = (si.small_parity_box(seed=2) if box == "noise32" else
         si.fourier_box(64, seed=1, amplitude=0.1, kmax=16.0, nu=1e-3))
    ref = run_oracle(orc, w, "fp32")
    o32, oacc = run_gpu(fd6, w, "fp32"), run_gpu(fd6, w, "fp32_acc64")

    def rms(a, b):
        return max(float(np.sqrt(np.mean((x - y) ** 2)) / np.max(np.abs(y)))
                   for x, y in zip(a, b))
    e32, eacc = rel_err(o32, ref), rel_err(oacc, ref)
    r32, racc = rms(o32, ref), rms(oacc, ref)
    print(f"{box} one step: fp32 {e32:.4e} (rms {r32:.4e}), fp32 + fp64 w {eacc:.4e} "
          f"(rms {racc:.4e})", flush=True)
    assert e32 <= TOL["fp32"]
    assert eacc <= 1.05 * e32 and racc <= r32


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_increments_match(fd6, orc, precision):
    """The change over one step (out - in), not only the state, matches."""
    w = si.small_parity_box(seed=3)
    ref = run_oracle(orc, w, precision)
    out = run_gpu(fd6, w, precision)
    base = oracle_inputs(w.fields, precision)
    inc_ref = [r - b for r, b in zip(ref, base)]
    inc_gpu = [o - b for o, b in zip(out, base)]
    tol = 1e-10 if precision == "fp64" else 1e-2
    assert rel_err(inc_gpu, inc_ref) <= tol


@pytest.mark.parametrize("shape", [(23, 29, 37), (6, 6, 6), (7, 70, 9), (40, 6, 130)])
def test_ragged_shapes_fp64(fd6, orc, shape):
    """Tails that do not fill a tile, the minimum size, and tall/wide boxes."""
    w = si.noise_box(shape, seed=5)
    ref = run_oracle(orc, w, "fp64", nsteps=2)
    for tile in range(fd6.tile_count()):
        out = run_gpu(fd6, w, "fp64", nsteps=2, tile=tile)
        e = rel_err(out, ref)
        print(f"{shape} tile {tile}: {e:.3e}", flush=True)
        assert e <= 1e-12, (shape, tile, e)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_acc64"])
def test_19p_variant_all_kernels(fd6, orc, precision):
    """Both passes of the 19-point method in every kernel shape: the direct
    kernels (ghost zones) and the z-sweeps (periodic images in the loader)."""
    w = si.small_parity_box(seed=1)
    ref = run_oracle(orc, w, precision, variant="19p")
    errs = {}
    for tile in range(fd6.tile_count()):
        out = run_gpu(fd6, w, precision, variant="19p", tile=tile)
        errs[tile] = rel_err(out, ref)
        print(f"19p {precision} tile {tile}: {errs[tile]:.3e}", flush=True)
    assert max(errs.values()) <= TOL[precision], errs


@pytest.mark.parametrize("shape", [(23, 29, 37), (6, 6, 6), (9, 11, 13), (40, 6, 130)])
def test_19p_ragged_and_wrapped_fp64(fd6, orc, shape):
    """Tails, the minimum size and boxes smaller than a tile (every halo cell
    is a periodic image), several steps."""
    w = si.noise_box(shape, seed=15)
    ref = run_oracle(orc, w, "fp64", variant="19p", nsteps=3)
    for tile in range(fd6.tile_count()):
        e = rel_err(run_gpu(fd6, w, "fp64", variant="19p", nsteps=3, tile=tile), ref)
        print(f"19p {shape} tile {tile}: {e:.3e}", flush=True)
        assert e <= 1e-12, (shape, tile, e)


def test_19p_sweep_tiles_are_bitwise_identical(fd6):
    w = si.noise_box((20, 21, 70), seed=18)
    outs = [run_gpu(fd6, w, "fp32", variant="19p", nsteps=2, tile=t)
            for t in range(1, fd6.tile_count())]
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_mid_box_several_steps_fp64(fd6, orc):
    """128^3-style random-phase fields on a smaller grid, 5 steps."""
    w = si.fourier_box(48, seed=0, amplitude=1e-2, kmax=8.0, nu=2e-3)
    ref = run_oracle(orc, w, "fp64", nsteps=5)
    for tile in range(1, fd6.tile_count()):
        out = run_gpu(fd6, w, "fp64", nsteps=5, tile=tile)
        assert rel_err(out, ref) <= 1e-11


@pytest.mark.parametrize("precision,shape", [("fp32", (20, 21, 70)), ("fp32", (32, 32, 32)),
                                             ("fp64", (32, 32, 32)),
                                             ("fp32_acc64", (32, 32, 32))])
def test_sweep_tiles_are_bitwise_identical(fd6, precision, shape):
    """Every z-sweep tile shape performs the same arithmetic per point."""
    w = si.noise_box(shape, seed=8)
    outs = [run_gpu(fd6, w, precision, nsteps=2, tile=t) for t in range(1, fd6.tile_count())]
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", ["55p", "19p"])
def test_zchunk_does_not_change_results(fd6, variant):
    """Chunk boundaries in z (1-plane chunks, ragged chunks, whole columns)
    leave every result bit unchanged."""
    w = si.noise_box((20, 21, 70), seed=19)
    outs = []
    for zc in (0, 1, 7, 16, 1000):
        box = fd6.Box(w.shape, "fp32", variant)
        box.set_tile(2)
        box.set_zchunk(zc)
        box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
        box.init_fields(w.fields)
        box.step(2)
        outs.append(box.get_fields())
        box.close()
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("variant,tile", [("55p", 6), ("55p", 0), ("19p", 6), ("19p", 0)])
def test_graph_mode_matches_eager(fd6, variant, tile):
    """Captured steps replayed several times, with eager work (exports,
    reductions) between the replays, equal the launch-by-launch path bit for
    bit; so do the reducing step (re-captured for a new target) and a
    re-capture after new parameters."""
    import torch
    w = si.noise_box((20, 21, 22), seed=23)

    def make(graph):
        box = fd6.Box(w.shape, "fp64", variant)
        box.set_tile(tile)
        box.set_graph(graph)
        box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
        box.init_fields(w.fields)
        return box

    eager, graph = make(False), make(True)
    for rnd in range(3):
        eager.step(2)
        graph.step(2)
        for a, b in zip(eager.get_fields(), graph.get_fields()):
            assert np.array_equal(a, b), rnd
        assert eager.reduce() == graph.reduce()
    for rnd in range(2):
        r1 = torch.zeros(8, dtype=torch.float64, device="cuda")
        r2 = torch.zeros(8, dtype=torch.float64, device="cuda")
        eager.step_reduce(3, r1)
        graph.step_reduce(3, r2)
        assert np.array_equal(r1.cpu().numpy(), r2.cpu().numpy()), rnd
    for box in (eager, graph):
        box.set_params(2 * w.nu, w.cs, w.dx, w.dy, w.dz, 0.5 * w.dt)
        box.step(3)
    for a, b in zip(eager.get_fields(), graph.get_fields()):
        assert np.array_equal(a, b)


def test_runs_are_deterministic(fd6):
    w = si.noise_box((16, 24, 40), seed=9)
    a = run_gpu(fd6, w, "fp32", nsteps=3)
    b = run_gpu(fd6, w, "fp32", nsteps=3)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("precision,variant,layout", [("fp64", "55p", "aos"), ("fp32", "55p", "aos"),
                                                      ("fp32", "55p", "soa"), ("fp64", "19p", "soa")])
def test_translation_equivariance_bitwise(fd6, precision, variant, layout):
    """Shifting the state by whole cells commutes with a step, bit for bit:
    the arithmetic at a point sees only its neighbourhood, through the
    loaders' periodic wrap, whatever tile, chunk or wave holds it.  The box
    is ragged (not a multiple of any tile) and the shift crosses tiles and
    the periodic seams in all three directions."""
    w = si.fourier_box(0, seed=7, amplitude=0.05, kmax=6.0, shape=(44, 37, 70))
    shift = (13, -9, 29)  # z, y, x

    def step(fields):
        box = fd6.Box(w.shape, precision, variant, layout=layout)
        box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
        box.init_fields(fields)
        box.step(2)
        out = box.get_fields()
        box.close()
        return out

    a = [np.roll(f, shift, axis=(0, 1, 2)) for f in step(w.fields)]
    b = step([np.roll(f, shift, axis=(0, 1, 2)) for f in w.fields])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_rest_state_bitwise(fd6):
    shape = (12, 10, 14)
    f = [np.full(shape, 0.25), np.zeros(shape), np.zeros(shape), np.zeros(shape)]
    for prec in ("fp64", "fp32"):
        box = fd6.Box(shape, prec)
        box.set_params(0.01, 1.0, 0.1, 0.1, 0.1, 0.05)
        box.init_fields(f)
        box.step(3)
        out = box.get_fields()
        for a, b in zip(out, si.as_float32_exact(f) if prec == "fp32" else f):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", ["55p", "19p"])
@pytest.mark.parametrize("tile", [0, 4])
def test_rhs_hook_fp64(fd6, orc, variant, tile):
    w = si.noise_box((18, 20, 22), seed=4)
    box = fd6.Box(w.shape, "fp64", variant)
    box.set_tile(tile)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    r = box.rhs()
    ref = orc.rhs(w.fields, w.nu, w.cs, w.dx, w.dy, w.dz, variant)
    assert rel_err(r, ref) <= 1e-12
    # the state is untouched by the hook
    for a, b in zip(box.get_fields(), w.fields):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_rhs_hook_beyond_the_staging_area(fd6, orc, layout):
    """The right-hand side of a box larger than the 2^22-value staging area
    (256 x 128 x 136: chunks of 128 planes and a ragged one of 8) is exported
    in z-chunks and matches the oracle's at every point."""
    w = si.fourier_box(0, seed=6, amplitude=0.05, kmax=8.0, shape=(136, 128, 256))
    box = fd6.Box(w.shape, "fp64", "55p", layout=layout)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    r = box.rhs()
    box.close()
    ref = orc.rhs(w.fields, w.nu, w.cs, w.dx, w.dy, w.dz, "55p")
    err = rel_err(r, ref)
    print(f"rhs hook 256x128x136 {layout}: rel err {err:.3e}", flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("variant,layout", [("55p", "soa"), ("55p", "aos"), ("19p", "soa")])
def test_rhs_hook_continuity_sums(fd6, variant, layout):
    """The GPU's own continuity right-hand side obeys the exact periodic-sum
    identities of the discrete equations (independently of the oracle's
    code): the divergence telescopes, so sum r_lnrho = -sum u . D lnrho to
    round-off (D from the np.roll formulation), and 0 for uniform ln rho."""
    from oracle import numpy_ref
    rng = np.random.default_rng(21)
    shape = (14, 19, 37)
    h = (0.3, 0.4, 0.5)  # dx, dy, dz
    u = [rng.normal(scale=0.1, size=shape) for _ in range(3)]
    lnrho = rng.normal(scale=0.05, size=shape)
    for lr in (np.full(shape, 0.3), lnrho):
        box = fd6.Box(shape, "fp64", variant, layout=layout)
        box.set_params(0.02, 1.0, h[0], h[1], h[2], 0.01)
        box.init_fields([lr] + u)
        r0 = box.rhs()[0]
        box.close()
        adv = sum(u[j] * numpy_ref.d1(lr, j, h[j]) for j in range(3))
        tol = 1e-13 * np.abs(r0).sum()
        assert abs(r0.sum() + adv.sum()) < tol
    # the identity is not met trivially (a sign error misses it by far)
    assert abs(r0.sum() - adv.sum()) > 1e6 * tol


def test_reductions_match_oracle(fd6, orc):
    w = si.fourier_box(40, seed=2, amplitude=0.1, kmax=6.0)
    for prec in ("fp64", "fp32"):
        box = fd6.Box(w.shape, prec)
        box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
        box.init_fields(w.fields)
        g = box.reduce()
        o = orc.reduce(oracle_inputs(w.fields, prec), w.dx, w.dy, w.dz)
        assert g["mass"] == pytest.approx(o["mass"], rel=1e-13)
        assert g["kinetic_energy"] == pytest.approx(o["kinetic_energy"], rel=1e-13)
        scale = np.sum(np.abs(oracle_inputs(w.fields, prec)[0]))
        assert abs(g["sum_lnrho"] - o["sum_lnrho"]) <= 1e-13 * scale
        assert g["umax"] == o["umax"]
        assert g["nonfinite"] == 0
        # repeated reductions are bitwise identical
        assert box.reduce() == g


def test_reduce_reports_nonfinite(fd6):
    shape = (8, 8, 8)
    f = [np.zeros(shape) for _ in range(4)]
    f[1][1, 2, 3] = np.nan
    f[3][4, 4, 4] = np.inf
    box = fd6.Box(shape, "fp64")
    box.set_params(0.01, 1.0, 0.1, 0.1, 0.1, 0.01)
    box.init_fields(f)
    with pytest.raises(fd6.Fd6Error) as e:
        box.reduce()
    assert e.value.status == -5
    r = box.reduce(allow_nonfinite=True)
    assert r["nonfinite"] == 2 and np.isnan(r["mass"]) and np.isnan(r["kinetic_energy"])


@pytest.mark.parametrize("variant,precision", [("55p", "fp32"), ("55p", "fp64"),
                                               ("19p", "fp32")])
def test_fused_diagnostics_count_nonfinite(fd6, variant, precision):
    """A NaN and an infinity planted in the state spread over their stencil
    neighbourhoods in one step; the diagnostics fused into the last substep
    count the same non-finite points as the standalone pass, and both report
    mass and kinetic energy as NaN."""
    import torch
    w = si.noise_box((20, 18, 40), seed=21)
    f = [a.copy() for a in w.fields]
    f[2][5, 6, 7] = np.nan
    f[0][12, 3, 30] = np.inf
    box = fd6.Box(w.shape, precision, variant)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(f)
    red = torch.zeros(8, dtype=torch.float64, device="cuda")
    box.step_reduce(1, red)
    fused = red.cpu().numpy()
    alone = box.reduce(allow_nonfinite=True)
    out = box.get_fields()
    box.close()
    bad = int(np.sum(~(np.isfinite(out[0]) & np.isfinite(out[1]) & np.isfinite(out[2]) &
                       np.isfinite(out[3]))))
    print(f"{variant} {precision}: {bad} non-finite points after one step", flush=True)
    assert bad > 2 and fused[4] == bad and alone["nonfinite"] == bad
    assert np.isnan(fused[0]) and np.isnan(fused[1])
    assert np.isnan(alone["mass"]) and np.isnan(alone["kinetic_energy"])


def test_checkpoint_restart_bitwise(fd6):
    """10 steps == 5 steps, get_fields / init_fields, 5 steps (w carries no
    state across steps because alpha(1) = 0)."""
    w = si.noise_box((16, 16, 16), seed=6)
    box = fd6.Box(w.shape, "fp64")
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    box.step(10)
    full = box.get_fields()
    box.init_fields(w.fields)
    box.step(5)
    mid = box.get_fields()
    box.init_fields(mid)
    box.step(5)
    for a, b in zip(box.get_fields(), full):
        assert np.array_equal(a, b)


def test_device_init_and_export(fd6):
    import torch
    w = si.noise_box((10, 12, 14), seed=12)
    box = fd6.Box(w.shape, "fp64")
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields([torch.from_numpy(f).cuda() for f in w.fields])
    box.step(1)
    dev = [t.cpu().numpy() for t in box.get_fields_device()]
    host = box.get_fields()
    for a, b in zip(dev, host):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("variant,tile", [("55p", 0), ("55p", 1), ("55p", 2), ("55p", 6),
                                          ("55p", 9), ("19p", 0), ("19p", 6), ("19p", 8)])
def test_step_reduce_matches_standalone_and_oracle(fd6, orc, variant, tile):
    """Diagnostics of the last step (fused into substep 3 -- the 55-point
    sweep, or pass 2 of the 19-point method -- for the z-sweep shapes, a
    separate pass for the direct shape) equal fd6_reduce of the same state up
    to summation order, and the oracle's reduction of the oracle's state;
    max |u| and the non-finite count exactly."""
    import torch
    w = si.noise_box((24, 20, 36), seed=13)
    box = fd6.Box(w.shape, "fp64", variant)
    box.set_tile(tile)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    red = torch.zeros(8, dtype=torch.float64, device="cuda")
    box.step_reduce(2, red)
    fused = red.cpu().numpy()
    alone = box.reduce()
    ref_state = orc.rk3(w.fields, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, 2)
    ref = orc.reduce(ref_state, w.dx, w.dy, w.dz)
    for key, i in (("mass", 0), ("kinetic_energy", 1)):
        assert fused[i] == pytest.approx(alone[key], rel=1e-13)
        assert fused[i] == pytest.approx(ref[key], rel=1e-12)
    assert abs(fused[2] - alone["sum_lnrho"]) <= 1e-12 * np.sum(np.abs(ref_state[0]))
    assert fused[3] == alone["umax"]
    assert fused[4] == 0.0
    # repeated runs are bitwise identical
    box.init_fields(w.fields)
    box.step_reduce(2, red)
    assert np.array_equal(red.cpu().numpy(), fused)


def test_step_reduce_falls_back_beyond_partial_capacity(fd6):
    """With more workgroups than fused-partial slots (1-plane chunks) the
    diagnostics come from the standalone pass: bitwise equal to fd6_reduce;
    the fused run agrees to rounding."""
    import torch
    w = si.noise_box((600, 64, 64), seed=22)
    red = torch.zeros(8, dtype=torch.float64, device="cuda")
    res = {}
    for zc in (1, 0):
        box = fd6.Box(w.shape, "fp32")
        box.set_tile(1)
        box.set_zchunk(zc)
        box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
        box.init_fields(w.fields)
        box.step_reduce(1, red)
        res[zc] = (red.cpu().numpy().copy(), box.reduce())
        box.close()
    fb, alone = res[1]
    assert fb[0] == alone["mass"] and fb[1] == alone["kinetic_energy"]
    assert fb[3] == alone["umax"]
    fused = res[0][0]
    assert fused[0] == pytest.approx(fb[0], rel=1e-13)
    assert fused[1] == pytest.approx(fb[1], rel=1e-12)
    assert fused[3] == fb[3]


def test_periodic_wrap_over_many_steps(fd6, orc):
    """Many steps on a box smaller than one tile in every direction: the
    z-sweep loader's periodic images (x, y and z wrap) stay exact."""
    w = si.noise_box((9, 11, 13), seed=21)
    ref = run_oracle(orc, w, "fp64", nsteps=6)
    for tile in range(1, fd6.tile_count()):
        out = run_gpu(fd6, w, "fp64", nsteps=6, tile=tile)
        assert rel_err(out, ref) <= 1e-12, tile
