"""GPU: the array-of-structures state layout (the alternative storage of the
discussion in Sec. 7), selected by FD6_LAYOUT_AOS.

Only the device layout changes, and every point goes through the same
arithmetic, so an AoS box reproduces the default layout bit for bit (state,
right-hand side, fused and standalone diagnostics, forced steps, graph
replays); against the FP64 oracle it meets the parity tolerances of one step
(FP64 1e-12, FP32 1e-5).
"""
import math

import numpy as np
import pytest

import synthetic_inputs as si

pytestmark = pytest.mark.gpu

EUNSUPPORTED = -6
TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp32_acc64": 1e-5}


@pytest.fixture(scope="module")
def fd6():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible ROCm GPU")
    import paper_1707_08900_amd as p
    return p


def aos_tiles(fd6):
    return [t for t in range(1, fd6.tile_count()) if t != 9]


def make(fd6, w, precision, layout, tile=None, zchunk=None):
    box = fd6.Box(w.shape, precision, "55p", layout=layout)
    if tile is not None:
        box.set_tile(tile)
    if zchunk is not None:
        box.set_zchunk(zchunk)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    return box


def rel_err(a, b):
    return max(float(np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300)) for x, y in zip(a, b))


def test_unsupported_forms_are_refused(fd6):
    box = fd6.Box((16, 16, 16), "fp32", "55p", layout="aos")
    for t in (0, 9):  # the direct kernels read ghost zones; shape 9 copies planes into LDS
        with pytest.raises(fd6.Fd6Error) as e:
            box.set_tile(t)
        assert e.value.status == EUNSUPPORTED
    box.set_tile(6)
    box.close()
    with pytest.raises(fd6.Fd6Error) as e:
        fd6.Box((16, 16, 16), "fp32", "19p", layout="aos")
    assert e.value.status == EUNSUPPORTED


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_acc64"])
def test_aos_matches_default_layout_bitwise(fd6, precision):
    """Ragged box (no dimension a multiple of a tile), every shape, 2 steps."""
    w = si.noise_box((21, 19, 70), seed=12)
    ref = make(fd6, w, precision, "soa", tile=6)
    ref.step(2)
    want = ref.get_fields()
    ref.close()
    for t in aos_tiles(fd6):
        box = make(fd6, w, precision, "aos", tile=t)
        box.step(2)
        got = box.get_fields()
        box.close()
        print(f"aos {precision} tile {t}", flush=True)
        for q in range(4):
            assert np.array_equal(got[q], want[q]), (t, q)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_aos_one_step_parity_with_oracle(fd6, orc, precision):
    w = si.small_parity_box(seed=5)
    base = si.as_float32_exact(w.fields) if precision == "fp32" else w.fields
    ref = orc.rk3(base, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, "55p", 1)
    box = make(fd6, w, precision, "aos")
    box.step(1)
    err = rel_err(box.get_fields(), ref)
    box.close()
    print(f"aos {precision} 32^3: rel err {err:.3e}", flush=True)
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_aos_rhs_and_diagnostics_match(fd6, precision):
    import torch
    w = si.noise_box((33, 40, 24), seed=4)
    boxes = {lay: make(fd6, w, precision, lay, tile=2, zchunk=9) for lay in ("soa", "aos")}
    r = {lay: b.rhs() for lay, b in boxes.items()}
    for q in range(4):
        assert np.array_equal(r["aos"][q], r["soa"][q])
    red = {}
    for lay, b in boxes.items():
        b.init_fields(w.fields)
        out = torch.zeros(8, dtype=torch.float64, device=b.device)
        b.step_reduce(2, out)  # fused diagnostics in substep 3
        red[lay] = (out.cpu().numpy()[:5], b.reduce())  # and the standalone pass
    assert np.array_equal(red["aos"][0], red["soa"][0])
    assert red["aos"][1] == red["soa"][1]
    f = {lay: b.get_fields() for lay, b in boxes.items()}
    for q in range(4):
        assert np.array_equal(f["aos"][q], f["soa"][q])
    for b in boxes.values():
        b.close()


def test_aos_forced_and_graph_steps_match(fd6):
    """Forced steps, eager and replayed, the last one with the fused
    diagnostics (the forced, reducing, AoS instantiation of the sweep)."""
    import torch
    w = si.noise_box((24, 30, 36), seed=8)
    draws = si.forcing_draws(4, 1.0, 2.0, 0.05, seed=2)
    res, reds = {}, {}
    for lay in ("soa", "aos"):
        for graph in (False, True):
            b = make(fd6, w, "fp32", lay, tile=12)
            b.set_graph(graph)
            red = torch.zeros(8, dtype=torch.float64, device=b.device)
            for i, d in enumerate(draws):
                b.set_forcing(d)
                if i + 1 < len(draws):
                    b.step(1)
                else:
                    b.step_reduce(1, red)
            res[(lay, graph)] = b.get_fields()
            reds[(lay, graph)] = red.cpu().numpy()[:5]
            b.close()
    want = res[("soa", False)]
    for key, got in res.items():
        for q in range(4):
            assert np.array_equal(got[q], want[q]), key
        assert np.array_equal(reds[key], reds[("soa", False)]), key


def test_aos_sound_wave_stays_on_the_closed_form(fd6):
    """A linear sound wave along x for 200 steps in the AoS layout: phase and
    amplitude of the discrete dispersion relation of the sixth-order D1 with
    RK3, as for the default layout."""
    # amplitude small enough that the quadratic terms (relative size ~ amp k t)
    # stay far below the tolerance
    n, k, amp, nu = 64, 3, 1e-8, 0.0
    h = 2 * math.pi / n
    x = np.arange(n) * h
    lnrho = np.broadcast_to(amp * np.sin(k * x), (n, n, n)).copy()
    zero = np.zeros((n, n, n))
    dt = 0.4 * h
    box = fd6.Box((n, n, n), "fp64", "55p", layout="aos")
    box.set_params(nu, 1.0, h, h, h, dt)
    box.init_fields([lnrho, zero, zero, zero])
    nsteps = 200
    box.step(nsteps)
    lr = box.get_fields()[0][0, 0, :]
    box.close()
    # discrete wave number of D1 (eqs. first_derivatives) and the RK3 growth
    th = k * h
    kd = (45 * math.sin(th) - 9 * math.sin(2 * th) + math.sin(3 * th)) / (30 * h)
    z = 1j * kd * dt  # eigenvalues +-i kd cs of the linear system
    g = 1 + z + z * z / 2 + z ** 3 / 6
    t_phase = nsteps * np.angle(g)
    a = abs(g) ** nsteps
    pred = amp * a * np.cos(t_phase) * np.sin(k * x)  # standing wave from rest
    assert np.max(np.abs(lr - pred)) <= 1e-5 * amp


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_acc64"])
def test_aos_ensemble_matches_single_boxes(fd6, precision):
    """Ensemble in the AoS layout (ragged boxes; z-chunked work items, and
    the packed deal of whole columns cut into pieces): each box equals its
    single-box run in the default layout bit for bit, and the per-box
    diagnostics equal the single-box ones."""
    shapes = [(21, 19, 70), (6, 6, 6), (33, 40, 24), (17, 9, 48), (40, 7, 13)]
    ws = [si.noise_box(s, seed=20 + i) for i, s in enumerate(shapes)]
    b = fd6.Batch(shapes, precision, layout="aos")
    b.set_params([(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt) for w in ws])
    for i, w in enumerate(ws):
        b.init_fields(i, w.fields)
    with pytest.raises(fd6.Fd6Error) as e:
        b.set_schedule(9, 0)
    assert e.value.status == EUNSUPPORTED
    for tile, zc in ((4, 8), (6, 0), (8, -2)):
        for i, w in enumerate(ws):
            b.init_fields(i, w.fields)
        b.set_schedule(tile, zc)
        b.step(2)
        red = b.reduce()
        for i, w in enumerate(ws):
            box = make(fd6, w, precision, "soa", tile=tile)
            box.step(2)
            want = box.get_fields()
            want_red = box.reduce()
            box.close()
            got = b.get_fields(i)
            for q in range(4):
                assert np.array_equal(got[q], want[q]), (tile, i, q)
            assert red[i] == want_red, (tile, i)
    b.close()


@pytest.mark.parametrize("layout", ["soa", "aos"])
def test_library_tuner_single_box(fd6, layout, tmp_path):
    """fd6_tune: a valid schedule for the layout, taken from the cache the
    second time, and a tuned box reproduces the default shape bit for bit."""
    w = si.noise_box((40, 24, 36), seed=17)
    cache = str(tmp_path / "tune.txt")
    box = make(fd6, w, "fp32", layout)
    default = box.get_schedule()
    assert default == (6, 0)
    tile, zc = box.tune(cache)
    assert 1 <= tile < fd6.tile_count() and (layout == "soa" or tile != 9)
    assert zc in (0, 40) or zc in (64, 128, 256)
    # the log: every shape the layout takes with the automatic chunk, then
    # the chunk lengths (here only nz = 40) for the fastest shape
    log = box.tune_log()
    shapes = [t for t, z, _ in log if z == 0]
    assert shapes == [t for t in range(1, fd6.tile_count()) if layout == "soa" or t != 9]
    assert all(ms > 0 for _, _, ms in log)
    fastest = min((ms, t) for t, z, ms in log if z == 0)[1]
    assert [(t, z) for t, z, _ in log if z != 0] == [(fastest, 40)]
    best = min(log, key=lambda e: e[2])
    assert (tile, zc) == (best[0], best[1])
    box.set_tile(default[0])
    box.set_zchunk(default[1])
    assert box.tune(cache) == (tile, zc)  # from the cache
    assert box.tune_log() == []
    assert len([ln for ln in open(cache).read().split("\n") if ln]) == 1
    box.init_fields(w.fields)
    box.step(2)
    got = box.get_fields()
    box.close()
    ref = make(fd6, w, "fp32", layout)
    ref.step(2)
    for a, b in zip(got, ref.get_fields()):
        assert np.array_equal(a, b)
    ref.close()


@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("shape", [(32, 32, 32), (23, 29, 37), (6, 6, 6), (40, 6, 70)])
def test_fused_substeps_bitwise_equal_to_plain_launches(fd6, orc, layout, shape):
    """Substeps 1 and 2 in one launch (temporal blocking): bit for bit the
    plain launches, with and without the fused diagnostics and in graph
    replay, on boxes smaller than the 16 x 16 tile and with ragged tails;
    and within the FP32 bound of the oracle."""
    import torch
    w = si.noise_box(shape, seed=31)
    ref = make(fd6, w, "fp32", layout)
    ref.step(3)
    want = ref.get_fields()
    red_ref = torch.zeros(8, dtype=torch.float64, device="cuda")
    ref.init_fields(w.fields)
    ref.step_reduce(2, red_ref)
    ref.close()
    box = make(fd6, w, "fp32", layout)
    box.set_fused_substeps(True)
    box.step(3)
    got = box.get_fields()
    for a, b in zip(got, want):
        assert np.array_equal(a, b), shape
    red = torch.zeros(8, dtype=torch.float64, device="cuda")
    for graph in (False, True):
        box.set_graph(graph)
        box.init_fields(w.fields)
        box.step_reduce(2, red)
        assert np.array_equal(red.cpu().numpy(), red_ref.cpu().numpy()), graph
    box.close()
    ref1 = orc.rk3(si.as_float32_exact(w.fields), w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, "55p", 3)
    err = max(float(np.max(np.abs(a - b)) / np.max(np.abs(b))) for a, b in zip(got, ref1))
    assert err <= 3e-5


def test_fused_substeps_refused_where_unsupported(fd6):
    w = si.noise_box((8, 8, 8), seed=1)
    for prec, var in (("fp64", "55p"), ("fp32_acc64", "55p"), ("fp32", "19p")):
        box = fd6.Box(w.shape, prec, var)
        with pytest.raises(fd6.Fd6Error) as ex:
            box.set_fused_substeps(True)
        assert ex.value.status == -6
        box.set_fused_substeps(False)
        box.close()
