"""GPU tests of the batched ensemble (one persistent launch per substep,
captured graph per step): every box must equal the single-box z-sweep run
with the same kernel shape bit for bit, and the FP64 oracle to 1e-12."""
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


def small_ensemble():
    shapes = [(12, 12, 12), (16, 20, 24), (32, 32, 32), (9, 14, 33), (20, 16, 16), (6, 6, 6)]
    ws = [si.noise_box(s, seed=40 + i, nu=2e-3 + 1e-3 * i) for i, s in enumerate(shapes)]
    return ws


def run_batch(fd6, ws, precision, nsteps, tile=3, zchunk=0, graph=True):
    b = fd6.Batch([w.shape for w in ws], precision)
    b.set_params([(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt) for w in ws])
    for i, w in enumerate(ws):
        b.init_fields(i, w.fields)
    if tile is not None:
        b.set_schedule(tile, zchunk)
    b.set_graph(graph)
    b.step(nsteps)
    out = [b.get_fields(i) for i in range(len(ws))]
    red = b.reduce()
    b.close()
    return out, red


def run_single(fd6, w, precision, nsteps, tile):
    box = fd6.Box(w.shape, precision)
    box.set_tile(tile)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(w.fields)
    box.step(nsteps)
    out = box.get_fields()
    red = box.reduce()
    box.close()
    return out, red


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("tile,zchunk", [(3, 0), (1, 8), (4, 0), (8, -1), (1, -1), (8, -2),
                                         (4, -2), (None, None)])
def test_batch_equals_single_box_runs_bitwise(fd6, precision, tile, zchunk):
    """(None, None): the default schedule, shape 8 with 64-plane chunks;
    zchunk -1: the balanced partition of the tile columns; -2: the packed deal
    of whole columns."""
    ws = small_ensemble()
    out, red = run_batch(fd6, ws, precision, 3, tile, zchunk)
    for i, w in enumerate(ws):
        ref, rref = run_single(fd6, w, precision, 3, 8 if tile is None else tile)
        for a, b in zip(out[i], ref):
            assert np.array_equal(a, b), (i, w.shape)
        assert red[i] == rref


def test_batch_fp64_matches_oracle(fd6, orc):
    ws = small_ensemble()
    out, _ = run_batch(fd6, ws, "fp64", 2)
    for i, w in enumerate(ws):
        ref = orc.rk3(w.fields, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, "55p", 2)
        err = max(float(np.max(np.abs(a - b)) / np.max(np.abs(b))) for a, b in zip(out[i], ref))
        assert err <= 1e-12, (i, err)


def test_graph_replay_equals_direct_launches(fd6):
    """Several replays (both starting parities) with eager work in between."""
    ws = small_ensemble()
    a, ra = run_batch(fd6, ws, "fp32", 5, graph=True)
    b, rb = run_batch(fd6, ws, "fp32", 5, graph=False)
    for x, y in zip(a, b):
        for p, q in zip(x, y):
            assert np.array_equal(p, q)
    assert ra == rb


def test_uneven_ensemble_sample(fd6, orc):
    """Eight boxes of the 64-box ensemble recipe (edges from {32,48,64,96})."""
    members = si.ensemble(nboxes=8)
    ws = [m.workload for m in members]
    out, _ = run_batch(fd6, ws, "fp32", 1)
    for i, w in enumerate(ws):
        inp = si.as_float32_exact(w.fields)
        ref = orc.rk3(inp, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, "55p", 1, 16)
        err = max(float(np.max(np.abs(a - b)) / np.max(np.abs(b))) for a, b in zip(out[i], ref))
        assert err <= 1e-5, (i, err)


def test_tuner_picks_a_valid_schedule_and_caches_it(fd6, tmp_path):
    """The library's autotuner: the chosen schedule is a z-sweep shape with
    one of the candidate chunk lengths, the ensemble still equals its
    single-box runs with that shape, and a second tuner call on the same
    ensemble takes the cached choice."""
    ws = small_ensemble()
    cache = str(tmp_path / "tune.txt")
    b = fd6.Batch([w.shape for w in ws], "fp32", layout="aos")
    b.set_params([(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt) for w in ws])
    for i, w in enumerate(ws):
        b.init_fields(i, w.fields)
    tile, zc = b.tune(cache)
    assert 1 <= tile < fd6.tile_count() and tile != 9 and zc in (0, 32, 48, 64, -1, -2)
    lines = open(cache).read().split("\n")
    assert len([ln for ln in lines if ln]) == 1 and lines[0].endswith(f" {tile} {zc}")
    b.set_schedule(1, 8)
    assert b.tune(cache) == (tile, zc)  # from the cache
    assert len([ln for ln in open(cache).read().split("\n") if ln]) == 1
    for i, w in enumerate(ws):
        b.init_fields(i, w.fields)
    b.step(2)
    for i, w in enumerate(ws):
        ref, _ = run_single(fd6, w, "fp32", 2, tile)
        for x, y in zip(b.get_fields(i), ref):
            assert np.array_equal(x, y), (i, w.shape)
    b.close()


def test_refused_schedule_leaves_the_schedule_in_force(fd6):
    """fd6_batch_set_schedule refuses chunks of 1-7 planes and bad shapes;
    the schedule in force, its work list and the results stay those of the
    last accepted call."""
    ws = small_ensemble()
    b = fd6.Batch([w.shape for w in ws], "fp32", layout="aos")
    b.set_params([(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt) for w in ws])
    for i, w in enumerate(ws):
        b.init_fields(i, w.fields)
    b.set_schedule(6, 16)
    for tile, zc, status in ((1, 1, -1), (6, 7, -1), (6, -3, -1), (0, 16, -1), (9, 16, -6),
                             (99, 16, -1)):
        with pytest.raises(fd6.Fd6Error) as ex:
            b.set_schedule(tile, zc)
        assert ex.value.status == status, (tile, zc)
        assert b.get_schedule() == (6, 16)
    b.step(2)
    for i, w in enumerate(ws):
        ref, _ = run_single(fd6, w, "fp32", 2, 6)
        for x, y in zip(b.get_fields(i), ref):
            assert np.array_equal(x, y), (i, w.shape)
    b.close()
