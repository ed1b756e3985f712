"""Host logic of the packed ensemble schedule (FD6_BATCH_PACKED): the column
deal in paper_1707_08900_amd/csrc/pack_columns.hpp, compiled on its own with
the host compiler and checked for exact coverage of every column, the
shortest-piece and cut limits, well-formed per-workgroup lists, and a largest
load no worse than the plain longest-first deal without cuts (computed here
independently)."""
import math
import os
import random
import shutil
import subprocess

import numpy as np
import pytest

import synthetic_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_08900_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <vector>
#include "pack_columns.hpp"
struct Item { int box, x0, y0, zb, ze; };
int main() {
    int tx, ty, G, refill, minc, n;
    if (scanf("%d %d %d %d %d %d", &tx, &ty, &G, &refill, &minc, &n) != 6) return 2;
    std::vector<Item> cols;
    for (int i = 0; i < n; ++i) {
        int nz, ny, nx;
        if (scanf("%d %d %d", &nz, &ny, &nx) != 3) return 2;
        for (int y0 = 0; y0 < ny; y0 += ty)
            for (int x0 = 0; x0 < nx; x0 += tx) cols.push_back(Item{i, x0, y0, 0, nz});
    }
    std::vector<Item> flat;
    std::vector<int> first;
    fd6::pack_columns(cols, G, refill, minc, &flat, &first);
    printf("%zu %zu\n", flat.size(), first.size());
    for (int f : first) printf("%d\n", f);
    for (const Item& it : flat) printf("%d %d %d %d %d\n", it.box, it.x0, it.y0, it.zb, it.ze);
    return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("pack")
    src, exe = d / "harness.cpp", d / "harness"
    src.write_text(HARNESS)
    # container bounds checks on: an index slip in the deal aborts the harness
    subprocess.run([cxx, "-O2", "-std=c++17", "-Wall", "-Werror", "-D_GLIBCXX_ASSERTIONS",
                    f"-I{CSRC}", str(src), "-o", str(exe)], check=True)
    return str(exe)


def run(exe, shapes, tx, ty, G, refill=6, minc=8):
    inp = f"{tx} {ty} {G} {refill} {minc} {len(shapes)}\n" + "".join(
        f"{nz} {ny} {nx}\n" for nz, ny, nx in shapes)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    lines = out.split("\n")
    nitems, nfirst = map(int, lines[0].split())
    first = [int(v) for v in lines[1:1 + nfirst]]
    items = [tuple(map(int, ln.split())) for ln in lines[1 + nfirst:1 + nfirst + nitems]]
    return first, items


def columns(shapes, tx, ty):
    return [(b, x0, y0, nz) for b, (nz, ny, nx) in enumerate(shapes)
            for y0 in range(0, ny, ty) for x0 in range(0, nx, tx)]


def lpt_no_cuts(shapes, tx, ty, G, refill):
    """Largest load of the plain deal: whole columns, longest first (stable),
    each to the least-loaded workgroup (lowest index among equals)."""
    import heapq
    costs = sorted((nz + refill for *_, nz in columns(shapes, tx, ty)), reverse=True)
    h = [(0, j) for j in range(G)]
    for c in costs:
        l, j = heapq.heappop(h)
        heapq.heappush(h, (l + c, j))
    return max(l for l, _ in h)


def check(shapes, tx, ty, G, first, items, refill=6, minc=8):
    cols = columns(shapes, tx, ty)
    nz_of = {(b, x0, y0): nz for b, x0, y0, nz in cols}
    # lists well formed
    assert len(first) == G + 1 and first[0] == 0 and first[-1] == len(items)
    assert all(a <= b for a, b in zip(first, first[1:]))
    # every plane of every column exactly once; pieces within the column
    cover = {k: np.zeros(nz, dtype=np.int64) for k, nz in nz_of.items()}
    pieces = {}
    for b, x0, y0, zb, ze in items:
        nz = nz_of[(b, x0, y0)]
        assert 0 <= zb < ze <= nz
        cover[(b, x0, y0)][zb:ze] += 1
        pieces.setdefault((b, x0, y0), []).append(ze - zb)
    for k, c in cover.items():
        assert np.all(c == 1), k
    # cut pieces keep at least minc planes; at most one cut per workgroup
    cut_cols = [k for k, p in pieces.items() if len(p) > 1]
    for k in cut_cols:
        assert min(pieces[k]) >= minc, (k, pieces[k])
    assert len(items) - len(cols) <= G
    loads = [sum(items[k][4] - items[k][3] + refill for k in range(first[L], first[L + 1]))
             for L in range(G)]
    return max(loads), sum(loads) / G, len(cut_cols)


def test_ensemble_of_the_benchmark(harness):
    """The 64-box ensemble (edges 32/48/64/96) with 32 x 8 tiles over 512
    workgroups: 1216 columns, a largest load of 212 plane steps (the deal
    without cuts: 226)."""
    shapes = [m.workload.shape for m in si.ensemble(64)]
    first, items = run(harness, shapes, 32, 8, 512)
    mk, mean, ncut = check(shapes, 32, 8, 512, first, items)
    assert len(columns(shapes, 32, 8)) == 1216
    assert lpt_no_cuts(shapes, 32, 8, 512, 6) == 226
    assert mk == 212 and mk <= 1.03 * mean and ncut == 120


@pytest.mark.parametrize("seed", range(12))
def test_random_ensembles(harness, seed):
    rng = random.Random(seed)
    n = rng.choice([1, 3, 17, 64])
    shapes = [(rng.randint(6, 120), rng.randint(6, 100), rng.randint(6, 100)) for _ in range(n)]
    tx, ty = rng.choice([(32, 8), (64, 4), (64, 8), (16, 16)])
    G = rng.choice([8, 64, 512])
    first, items = run(harness, shapes, tx, ty, G)
    mk, mean, _ = check(shapes, tx, ty, G, first, items)
    assert mk <= lpt_no_cuts(shapes, tx, ty, G, 6)


def test_more_workgroups_than_columns(harness):
    """Few columns, many workgroups: columns are cut into pieces of at least 8
    planes; a column too short to cut (6 or 9 planes) stays whole."""
    shapes = [(12, 12, 12), (16, 20, 24), (32, 32, 32), (9, 14, 33), (20, 16, 16), (6, 6, 6)]
    first, items = run(harness, shapes, 32, 8, 512)
    mk, _, ncut = check(shapes, 32, 8, 512, first, items)
    assert ncut > 0 and mk < lpt_no_cuts(shapes, 32, 8, 512, 6)


def test_many_columns_per_workgroup_keep_whole_columns(harness):
    """When the deal without cuts is already within 0.5% of the mean cost (many
    columns per workgroup), the packed deal keeps every column whole."""
    shapes = [(e, e, e) for e in (32 + 16 * (i % 5) for i in range(6000))]
    ncols = len(columns(shapes, 32, 8))
    lo = math.ceil(sum(nz + 6 for *_, nz in columns(shapes, 32, 8)) / 512)
    assert lpt_no_cuts(shapes, 32, 8, 512, 6) * 200 <= lo * 201  # the premise
    first, items = run(harness, shapes, 32, 8, 512)
    mk, _, ncut = check(shapes, 32, 8, 512, first, items)
    assert ncut == 0 and len(items) == ncols and mk <= 1.005 * lo
