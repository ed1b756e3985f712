"""Kernel-shape tuning of a box, reported from Python.

The search itself is the library's (fd6_tune, C ABI): every z-sweep shape the
box's layout takes with the automatic z-chunk, then the z-chunk lengths 64,
128, 256 (those below nz) and nz for the fastest shape, each on reducing
steps timed with HIP events, keeping the fastest pair.  This module only runs
it and returns the timings the library logged (fd6_get_tune_log).  Tuning
runs real steps, so it advances the box's state: call it before init_fields
of the actual run, or re-initialise afterwards.
"""
from __future__ import annotations

from typing import Optional

from . import Box


def tune(box: Box, cache_path: Optional[str] = None) -> dict:
    """Tune the box's schedule with the library's tuner; returns {tile,
    zchunk, ms, timings (shape -> ms per step, automatic chunk),
    zchunk_timings (chunk -> ms per step, chosen shape)}."""
    tile, zchunk = box.tune(cache_path)
    log = box.tune_log()
    shapes = {str(t): ms for t, z, ms in log if z == 0}
    chunks = {str(z): ms for t, z, ms in log if z != 0 and t == tile}
    best = [ms for t, z, ms in log if (t, z) == (tile, zchunk)]
    return {"tile": tile, "zchunk": zchunk, "ms": best[-1] if best else None,
            "timings": shapes, "zchunk_timings": chunks}


def main(argv=None) -> int:
    """Tune a random-phase box of the benchmark's kind and print the library's
    trial log as one JSON line (ms per reducing step for every shape with the
    automatic z-chunk, then the z-chunk lengths of the fastest shape)."""
    import argparse
    import json

    import torch

    import synthetic_inputs as si

    ap = argparse.ArgumentParser(description=main.__doc__.split("\n")[0])
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--precision", choices=("fp32", "fp64", "fp32_acc64"), default="fp32")
    ap.add_argument("--layout", choices=("aos", "soa"), default="aos")
    ap.add_argument("--variant", choices=("55p", "19p"), default="55p")
    a = ap.parse_args(argv)
    w = si.mid_box(a.size) if a.size <= 128 else si.large_box(a.size)
    box = Box(w.shape, a.precision, a.variant, layout=a.layout)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields([torch.from_numpy(f).cuda() for f in w.fields])
    res = tune(box)
    box.close()
    res.update({"size": a.size, "precision": a.precision, "layout": a.layout,
                "variant": a.variant, "device": torch.cuda.get_device_name(0)})
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    import sys
    sys.exit(main())
