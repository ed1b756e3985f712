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
