"""Autotuner for the substep kernel shape (55-point and 19-point methods).

Times every kernel shape the library offers (fd6_tile_count) on the caller's
own box with HIP events, then a few z-chunk lengths for the fastest shape,
keeps the fastest pair, and caches the choice in a JSON
file keyed by grid shape, precision, variant, layout and device name (path from
FD6_TUNE_CACHE, default ~/.cache/fd6_tune.json).  Tuning runs real steps, so
it advances the box's state: call it before init_fields of the actual run,
or re-initialise afterwards.  The library's own tuner (fd6_tune, Box.tune)
makes the same choice in C for callers without Python; this one also returns
the timing of every candidate.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

import torch

from . import Box, Fd6Error, tile_count

FD6_EUNSUPPORTED = -6


def _cache_path() -> str:
    return os.environ.get("FD6_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fd6_tune.json"))


def _key(box: Box) -> str:
    name = torch.cuda.get_device_name(box.device)
    nz, ny, nx = box.shape
    return f"{name}|{nx}x{ny}x{nz}|{box.precision}|{box.variant}|{box.layout}"


def _load() -> Dict[str, dict]:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_tile(box: Box, tile: int, steps: int = 3, reduce: bool = False) -> float:
    """Milliseconds per full RK3 step with the given kernel shape (reduce:
    steps that also produce the FP64 diagnostics, as step_reduce does)."""
    box.set_tile(tile)
    red = torch.zeros(8, dtype=torch.float64, device=box.device) if reduce else None

    def run(n):
        for _ in range(n):
            if reduce:
                box.step_reduce(1, red)
            else:
                box.step(1)

    run(1)  # warm-up (code object load, caches)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(box.stream)
    run(steps)
    e1.record(box.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(box: Box, steps: int = 3, use_cache: bool = True,
         candidates: Optional[list] = None, zchunks: Optional[list] = None,
         reduce: bool = False) -> dict:
    """Pick the fastest kernel shape, then z-chunk length, for this box;
    returns {tile, zchunk, ms, timings, zchunk_timings}."""
    key = _key(box) + ("|reduce" if reduce else "")
    cache = _load() if use_cache else {}
    if use_cache and key in cache and "zchunk" in cache[key]:
        box.set_tile(cache[key]["tile"])
        box.set_zchunk(cache[key]["zchunk"])
        return cache[key]
    box.set_zchunk(0)
    tiles = candidates if candidates is not None else list(range(1, tile_count()))
    timings = {}
    for t in tiles:
        try:
            timings[t] = time_tile(box, t, steps, reduce)
        except Fd6Error as e:  # a shape the box's layout does not take
            if e.status != FD6_EUNSUPPORTED:
                raise
    best = min(timings, key=timings.get)
    box.set_tile(best)
    nz = box.shape[0]
    zcs = zchunks if zchunks is not None else sorted({z for z in (64, 128, 256) if z < nz} | {nz})
    ztimes = {}  # explicit lengths only, so the choice is reproducible
    for z in zcs:
        box.set_zchunk(z)
        ztimes[z] = time_tile(box, best, steps, reduce)
    zbest = min(ztimes, key=ztimes.get)
    box.set_zchunk(zbest)
    result = {"tile": best, "zchunk": zbest, "ms": ztimes[zbest],
              "timings": {str(k): v for k, v in timings.items()},
              "zchunk_timings": {str(k): v for k, v in ztimes.items()}}
    if use_cache:
        cache[key] = result
        path = _cache_path()
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return result
