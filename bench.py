#!/usr/bin/env python3
"""Throughput benchmark of the full RK3 step on one MI355X.

Headline workload (the single-box FP32 throughput configuration): a 512^3
periodic box, FP32 storage and arithmetic, 55-point discretisation, fields
lnrho and u as sums of 16 random-phase Fourier modes with |k| <= 16 and
amplitude 0.1, nu = 1e-3, cs = 1, dt = 0.4 CFL, and FP64 global reductions
(mass, kinetic energy, sum lnrho, max |u|, non-finite count) computed on the
device after every step.  One step = 3 substeps, each one fused
right-hand-side + 2N-RK3 z-sweep kernel that resolves the periodic images in
its loader; the third also produces the reductions' partials.  The state is
stored as an array of structures (the four values of a point adjacent)
unless --layout soa.  Kernel shape and z-chunk come from the library's
autotuner.

Beside it, on the same GPU ("forms"): the FP64 and FP32 + FP64-RK3-register
precision forms, the other layout and the 19-point method at 512^3; the FP32
step at 256^3, 384^3 and 640^3, the FP32 and FP64 steps at 128^3 (a state
the last-level cache holds) and at 768^3 (linear sound wave); the 64-box
ensemble in both layouts; the forced 19-point 256^3 run.  Every form states
its error against the FP64 oracle on the same inputs: full fields after one
step at 128^3 to 640^3 and for all 64 ensemble boxes, the wave's x-profile
against the oracle's exact slab replica at 768^3.

Prints ONE JSON line (metric, value in grid-point updates/s, roofline of the
dominant kernel measured with HIP events on its stream, the FP64 oracle's
rate on the host CPU, and the forms).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per grid-point update (one full RK3 step), the
# method's own minimum: state read once per substep, w read when alpha != 0
# and written when it is needed again, output written once; ghosts and halo
# re-reads excluded.  55-point: 40 field accesses per step (16 of them to w);
# 19-point: 76 (28 to w).
ALG_BYTES = {("55p", "fp32"): 160, ("55p", "fp64"): 320, ("55p", "fp32_acc64"): 224,
             ("19p", "fp32"): 304, ("19p", "fp64"): 608, ("19p", "fp32_acc64"): 416}
LAUNCHES = {"55p": 3, "19p": 6}  # substep kernel launches per step
PREC_TAG = {"fp32": "f32", "fp64": "f64", "fp32_acc64": "f32w64"}
DTYPE = {"fp32": "f32", "fp64": "f64", "fp32_acc64": "f32 state, f64 RK3 register"}
PNAME = {"fp32": "FP32", "fp64": "FP64", "fp32_acc64": "FP32 state with FP64 RK3 register"}
VNAME = {"55p": "55-point fused substep", "19p": "19-point two-pass substep"}


def traffic_file(variant, precision, n):
    """Committed counter record of the headline kernel of one form."""
    kern = "substep55" if variant == "55p" else "substep19"
    return os.path.join(ROOT, "profiles", f"traffic_{kern}_{precision}_{n}.json")


def kernel_srcs(variant, precision):
    """Sources whose hash a counter record must match."""
    t = PREC_TAG[precision]
    files = ["sweep_common.hpp", "sweep_substep.hpp", f"substep55_{t}.hip"]
    files += [f"substep55_aos_{t}.hip"] if variant == "55p" else ["substep19.hip"]
    # build.py holds the compiler options, which shape the machine code too
    return ([os.path.join(ROOT, "paper_1707_08900_amd", "csrc", f) for f in files] +
            [os.path.join(ROOT, "paper_1707_08900_amd", "build.py")])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(shape, layout, variant="55p", precision="fp32", n=512):
    """HBM bytes per launch from the committed rocprofv3 counter records (one
    per kernel shape, z-chunk and layout), if one was taken on the current
    kernel source with the schedule and layout of this run."""
    try:
        with open(traffic_file(variant, precision, n)) as f:
            recs = json.load(f)
    except (OSError, ValueError):
        return None
    sha = source_sha(kernel_srcs(variant, precision))
    for t in (recs.get("records", []) if isinstance(recs, dict) else []):
        if (t.get("kernel_source_sha") == sha and t.get("layout", "soa") == layout and
                (t.get("tile"), t.get("zchunk")) == (shape.get("tile"), shape.get("zchunk"))):
            return t.get("traffic_bytes_per_launch")
    return None


def device_copy(torch, nrep):
    """A plain 1 GiB device-to-device copy, the streaming reference (and the
    calibration kernel of the rocprofv3 traffic counters); GB/s read + write."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(nrep):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2 * src.numel() * 4 * nrep / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def cpu_threads():
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set (the host's share per GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(n, 1)


def host_cpu():
    """(model name, physical cores, logical CPUs) of the host."""
    model, cores = "unknown CPU", set()
    try:
        phys = core = None
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == "unknown CPU":
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("physical id"):
                    phys = line.split(":", 1)[1].strip()
                elif line.startswith("core id"):
                    core = line.split(":", 1)[1].strip()
                elif not line.strip():
                    if core is not None:
                        cores.add((phys, core))
                    phys = core = None
    except OSError:
        pass
    return model, (len(cores) or None), os.cpu_count()


def rel_errs(out, ref):
    """Per field ||gpu - oracle||_inf / ||oracle||_inf."""
    import numpy as np
    return [float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))
            for a, b in zip(out, ref)]


def timed_steps(torch, box, red, steps, warmup, timing=True):
    for _ in range(warmup):
        box.step_reduce(1, red)
    torch.cuda.synchronize()
    if timing:
        box.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(box.stream)
    for _ in range(steps):
        box.step_reduce(1, red)
    e1.record(box.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    tm = box.get_timing() if timing else None
    if timing:
        box.set_timing(False)
    return wall, ev_ms, tm


def run_form(torch, fd6, w, dev_fields, prec, var, layout, steps, warmup, tile=None, zchunk=0,
             graph=False, error_steps=1, fused12=False):
    """Tune (or fix) the schedule, time `steps` reducing steps after `warmup`,
    then run `error_steps` steps from the initial state in the same schedule
    and return the state (FP64 device tensors) for the error check."""
    from paper_1707_08900_amd import tune as tuner
    n3 = int(w.shape[0]) * int(w.shape[1]) * int(w.shape[2])
    box = fd6.Box(w.shape, prec, var, layout=layout)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(dev_fields)
    if tile is None:
        tuned = tuner.tune(box)
    else:
        box.set_tile(tile)
        box.set_zchunk(zchunk)
        tuned = {"tile": tile, "zchunk": zchunk}
    box.set_fused_substeps(fused12)
    box.init_fields(dev_fields)
    red = torch.zeros(8, dtype=torch.float64, device="cuda")
    wall, ev_ms, (kms, klaunch, gms, glaunch) = timed_steps(torch, box, red, steps, warmup)
    v = n3 * steps / (ev_ms * 1e-3)
    alg_launch = n3 * ALG_BYTES[(var, prec)] / (2 if fused12 else LAUNCHES[var])
    avg_launch_s = kms * 1e-3 / klaunch
    res = {"updates_per_s": v, "ms_per_step": ev_ms / steps,
           "hbm_frac_step": v * ALG_BYTES[(var, prec)] / (HBM_PEAK_GBS * 1e9),
           "kernel_avg_launch_us": avg_launch_s * 1e6,
           "kernel_hbm_frac": alg_launch / avg_launch_s / (HBM_PEAK_GBS * 1e9),
           "kernel_shape": {"tile": tuned["tile"], "zchunk": tuned["zchunk"]},
           "host_wall_ms_per_step": wall * 1e3 / steps,
           "diagnostics": red[:5].cpu().tolist()}
    extra = {"tuned": tuned, "kms": kms, "klaunch": klaunch, "gms": gms, "glaunch": glaunch}
    if graph:
        box.set_graph(True)
        _, gev_ms, _ = timed_steps(torch, box, red, steps, 2, timing=False)
        box.set_graph(False)
        res["graph_ms_per_step"] = gev_ms / steps
        res["graph_updates_per_s"] = n3 * steps / (gev_ms * 1e-3)
    out = None
    if error_steps > 0:
        box.init_fields(dev_fields)
        box.step_reduce(error_steps, red)
        out = box.get_fields_device()
    box.close()
    return res, extra, out


class OracleSteps:
    """One-step FP64 oracle results of a workload, computed once per (method,
    input precision): FP64 inputs, or the FP32-rounded inputs the FP32 forms
    start from."""

    def __init__(self, orc, si, w, threads):
        self.orc, self.si, self.w, self.threads = orc, si, w, threads
        self.cache, self.seconds = {}, {}

    def get(self, var, prec):
        key = (var, "fp64" if prec == "fp64" else "fp32")
        if key not in self.cache:
            w = self.w
            inp = w.fields if key[1] == "fp64" else self.si.as_float32_exact(w.fields)
            t0 = time.perf_counter()
            self.cache[key] = self.orc.rk3(inp, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, var, 1,
                                           self.threads)
            self.seconds[key] = time.perf_counter() - t0
            log(f"oracle step {key}: {self.seconds[key]:.2f} s on {self.threads} threads")
        return self.cache[key]

    def drop(self, var, prec):
        self.cache.pop((var, "fp64" if prec == "fp64" else "fp32"), None)


def with_error(res, out, ref):
    e = rel_errs([t.cpu().numpy() for t in out], ref)
    res["rel_err_1step"] = max(e)
    res["rel_err_1step_fields"] = e
    res["error_measure"] = "full fields after one step vs the FP64 oracle on the same inputs"


def batch_form(torch, fd6, orc, si, steps, threads, layout="aos", schedule=None, check=True):
    """64 independent boxes (edges from {32, 48, 64, 96}, per-box nu and
    amplitude, FP32), one persistent launch per substep, graph per step.
    The kernel shape and z-chunk are tuned on the ensemble itself by the
    library's autotuner (or fixed by `schedule`); every box is then checked
    against the oracle after one step."""
    import numpy as np
    members = si.ensemble(64)
    ws = [m.workload for m in members]
    pts = sum(int(np.prod(w.shape)) for w in ws)
    b = fd6.Batch([w.shape for w in ws], "fp32", layout=layout)
    b.set_params([(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt) for w in ws])

    def reinit():
        for i, w in enumerate(ws):
            b.init_fields(i, w.fields)

    reinit()
    t0 = time.perf_counter()
    if schedule is None:
        best = b.tune()  # the library's autotuner (every shape x chunk choice)
    else:
        b.set_schedule(*schedule)
        best = b.get_schedule()
    tune_s = time.perf_counter() - t0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reinit()
    b.step(20)  # untimed: the step time settles 10-20 steps after a change of schedule
    torch.cuda.synchronize()
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    red = b.reduce()
    # error: every box after one step from its initial state
    errs = [float("nan")] * len(ws)
    if check:
        reinit()
        b.step(1)
        for i, w in enumerate(ws):
            ref = orc.rk3(si.as_float32_exact(w.fields), w.nu, w.cs, w.dx, w.dy, w.dz, w.dt,
                          "55p", 1, threads)
            errs[i] = max(rel_errs(b.get_fields(i), ref))
    b.close()
    by_edge = {}
    for w, e in zip(ws, errs):
        by_edge[str(w.shape[0])] = max(by_edge.get(str(w.shape[0]), 0.0), e)
    return {"updates_per_s": pts / (ms * 1e-3), "ms_per_step": ms, "boxes": len(ws),
            "points": pts, "sizes": sorted(set(w.shape[0] for w in ws)),
            "schedule": {"tile": best[0], "zchunk": best[1]},
            "tuning_s": round(tune_s, 2),
            "hbm_frac_step": pts / (ms * 1e-3) * ALG_BYTES[("55p", "fp32")] / (HBM_PEAK_GBS * 1e9),
            "all_finite": all(r["nonfinite"] == 0 for r in red),
            "rel_err_1step": max(errs), "rel_err_1step_by_edge": by_edge,
            "error_measure": "all 64 boxes, full fields after one step vs the FP64 oracle on "
                             "the same FP32-rounded inputs"}


def forced_form(torch, fd6, si, steps):
    """The forced-turbulence configuration of Sec. 6: 19-point method, 256^3,
    nu = 1.4e-4, FP32, a new forcing mode drawn every step (isotropic shell
    1 <= |k| <= 3, f0 = 0.02), next to the same steps without the force."""
    from paper_1707_08900_amd import tune as tuner
    n = 256
    w = si.fourier_box(n, seed=0, amplitude=0.1, kmax=16.0, nu=1.4e-4)
    draws = si.forcing_draws(steps + 2, 1.0, 3.0, 0.02, seed=0)
    dev = [torch.from_numpy(f).cuda() for f in w.fields]
    box = fd6.Box(w.shape, "fp32", "19p")
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    box.init_fields(dev)
    tuned = tuner.tune(box)
    res = {}
    for forced in (True, False):
        box.init_fields(dev)
        box.set_forcing(draws[0] if forced else None)
        box.step(2)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(box.stream)
        for s in range(steps):
            if forced:
                box.set_forcing(draws[2 + s])
            box.step(1)
        e1.record(box.stream)
        e1.synchronize()
        res[forced] = e0.elapsed_time(e1) / steps
    box.close()
    return {"updates_per_s": n ** 3 / (res[True] * 1e-3), "ms_per_step": res[True],
            "unforced_ms_per_step": res[False], "schedule": {"tile": tuned["tile"],
                                                             "zchunk": tuned["zchunk"]},
            "workload": "256^3, 19-point, FP32, nu = 1.4e-4, force drawn every step from "
                        "1 <= |k| <= 3, f0 = 0.02"}


SOUND_A, SOUND_K = 1e-4, 4


def sound_form(torch, fd6, orc, si, n, prec, steps, warmup, err_steps, threads):
    """The 768^3 linear sound wave (lnrho = 1e-4 sin(4x), u = 0, nu = 1e-4,
    dt = 0.4 dx): step rate, and after err_steps steps the x-profile against
    the oracle's exact n x 8 x 8 slab replica (the fields never vary in y
    and z) plus the spread across columns."""
    slab = si.sound_wave_box(shape=(8, 8, n), amplitude=SOUND_A, k=SOUND_K)
    h = 2 * math.pi / n

    class W:  # the n^3 box with the slab's parameters
        shape, nu, cs, dx, dy, dz, dt = (n, n, n), slab.nu, slab.cs, h, h, h, slab.dt
    x = torch.arange(n, dtype=torch.float64, device="cuda") * h
    lnrho = (SOUND_A * torch.sin(SOUND_K * x)).expand(n, n, n).contiguous()
    zero = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    dev = [lnrho, zero, zero, zero]
    res, extra, out = run_form(torch, fd6, W, dev, prec, "55p", "aos", steps, warmup,
                               error_steps=err_steps)
    del dev, lnrho, zero
    res["workload"] = (f"{n}^3 linear sound wave, lnrho = 1e-4 sin(4x), u = 0, nu = 1e-4, "
                       f"dt = 0.4 dx")
    if err_steps == 0:  # rate only (--no-check)
        return res, extra
    lr, ux = out[0], out[1]
    spread = float((lr - lr[0:1, 0:1, :]).abs().max()) / SOUND_A
    prof = [lr[0, 0].cpu().numpy(), ux[0, 0].cpu().numpy()]
    del out, lr, ux
    torch.cuda.empty_cache()
    f = slab.fields if prec == "fp64" else si.as_float32_exact(slab.fields)
    ref = orc.rk3(f, slab.nu, slab.cs, h, h, h, slab.dt, "55p", err_steps, threads)
    import numpy as np
    e = max(float(np.max(np.abs(prof[0] - ref[0][0, 0]))),
            float(np.max(np.abs(prof[1] - ref[1][0, 0])))) / SOUND_A
    res.update({"rel_err_profile": e, "column_spread": spread, "error_steps": err_steps,
                "error_measure": f"x-profiles of lnrho and ux after {err_steps} steps vs the "
                                 f"oracle's exact {n}x8x8 slab replica, relative to the "
                                 f"amplitude 1e-4"})
    return res, extra


def cpu_baseline(orefs, w, threads, oracle_key):
    """FP64 oracle rate: one full RK3 step of the whole workload on the host
    threads (the step the GPU forms are checked against), and one step of its
    first 48 z-planes (as a periodic box) on one thread."""
    orc, si = orefs.orc, orefs.si
    orefs.get(*oracle_key)
    dt = orefs.seconds[(oracle_key[0], "fp64" if oracle_key[1] == "fp64" else "fp32")]
    nzs = w.shape[0]
    pts = nzs * w.shape[1] * w.shape[2]
    nz1 = min(48, nzs)
    s1 = [f[:nz1].copy() for f in w.fields]
    t0 = time.perf_counter()
    orc.rk3(s1, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, "55p", 1, 1)
    dt1 = time.perf_counter() - t0
    model, phys, logical = host_cpu()
    return {"value": pts / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "value_1core": nz1 * w.shape[1] * w.shape[2] / dt1,
            "host_cpu": model, "host_physical_cores": phys, "host_logical_cpus": logical,
            "sample": f"the whole {w.shape[2]}x{w.shape[1]}x{nzs} workload, one RK3 step, FP64 "
                      f"C oracle with {threads} OpenMP threads, all the host threads this "
                      f"process may use ({dt:.2f} s); value_1core: its first {nz1} z-planes as "
                      f"a periodic box on 1 thread ({dt1:.2f} s); host CPU: {model}, "
                      f"{phys} physical cores, {logical} logical CPUs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other precision, layout, method and size forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle error checks")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched ensemble form")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched ensemble and print its entry (profiling); "
                         "--tile/--zchunk fix its schedule, --layout its layout")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration for rocprofv3)")
    ap.add_argument("--tile", type=int, default=None,
                    help="kernel shape of the headline run (skips the autotuner)")
    ap.add_argument("--zchunk", type=int, default=0,
                    help="z-chunk length with --tile (0: automatic)")
    ap.add_argument("--layout", choices=("aos", "soa"), default="aos",
                    help="device layout of the headline box's state (55-point only)")
    ap.add_argument("--precision", choices=("fp32", "fp64", "fp32_acc64"), default="fp32",
                    help="precision form of the headline box (profiling the other forms)")
    ap.add_argument("--variant", choices=("55p", "19p"), default="55p",
                    help="method of the headline box (profiling the other forms)")
    ap.add_argument("--sound-wave", action="store_true",
                    help="headline box holds the linear sound wave of the 768^3 form instead of "
                         "the random-phase fields (profiling that form at --size)")
    ap.add_argument("--fused12", action="store_true",
                    help="headline box with substeps 1 and 2 fused in one launch (FP32, "
                         "55-point; profiling the temporal-blocking schedule)")
    a = ap.parse_args()
    if a.variant == "19p":
        a.layout = "soa"  # the 19-point passes keep one array per field
    prec, var = a.precision, a.variant

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a box runs on "
              "one MI355X; splitting it into z slabs with a 3-plane halo exchange per substep "
              "is not implemented). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1707_08900_amd as fd6
    import synthetic_inputs as si
    threads = cpu_threads()

    if a.batch_only:
        import oracle
        oracle.build(force=False)
        if a.calibrate_copy:
            log(f"device copy 1 GiB: {device_copy(torch, 3):.0f} GB/s (read + write)")
        sched = (a.tile, a.zchunk) if a.tile is not None else None
        bf = batch_form(torch, fd6, oracle, si, a.steps, threads, layout=a.layout,
                        schedule=sched, check=not a.no_check)
        log(f"batched aos: {bf['ms_per_step']:.3f} ms/step, {bf['updates_per_s'] / 1e9:.2f} G "
            f"updates/s, schedule {bf['schedule']}, rel err {bf['rel_err_1step']:.3e}")
        print(json.dumps({"metric": "batched grid-point updates/s", "value": bf["updates_per_s"],
                          "unit": "updates/s", "batched_fp32": bf}), flush=True)
        return

    n = a.size
    t0 = time.perf_counter()
    w = si.sound_wave_box(n, amplitude=SOUND_A, k=SOUND_K) if a.sound_wave else si.large_box(n)
    log(f"inputs {n}^3 generated in {time.perf_counter() - t0:.1f} s; dt = {w.dt:.4e}")

    copy_gbs = device_copy(torch, 3 if a.calibrate_copy else 5)
    log(f"device copy 1 GiB: {copy_gbs:.0f} GB/s (read + write)")

    dev_fields = [torch.from_numpy(f).cuda() for f in w.fields]
    hk = "fp32" if (prec, var, n) == ("fp32", "55p", 512) else "headline"
    head, hx, hout = run_form(torch, fd6, w, dev_fields, prec, var, a.layout, a.steps, a.warmup,
                              tile=a.tile, zchunk=a.zchunk, graph=True,
                              error_steps=0 if a.no_check else 1, fused12=a.fused12)
    tuned = hx["tuned"]
    log(f"kernel shape: {tuned}")
    ms_per_step = head["ms_per_step"]
    value = head["updates_per_s"]
    log(f"{prec} {var} {a.layout} {n}^3: {ms_per_step:.3f} ms/step, {value / 1e9:.2f} G updates/s; "
        f"graph replay {head['graph_ms_per_step']:.3f} ms/step")

    # dominant kernel: the fused 55-point substep kernel (19-point: the
    # average of its two passes)
    alg_per_launch = n ** 3 * ALG_BYTES[(var, prec)] / (2 if a.fused12 else LAUNCHES[var])
    avg_launch_s = hx["kms"] * 1e-3 / hx["klaunch"]
    achieved = alg_per_launch / avg_launch_s / 1e9
    traffic = load_traffic(tuned, a.layout, var, prec, n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "kernel": ("substep55_fused12 + substep55_sweep_red (average per launch)"
                           if a.fused12 else
                           f"substep55_sweep (fused RHS + RK3, {a.layout} layout)" if var == "55p"
                           else "substep19_pass1 / substep19_pass2 (average per launch)"),
                "avg_launch_us": round(avg_launch_s * 1e6, 2), "launches": hx["klaunch"],
                "alg_bytes_per_launch": alg_per_launch,
                "ghost_fill_us_per_launch": round(hx["gms"] * 1e3 / max(hx["glaunch"], 1), 2),
                "device_copy_gbs": round(copy_gbs, 1)}

    import oracle
    oracle.build(force=False)
    orefs = OracleSteps(oracle, si, w, threads)
    forms = {hk: head}
    if not a.no_check:
        with_error(head, hout, orefs.get(var, prec))
        log(f"headline rel err after one step (full fields): {head['rel_err_1step']:.3e}")
    del hout
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(orefs, w, threads, (var, prec))
        log(f"cpu oracle: {cpu['value'] / 1e6:.2f} M updates/s on {threads} threads")

    if not a.no_forms:
        other = "soa" if a.layout == "aos" else "aos"
        # grouped by the oracle step they are checked against
        plan = [("fp32", "55p", other), ("fp32_acc64", "55p", "aos"),
                ("fp64", "55p", "aos"), ("fp64", "55p", "soa"),
                ("fp32", "19p", "soa"), ("fp64", "19p", "soa")]
        for i, (fprec, fvar, lay) in enumerate(plan):
            if (fprec, fvar, lay) == (prec, var, a.layout):
                continue
            entry, _, out = run_form(torch, fd6, w, dev_fields, fprec, fvar, lay, a.steps, 2,
                                     error_steps=0 if a.no_check else 1)
            if not a.no_check:
                with_error(entry, out, orefs.get(fvar, fprec))
            del out
            key = f"{fprec}_{fvar}" + (f"_{lay}" if fvar == "55p" else "")
            forms[key] = entry
            log(f"{key}: {entry['ms_per_step']:.3f} ms/step, "
                f"{entry['updates_per_s'] / 1e9:.2f} G updates/s, "
                f"rel err {entry.get('rel_err_1step', float('nan')):.3e}")
            # free an oracle step once no later form is checked against it
            okey = (fvar, fprec == "fp64")
            if all((v2, p2 == "fp64") != okey for p2, v2, _ in plan[i + 1:]):
                orefs.drop(fvar, fprec)
        orefs.cache.clear()
        base64 = forms.get("fp64_55p_aos", {}).get("updates_per_s")
        if base64:
            for k, e in forms.items():
                e["speed_vs_fp64_55p"] = e["updates_per_s"] / base64
    del dev_fields
    torch.cuda.empty_cache()

    if not a.no_forms and n == 512:
        # the size sweep: 256^3, 384^3 and 640^3 (random-phase, full-field
        # error) and 768^3 (the linear sound wave, profile error), FP32 and
        # FP64 at 768^3
        for ns in (256, 384, 640):
            wn = si.large_box(ns)
            dn = [torch.from_numpy(f).cuda() for f in wn.fields]
            en, _, out = run_form(torch, fd6, wn, dn, "fp32", "55p", "aos", a.steps, 2,
                                  error_steps=0 if a.no_check else 1)
            del dn
            if not a.no_check:
                with_error(en, out, OracleSteps(oracle, si, wn, threads).get("55p", "fp32"))
            en["workload"] = f"{ns}^3 random-phase |k|<=16 A=0.1, nu=1e-3"
            forms[f"fp32_55p_aos_{ns}"] = en
            del out, wn
            torch.cuda.empty_cache()
            log(f"fp32 {ns}^3: {en['ms_per_step']:.3f} ms/step, "
                f"{en['updates_per_s'] / 1e9:.2f} G updates/s, kernel "
                f"{en['kernel_hbm_frac']:.3f} of HBM peak")
        # 128^3 (16 random-phase modes, |k| <= 8, A = 1e-2, nu = 2e-3): the
        # state of a step (about 100 MB in FP32) stays in the last-level
        # cache between launches, so its fraction is not an HBM figure
        w128 = si.mid_box(128)
        d128 = [torch.from_numpy(f).cuda() for f in w128.fields]
        o128 = None if a.no_check else OracleSteps(oracle, si, w128, threads)
        for p128 in ("fp32", "fp64"):
            e128, _, out = run_form(torch, fd6, w128, d128, p128, "55p", "aos", max(a.steps, 100),
                                    5, graph=True, error_steps=0 if a.no_check else 1)
            if o128 is not None:
                with_error(e128, out, o128.get("55p", p128))
            e128["workload"] = ("128^3 random-phase |k|<=8 A=1e-2, nu=2e-3 (state held in the "
                                "last-level cache)")
            forms[f"{p128}_55p_aos_128"] = e128
            del out
            log(f"{p128} 128^3: {e128['ms_per_step']:.3f} ms/step, "
                f"{e128['updates_per_s'] / 1e9:.2f} G updates/s; graph replay "
                f"{e128['graph_ms_per_step']:.3f} ms/step, "
                f"{e128['graph_updates_per_s'] / 1e9:.2f} G updates/s")
        del d128
        for sprec in ("fp32", "fp64"):
            e768, _ = sound_form(torch, fd6, oracle, si, 768, sprec, a.steps, 2,
                                 0 if a.no_check else 100, threads)
            forms[f"{sprec}_55p_aos_768"] = e768
            log(f"{sprec} 768^3: {e768['ms_per_step']:.3f} ms/step, "
                f"{e768['updates_per_s'] / 1e9:.2f} G updates/s, kernel "
                f"{e768['kernel_hbm_frac']:.3f} of HBM peak, profile err "
                f"{e768.get('rel_err_profile', float('nan')):.3e}")
            torch.cuda.empty_cache()
        f32, f64 = forms["fp32_55p_aos_768"], forms["fp64_55p_aos_768"]
        f32["speed_vs_fp64_768"] = f32["updates_per_s"] / f64["updates_per_s"]

    if not a.no_forms:
        forms["forced_fp32_19p_256"] = forced_form(torch, fd6, si, max(10, a.steps // 2))
        ff = forms["forced_fp32_19p_256"]
        log(f"forced 19p 256^3: {ff['ms_per_step']:.3f} ms/step with a new force each step, "
            f"{ff['unforced_ms_per_step']:.3f} ms/step unforced")

    if not a.no_batch:
        for lay, key in (("aos", "batched_fp32"), ("soa", "batched_fp32_soa")):
            forms[key] = batch_form(torch, fd6, oracle, si, a.steps, threads, layout=lay)
            bf = forms[key]
            log(f"batched {lay}: {bf['ms_per_step']:.3f} ms/step, "
                f"{bf['updates_per_s'] / 1e9:.2f} G updates/s ({bf['boxes']} boxes, "
                f"{bf['points']} points, schedule {bf['schedule']}), "
                f"rel err {bf['rel_err_1step']:.3e}")
            if "fp64_55p_aos" in forms:
                bf["speed_vs_fp64_55p"] = (bf["updates_per_s"] /
                                           forms["fp64_55p_aos"]["updates_per_s"])

    out = {
        "metric": "grid-point updates/s per full RK3 step + % HBM roofline (FP64 vs FP32 vs batched)",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": f"{n}^3 periodic box, {PNAME[prec]}, {VNAME[var]}, 16 random-phase "
                               f"modes |k|<=16 A=0.1, nu=1e-3, cs=1, dt=0.4 CFL, FP64 reductions "
                               f"every step",
                   "grid": [n, n, n], "precision": prec, "variant": var,
                   "layout": a.layout, "kernel_shape": {"tile": tuned["tile"],
                                                        "zchunk": tuned["zchunk"]}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "hbm_frac_step": value * ALG_BYTES[(var, prec)] / (HBM_PEAK_GBS * 1e9),
        "rel_err_1step": head.get("rel_err_1step"),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
