#!/usr/bin/env python3
"""Throughput benchmark of the full RK3 step on one MI355X.

Workload (the single-box FP32 throughput configuration): a 512^3 periodic
box, FP32 storage and arithmetic, 55-point discretisation, fields lnrho and u
as sums of 16 random-phase Fourier modes with |k| <= 16 and amplitude 0.1,
nu = 1e-3, cs = 1, dt = 0.4 CFL, and FP64 global reductions (mass, kinetic
energy, sum lnrho, max |u|, non-finite count) computed on the device after
every step.  One step = 3 substeps, each one fused right-hand-side + 2N-RK3
z-sweep kernel that resolves the periodic images in its loader; the third
also produces the reductions' partials.  The state is stored as an array of
structures (the four values of a point adjacent) unless --layout soa.

Prints ONE JSON line (metric, value in grid-point updates/s, roofline of the
dominant kernel measured with HIP events on its stream, the FP64 oracle's
rate on the host CPU, and the other precision forms on the same GPU).
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
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source with the same layout, kernel shape and
    z-chunk length."""
    try:
        with open(traffic_file(variant, precision, n)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != source_sha(kernel_srcs(variant, precision)):
        return None
    if (t.get("tile"), t.get("zchunk")) != (shape.get("tile"), shape.get("zchunk")):
        return None
    if t.get("layout", "soa") != layout:
        return None
    return t.get("traffic_bytes_per_launch")


def make_box(fd6, w, dev_fields, precision, variant, tune=True, layout="soa"):
    box = fd6.Box(w.shape, precision, variant, layout=layout)
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    tuned = None
    if tune:
        from paper_1707_08900_amd import tune as tuner
        box.init_fields(dev_fields)
        tuned = tuner.tune(box, steps=2, use_cache=False, reduce=True)
    box.init_fields(dev_fields)
    return box, tuned


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


def sample_error(orc, fd6, si, w, dev_fields, precision, variant, nsamples=6, layout="soa"):
    """Max over sampled points of |gpu - oracle| / max|field| after one step
    from the workload's initial state (oracle on local patches)."""
    import numpy as np
    box, _ = make_box(fd6, w, dev_fields, precision, variant, tune=False, layout=layout)
    box.step(1)
    out = box.get_fields_device()
    box.close()
    inp = si.as_float32_exact(w.fields) if precision != "fp64" else w.fields
    rng = np.random.default_rng(123)
    nz, ny, nx = w.shape
    worst = 0.0
    scale = [max(float(np.max(np.abs(f))), 1e-300) for f in inp]
    for _ in range(nsamples):
        c = (int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx)))
        ref = orc.rk3_point(inp, c, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, variant, 1)
        for q in range(4):
            worst = max(worst, abs(float(out[q][c].item()) - ref[q]) / scale[q])
    return worst


def batch_form(torch, fd6, si, steps, layout="aos"):
    """64 independent boxes (edges from {32, 48, 64, 96}, per-box nu and
    amplitude, FP32), one persistent launch per substep, graph per step.
    The kernel shape and z-chunk are tuned on the ensemble itself by the
    library's autotuner."""
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
    best = b.tune()  # the library's autotuner (every shape x chunks 0, 32, 48, 64)
    tune_s = time.perf_counter() - t0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reinit()
    b.step(2)
    torch.cuda.synchronize()
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    red = b.reduce()
    b.close()
    return {"updates_per_s": pts / (ms * 1e-3), "ms_per_step": ms, "boxes": len(ws),
            "points": pts, "sizes": sorted(set(w.shape[0] for w in ws)),
            "schedule": {"tile": best[0], "zchunk": best[1]},
            "tuning_s": round(tune_s, 2),
            "hbm_frac_step": pts / (ms * 1e-3) * ALG_BYTES[("55p", "fp32")] / (HBM_PEAK_GBS * 1e9),
            "all_finite": all(r["nonfinite"] == 0 for r in red)}


def forced_form(torch, fd6, si, steps):
    """The forced-turbulence configuration of Sec. 6: 19-point method, 256^3,
    nu = 1.4e-4, FP32, a new forcing mode drawn every step (isotropic shell
    1 <= |k| <= 3, f0 = 0.02), next to the same steps without the force."""
    n = 256
    w = si.fourier_box(n, seed=0, amplitude=0.1, kmax=16.0, nu=1.4e-4)
    draws = si.forcing_draws(steps + 2, 1.0, 3.0, 0.02, seed=0)
    dev = [torch.from_numpy(f).cuda() for f in w.fields]
    box = fd6.Box(w.shape, "fp32", "19p")
    box.set_params(w.nu, w.cs, w.dx, w.dy, w.dz, w.dt)
    from paper_1707_08900_amd import tune as tuner
    box.init_fields(dev)
    tuned = tuner.tune(box, steps=2, use_cache=False)
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


def cpu_baseline(orc, si, w, threads):
    """FP64 oracle rate on a bounded sample of the workload: one full RK3
    step of the whole box on the host threads, and one step of its first 48
    z-planes (as a periodic box) on one thread; about 10-15 s in all."""
    warm = [f[:8].copy() for f in w.fields]
    orc.rk3(warm, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, "55p", 1, threads)  # load, thread pool
    nzs = w.shape[0]
    t0 = time.perf_counter()
    orc.rk3(w.fields, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, "55p", 1, threads)
    dt = time.perf_counter() - t0
    pts = nzs * w.shape[1] * w.shape[2]
    # the same oracle on one core
    nz1 = min(48, nzs)
    s1 = [f[:nz1].copy() for f in w.fields]
    t0 = time.perf_counter()
    orc.rk3(s1, w.nu, w.cs, w.dx, w.dy, w.dz, w.dt, "55p", 1, 1)
    dt1 = time.perf_counter() - t0
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": pts / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "value_1core": nz1 * w.shape[1] * w.shape[2] / dt1,
            "sample": f"the whole {w.shape[2]}x{w.shape[1]}x{nzs} workload, one RK3 step, FP64 "
                      f"C oracle with {threads} OpenMP threads ({dt:.2f} s); value_1core: its "
                      f"first {nz1} z-planes as a periodic box on 1 thread ({dt1:.2f} s); "
                      f"host CPU: {cpu}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--no-forms", action="store_true", help="skip the FP64/ACC64/19p forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled oracle check")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched ensemble form")
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
    a = ap.parse_args()
    if a.variant == "19p":
        a.layout = "soa"  # the 19-point passes keep one array per field
    prec, var = a.precision, a.variant
    launches_per_step = 3 if var == "55p" else 6

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a box runs on "
              "one MI355X; splitting it into z slabs with a 3-plane halo exchange per substep "
              "is not implemented). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1707_08900_amd as fd6
    import synthetic_inputs as si

    n = a.size
    t0 = time.perf_counter()
    w = si.large_box(n)
    log(f"inputs {n}^3 generated in {time.perf_counter() - t0:.1f} s; dt = {w.dt:.4e}")

    # streaming reference: a plain 1 GiB device-to-device copy (also the
    # calibration kernel of the rocprofv3 traffic counters)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3 if a.calibrate_copy else 5):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    copy_gbs = 2 * src.numel() * 4 * (3 if a.calibrate_copy else 5) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    log(f"device copy 1 GiB: {copy_gbs:.0f} GB/s (read + write)")

    dev_fields = [torch.from_numpy(f).cuda() for f in w.fields]
    red = torch.zeros(8, dtype=torch.float64, device="cuda")
    box, tuned = make_box(fd6, w, dev_fields, prec, var, tune=a.tile is None,
                          layout=a.layout)
    if a.tile is not None:
        box.set_tile(a.tile)
        box.set_zchunk(a.zchunk)
        tuned = {"tile": a.tile, "zchunk": a.zchunk}
    log(f"kernel shape: {tuned}")
    wall, ev_ms, (kms, klaunch, gms, glaunch) = timed_steps(torch, box, red, a.steps, a.warmup)
    r = red.cpu().numpy()
    # the same steps replayed from a captured graph per step (no per-launch
    # events in this mode)
    box.set_graph(True)
    _, gev_ms, _ = timed_steps(torch, box, red, a.steps, 2, timing=False)
    box.set_graph(False)
    box.close()
    ms_per_step = ev_ms / a.steps
    value = n ** 3 * a.steps / (ev_ms * 1e-3)
    log(f"{prec} {var} {a.layout} {n}^3: {ms_per_step:.3f} ms/step, {value / 1e9:.2f} G updates/s "
        f"(host wall {wall * 1e3 / a.steps:.3f} ms/step); mass {r[0]:.10e} ke {r[1]:.6e}")

    # dominant kernel: the fused 55-point substep kernel (19-point: the
    # average of its two passes)
    alg_per_launch = n ** 3 * ALG_BYTES[(var, prec)] / launches_per_step
    avg_launch_s = kms * 1e-3 / klaunch
    achieved = alg_per_launch / avg_launch_s / 1e9
    traffic = load_traffic(tuned, a.layout, var, prec, n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "kernel": (f"substep55_sweep (fused RHS + RK3, {a.layout} layout)" if var == "55p"
                           else "substep19_pass1 / substep19_pass2 (average per launch)"),
                "avg_launch_us": round(avg_launch_s * 1e6, 2), "launches": klaunch,
                "alg_bytes_per_launch": alg_per_launch,
                "ghost_fill_us_per_launch": round(gms * 1e3 / max(glaunch, 1), 2),
                "device_copy_gbs": round(copy_gbs, 1)}

    import oracle
    forms = {}
    step_alg = ALG_BYTES[(var, prec)]
    hk = "fp32" if (prec, var) == ("fp32", "55p") else "headline"  # key of the headline form
    forms[hk] = {"updates_per_s": value, "ms_per_step": ms_per_step,
                 "hbm_frac_step": value * step_alg / (HBM_PEAK_GBS * 1e9)}
    forms[f"{hk}_graph"] = {"updates_per_s": n ** 3 * a.steps / (gev_ms * 1e-3),
                           "ms_per_step": gev_ms / a.steps}
    log(f"{prec} {var} {n}^3 graph replay: {gev_ms / a.steps:.3f} ms/step")
    if not a.no_check:
        forms[hk]["sample_rel_err_1step"] = sample_error(oracle, fd6, si, w, dev_fields,
                                                         prec, var, layout=a.layout)
    if not a.no_forms:
        k2 = max(5, a.steps // 5)
        other = "soa" if a.layout == "aos" else "aos"
        for fprec, fvar, lay in (("fp64", "55p", "aos"), ("fp64", "55p", "soa"),
                                 ("fp32_acc64", "55p", "aos"), ("fp32", "55p", other),
                                 ("fp32", "19p", "soa"), ("fp64", "19p", "soa")):
            b2, tn = make_box(fd6, w, dev_fields, fprec, fvar, layout=lay)
            wl, em, tm = timed_steps(torch, b2, red, k2, 2)
            b2.close()
            v = n ** 3 * k2 / (em * 1e-3)
            entry = {"updates_per_s": v, "ms_per_step": em / k2,
                     "hbm_frac_step": v * ALG_BYTES[(fvar, fprec)] / (HBM_PEAK_GBS * 1e9),
                     "speed_vs_fp64_55p": None}
            entry["kernel_shape"] = {"tile": tn["tile"], "zchunk": tn["zchunk"]}
            if not a.no_check:
                entry["sample_rel_err_1step"] = sample_error(oracle, fd6, si, w, dev_fields,
                                                             fprec, fvar, layout=lay)
            key = f"{fprec}_{fvar}" + (f"_{lay}" if fvar == "55p" else "")
            forms[key] = entry
            log(f"{key}: {em / k2:.3f} ms/step, {v / 1e9:.2f} G updates/s")
        base64 = forms["fp64_55p_aos"]["updates_per_s"]
        forms[hk]["speed_vs_fp64_55p"] = value / base64
        for k, e in forms.items():
            if k != hk:
                e["speed_vs_fp64_55p"] = e["updates_per_s"] / base64

    if not a.no_forms:
        forms["forced_fp32_19p_256"] = forced_form(torch, fd6, si, max(10, a.steps // 2))
        ff = forms["forced_fp32_19p_256"]
        log(f"forced 19p 256^3: {ff['ms_per_step']:.3f} ms/step with a new force each step, "
            f"{ff['unforced_ms_per_step']:.3f} ms/step unforced")

    if not a.no_batch:
        for lay, key in (("aos", "batched_fp32"), ("soa", "batched_fp32_soa")):
            forms[key] = batch_form(torch, fd6, si, max(10, a.steps // 2), layout=lay)
            bf = forms[key]
            log(f"batched {lay}: {bf['ms_per_step']:.3f} ms/step, "
                f"{bf['updates_per_s'] / 1e9:.2f} G updates/s ({bf['boxes']} boxes, "
                f"{bf['points']} points, schedule {bf['schedule']})")
            if "fp64_55p_aos" in forms:
                bf["speed_vs_fp64_55p"] = (bf["updates_per_s"] /
                                           forms["fp64_55p_aos"]["updates_per_s"])

    cpu = None
    if not a.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        oracle.build(force=False)
        cpu = cpu_baseline(oracle, si, w, threads)
        log(f"cpu oracle: {cpu['value'] / 1e6:.2f} M updates/s on {threads} threads")

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
                   "layout": a.layout, "kernel_shape": tuned},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "hbm_frac_step": value * step_alg / (HBM_PEAK_GBS * 1e9),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
