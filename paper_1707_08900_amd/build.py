"""Build libfd6.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1707_08900_amd.build [--verbose] [--resource-usage] [--incremental]
       python -m paper_1707_08900_amd.build --host-sanitize --out DIR
         (host code instrumented with AddressSanitizer and UndefinedBehaviorSanitizer,
          device code unchanged; the library and its objects go to DIR)
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfd6.so")
SOURCES = ["aux_kernels.hip", "substep55_f32.hip", "substep55_f64.hip", "substep55_f32w64.hip",
           "substep55_aos_f32.hip", "substep55_aos_f64.hip", "substep55_aos_f32w64.hip",
           "substep19.hip", "reduce_static.hip", "fused12_f32.hip", "fd6_abi.cpp"]

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code.  Multiply-adds
# are fused only within one expression (-ffp-contract=on), so the rounding of
# every stencil sum is fixed by the source and does not depend on how a kernel
# is unrolled or inlined: all z-sweep shapes and the batched form agree bit
# for bit.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-ffp-contract=on",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-Wno-unknown-warning-option"]


# Per-unit options.  The FP64 sweep kernels run at one wave per SIMD (they need
# about 430 registers), so latency is hidden only by instruction-level
# parallelism inside the wave: the scheduler's max-ILP strategy orders them for
# that (512^3 AoS: 3640 -> 3525 us per launch; 32 x 8 with one array per field
# 4268 -> 3742 us).  It slows the two-wave FP32 kernels (1462 -> 1583 us), so it
# is applied to the FP64 units only.  Scheduling does not change results.
UNIT_FLAGS = {
    "substep55_f64.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
    "substep55_aos_f64.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


# Host-side sanitizers only: each flag applies to the host compilation.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer"]


def _up_to_date(src: str, obj: str) -> bool:
    """The object is newer than its source, every header of the library and
    this file (which holds the compiler options)."""
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src), os.path.abspath(__file__)]
    with open(deps[0]) as f:
        if "fd6.h" in f.read():
            deps.append(os.path.join(HERE, "..", "include", "fd6.h"))
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    return all(os.path.getmtime(d) < t for d in deps)


def _compile(src: str, resource_usage: bool, incremental: bool = False, build_dir: str = BUILD,
             extra=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    if incremental and not resource_usage and _up_to_date(src, obj):
        return obj
    cmd = [HIPCC, *COMMON, *UNIT_FLAGS.get(src, []), *extra, "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", obj]
    if resource_usage:
        cmd.insert(1, "-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if resource_usage:
        sys.stderr.write(r.stderr)
    return obj


def build(verbose: bool = False, resource_usage: bool = False, incremental: bool = False,
          host_sanitize: bool = False, out_dir: str = None) -> str:
    """Compile every unit (incremental: only units older than their source, a
    header or this file) and link libfd6.so (in out_dir if given, else in the
    package)."""
    build_dir = os.path.join(out_dir, "_build") if out_dir else BUILD
    lib = os.path.join(out_dir, "libfd6.so") if out_dir else LIB
    extra = HOST_SANITIZE if host_sanitize else []
    os.makedirs(build_dir, exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, resource_usage, incremental, build_dir, extra),
                           SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--resource-usage", action="store_true")
    ap.add_argument("--incremental", action="store_true",
                    help="skip units whose object is newer than every source and header")
    ap.add_argument("--host-sanitize", action="store_true",
                    help="instrument the host code with AddressSanitizer and UBSan")
    ap.add_argument("--out", default=None, help="directory for the library and its objects")
    a = ap.parse_args()
    build(verbose=True, resource_usage=a.resource_usage, incremental=a.incremental,
          host_sanitize=a.host_sanitize, out_dir=a.out)
