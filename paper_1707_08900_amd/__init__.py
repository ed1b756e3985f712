"""MI355X (gfx950) per-substep kernel of a sixth-order finite-difference solver
for isothermal compressible hydrodynamics (Pekkila et al. 2017).

This module is a thin ctypes binding over ``libfd6.so`` (C ABI declared in
``include/fd6.h``): argument marshalling only.  Every step of the computation
runs in the library's HIP kernels; PyTorch provides the device workspace and
the HIP stream.  There is no CPU fallback: without the built library every
entry point raises ImportError (``library()``), and without a GPU creating a
box fails.

Box: one periodic box (55- or 19-point method, FP64 / FP32 / FP32 + FP64 RK3
register, state stored per field or as an array of structures).  Batch: an
ensemble of boxes advanced by one persistent launch per substep, with the
library's schedule autotuner.  tune.tune(): the kernel-shape autotuner of a
box.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch  # loaded first: its HIP runtime is the one the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
# FD6_LIB selects another build of the library (e.g. a host-sanitizer build)
LIB_PATH = os.environ.get("FD6_LIB") or os.path.join(_HERE, "libfd6.so")

PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_acc64": 2}
VARIANTS = {"55p": 0, "19p": 1}
LAYOUTS = {"soa": 0, "aos": 1}  # fd6_desc.flags: 0, FD6_LAYOUT_AOS
STATUS = {0: "FD6_OK", -1: "FD6_EINVAL", -2: "FD6_ESTATE", -3: "FD6_ENOMEM", -4: "FD6_EHIP",
          -5: "FD6_ENONFINITE", -6: "FD6_EUNSUPPORTED"}
# z-chunk values of Batch.set_schedule beside chunk lengths (FD6_BATCH_BALANCED,
# FD6_BATCH_PACKED in include/fd6.h)
BATCH_BALANCED = -1
BATCH_PACKED = -2

# every symbol the header declares
ABI_SYMBOLS = (
    "fd6_abi_version", "fd6_status_string", "fd6_workspace_bytes", "fd6_create", "fd6_destroy",
    "fd6_set_stream", "fd6_set_params", "fd6_init_fields", "fd6_init_fields_device",
    "fd6_rk3_step", "fd6_rk3_step_reduce", "fd6_get_fields", "fd6_get_fields_device", "fd6_reduce", "fd6_rhs",
    "fd6_reduce_device", "fd6_tile_count", "fd6_set_tile", "fd6_set_zchunk", "fd6_set_graph",
    "fd6_get_schedule", "fd6_tune", "fd6_get_tune_log",
    "fd6_set_forcing", "fd6_set_timing", "fd6_set_fused_substeps",
    "fd6_get_timing",
    "fd6_last_error", "fd6_batch_workspace_bytes", "fd6_batch_create", "fd6_batch_destroy",
    "fd6_batch_set_params", "fd6_batch_init_fields", "fd6_batch_set_schedule",
    "fd6_batch_tune", "fd6_batch_get_schedule",
    "fd6_batch_set_graph", "fd6_batch_step", "fd6_batch_get_fields", "fd6_batch_reduce",
    "fd6_batch_last_error", "fd6_reduce_fields_static",
)


class Fd6Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class Fd6Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("nu", "cs", "dx", "dy", "dz", "dt")]


class Fd6Forcing(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("kx", "ky", "kz", "ex", "ey", "ez", "f0", "phase")]


class Fd6Reductions(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("kinetic_energy", ctypes.c_double),
                ("sum_lnrho", ctypes.c_double), ("umax", ctypes.c_double),
                ("nonfinite", ctypes.c_int64)]


class Fd6Error(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        msg = f"{what}: {STATUS.get(status, status)}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


def _declare(lib):
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    sig = {
        "fd6_abi_version": (I, []),
        "fd6_status_string": (ctypes.c_char_p, [I]),
        "fd6_workspace_bytes": (I, [ctypes.POINTER(Fd6Desc), ctypes.POINTER(ctypes.c_size_t)]),
        "fd6_create": (I, [ctypes.POINTER(Fd6Desc), P, ctypes.c_size_t, P, ctypes.POINTER(P)]),
        "fd6_destroy": (I, [P]),
        "fd6_set_stream": (I, [P, P]),
        "fd6_set_params": (I, [P, ctypes.POINTER(Fd6Params)]),
        "fd6_init_fields": (I, [P, D, D, D, D]),
        "fd6_init_fields_device": (I, [P, P, P, P, P]),
        "fd6_rk3_step": (I, [P, ctypes.c_int32]),
        "fd6_rk3_step_reduce": (I, [P, ctypes.c_int32, P]),
        "fd6_get_fields": (I, [P, D, D, D, D]),
        "fd6_get_fields_device": (I, [P, P, P, P, P]),
        "fd6_reduce": (I, [P, ctypes.POINTER(Fd6Reductions)]),
        "fd6_rhs": (I, [P, D, D, D, D]),
        "fd6_reduce_device": (I, [P, P]),
        "fd6_set_timing": (I, [P, I]),
        "fd6_get_timing": (I, [P, D, ctypes.POINTER(ctypes.c_int64), D,
                                ctypes.POINTER(ctypes.c_int64)]),
        "fd6_tile_count": (I, []),
        "fd6_set_tile": (I, [P, ctypes.c_int32]),
        "fd6_set_zchunk": (I, [P, ctypes.c_int32]),
        "fd6_set_graph": (I, [P, ctypes.c_int32]),
        "fd6_set_fused_substeps": (I, [P, ctypes.c_int32]),
        "fd6_set_forcing": (I, [P, ctypes.POINTER(Fd6Forcing)]),
        "fd6_last_error": (ctypes.c_char_p, [P]),
        "fd6_batch_workspace_bytes": (I, [ctypes.c_int32, ctypes.POINTER(Fd6Desc),
                                          ctypes.POINTER(ctypes.c_size_t)]),
        "fd6_batch_create": (I, [ctypes.c_int32, ctypes.POINTER(Fd6Desc), P, ctypes.c_size_t, P,
                                 ctypes.POINTER(P)]),
        "fd6_batch_destroy": (I, [P]),
        "fd6_batch_set_params": (I, [P, ctypes.POINTER(Fd6Params)]),
        "fd6_batch_init_fields": (I, [P, ctypes.c_int32, D, D, D, D]),
        "fd6_batch_set_schedule": (I, [P, ctypes.c_int32, ctypes.c_int32]),
        "fd6_tune": (I, [P, ctypes.c_char_p]),
        "fd6_get_schedule": (I, [P, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int32)]),
        "fd6_get_tune_log": (I, [P, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int32)]),
        "fd6_batch_tune": (I, [P, ctypes.c_char_p]),
        "fd6_batch_get_schedule": (I, [P, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
        "fd6_batch_set_graph": (I, [P, ctypes.c_int32]),
        "fd6_batch_step": (I, [P, ctypes.c_int32]),
        "fd6_batch_get_fields": (I, [P, ctypes.c_int32, D, D, D, D]),
        "fd6_batch_reduce": (I, [P, ctypes.POINTER(Fd6Reductions)]),
        "fd6_batch_last_error": (ctypes.c_char_p, [P]),
        "fd6_reduce_fields_static": (I, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, P, P, P, P, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def library():
    """Load libfd6.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1707_08900_amd.build`")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def workspace_bytes(shape, precision="fp32", variant="55p", layout="soa") -> int:
    nz, ny, nx = shape
    d = Fd6Desc(nx, ny, nz, PRECISIONS[precision], VARIANTS[variant], LAYOUTS[layout])
    out = ctypes.c_size_t()
    rc = library().fd6_workspace_bytes(ctypes.byref(d), ctypes.byref(out))
    if rc != 0:
        raise Fd6Error(rc, "fd6_workspace_bytes")
    return out.value


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Box:
    """One periodic box: lnrho, ux, uy, uz of shape (nz, ny, nx) on the GPU.

    layout: device layout of the state, "soa" (one array per field) or "aos"
    (the four values of a point adjacent; 55-point method only)."""

    def __init__(self, shape: Sequence[int], precision: str = "fp32", variant: str = "55p",
                 device: str = "cuda:0", stream: Optional[torch.cuda.Stream] = None,
                 layout: str = "soa"):
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1707_08900_amd needs a ROCm GPU (gfx950); none is visible")
        self.lib = library()
        self.shape = tuple(int(s) for s in shape)
        self.precision, self.variant, self.layout = precision, variant, layout
        self.device = torch.device(device)
        nz, ny, nx = self.shape
        self.desc = Fd6Desc(nx, ny, nz, PRECISIONS[precision], VARIANTS[variant], LAYOUTS[layout])
        nbytes = workspace_bytes(self.shape, precision, variant, layout)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        self._check(self.lib.fd6_create(ctypes.byref(self.desc), ctypes.c_void_p(aligned),
                                        nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                        ctypes.byref(h)), "fd6_create", handle=False)
        self.h = h
        self.params = None

    # -- helpers --------------------------------------------------------
    def _check(self, rc, what, handle=True):
        if rc != 0:
            detail = ""
            if handle and getattr(self, "h", None):
                detail = (self.lib.fd6_last_error(self.h) or b"").decode()
            raise Fd6Error(rc, what, detail)
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.fd6_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API --------------------------------------------------------------
    def set_stream(self, stream: torch.cuda.Stream):
        self.stream = stream
        self._check(self.lib.fd6_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)),
                    "fd6_set_stream")

    def set_params(self, nu, cs, dx, dy, dz, dt):
        self.params = Fd6Params(nu, cs, dx, dy, dz, dt)
        self._check(self.lib.fd6_set_params(self.h, ctypes.byref(self.params)), "fd6_set_params")

    def init_fields(self, fields):
        """fields: four float64 arrays (numpy on the host, or torch on this device)."""
        if all(isinstance(f, torch.Tensor) and f.is_cuda for f in fields):
            ts = [f.contiguous() for f in fields]
            for t in ts:
                assert t.dtype == torch.float64 and tuple(t.shape) == self.shape
            self._keep = ts
            self._check(self.lib.fd6_init_fields_device(
                self.h, *[ctypes.c_void_p(t.data_ptr()) for t in ts]), "fd6_init_fields_device")
            return
        arrs = [np.ascontiguousarray(f, dtype=np.float64) for f in fields]
        for a in arrs:
            assert a.shape == self.shape, (a.shape, self.shape)
        self._check(self.lib.fd6_init_fields(self.h, *[_dptr(a) for a in arrs]),
                    "fd6_init_fields")

    def step(self, nsteps: int = 1):
        self._check(self.lib.fd6_rk3_step(self.h, int(nsteps)), "fd6_rk3_step")

    def step_reduce(self, nsteps: int, out: torch.Tensor):
        """Advance and leave the FP64 diagnostics of the final state in `out`
        (float64 device tensor, >= 5 elements), asynchronously."""
        assert out.dtype == torch.float64 and out.is_cuda and out.numel() >= 5
        self._check(self.lib.fd6_rk3_step_reduce(self.h, int(nsteps),
                                                 ctypes.c_void_p(out.data_ptr())),
                    "fd6_rk3_step_reduce")

    def get_fields(self):
        out = [np.empty(self.shape) for _ in range(4)]
        self._check(self.lib.fd6_get_fields(self.h, *[_dptr(a) for a in out]), "fd6_get_fields")
        return out

    def get_fields_device(self):
        out = [torch.empty(self.shape, dtype=torch.float64, device=self.device) for _ in range(4)]
        self._check(self.lib.fd6_get_fields_device(
            self.h, *[ctypes.c_void_p(t.data_ptr()) for t in out]), "fd6_get_fields_device")
        return out

    def rhs(self):
        out = [np.empty(self.shape) for _ in range(4)]
        self._check(self.lib.fd6_rhs(self.h, *[_dptr(a) for a in out]), "fd6_rhs")
        return out

    def reduce(self, allow_nonfinite: bool = False):
        r = Fd6Reductions()
        rc = self.lib.fd6_reduce(self.h, ctypes.byref(r))
        if rc != 0 and not (allow_nonfinite and rc == -5):
            self._check(rc, "fd6_reduce")
        return {"mass": r.mass, "kinetic_energy": r.kinetic_energy, "sum_lnrho": r.sum_lnrho,
                "umax": r.umax, "nonfinite": int(r.nonfinite)}

    def reduce_device(self, out: torch.Tensor):
        """Enqueue the FP64 diagnostics into a 5-element float64 device tensor."""
        assert out.dtype == torch.float64 and out.is_cuda and out.numel() >= 5
        self._check(self.lib.fd6_reduce_device(self.h, ctypes.c_void_p(out.data_ptr())),
                    "fd6_reduce_device")

    def set_timing(self, enable: bool):
        self._check(self.lib.fd6_set_timing(self.h, 1 if enable else 0), "fd6_set_timing")

    def get_timing(self):
        """(kernel_ms, kernel_launches, ghost_ms, ghost_launches) since set_timing(True)."""
        km, kn, gm, gn = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.fd6_get_timing(self.h, ctypes.byref(km), ctypes.byref(kn),
                                            ctypes.byref(gm), ctypes.byref(gn)), "fd6_get_timing")
        return km.value, kn.value, gm.value, gn.value

    def set_tile(self, tile: int):
        self._check(self.lib.fd6_set_tile(self.h, int(tile)), "fd6_set_tile")

    def set_zchunk(self, zchunk: int):
        """z-chunk length of the sweep kernels (0: automatic)."""
        self._check(self.lib.fd6_set_zchunk(self.h, int(zchunk)), "fd6_set_zchunk")

    def get_schedule(self):
        """(kernel shape, z-chunk length) currently in use."""
        t, z = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.fd6_get_schedule(self.h, ctypes.byref(t), ctypes.byref(z)),
                    "fd6_get_schedule")
        return t.value, z.value

    def tune(self, cache_path: Optional[str] = None):
        """The library's autotuner (fd6_tune; advances the state, so set the
        fields again afterwards).  Returns (tile, zchunk); tune_log() lists
        the candidates it timed."""
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.fd6_tune(self.h, path), "fd6_tune")
        return self.get_schedule()

    def tune_log(self):
        """[(tile, zchunk, ms per step)] timed by the last tune() call."""
        n = ctypes.c_int32()
        self._check(self.lib.fd6_get_tune_log(self.h, None, None, None, 0, ctypes.byref(n)),
                    "fd6_get_tune_log")
        k = n.value
        t, z, m = (ctypes.c_int32 * k)(), (ctypes.c_int32 * k)(), (ctypes.c_float * k)()
        self._check(self.lib.fd6_get_tune_log(self.h, t, z, m, k, ctypes.byref(n)),
                    "fd6_get_tune_log")
        return [(t[i], z[i], float(m[i])) for i in range(k)]

    def set_forcing(self, forcing=None):
        """External force (one mode of eq. forcing) for the following steps:
        ``{"k": (kx, ky, kz), "e": (ex, ey, ez), "f0": f0, "phase": phi}``, or
        None to switch it off."""
        if forcing is None:
            self._check(self.lib.fd6_set_forcing(self.h, None), "fd6_set_forcing")
            return
        f = Fd6Forcing(*[float(v) for v in forcing["k"]], *[float(v) for v in forcing["e"]],
                       float(forcing["f0"]), float(forcing["phase"]))
        self._check(self.lib.fd6_set_forcing(self.h, ctypes.byref(f)), "fd6_set_forcing")

    def set_fused_substeps(self, enable: bool):
        """Run substeps 1 and 2 of every step as one launch (temporal
        blocking; FP32, 55-point; experimental, off by default)."""
        self._check(self.lib.fd6_set_fused_substeps(self.h, 1 if enable else 0),
                    "fd6_set_fused_substeps")

    def set_graph(self, enable: bool):
        """Replay each step as a captured HIP graph."""
        self._check(self.lib.fd6_set_graph(self.h, 1 if enable else 0), "fd6_set_graph")


class Batch:
    """An ensemble of independent periodic boxes advanced together on the GPU
    (one persistent launch per substep, a captured graph per step); layout as
    for Box, one for every box."""

    def __init__(self, shapes, precision: str = "fp32", device: str = "cuda:0",
                 stream: Optional[torch.cuda.Stream] = None, layout: str = "soa"):
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1707_08900_amd needs a ROCm GPU (gfx950); none is visible")
        self.lib = library()
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.n = len(self.shapes)
        self.precision, self.layout = precision, layout
        self.device = torch.device(device)
        arr = (Fd6Desc * self.n)()
        for i, (nz, ny, nx) in enumerate(self.shapes):
            arr[i] = Fd6Desc(nx, ny, nz, PRECISIONS[precision], VARIANTS["55p"], LAYOUTS[layout])
        self._descs = arr
        need = ctypes.c_size_t()
        rc = self.lib.fd6_batch_workspace_bytes(self.n, arr, ctypes.byref(need))
        if rc != 0:
            raise Fd6Error(rc, "fd6_batch_workspace_bytes")
        self._ws = torch.empty(need.value + 256, dtype=torch.uint8, device=self.device)
        aligned = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = self.lib.fd6_batch_create(self.n, arr, ctypes.c_void_p(aligned), need.value,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise Fd6Error(rc, "fd6_batch_create")
        self.h = h

    def _check(self, rc, what):
        if rc != 0:
            detail = (self.lib.fd6_batch_last_error(self.h) or b"").decode()
            raise Fd6Error(rc, what, detail)

    def close(self):
        if getattr(self, "h", None):
            self.lib.fd6_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        """params: sequence of (nu, cs, dx, dy, dz, dt), one per box."""
        arr = (Fd6Params * self.n)(*[Fd6Params(*p) for p in params])
        self._check(self.lib.fd6_batch_set_params(self.h, arr), "fd6_batch_set_params")

    def init_fields(self, box: int, fields):
        arrs = [np.ascontiguousarray(f, dtype=np.float64) for f in fields]
        for a in arrs:
            assert a.shape == self.shapes[box]
        self._check(self.lib.fd6_batch_init_fields(self.h, box, *[_dptr(a) for a in arrs]),
                    "fd6_batch_init_fields")

    def set_schedule(self, tile: int, zchunk: int = 0):
        """Kernel shape and work distribution: zchunk >= 0 (chunks of at most
        zchunk planes, 0 = whole boxes, dealt in turn), BATCH_BALANCED or
        BATCH_PACKED."""
        self._check(self.lib.fd6_batch_set_schedule(self.h, tile, zchunk), "fd6_batch_set_schedule")

    def get_schedule(self):
        t, z = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.fd6_batch_get_schedule(self.h, ctypes.byref(t), ctypes.byref(z)),
                    "fd6_batch_get_schedule")
        return t.value, z.value

    def tune(self, cache_path: Optional[str] = None):
        """Time the schedules in the library's autotuner and keep the fastest
        (advances every box; set the fields again afterwards).  Returns
        (tile, zchunk)."""
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.fd6_batch_tune(self.h, path), "fd6_batch_tune")
        return self.get_schedule()

    def set_graph(self, enable: bool):
        self._check(self.lib.fd6_batch_set_graph(self.h, 1 if enable else 0), "fd6_batch_set_graph")

    def step(self, nsteps: int = 1):
        self._check(self.lib.fd6_batch_step(self.h, int(nsteps)), "fd6_batch_step")

    def get_fields(self, box: int):
        out = [np.empty(self.shapes[box]) for _ in range(4)]
        self._check(self.lib.fd6_batch_get_fields(self.h, box, *[_dptr(a) for a in out]),
                    "fd6_batch_get_fields")
        return out

    def reduce(self):
        arr = (Fd6Reductions * self.n)()
        rc = self.lib.fd6_batch_reduce(self.h, arr)
        if rc not in (0, -5):
            self._check(rc, "fd6_batch_reduce")
        return [{"mass": r.mass, "kinetic_energy": r.kinetic_energy, "sum_lnrho": r.sum_lnrho,
                 "umax": r.umax, "nonfinite": int(r.nonfinite)} for r in arr]


def tile_count() -> int:
    return library().fd6_tile_count()


def reduce_fields_static(fields, dx: float, dy: float, dz: float, out: torch.Tensor,
                         stream: Optional[torch.cuda.Stream] = None) -> None:
    """FP64 diagnostics of four compact device tensors (float32 or float64,
    shape (nz, ny, nx)) into the 5-element float64 device tensor `out`,
    asynchronously, through the library entry point that allocates nothing
    (its partial sums live in a static device array shared by every call on
    the device)."""
    ts = list(fields)
    assert len(ts) == 4 and all(t.is_cuda and t.is_contiguous() for t in ts)
    dt = ts[0].dtype
    assert ts[0].dim() == 3 and all(t.dtype == dt and t.shape == ts[0].shape for t in ts)
    prec = {torch.float64: PRECISIONS["fp64"], torch.float32: PRECISIONS["fp32"]}[dt]
    assert out.dtype == torch.float64 and out.is_cuda and out.numel() >= 5
    assert all(t.device == ts[0].device for t in ts) and out.device == ts[0].device
    nz, ny, nx = (int(v) for v in ts[0].shape)
    st = stream if stream is not None else torch.cuda.current_stream(ts[0].device)
    # the library takes the static array of the current device
    with torch.cuda.device(ts[0].device):
        rc = library().fd6_reduce_fields_static(
            nx, ny, nz, prec, *[ctypes.c_void_p(t.data_ptr()) for t in ts], float(dx),
            float(dy), float(dz), ctypes.c_void_p(st.cuda_stream),
            ctypes.c_void_p(out.data_ptr()))
    if rc != 0:
        raise Fd6Error(rc, "fd6_reduce_fields_static")
