"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/fd6.h declares, and its validation layer rejects
bad arguments and out-of-order calls without touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fd6.h")


def header_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fd6_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def pkg():
    import paper_1707_08900_amd as p
    if not os.path.exists(p.LIB_PATH):
        pytest.fail("libfd6.so is not built (python -m paper_1707_08900_amd.build)")
    return p


def test_exports_every_declared_symbol(pkg):
    lib = pkg.library()
    declared = header_symbols()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(pkg.ABI_SYMBOLS)


def test_version_and_status_strings(pkg):
    lib = pkg.library()
    assert lib.fd6_abi_version() == 1
    for s in range(-6, 1):
        assert lib.fd6_status_string(s)
    assert lib.fd6_status_string(-99) == b"unknown status"


def desc(nx=32, ny=32, nz=32, prec=1, var=0, flags=0):
    import paper_1707_08900_amd as p
    return p.Fd6Desc(nx, ny, nz, prec, var, flags)


def test_workspace_bytes_validation(pkg):
    lib = pkg.library()
    out = ctypes.c_size_t()
    assert lib.fd6_workspace_bytes(ctypes.byref(desc()), ctypes.byref(out)) == 0
    fp32 = out.value
    assert lib.fd6_workspace_bytes(ctypes.byref(desc(prec=0)), ctypes.byref(out)) == 0
    assert out.value > fp32  # FP64 needs more
    for bad in (desc(nx=5), desc(ny=0), desc(nz=4097), desc(prec=3), desc(var=2),
                desc(flags=2), desc(flags=-1)):
        assert lib.fd6_workspace_bytes(ctypes.byref(bad), ctypes.byref(out)) == -1
    assert lib.fd6_workspace_bytes(None, ctypes.byref(out)) == -1
    assert lib.fd6_workspace_bytes(ctypes.byref(desc()), None) == -1


def test_aos_layout_flag(pkg):
    """FD6_LAYOUT_AOS: same workspace as one array per field, 55-point only."""
    lib = pkg.library()
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    for prec in (0, 1, 2):
        assert lib.fd6_workspace_bytes(ctypes.byref(desc(prec=prec)), ctypes.byref(a)) == 0
        assert lib.fd6_workspace_bytes(ctypes.byref(desc(prec=prec, flags=1)),
                                       ctypes.byref(b)) == 0
        assert a.value == b.value
    assert lib.fd6_workspace_bytes(ctypes.byref(desc(var=1, flags=1)), ctypes.byref(a)) == -6
    assert pkg.workspace_bytes((20, 24, 28), "fp64", "55p", "aos") == \
        pkg.workspace_bytes((20, 24, 28), "fp64", "55p")
    # an ensemble takes one layout for all its boxes
    ds = (pkg.Fd6Desc * 2)(desc(), desc(flags=1))
    assert lib.fd6_batch_workspace_bytes(2, ds, ctypes.byref(a)) == -1
    ds = (pkg.Fd6Desc * 2)(desc(flags=1), desc(nx=48, flags=1))
    assert lib.fd6_batch_workspace_bytes(2, ds, ctypes.byref(a)) == 0
    ds0 = (pkg.Fd6Desc * 2)(desc(), desc(nx=48))
    assert lib.fd6_batch_workspace_bytes(2, ds0, ctypes.byref(b)) == 0
    assert a.value == b.value


def test_workspace_grows_with_19p_div_field(pkg):
    lib = pkg.library()
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    lib.fd6_workspace_bytes(ctypes.byref(desc(var=0)), ctypes.byref(a))
    lib.fd6_workspace_bytes(ctypes.byref(desc(var=1)), ctypes.byref(b))
    assert b.value > a.value


def test_create_validation_and_state_machine(pkg):
    """Everything here stays in host code: fd6_create only carves the
    workspace pointer, and validation precedes every device call."""
    lib = pkg.library()
    d = desc(nx=8, ny=8, nz=8, prec=0)
    need = ctypes.c_size_t()
    lib.fd6_workspace_bytes(ctypes.byref(d), ctypes.byref(need))
    fake = ctypes.c_void_p(1 << 40)  # aligned, never dereferenced by create
    h = ctypes.c_void_p()
    assert lib.fd6_create(ctypes.byref(d), fake, need.value - 1, None, ctypes.byref(h)) == -3
    assert lib.fd6_create(ctypes.byref(d), ctypes.c_void_p((1 << 40) + 8), need.value, None,
                          ctypes.byref(h)) == -1
    assert lib.fd6_create(ctypes.byref(d), None, need.value, None, ctypes.byref(h)) == -1
    assert lib.fd6_create(ctypes.byref(d), fake, need.value, None, None) == -1
    assert lib.fd6_create(ctypes.byref(d), fake, need.value, None, ctypes.byref(h)) == 0
    try:
        # step / get / reduce / rhs before params and fields
        assert lib.fd6_rk3_step(h, 1) == -2
        r = pkg.Fd6Reductions()
        assert lib.fd6_reduce(h, ctypes.byref(r)) == -2
        buf = (ctypes.c_double * 512)()
        assert lib.fd6_get_fields(h, buf, buf, buf, buf) == -2
        assert lib.fd6_rhs(h, buf, buf, buf, buf) == -2
        assert lib.fd6_rk3_step(h, -1) == -1
        # parameter validation
        good = pkg.Fd6Params(1e-3, 1.0, 0.1, 0.1, 0.1, 0.01)
        for field, val in (("nu", -1.0), ("cs", float("nan")), ("dx", 0.0), ("dy", -0.1),
                           ("dz", float("inf")), ("dt", 0.0)):
            p = pkg.Fd6Params(*[getattr(good, n) for n in ("nu", "cs", "dx", "dy", "dz", "dt")])
            setattr(p, field, val)
            assert lib.fd6_set_params(h, ctypes.byref(p)) == -1, field
        assert lib.fd6_set_params(h, ctypes.byref(good)) == 0
        assert lib.fd6_rk3_step(h, 1) == -2  # fields still missing
        assert lib.fd6_init_fields(h, None, buf, buf, buf) == -1
        # tile selection
        n = lib.fd6_tile_count()
        assert n >= 2
        assert lib.fd6_set_tile(h, n) == -1
        assert lib.fd6_set_tile(h, -1) == -1
        assert lib.fd6_set_tile(h, 0) == 0
        assert lib.fd6_set_graph(h, 1) == 0 and lib.fd6_set_graph(h, 0) == 0
        # forcing validation (host only)
        F = pkg.Fd6Forcing
        good_f = F(1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.01, 0.5)
        assert lib.fd6_set_forcing(h, ctypes.byref(good_f)) == 0
        assert lib.fd6_set_forcing(h, None) == 0
        for bad in (F(0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.01, 0.5),      # k = 0
                    F(1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.01, 0.5),      # e parallel to k
                    F(1.0, 0.0, 0.0, 0.0, 2.0, 0.0, 0.01, 0.5),      # |e| != 1
                    F(1.0, 0.0, 0.0, 0.0, 1.0, 0.0, -0.01, 0.5),     # f0 < 0
                    F(1.0, float("nan"), 0.0, 0.0, 1.0, 0.0, 0.01, 0.5)):
            assert lib.fd6_set_forcing(h, ctypes.byref(bad)) == -1
        assert lib.fd6_set_forcing(None, ctypes.byref(good_f)) == -1
        assert lib.fd6_set_graph(None, 1) == -1
        assert lib.fd6_set_zchunk(h, -1) == -1
        assert lib.fd6_set_zchunk(h, 0) == 0 and lib.fd6_set_zchunk(h, 10 ** 6) == 0
        assert lib.fd6_last_error(h) == b""
    finally:
        assert lib.fd6_destroy(h) == 0
    assert lib.fd6_destroy(None) == 0
    assert lib.fd6_last_error(None) == b""


def test_batch_validation(pkg):
    lib = pkg.library()
    out = ctypes.c_size_t()
    arr = (pkg.Fd6Desc * 3)(desc(8, 8, 8), desc(16, 12, 10), desc(32, 32, 32))
    assert lib.fd6_batch_workspace_bytes(3, arr, ctypes.byref(out)) == 0
    single = ctypes.c_size_t()
    lib.fd6_workspace_bytes(ctypes.byref(desc(32, 32, 32)), ctypes.byref(single))
    assert out.value > 0
    assert lib.fd6_batch_workspace_bytes(0, arr, ctypes.byref(out)) == -1
    mixed = (pkg.Fd6Desc * 2)(desc(8, 8, 8, prec=0), desc(8, 8, 8, prec=1))
    assert lib.fd6_batch_workspace_bytes(2, mixed, ctypes.byref(out)) == -1
    v19 = (pkg.Fd6Desc * 1)(desc(8, 8, 8, var=1))
    assert lib.fd6_batch_workspace_bytes(1, v19, ctypes.byref(out)) == -6
    bad = (pkg.Fd6Desc * 1)(desc(5, 8, 8))
    assert lib.fd6_batch_workspace_bytes(1, bad, ctypes.byref(out)) == -1
    # state machine without a device: create only carves the pointer
    lib.fd6_batch_workspace_bytes(3, arr, ctypes.byref(out))
    h = ctypes.c_void_p()
    assert lib.fd6_batch_create(3, arr, ctypes.c_void_p(1 << 40), out.value - 1, None,
                                ctypes.byref(h)) == -3
    assert lib.fd6_batch_create(3, arr, ctypes.c_void_p(1 << 40), out.value, None,
                                ctypes.byref(h)) == 0
    try:
        assert lib.fd6_batch_step(h, 1) == -2
        assert lib.fd6_batch_set_schedule(h, 0, 0) == -1
        assert lib.fd6_batch_set_schedule(h, 1, -3) == -1  # -1, -2: balanced, packed
        buf = (ctypes.c_double * 8)()
        assert lib.fd6_batch_init_fields(h, 3, buf, buf, buf, buf) == -1
        assert lib.fd6_batch_get_fields(h, 0, buf, buf, buf, buf) == -2
    finally:
        assert lib.fd6_batch_destroy(h) == 0


def test_batch_tuner_argument_checks(pkg):
    lib = pkg.library()
    t, z = ctypes.c_int32(), ctypes.c_int32()
    assert lib.fd6_batch_tune(None, None) == -1
    assert lib.fd6_batch_tune(None, b"/nonexistent/cache") == -1
    assert lib.fd6_batch_get_schedule(None, ctypes.byref(t), ctypes.byref(z)) == -1


def test_box_tuner_argument_checks(pkg):
    lib = pkg.library()
    t, z = ctypes.c_int32(), ctypes.c_int32()
    assert lib.fd6_tune(None, None) == -1
    assert lib.fd6_get_schedule(None, ctypes.byref(t), ctypes.byref(z)) == -1
    # the tuning log: argument checks, and empty before any tuning
    d = desc(nx=8, ny=8, nz=8, prec=1)
    need = ctypes.c_size_t()
    lib.fd6_workspace_bytes(ctypes.byref(d), ctypes.byref(need))
    h = ctypes.c_void_p()
    assert lib.fd6_create(ctypes.byref(d), ctypes.c_void_p(1 << 40), need.value, None,
                          ctypes.byref(h)) == 0
    try:
        n = ctypes.c_int32(-1)
        assert lib.fd6_get_tune_log(h, None, None, None, 0, ctypes.byref(n)) == 0 and n.value == 0
        assert lib.fd6_get_tune_log(h, None, None, None, 0, None) == -1
        assert lib.fd6_get_tune_log(h, None, None, None, -1, ctypes.byref(n)) == -1
        assert lib.fd6_get_tune_log(h, None, None, None, 4, ctypes.byref(n)) == -1
        assert lib.fd6_get_tune_log(None, None, None, None, 0, ctypes.byref(n)) == -1
    finally:
        lib.fd6_destroy(h)


def test_batch_schedule_rejects_short_chunks_before_any_device_call(pkg):
    """Chunks of 1-7 planes are refused up front (FD6_EINVAL), so the check
    needs no device."""
    lib = pkg.library()
    arr = (pkg.Fd6Desc * 2)(desc(8, 8, 8), desc(16, 12, 10))
    out = ctypes.c_size_t()
    assert lib.fd6_batch_workspace_bytes(2, arr, ctypes.byref(out)) == 0
    h = ctypes.c_void_p()
    assert lib.fd6_batch_create(2, arr, ctypes.c_void_p(1 << 40), out.value, None,
                                ctypes.byref(h)) == 0
    try:
        for zc in range(1, 8):
            assert lib.fd6_batch_set_schedule(h, 6, zc) == -1, zc
        t, z = ctypes.c_int32(), ctypes.c_int32()
        assert lib.fd6_batch_get_schedule(h, ctypes.byref(t), ctypes.byref(z)) == 0
        assert (t.value, z.value) == (8, 64)  # the default stays in force
    finally:
        lib.fd6_batch_destroy(h)


def test_reduce_fields_static_validation(pkg):
    """The no-allocation diagnostics entry point rejects bad arguments before
    touching the device."""
    lib = pkg.library()
    P = ctypes.c_void_p
    f = [P(256 * (i + 1)) for i in range(4)]  # never dereferenced on these paths
    out = P(4096)
    ok = (8, 8, 8, 1, *f, 0.1, 0.1, 0.1, None, out)
    names = ["nx", "ny", "nz", "prec", "f0", "f1", "f2", "f3", "dx", "dy", "dz", "st", "out"]

    def call(**over):
        a = list(ok)
        for k, v in over.items():
            a[names.index(k)] = v
        return lib.fd6_reduce_fields_static(*a)

    for bad in ({"nx": 0}, {"ny": -1}, {"nz": 4097}, {"prec": 3}, {"prec": -1},
                {"f0": None}, {"f3": None}, {"out": None}, {"dx": 0.0}, {"dy": -1.0},
                {"dz": float("nan")}, {"dx": float("inf")}):
        assert call(**bad) == -1, bad


def test_binding_constants_match_the_header(pkg):
    """Status codes, precisions, methods, layout flag and the special schedule
    values of the binding equal the header's definitions."""
    src = open(HEADER).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(
        r"#define\s+(FD6_\w+)\s+\(?(-?\d+)\)?", src)}
    enums = {m.group(1): int(m.group(2)) for m in re.finditer(
        r"\b(FD6_[A-Z0-9_]+)\s*=\s*(-?\d+)", src)}
    both = {**enums, **defs}
    assert pkg.BATCH_BALANCED == both["FD6_BATCH_BALANCED"]
    assert pkg.BATCH_PACKED == both["FD6_BATCH_PACKED"]
    for code, name in pkg.STATUS.items():
        assert both[name] == code, name
    assert pkg.LAYOUTS["aos"] == both["FD6_LAYOUT_AOS"]
    assert pkg.PRECISIONS == {"fp64": both["FD6_FP64"], "fp32": both["FD6_FP32"],
                              "fp32_acc64": both["FD6_FP32_ACC64"]}
    assert pkg.VARIANTS == {"55p": both["FD6_55P"], "19p": both["FD6_19P"]}
