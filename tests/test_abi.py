"""Host-side checks of the C ABI (no device work): the library loads, exports
every entry point include/eik.h declares, sizes workspaces and rejects invalid
arguments before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eik.h")

eik = pytest.importorskip("paper_2106_15869_amd")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eik_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(eik.LIB_PATH):
        pytest.fail("libeik.so is not built (python -m paper_2106_15869_amd.build)")
    return eik.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert set(names) == set(eik.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version_and_status_strings(lib):
    header = int(re.search(r"#define EIK_ABI_VERSION (\d+)", open(HEADER).read()).group(1))
    assert eik.eik_abi_version() == header == eik.EIK_ABI_VERSION
    assert eik.eik_status_string(0) == "EIK_OK"
    assert eik.eik_status_string(2) == "EIK_ERR_NO_CONVERGENCE"
    assert eik.eik_status_string(99) == "EIK_UNKNOWN_STATUS"


def test_default_options(lib):
    o = eik.EikOptions()
    lib.eik_default_options(ctypes.byref(o))
    assert o.dtype == eik.EIK_FLOAT32 and o.variant == eik.EIK_VARIANT_TILE
    assert o.flags == 0 and o.max_iters == 0 and not o.workspace
    assert o.order_min == 0 and o.workgroups == 0


def test_options_struct_layout():
    # mirrors eik_options in include/eik.h on LP64
    assert ctypes.sizeof(eik.EikOptions) == 112
    assert eik.EikOptions.order_min.offset == 104 and eik.EikOptions.workgroups.offset == 108
    assert ctypes.sizeof(eik.EikTuneEntry) == 32
    assert eik.EikOptions.max_iters.offset == 24
    assert eik.EikOptions.stats.offset == 72
    assert ctypes.sizeof(eik.EikStats) == 128 + 80
    assert eik.EikStats.evals_early.offset == 120


def test_struct_layout_matches_c_compiler(tmp_path):
    """Offsets and sizes of the ctypes mirrors equal what a C compiler makes
    of include/eik.h."""
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "eik.h"\n'
        'int main(void) { printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(eik_options),'
        ' sizeof(eik_stats), offsetof(eik_options, max_iters), offsetof(eik_options, stats),'
        ' offsetof(eik_stats, evals_check), offsetof(eik_stats, evals_early),'
        ' offsetof(eik_stats, kernel_launches), offsetof(eik_stats, kernel_ms),'
        ' offsetof(eik_options, spacing), offsetof(eik_options, order_min), offsetof(eik_options, workgroups),'
        ' sizeof(eik_tune_entry), offsetof(eik_tune_entry, order_min), offsetof(eik_tune_entry, workgroups));'
        ' return 0; }\n')
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(eik.EikOptions), ctypes.sizeof(eik.EikStats), eik.EikOptions.max_iters.offset,
            eik.EikOptions.stats.offset, eik.EikStats.evals_check.offset, eik.EikStats.evals_early.offset,
            eik.EikStats.kernel_launches.offset,
            eik.EikStats.kernel_ms.offset, eik.EikOptions.spacing.offset, eik.EikOptions.order_min.offset,
            eik.EikOptions.workgroups.offset, ctypes.sizeof(eik.EikTuneEntry), eik.EikTuneEntry.order_min.offset,
            eik.EikTuneEntry.workgroups.offset]
    assert got == want


def test_workspace_size(lib):
    o = eik.make_options(eik.EIK_FLOAT32, "node")
    n = 64 * 64
    ws = eik.eik_workspace_size((64, 64), o)
    assert ws >= 13 * n  # labels + stamps + two lists
    od = eik.make_options(eik.EIK_FLOAT64, "node", deterministic=True)
    assert eik.eik_workspace_size((64, 64), od) >= ws + 8 * n
    assert eik.eik_workspace_size((7, 9, 5), eik.make_options(eik.EIK_FLOAT32, "tile")) > 0
    # FIM keeps a third (converged) list
    assert eik.eik_workspace_size((64, 64), eik.make_options(eik.EIK_FLOAT32, "fim")) >= ws + 4 * 7 * n
    # invalid shapes give 0
    assert eik.eik_workspace_size((0, 5), o) == 0
    assert eik.eik_workspace_size((5,), o) == 0
    assert eik.eik_workspace_size((2, 2, 2, 2), o) == 0
    assert eik.eik_workspace_size((1 << 16, 1 << 16), o) == 0


def _solve_raw(lib, dims, h=1.0, sources=(0,), eps=0.0, opt=None, F=0x1000, phi=0x2000):
    d = np.asarray(dims, dtype=np.int64)
    s = np.asarray(sources, dtype=np.int64)
    return lib.eik_solve(F, len(d), d.ctypes.data, h, s.ctypes.data if s.size else None, len(s),
                         eps, phi, ctypes.byref(opt) if opt is not None else None)


@pytest.mark.parametrize("kwargs,why", [
    (dict(dims=(4,)), "ndim"),
    (dict(dims=(4, 0)), "dim"),
    (dict(dims=(4, 4), h=0.0), "h"),
    (dict(dims=(4, 4), h=float("nan")), "h"),
    (dict(dims=(4, 4), h=float("inf")), "h"),
    (dict(dims=(4, 4), eps=-1.0), "eps"),
    (dict(dims=(4, 4), sources=()), "source"),
    (dict(dims=(4, 4), sources=(16,)), "range"),
    (dict(dims=(4, 4), sources=(-1,)), "range"),
    (dict(dims=(4, 4), F=None), "NULL"),
    (dict(dims=(4, 4), phi=None), "NULL"),
    (dict(dims=(4, 4), phi=0x1000), "alias"),
])
def test_invalid_arguments_rejected_before_device_work(lib, kwargs, why):
    rc = _solve_raw(lib, **kwargs)
    assert rc == eik.EIK_ERR_INVALID_ARGUMENT
    assert why.lower() in lib.eik_last_error().decode().lower()


def test_invalid_options_rejected(lib):
    o = eik.make_options(eik.EIK_FLOAT32, "tile", deterministic=True)
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT
    o = eik.make_options(eik.EIK_FLOAT32, "node")
    o.dtype = 7
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT
    o = eik.make_options(eik.EIK_FLOAT32, "node", async_=True)  # no workspace
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT
    o = eik.make_options(eik.EIK_FLOAT32, "node")
    o.workspace = 0x1001  # misaligned
    o.workspace_bytes = 1 << 20
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT
    o = eik.make_options(eik.EIK_FLOAT32, "node")
    o.workspace = 0x100000
    o.workspace_bytes = 16  # too small
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_OUT_OF_MEMORY
    o = eik.make_options(eik.EIK_FLOAT32, "node")
    o.flags = 64
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT
    o = eik.make_options(eik.EIK_FLOAT32, "node", profile=True, async_=True)
    o.workspace = 0x100000
    o.workspace_bytes = 1 << 30
    o.max_iters = 10
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT  # profile needs a sync
    o = eik.make_options(eik.EIK_FLOAT32, "fim", skip_remedy=True)
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT  # FIM has no remedy
    assert "remedy" in lib.eik_last_error().decode()
    o = eik.make_options(eik.EIK_FLOAT32, "fim", deterministic=True)
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT
    o = eik.make_options(eik.EIK_FLOAT32, "node", fifo=True)
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT  # a tile-schedule choice
    o = eik.make_options(eik.EIK_FLOAT32, "node")
    o.variant = 3
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT


def test_bad_source_values_rejected(lib):
    o = eik.make_options(eik.EIK_FLOAT32, "node")
    vals = np.array([np.nan])
    o.source_values = vals.ctypes.data
    assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT


def test_apply_local_and_adjoint_validation(lib):
    d = np.asarray((4, 4), dtype=np.int64)
    assert lib.eik_apply_local(0x1000, 0x2000, 2, d.ctypes.data, 1.0, 0x2000, None) == \
        eik.EIK_ERR_INVALID_ARGUMENT
    assert lib.eik_apply_local(0x1000, 0x2000, 2, d.ctypes.data, -1.0, 0x3000, None) == \
        eik.EIK_ERR_INVALID_ARGUMENT
    s = np.asarray([99], dtype=np.int64)
    assert lib.eik_adjoint(0x1000, 0x2000, 2, d.ctypes.data, 1.0, s.ctypes.data, 1, 0x3000, 0x4000,
                           None) == eik.EIK_ERR_INVALID_ARGUMENT


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        eik.solve(torch.ones(4, 4), 1.0, [0])


def _inst(shapes, h=1.0, nsrc=1):
    arr = (eik.EikInstance * len(shapes))()
    for k, sh in enumerate(shapes):
        for j, v in enumerate(sh):
            arr[k].dims[j] = v
        arr[k].h = h
        arr[k].n_sources = nsrc
    return arr


def test_batch_workspace_size(lib):
    o = eik.make_options(eik.EIK_FLOAT32, "tile")
    one = lib.eik_batch_workspace_size(2, _inst([(64, 64)]), 1, ctypes.byref(o))
    assert one == eik.eik_workspace_size((64, 64), o)
    many = lib.eik_batch_workspace_size(2, _inst([(64, 64), (30, 70), (1, 9)]), 3, ctypes.byref(o))
    assert many > one
    assert lib.eik_batch_workspace_size(2, _inst([(64, 0)]), 1, ctypes.byref(o)) == 0
    assert lib.eik_batch_workspace_size(4, _inst([(4, 4)]), 1, ctypes.byref(o)) == 0
    assert lib.eik_adjoint_batch_workspace_size(3, _inst([(8, 9, 10), (3, 3, 3)]), 2, ctypes.byref(o)) > 0
    node = eik.make_options(eik.EIK_FLOAT32, "node")
    assert lib.eik_batch_workspace_size(2, _inst([(8, 8)]), 1, ctypes.byref(node)) == 0


@pytest.mark.parametrize("case,why", [
    ("no_instances", "instance"),
    ("bad_dim", "dim"),
    ("bad_h", "h"),
    ("no_source", "source"),
    ("source_range", "range"),
    ("null_sources", "null"),
])
def test_batch_invalid_arguments(lib, case, why):
    shapes = [(8, 8), (5, 7)]
    inst = _inst(shapes)
    src = np.array([0, 34], dtype=np.int64)
    n = len(shapes)
    if case == "no_instances":
        n = 0
    elif case == "bad_dim":
        inst[1].dims[0] = 0
    elif case == "bad_h":
        inst[0].h = float("nan")
    elif case == "no_source":
        inst[1].n_sources = 0
    elif case == "source_range":
        src[1] = 35  # 5 x 7 grid has 35 nodes
    o = eik.make_options(eik.EIK_FLOAT32, "tile")
    sp = None if case == "null_sources" else src.ctypes.data
    rc = lib.eik_solve_batch(0x1000, 2, inst, n, sp, 0.0, 0x2000, ctypes.byref(o))
    assert rc == eik.EIK_ERR_INVALID_ARGUMENT
    assert why in lib.eik_last_error().decode().lower()


def test_batch_needs_tile_variant(lib):
    o = eik.make_options(eik.EIK_FLOAT32, "node")
    src = np.array([0], dtype=np.int64)
    rc = lib.eik_solve_batch(0x1000, 2, _inst([(8, 8)]), 1, src.ctypes.data, 0.0, 0x2000, ctypes.byref(o))
    assert rc == eik.EIK_ERR_UNSUPPORTED


def test_tune_validation(lib):
    d = np.asarray((16, 16), dtype=np.int64)
    s = np.asarray([0], dtype=np.int64)
    n = ctypes.c_int32(-1)
    assert lib.eik_tune(0x1000, 2, d.ctypes.data, 1.0, s.ctypes.data, 1, 0.0, 0x2000, None, None, 0,
                        ctypes.byref(n)) == eik.EIK_ERR_INVALID_ARGUMENT
    assert n.value == 0
    o = eik.make_options(eik.EIK_FLOAT32, "tile", async_=True)
    assert lib.eik_tune(0x1000, 2, d.ctypes.data, 1.0, s.ctypes.data, 1, 0.0, 0x2000, ctypes.byref(o), None, 0,
                        None) == eik.EIK_ERR_INVALID_ARGUMENT
    o = eik.make_options(eik.EIK_FLOAT32, "tile")
    assert lib.eik_tune(0x1000, 2, d.ctypes.data, 1.0, s.ctypes.data, 1, 0.0, None, ctypes.byref(o), None, 0,
                        None) == eik.EIK_ERR_INVALID_ARGUMENT
    # the solve's own checks run before the cache is consulted or any device
    # work: a source out of range, phi aliasing F, a bad h or eps
    bad = np.asarray([256], dtype=np.int64)
    for args, why in [((0x1000, bad, 1.0, 0.0, 0x2000), "range"), ((0x1000, s, 1.0, 0.0, 0x1000), "alias"),
                      ((0x1000, s, -1.0, 0.0, 0x2000), "h must"), ((0x1000, s, 1.0, -1.0, 0x2000), "eps")]:
        F, src, h, eps, scratch = args
        assert lib.eik_tune(F, 2, d.ctypes.data, h, src.ctypes.data, 1, eps, scratch, ctypes.byref(o), None, 0,
                            None) == eik.EIK_ERR_INVALID_ARGUMENT, why
        assert why in lib.eik_last_error().decode()


@pytest.mark.parametrize("sp,ok", [((0.5, 2.0, 0.0), True), ((0.5, -1.0, 0.0), False), ((0.5, 0.0, 0.0), False),
                                   ((0.5, 1.0, 3.0), False), ((float("inf"), 1.0, 0.0), False)])
def test_spacing_validation(lib, sp, ok):
    """2D problems take two positive spacings (dims order) and a zero third;
    an invalid combination is rejected before any device work."""
    o = eik.make_options(eik.EIK_FLOAT32, "node", spacing=sp)
    # a too-small workspace stops a valid call right after validation, before
    # any device work
    o.workspace = 0x100000
    o.workspace_bytes = 16
    rc = _solve_raw(lib, (4, 4), opt=o)
    if ok:
        assert rc == eik.EIK_ERR_OUT_OF_MEMORY
    else:
        assert rc == eik.EIK_ERR_INVALID_ARGUMENT and "spacing" in lib.eik_last_error().decode()


def test_spacing_rejected_for_batches(lib):
    o = eik.make_options(eik.EIK_FLOAT32, "tile", spacing=(1.0, 2.0))
    src = np.array([0], dtype=np.int64)
    rc = lib.eik_solve_batch(0x1000, 2, _inst([(8, 8)]), 1, src.ctypes.data, 0.0, 0x2000, ctypes.byref(o))
    assert rc == eik.EIK_ERR_UNSUPPORTED


def test_async_status_rejects_bad_workspace(lib):
    """eik_async_status validates its workspace pointer on the host, before
    any device call."""
    assert lib.eik_async_status(None, None) == eik.EIK_ERR_INVALID_ARGUMENT
    assert b"NULL" in lib.eik_last_error()
    assert lib.eik_async_status(0x1010, None) == eik.EIK_ERR_INVALID_ARGUMENT
    assert b"aligned" in lib.eik_last_error()


def _noalloc_raw(lib, dims, opt=None, F=0x1000, phi=0x2000, sources=(0,)):
    d = np.asarray(dims, dtype=np.int64)
    s = np.asarray(sources, dtype=np.int64)
    return lib.eik_solve_noalloc(F, len(d), d.ctypes.data, 1.0, s.ctypes.data, len(s), 0.0, phi,
                                 ctypes.byref(opt) if opt is not None else None)


def test_noalloc_rejects_before_device_work(lib):
    """eik_solve_noalloc answers these on the host: a problem whose workspace
    exceeds the 128 MiB static scratch, a caller workspace, asynchronous or
    profiled calls, and eik_solve's own argument checks."""
    big = (512, 512, 512)
    o = eik.make_options(eik.EIK_FLOAT32, "tile")
    assert eik.eik_workspace_size(big, o) > 128 << 20
    assert _noalloc_raw(lib, big, o) == eik.EIK_ERR_OUT_OF_MEMORY
    assert b"static scratch" in lib.eik_last_error()
    node = eik.make_options(eik.EIK_FLOAT32, "node")
    assert eik.eik_workspace_size((2048, 2048), node) > 128 << 20
    assert _noalloc_raw(lib, (2048, 2048), node) == eik.EIK_ERR_OUT_OF_MEMORY
    ws = eik.make_options(eik.EIK_FLOAT32, "tile")
    ws.workspace = 0x10000
    ws.workspace_bytes = 1 << 20
    assert _noalloc_raw(lib, (8, 8), ws) == eik.EIK_ERR_INVALID_ARGUMENT
    assert b"workspace must be NULL" in lib.eik_last_error()
    a = eik.make_options(eik.EIK_FLOAT32, "tile", async_=True, max_iters=10)
    assert _noalloc_raw(lib, (8, 8), a) == eik.EIK_ERR_UNSUPPORTED
    p = eik.make_options(eik.EIK_FLOAT32, "tile", profile=True)
    assert _noalloc_raw(lib, (8, 8), p) == eik.EIK_ERR_UNSUPPORTED
    assert _noalloc_raw(lib, (8, 8), sources=(64,)) == eik.EIK_ERR_INVALID_ARGUMENT
    assert _noalloc_raw(lib, (8, 8), phi=0x1000) == eik.EIK_ERR_INVALID_ARGUMENT
    assert _noalloc_raw(lib, (8, 8), F=None) == eik.EIK_ERR_INVALID_ARGUMENT
    bad = eik.make_options(eik.EIK_FLOAT32, "tile")
    bad.flags = 1 << 31
    assert _noalloc_raw(lib, (8, 8), bad) == eik.EIK_ERR_INVALID_ARGUMENT


@pytest.mark.parametrize("field,value,ok", [
    ("order_min", -1, False), ("order_min", 1, True), ("order_min", 4096, True),
    ("workgroups", -8, False), ("workgroups", 12, False), ("workgroups", 2056, False),
    ("workgroups", 8, True), ("workgroups", 1536, True), ("workgroups", 2048, True),
])
def test_schedule_options_validated(lib, field, value, ok):
    """order_min >= 0; workgroups 0 or a multiple of 8 up to 2048 (host checks,
    before device work: the valid ones are seen through the size query)."""
    o = eik.make_options(eik.EIK_FLOAT32, "tile", **{field: value})
    if ok:
        assert eik.eik_workspace_size((16, 16), o) > 0
    else:
        assert _solve_raw(lib, (4, 4), opt=o) == eik.EIK_ERR_INVALID_ARGUMENT
        assert field.split("_")[0] in lib.eik_last_error().decode()
