"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/pic.h declares, and rejects bad arguments before any
launch with the documented status."""
import ctypes as C
import os
import re

import pytest

from paper_2101_12149_amd import _lib
from paper_2101_12149_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pic.h")).read()
    return re.findall(r"PIC_API\s+[\w\s\*]+?\b(pic_\w+)\s*\(", text)


def test_header_declares_the_entry_points():
    names = set(_declared())
    for n in ("pic_sort_tiles", "pic_gather", "pic_push", "pic_deposit", "pic_yee", "pic_step",
              "pic_step_adjoint", "pic_reduce", "pic_workspace_bytes", "pic_last_error", "pic_tile_count"):
        assert n in names
    assert names == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for n in _declared():
        assert hasattr(lib, n), n


def _grid(**kw):
    g = wl.plasma_grid((16, 16, 16), 3)
    for k, v in kw.items():
        setattr(g, k, v)
    return g


def test_workspace_bytes_grows_with_particles_and_rejects_bad_grids():
    g = _grid()
    a = _lib.pic_workspace_bytes(g, "f64", 0)
    b = _lib.pic_workspace_bytes(g, "f64", 1000)
    c = _lib.pic_workspace_bytes(g, "f32", 1000)
    assert a > 0 and b > a and c < b
    assert _lib.pic_workspace_bytes(_grid(order=2), "f64", 10) == 0
    assert _lib.pic_workspace_bytes(_grid(n=(3, 16, 16)), "f64", 10) == 0
    assert _lib.pic_tile_count(_grid(tile=(8, 8, 8)), "f64") in (8, 16, 32, 64)


def test_tile_shape_resolves_the_automatic_choices():
    """The automatic tile is the largest divisor of n not above 8 with one
    cell of slack; while the LDS regions do not fit, the largest tile edge
    halves before the slack is dropped; on a grid of fewer than 512 tiles an
    automatic edge of 8 or more halves (largest first) until there are 512
    or none is left to halve; a fixed tile that cannot hold the
    slack keeps the tile and drops the slack."""
    big = wl.plasma_grid((256, 256, 256), 3)
    assert _lib.pic_tile_shape(big, "f32") == ((8, 8, 8), 1)
    assert _lib.pic_tile_shape(big, "f64") == ((8, 8, 4), 1)
    assert _lib.pic_tile_shape(wl.plasma_grid((12, 16, 20), 3), "f32") == ((6, 4, 5), 1)
    assert _lib.pic_tile_shape(wl.plasma_grid((32, 32, 32), 1), "f64") == ((4, 4, 4), 1)
    assert _lib.pic_tile_shape(wl.plasma_grid((64, 64, 64), 3), "f64") == ((8, 8, 4), 1)
    assert _lib.pic_tile_shape(wl.plasma_grid((16, 16, 16), 3), "f32") == ((4, 4, 4), 1)
    fixed = wl.plasma_grid((16, 16, 16), 3)
    fixed.tile = (8, 8, 8)
    assert _lib.pic_tile_shape(fixed, "f64") == ((8, 8, 8), 0)
    for g, dt in ((big, "f32"), (big, "f64"), (fixed, "f64")):
        t, _ = _lib.pic_tile_shape(g, dt)
        assert _lib.pic_tile_count(g, dt) == (g.n[0] // t[0]) * (g.n[1] // t[1]) * (g.n[2] // t[2])
    with pytest.raises(_lib.PicError):
        _lib.pic_tile_shape(_grid(order=2), "f64")


def _raw_call_step(grid, dtype="f64"):
    lib = _lib.load()
    g = _lib.make_grid(grid, dtype)
    sp = _lib.pic_species()
    sp.n = 0
    sp.m, sp.q = 1.0, -1.0
    f = _lib.pic_fields()
    for m in range(3):
        f.E[m] = f.B[m] = f.J[m] = 0x1000      # never dereferenced: validation fails first
    src = _lib.pic_source()
    src.k_plane = -1
    st = lib.pic_step(C.byref(g), C.byref(sp), C.byref(f), C.byref(src), 0, 1, 0, None, None, 0, None, None)
    return st, lib.pic_last_error().decode()


def test_noalloc_step_refuses_sizes_beyond_its_static_scratch():
    """pic_step_noalloc checks the scratch its grid and particle count need
    against the static array before anything is launched: a 256^3 grid (its
    per-cell buffers alone exceed 128 MiB) is refused with PIC_E_WORKSPACE."""
    lib = _lib.load()
    big = wl.plasma_grid((256, 256, 256), 3)
    assert _lib.pic_workspace_bytes(big, "f32", 0) > _lib.NOALLOC_SCRATCH_BYTES
    assert _lib.pic_workspace_bytes(wl.plasma_grid((64, 64, 64), 3), "f64", 64 ** 3 * 4) \
        <= _lib.NOALLOC_SCRATCH_BYTES
    g = _lib.make_grid(big, "f32")
    sp = _lib.pic_species()
    sp.n = 0
    sp.m, sp.q = 1.0, -1.0
    f = _lib.pic_fields()
    for m in range(3):
        f.E[m] = f.B[m] = f.J[m] = 0x1000      # never dereferenced: the size check fails first
    st = lib.pic_step_noalloc(C.byref(g), C.byref(sp), C.byref(f), None, 0, 1, 0, None, None, None)
    assert st == 4 and "scratch" in lib.pic_last_error().decode()


def test_cfl_violation_is_rejected():
    g = _grid()
    g.dt = g.d[0] / (3 ** 0.5) * 1.01
    st, msg = _raw_call_step(g)
    assert st == 2 and "CFL" in msg


def test_unsupported_order_and_dtype():
    st, _ = _raw_call_step(_grid(order=2))
    assert st == 3
    lib = _lib.load()
    g = _lib.make_grid(_grid(), "f64")
    g.dtype = 7
    assert lib.pic_workspace_bytes(C.byref(g), 10) == 0


def test_missing_workspace_and_null_pointers():
    st, msg = _raw_call_step(_grid())
    assert st == 4 and "workspace" in msg
    lib = _lib.load()
    g = _lib.make_grid(_grid(), "f64")
    assert lib.pic_step(C.byref(g), None, None, None, 0, 1, 0, None, None, 0, None, None) == 1
    sp = _lib.pic_species()
    sp.n = 5
    sp.m = 1.0
    assert lib.pic_gather(C.byref(g), C.byref(sp), None, (C.c_void_p * 3)(), (C.c_void_p * 3)(), None) == 1
    assert "NULL" in lib.pic_last_error().decode()


def test_bad_tile_and_negative_steps():
    st, msg = _raw_call_step(_grid(tile=(5, 8, 8)))
    assert st == 1 and "tile" in msg
    lib = _lib.load()
    g = _lib.make_grid(_grid(), "f64")
    sp = _lib.pic_species()
    sp.m = 1.0
    f = _lib.pic_fields()
    for m in range(3):
        f.E[m] = f.B[m] = f.J[m] = 0x1000
    assert lib.pic_step(C.byref(g), C.byref(sp), C.byref(f), None, 0, -1, 0, None, None, 0, None, None) == 1
    assert lib.pic_step(C.byref(g), C.byref(sp), C.byref(f), None, 0, 1, 4, None, None, 0, None, None) == 1


def test_solver_and_pusher_are_validated_with_each_solvers_cfl_limit():
    """Yee is stable up to c dt = 1/sqrt(sum 1/d^2), CKC up to c dt = min d:
    a step between the two is refused for Yee and accepted for CKC; unknown
    solver or pusher codes are unsupported."""
    import dataclasses
    g = wl.Grid((16, 16, 16), (0.2, 0.25, 0.3), 0.19)
    with pytest.raises(_lib.PicError) as e:
        _lib.pic_tile_shape(g, "f64")
    assert e.value.status == 2
    assert _lib.pic_tile_count(dataclasses.replace(g, solver=1), "f64") > 0
    with pytest.raises(_lib.PicError) as e:
        _lib.pic_tile_shape(dataclasses.replace(g, solver=1, dt=0.203), "f64")
    assert e.value.status == 2
    for bad in (dict(solver=2), dict(pusher=-1)):
        with pytest.raises(_lib.PicError) as e:
            _lib.pic_tile_shape(dataclasses.replace(g, dt=0.05, **bad), "f64")
        assert e.value.status == 3


def test_gather_filter_takes_twelve_field_arrays_of_workspace():
    """Filtered E, B and their adjoints: six field arrays each; non-finite
    taps are refused."""
    import dataclasses
    import numpy as np
    g = wl.plasma_grid((16, 16, 16), 3)
    taps = np.tile([0.5, 0.25, 0.0, 0.0], (6, 1))
    plain = _lib.pic_workspace_bytes(g, "f64", 1000)
    filt = _lib.pic_workspace_bytes(dataclasses.replace(g, gather_filter=taps), "f64", 1000)
    assert filt - plain == 12 * 16 ** 3 * 8
    bad = taps.copy()
    bad[2, 1] = np.nan
    with pytest.raises(_lib.PicError) as e:
        _lib.pic_tile_shape(dataclasses.replace(g, gather_filter=bad), "f64")
    assert e.value.status == 1


def test_atomic_probe_library_loads():
    """The throughput probe that bench.py --atomic-micro runs is built beside
    the library and exports its two entry points (nothing is launched here)."""
    lib = C.CDLL(os.path.join(ROOT, "paper_2101_12149_amd", "libpic355_micro.so"))
    assert lib.picmb_num_modes() == 10
    assert hasattr(lib, "picmb_run")
    ms, ops = C.c_double(), C.c_double()
    assert lib.picmb_run(99, 1, 1, 1, 1, C.byref(ms), C.byref(ops)) == -1   # bad mode: refused before any call
