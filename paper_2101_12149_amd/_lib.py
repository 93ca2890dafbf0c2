"""ctypes binding of libpic355.so (include/pic.h).

Argument marshalling only: every function here forwards to the C entry point
of the same name; all arithmetic runs in the HIP kernels.  Tensors must be
contiguous CUDA (HIP) tensors of the grid dtype; the stream is torch's
current stream.  If the library has not been built, loading raises.
"""
import ctypes as C
import os
import threading

import numpy as np

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic355.so")

PIC_F32, PIC_F64 = 0, 1
STATUS = {0: "PIC_OK", 1: "PIC_E_INVALID", 2: "PIC_E_CFL", 3: "PIC_E_UNSUPPORTED", 4: "PIC_E_WORKSPACE",
          5: "PIC_E_STATE", 6: "PIC_E_DEVICE"}


class PicError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class pic_grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("d", C.c_double * 3), ("dt", C.c_double), ("c", C.c_double),
                ("eps0", C.c_double), ("order", C.c_int32), ("dtype", C.c_int32), ("tile", C.c_int32 * 3),
                ("slack", C.c_int32), ("pusher", C.c_int32), ("solver", C.c_int32),
                ("gather_filter", C.c_void_p)]


class pic_species(C.Structure):
    _fields_ = [("n", C.c_int64), ("cell", C.c_void_p * 3), ("off", C.c_void_p * 3), ("u", C.c_void_p * 3),
                ("w", C.c_void_p), ("w0", C.c_double), ("q", C.c_double), ("m", C.c_double)]


class pic_fields(C.Structure):
    _fields_ = [("E", C.c_void_p * 3), ("B", C.c_void_p * 3), ("J", C.c_void_p * 3)]


class pic_source(C.Structure):
    _fields_ = [("k_plane", C.c_int32), ("amp", C.c_void_p), ("g", C.c_void_p), ("n_g", C.c_int64)]


class pic_adjoint(C.Structure):
    _fields_ = [("lx", C.c_void_p * 3), ("lu", C.c_void_p * 3), ("lE", C.c_void_p * 3), ("lB", C.c_void_p * 3)]


EXPORTS = ("pic_workspace_bytes", "pic_tile_count", "pic_tile_shape", "pic_sort_tiles", "pic_gather", "pic_push",
           "pic_deposit", "pic_yee", "pic_step", "pic_step_noalloc", "pic_step_adjoint", "pic_reduce",
           "pic_gauss_residual", "pic_energy_loss", "pic_timing", "pic_last_error")
TIMING_CATEGORIES = ("sort", "particles", "yee", "reduce", "adjoint_fields", "adjoint_particles", "strays")

_lock = threading.Lock()
_lib = None


def load():
    """Load libpic355.so (raises if it is missing: there is no fallback)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                                   "(python paper_2101_12149_amd/build.py)")
            lib = C.CDLL(LIB_PATH)
            P = C.POINTER
            V3 = C.c_void_p * 3
            lib.pic_workspace_bytes.restype = C.c_size_t
            lib.pic_workspace_bytes.argtypes = [P(pic_grid), C.c_int64]
            lib.pic_tile_count.restype = C.c_int64
            lib.pic_tile_count.argtypes = [P(pic_grid)]
            lib.pic_tile_shape.restype = C.c_int
            lib.pic_tile_shape.argtypes = [P(pic_grid), C.c_void_p, C.c_void_p]
            lib.pic_sort_tiles.restype = C.c_int
            lib.pic_sort_tiles.argtypes = [P(pic_grid), P(pic_species), C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_size_t, C.c_void_p]
            lib.pic_gather.restype = C.c_int
            lib.pic_gather.argtypes = [P(pic_grid), P(pic_species), P(pic_fields), V3, V3, C.c_void_p]
            lib.pic_push.restype = C.c_int
            lib.pic_push.argtypes = [P(pic_grid), P(pic_species), V3, V3, C.c_void_p]
            lib.pic_deposit.restype = C.c_int
            lib.pic_deposit.argtypes = [P(pic_grid), P(pic_species), P(pic_species), P(pic_fields), C.c_void_p]
            lib.pic_yee.restype = C.c_int
            lib.pic_yee.argtypes = [P(pic_grid), P(pic_fields), P(pic_source), C.c_int64, C.c_void_p]
            lib.pic_step.restype = C.c_int
            lib.pic_step.argtypes = [P(pic_grid), P(pic_species), P(pic_fields), P(pic_source), C.c_int64,
                                     C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                     C.c_void_p]
            lib.pic_step_noalloc.restype = C.c_int
            lib.pic_step_noalloc.argtypes = [P(pic_grid), P(pic_species), P(pic_fields), P(pic_source), C.c_int64,
                                             C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
            lib.pic_step_adjoint.restype = C.c_int
            lib.pic_step_adjoint.argtypes = [P(pic_grid), P(pic_species), P(pic_fields), C.c_void_p, P(pic_source),
                                             C.c_int64, P(pic_adjoint), C.c_void_p, C.c_void_p, C.c_size_t,
                                             C.c_void_p]
            lib.pic_reduce.restype = C.c_int
            lib.pic_reduce.argtypes = [P(pic_grid), P(pic_species), P(pic_fields), C.c_void_p, C.c_void_p,
                                       C.c_size_t, C.c_void_p]
            lib.pic_gauss_residual.restype = C.c_int
            lib.pic_gauss_residual.argtypes = [P(pic_grid), P(pic_species), P(pic_fields), C.c_void_p, C.c_void_p,
                                               C.c_size_t, C.c_void_p]
            lib.pic_energy_loss.restype = C.c_int
            lib.pic_energy_loss.argtypes = [P(pic_grid), P(pic_fields), C.c_int64, C.c_double, P(pic_adjoint),
                                            C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
            lib.pic_timing.restype = C.c_int
            lib.pic_timing.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_int]
            lib.pic_last_error.restype = C.c_char_p
            lib.pic_last_error.argtypes = []
            _lib = lib
    return _lib


# ---------------------------------------------------------------------------
# marshalling

def _dtype_code(dtype):
    if isinstance(dtype, int) and dtype in (PIC_F32, PIC_F64):
        return dtype
    if dtype in ("f64", torch.float64):
        return PIC_F64
    if dtype in ("f32", torch.float32):
        return PIC_F32
    raise ValueError(f"unsupported dtype {dtype}")


def _tdtype(code):
    return torch.float64 if code == PIC_F64 else torch.float32


def make_grid(grid, dtype):
    g = pic_grid()
    g.n[:] = [int(v) for v in grid.n]
    g.d[:] = [float(v) for v in grid.d]
    g.dt, g.c, g.eps0 = float(grid.dt), float(grid.c), float(grid.eps0)
    g.order = int(grid.order)
    g.dtype = _dtype_code(dtype)
    t = getattr(grid, "tile", (0, 0, 0)) or (0, 0, 0)
    g.tile[:] = [int(v) for v in t]
    g.slack = int(getattr(grid, "slack", -1))
    g.pusher = int(getattr(grid, "pusher", 0))
    g.solver = int(getattr(grid, "solver", 0))
    gf = getattr(grid, "gather_filter", None)
    if gf is not None:
        gf = np.ascontiguousarray(np.asarray(gf, dtype=np.float64).reshape(6, 4))
        g._filter = gf               # kept alive with the struct
        g.gather_filter = gf.ctypes.data
    return g


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


def make_species(sp, code):
    tdt = _tdtype(code)
    n = int(sp.cell.shape[1])
    s = pic_species()
    s.n = n
    for d in range(3):
        s.cell[d] = _ptr(sp.cell[d], torch.int32, "cell")
        s.off[d] = _ptr(sp.off[d], tdt, "off")
        s.u[d] = _ptr(sp.u[d], tdt, "u")
    s.w = _ptr(sp.w, tdt, "w") if sp.w is not None else None
    s.w0, s.q, s.m = float(sp.w0), float(sp.q), float(sp.m)
    return s


def make_fields(f, code, need_j=True):
    tdt = _tdtype(code)
    s = pic_fields()
    for m in range(3):
        s.E[m] = _ptr(f.E[m], tdt, "E")
        s.B[m] = _ptr(f.B[m], tdt, "B")
        s.J[m] = _ptr(f.J[m], tdt, "J") if (need_j or f.J is not None) else None
    return s


def make_source(src, code):
    s = pic_source()
    if src is None or src.k_plane < 0:
        s.k_plane = -1
        return s, None
    import numpy as np
    g = np.ascontiguousarray(src.g, dtype=np.float64)
    s.k_plane = int(src.k_plane)
    s.amp = _ptr(src.amp, _tdtype(code), "amp")
    s.g = g.ctypes.data
    s.n_g = int(g.shape[0])
    return s, g


def _vec(ts, code, name):
    v = (C.c_void_p * 3)()
    for m in range(3):
        v[m] = _ptr(ts[m], _tdtype(code), name)
    return v


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(status):
    if status != 0:
        msg = load().pic_last_error()
        raise PicError(status, msg.decode() if msg else "")


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)

def pic_workspace_bytes(grid, dtype, n_particles):
    g = make_grid(grid, dtype)
    return int(load().pic_workspace_bytes(C.byref(g), int(n_particles)))


def pic_tile_count(grid, dtype):
    g = make_grid(grid, dtype)
    return int(load().pic_tile_count(C.byref(g)))


def pic_tile_shape(grid, dtype):
    """(tile edge per direction, slack) the library uses for this grid."""
    g = make_grid(grid, dtype)
    t = (C.c_int32 * 3)()
    sl = C.c_int32()
    _check(load().pic_tile_shape(C.byref(g), C.cast(t, C.c_void_p), C.cast(C.pointer(sl), C.c_void_p)))
    return tuple(t), sl.value


def tile_geometry(grid, dtype):
    """Tile edges, tiles per direction and slack as a dict."""
    t, sl = pic_tile_shape(grid, dtype)
    return {"tile": t, "ntiles_xyz": tuple(int(grid.n[d]) // t[d] for d in range(3)), "slack": sl}


def workspace(grid, dtype, n_particles, device="cuda"):
    """A device byte tensor large enough for every call on this grid."""
    nb = pic_workspace_bytes(grid, dtype, n_particles)
    if nb == 0:
        raise PicError(1, "invalid grid")
    return torch.empty(nb + 256, dtype=torch.uint8, device=device)


def _ws_ptr(ws):
    p = ws.data_ptr()
    pa = (p + 255) & ~255
    return pa, ws.numel() - (pa - p)


def pic_sort_tiles(grid, sp, tile_start, ws, perm=None, dtype=None):
    code = _dtype_code(dtype or sp.off.dtype)
    g, s = make_grid(grid, code), make_species(sp, code)
    wp, wn = _ws_ptr(ws)
    _check(load().pic_sort_tiles(C.byref(g), C.byref(s), _ptr(tile_start, torch.int32, "tile_start"),
                                 _ptr(perm, torch.int32, "perm") if perm is not None else None, wp, wn, _stream()))


def pic_gather(grid, sp, fields, Ep=None, Bp=None):
    code = _dtype_code(sp.off.dtype)
    n = int(sp.cell.shape[1])
    if Ep is None:
        Ep = torch.empty((3, n), dtype=_tdtype(code), device=sp.off.device)
    if Bp is None:
        Bp = torch.empty((3, n), dtype=_tdtype(code), device=sp.off.device)
    g, s, f = make_grid(grid, code), make_species(sp, code), make_fields(fields, code, need_j=False)
    _check(load().pic_gather(C.byref(g), C.byref(s), C.byref(f), _vec(Ep, code, "Ep"), _vec(Bp, code, "Bp"),
                             _stream()))
    return Ep, Bp


def pic_push(grid, sp, Ep, Bp):
    code = _dtype_code(sp.off.dtype)
    g, s = make_grid(grid, code), make_species(sp, code)
    _check(load().pic_push(C.byref(g), C.byref(s), _vec(Ep, code, "Ep"), _vec(Bp, code, "Bp"), _stream()))


def pic_deposit(grid, before, after, fields):
    code = _dtype_code(before.off.dtype)
    g, s0, s1, f = make_grid(grid, code), make_species(before, code), make_species(after, code), \
        make_fields(fields, code)
    _check(load().pic_deposit(C.byref(g), C.byref(s0), C.byref(s1), C.byref(f), _stream()))


def pic_yee(grid, fields, src=None, step=0):
    code = _dtype_code(fields.E.dtype)
    g, f = make_grid(grid, code), make_fields(fields, code)
    so, keep = make_source(src, code)
    _check(load().pic_yee(C.byref(g), C.byref(f), C.byref(so), int(step), _stream()))
    del keep


def pic_step(grid, sp, fields, src, step0, nsteps, sort_every, tile_start, ws, diag=None):
    code = _dtype_code(sp.off.dtype)
    g, s, f = make_grid(grid, code), make_species(sp, code), make_fields(fields, code)
    so, keep = make_source(src, code)
    wp, wn = _ws_ptr(ws)
    _check(load().pic_step(C.byref(g), C.byref(s), C.byref(f), C.byref(so), int(step0), int(nsteps),
                           int(sort_every), _ptr(tile_start, torch.int32, "tile_start") if tile_start is not None
                           else None, wp, wn, _ptr(diag, torch.float64, "diag") if diag is not None else None,
                           _stream()))
    del keep


def pic_step_noalloc(grid, sp, fields, src, step0, nsteps, sort_every, tile_start, diag=None):
    """pic_step without a workspace: the library's static scratch array."""
    code = _dtype_code(sp.off.dtype)
    g, s, f = make_grid(grid, code), make_species(sp, code), make_fields(fields, code)
    so, keep = make_source(src, code)
    _check(load().pic_step_noalloc(C.byref(g), C.byref(s), C.byref(f), C.byref(so), int(step0), int(nsteps),
                                   int(sort_every), _ptr(tile_start, torch.int32, "tile_start")
                                   if tile_start is not None else None,
                                   _ptr(diag, torch.float64, "diag") if diag is not None else None, _stream()))
    del keep


NOALLOC_SCRATCH_BYTES = 128 << 20


def make_adjoint(lam, code):
    a = pic_adjoint()
    n = int(lam.lx.shape[1]) if lam.lx is not None else 0
    for m in range(3):
        a.lx[m] = _ptr(lam.lx[m], _tdtype(code), "lx") if n > 0 else None
        a.lu[m] = _ptr(lam.lu[m], _tdtype(code), "lu") if n > 0 else None
        a.lE[m] = _ptr(lam.lE[m], _tdtype(code), "lE")
        a.lB[m] = _ptr(lam.lB[m], _tdtype(code), "lB")
    return a


def pic_step_adjoint(grid, sp, fields, src, step, lam, dA, ws, tile_start=None):
    """lam: object with lx, lu (3, N) and lE, lB (3, nz, ny, nx) device tensors;
    tile_start: the binning of sp (or None for the untiled kernel)."""
    code = _dtype_code(sp.off.dtype)
    g, s, f = make_grid(grid, code), make_species(sp, code), make_fields(fields, code, need_j=False)
    so, keep = make_source(src, code)
    a = make_adjoint(lam, code)
    wp, wn = _ws_ptr(ws)
    _check(load().pic_step_adjoint(C.byref(g), C.byref(s), C.byref(f),
                                   _ptr(tile_start, torch.int32, "tile_start") if tile_start is not None else None,
                                   C.byref(so), int(step), C.byref(a),
                                   _ptr(dA, torch.float64, "dA") if dA is not None else None, wp, wn, _stream()))
    del keep


def pic_reduce(grid, sp, fields, ws, out=None):
    code = _dtype_code(fields.E.dtype)
    if out is None:
        out = torch.empty(5, dtype=torch.float64, device=fields.E.device)
    g, f = make_grid(grid, code), make_fields(fields, code, need_j=False)
    s = make_species(sp, code) if sp is not None else None
    wp, wn = _ws_ptr(ws)
    _check(load().pic_reduce(C.byref(g), C.byref(s) if s is not None else None, C.byref(f),
                             _ptr(out, torch.float64, "out"), wp, wn, _stream()))
    return out


def pic_gauss_residual(grid, sp, fields, ws, out=None):
    """(|div E - rho/eps0|_2, |rho/eps0|_2, species charge) as a device double[3]."""
    code = _dtype_code(sp.off.dtype)
    g, s, f = make_grid(grid, code), make_species(sp, code), make_fields(fields, code, need_j=False)
    if out is None:
        out = torch.zeros(3, dtype=torch.float64, device=sp.off.device)
    wp, wn = _ws_ptr(ws)
    _check(load().pic_gauss_residual(C.byref(g), C.byref(s), C.byref(f), _ptr(out, torch.float64, "out"), wp, wn,
                                     _stream()))
    return out


def pic_energy_loss(grid, fields, lam, ws, seed=1.0, out=None):
    """L = U_E + U_B into out (device float64 [1]) and the seed of the reverse
    sweep into lam (lE, lB scaled fields; lx, lu zeroed)."""
    code = _dtype_code(fields.E.dtype)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=fields.E.device)
    g, f = make_grid(grid, code), make_fields(fields, code, need_j=False)
    a = make_adjoint(lam, code)
    n = int(lam.lx.shape[1]) if lam.lx is not None else 0
    wp, wn = _ws_ptr(ws)
    _check(load().pic_energy_loss(C.byref(g), C.byref(f), n, float(seed), C.byref(a),
                                  _ptr(out, torch.float64, "out"), wp, wn, _stream()))
    return out


def pic_timing(enable):
    """Read and reset the per-category kernel times, then switch timing on or
    off.  Returns {category: (milliseconds, launches)}."""
    n = len(TIMING_CATEGORIES)
    ms = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    _check(load().pic_timing(1 if enable else 0, C.cast(ms, C.c_void_p), C.cast(cnt, C.c_void_p), n))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(TIMING_CATEGORIES)}


def pic_last_error():
    m = load().pic_last_error()
    return m.decode() if m else ""
