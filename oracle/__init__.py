"""FP64 CPU oracle of the electromagnetic PIC step (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It never imports the product package
and the product never imports it.  The arithmetic lives in ``oracle.c``; this
module only marshals numpy arrays into the C structs.

Inputs are duck-typed so that any container with the right attributes works:
  grid:    n (nx,ny,nz), d (dx,dy,dz), dt, c, eps0, order
  species: cell (3,N) int32, off (3,N) float64, u (3,N) float64,
           w (N,) float64 or None, w0, q, m
  fields:  E, B, J, each (3, nz, ny, nx) float64 (x fastest)
  source:  k_plane, amp (ny, nx) float64, g (nsteps,) float64   (or None)
All arrays are modified in place where the C function writes.
"""
import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build():
    """Compile the oracle with gcc (plain -O2, IEEE arithmetic, OpenMP)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
                           "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)


class _Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("d", C.c_double * 3), ("dt", C.c_double),
                ("c", C.c_double), ("eps0", C.c_double), ("order", C.c_int32), ("pusher", C.c_int32),
                ("solver", C.c_int32), ("gather_filter", C.c_void_p)]


class _Species(C.Structure):
    _fields_ = [("n", C.c_int64), ("cell", C.c_void_p * 3), ("off", C.c_void_p * 3),
                ("u", C.c_void_p * 3), ("w", C.c_void_p), ("w0", C.c_double),
                ("q", C.c_double), ("m", C.c_double)]


class _Fields(C.Structure):
    _fields_ = [("E", C.c_void_p * 3), ("B", C.c_void_p * 3), ("J", C.c_void_p * 3)]


class _Source(C.Structure):
    _fields_ = [("k_plane", C.c_int32), ("amp", C.c_void_p), ("g", C.c_void_p), ("n_g", C.c_int64)]


class _Adjoint(C.Structure):
    _fields_ = [("lx", C.c_void_p * 3), ("lu", C.c_void_p * 3), ("lE", C.c_void_p * 3),
                ("lB", C.c_void_p * 3)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
                build()
            lib = C.CDLL(_SO)
            P = C.POINTER
            lib.or_num_threads.restype = C.c_int
            lib.or_set_num_threads.argtypes = [C.c_int]
            lib.or_shape.restype = C.c_double
            lib.or_shape.argtypes = [C.c_int, C.c_double]
            lib.or_dshape.restype = C.c_double
            lib.or_dshape.argtypes = [C.c_int, C.c_double]
            lib.or_gather.argtypes = [P(_Grid), P(_Species), P(_Fields), C.c_void_p * 3, C.c_void_p * 3]
            lib.or_push.argtypes = [P(_Grid), P(_Species), C.c_void_p * 3, C.c_void_p * 3]
            lib.or_deposit.argtypes = [P(_Grid), P(_Species), P(_Species), P(_Fields)]
            lib.or_rho.argtypes = [P(_Grid), P(_Species), C.c_void_p]
            lib.or_ckc_coeffs.argtypes = [P(_Grid), C.c_void_p]
            lib.or_yee.argtypes = [P(_Grid), P(_Fields), P(_Source), C.c_int64]
            lib.or_reduce.argtypes = [P(_Grid), P(_Species), P(_Fields), C.c_void_p]
            lib.or_gauss.argtypes = [P(_Grid), P(_Species), P(_Fields), C.c_void_p, C.c_void_p]
            lib.or_step.argtypes = [P(_Grid), P(_Species), P(_Fields), P(_Source), C.c_int64,
                                    C.c_int32, C.c_void_p]
            lib.or_loss.restype = C.c_double
            lib.or_loss.argtypes = [P(_Grid), P(_Fields), P(_Adjoint), C.c_int64]
            lib.or_step_adjoint.argtypes = [P(_Grid), P(_Species), P(_Fields), P(_Source), C.c_int64,
                                            P(_Adjoint), C.c_void_p]
            _lib = lib
    return _lib


def _f64(a, name):
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous):
        raise TypeError(f"{name} must be a C-contiguous float64 numpy array")
    return a


def _ptr(a):
    return a.ctypes.data


def _grid(g):
    s = _Grid()
    s.n[:] = [int(v) for v in g.n]
    s.d[:] = [float(v) for v in g.d]
    s.dt, s.c, s.eps0, s.order = float(g.dt), float(g.c), float(g.eps0), int(g.order)
    s.pusher = int(getattr(g, "pusher", 0))
    if s.pusher not in (0, 1):
        raise ValueError("pusher must be 0 (Boris) or 1 (Vay)")
    s.solver = int(getattr(g, "solver", 0))
    if s.solver not in (0, 1):
        raise ValueError("solver must be 0 (Yee) or 1 (CKC)")
    gf = getattr(g, "gather_filter", None)
    if gf is not None:
        gf = np.ascontiguousarray(np.asarray(gf, dtype=np.float64).reshape(6, 4))
        s._filter = gf            # kept alive with the struct
        s.gather_filter = gf.ctypes.data
    return s


def _species(sp):
    cell, off, u = sp.cell, sp.off, sp.u
    if not (isinstance(cell, np.ndarray) and cell.dtype == np.int32 and cell.flags.c_contiguous
            and cell.ndim == 2 and cell.shape[0] == 3):
        raise TypeError("cell must be a C-contiguous (3, N) int32 numpy array")
    _f64(off, "off")
    _f64(u, "u")
    n = cell.shape[1]
    if off.shape != (3, n) or u.shape != (3, n):
        raise ValueError("off and u must be (3, N)")
    s = _Species()
    s.n = n
    for d in range(3):
        s.cell[d] = _ptr(cell[d])
        s.off[d] = _ptr(off[d])
        s.u[d] = _ptr(u[d])
    if sp.w is not None:
        w = _f64(sp.w, "w")
        if w.shape != (n,):
            raise ValueError("w must be (N,)")
        s.w = _ptr(w)
    else:
        s.w = None
    s.w0, s.q, s.m = float(sp.w0), float(sp.q), float(sp.m)
    return s


def _fields(f, grid):
    shape = (3, int(grid.n[2]), int(grid.n[1]), int(grid.n[0]))
    s = _Fields()
    for name in ("E", "B", "J"):
        a = _f64(getattr(f, name), name)
        if a.shape != shape:
            raise ValueError(f"{name} must have shape {shape}")
        arr = getattr(s, name)
        for m in range(3):
            arr[m] = _ptr(a[m])
    return s


def _source(src, grid):
    s = _Source()
    if src is None or src.k_plane < 0:
        s.k_plane = -1
        return s, None
    amp = _f64(src.amp, "amp")
    if amp.shape != (int(grid.n[1]), int(grid.n[0])):
        raise ValueError("amp must be (ny, nx)")
    g = np.ascontiguousarray(src.g, dtype=np.float64)
    s.k_plane, s.amp, s.g, s.n_g = int(src.k_plane), _ptr(amp), _ptr(g), g.shape[0]
    return s, g  # keep g alive


def _vec3(arrs):
    v = (C.c_void_p * 3)()
    for m in range(3):
        v[m] = _ptr(_f64(arrs[m], "vector component"))
    return v


def num_threads():
    return int(_load().or_num_threads())


def set_num_threads(n):
    """Thread count of the oracle's later parallel loops (OpenMP); only
    the summation order of the per-thread current buffers depends on it."""
    _load().or_set_num_threads(int(n))


def shape(order, r):
    lib = _load()
    return np.array([lib.or_shape(order, float(x)) for x in np.ravel(r)]).reshape(np.shape(r))


def dshape(order, r):
    lib = _load()
    return np.array([lib.or_dshape(order, float(x)) for x in np.ravel(r)]).reshape(np.shape(r))


def gather(grid, sp, fields):
    """Fields at the particles: returns (Ep, Bp), each (3, N)."""
    lib = _load()
    n = sp.cell.shape[1]
    Ep = np.zeros((3, n))
    Bp = np.zeros((3, n))
    g, s, f = _grid(grid), _species(sp), _fields(fields, grid)
    lib.or_gather(C.byref(g), C.byref(s), C.byref(f), _vec3(Ep), _vec3(Bp))
    return Ep, Bp


def push(grid, sp, Ep, Bp):
    """Boris momentum update and position update, in place."""
    lib = _load()
    g, s = _grid(grid), _species(sp)
    lib.or_push(C.byref(g), C.byref(s), _vec3(Ep), _vec3(Bp))


def deposit(grid, before, after, fields):
    """J += Esirkepov current of particles moving from before to after."""
    lib = _load()
    g, s0, s1, f = _grid(grid), _species(before), _species(after), _fields(fields, grid)
    lib.or_deposit(C.byref(g), C.byref(s0), C.byref(s1), C.byref(f))


def rho(grid, sp):
    """Nodal charge density, (nz, ny, nx)."""
    lib = _load()
    out = np.zeros((int(grid.n[2]), int(grid.n[1]), int(grid.n[0])))
    g, s = _grid(grid), _species(sp)
    lib.or_rho(C.byref(g), C.byref(s), _ptr(out))
    return out


def ckc_coeffs(grid):
    """(3, 4) array: (alpha, beta_p, beta_q, gamma) of the CKC averaging of
    the differences along x, y, z (p, q = the next two axes cyclically)."""
    lib = _load()
    out = np.zeros(12)
    g = _grid(grid)
    lib.or_ckc_coeffs(C.byref(g), _ptr(out))
    return out.reshape(3, 4)


def yee(grid, fields, src=None, step=0):
    lib = _load()
    g, f = _grid(grid), _fields(fields, grid)
    s, keep = _source(src, grid)
    lib.or_yee(C.byref(g), C.byref(f), C.byref(s), int(step))
    del keep


def reduce(grid, sp, fields):
    """[U_E, U_B, kinetic, charge, z-momentum] in FP64."""
    lib = _load()
    out = np.zeros(5)
    g, f = _grid(grid), _fields(fields, grid)
    s = _species(sp) if sp is not None else None
    lib.or_reduce(C.byref(g), C.byref(s) if s is not None else None, C.byref(f), _ptr(out))
    return out


def gauss(grid, sp, fields):
    """Gauss-law residual: (res (nz, ny, nx) = div E - rho/eps0 per node with
    the neutralising background, [|res|_2, |rho/eps0|_2, species charge])."""
    lib = _load()
    res = np.zeros((int(grid.n[2]), int(grid.n[1]), int(grid.n[0])))
    out = np.zeros(3)
    g, s, f = _grid(grid), _species(sp), _fields(fields, grid)
    lib.or_gauss(C.byref(g), C.byref(s), C.byref(f), _ptr(res), _ptr(out))
    return res, out


def step(grid, sp, fields, src=None, step0=0, nsteps=1):
    """Advance nsteps full PIC steps in place; returns diag (nsteps, 5)."""
    lib = _load()
    diag = np.zeros((max(nsteps, 1), 5))
    g, s, f = _grid(grid), _species(sp), _fields(fields, grid)
    so, keep = _source(src, grid)
    lib.or_step(C.byref(g), C.byref(s), C.byref(f), C.byref(so), int(step0), int(nsteps), _ptr(diag))
    del keep
    return diag[:nsteps]


class Adjoint:
    """Adjoint state: lx, lu (3, N); lE, lB (3, nz, ny, nx)."""

    def __init__(self, grid, n):
        shape = (3, int(grid.n[2]), int(grid.n[1]), int(grid.n[0]))
        self.lx = np.zeros((3, n))
        self.lu = np.zeros((3, n))
        self.lE = np.zeros(shape)
        self.lB = np.zeros(shape)

    def _struct(self):
        a = _Adjoint()
        for m in range(3):
            a.lx[m] = _ptr(_f64(self.lx, "lx")[m])
            a.lu[m] = _ptr(_f64(self.lu, "lu")[m])
            a.lE[m] = _ptr(_f64(self.lE, "lE")[m])
            a.lB[m] = _ptr(_f64(self.lB, "lB")[m])
        return a


def loss(grid, fields, n_particles=0):
    """L = U_E + U_B and its terminal adjoint."""
    lib = _load()
    lam = Adjoint(grid, n_particles)
    g, f = _grid(grid), _fields(fields, grid)
    a = lam._struct()
    L = lib.or_loss(C.byref(g), C.byref(f), C.byref(a), int(n_particles))
    return L, lam


def step_adjoint(grid, sp, fields, src, step_index, lam, dA):
    """Reverse one step: lam (state n+1) -> lam (state n); dA (ny, nx) +=."""
    lib = _load()
    g, s, f = _grid(grid), _species(sp), _fields(fields, grid)
    so, keep = _source(src, grid)
    a = lam._struct()
    dptr = _ptr(_f64(dA, "dA")) if dA is not None else None
    lib.or_step_adjoint(C.byref(g), C.byref(s), C.byref(f), C.byref(so), int(step_index), C.byref(a), dptr)
    del keep


def rollout_grad(grid, sp, fields, src, step0, nsteps):
    """Forward nsteps from copies of the inputs, then reverse.

    Returns (L, dL/du0 (3, N), dL/dA (ny, nx) or None, final species, final fields).
    Every intermediate state is stored (intended for small test cases)."""
    states = []
    s = _copy_species(sp)
    f = _copy_fields(fields)
    for it in range(nsteps):
        states.append((_copy_species(s), _copy_fields(f)))
        step(grid, s, f, src, step0 + it, 1)
    L, lam = loss(grid, f, s.cell.shape[1])
    dA = np.zeros((int(grid.n[1]), int(grid.n[0]))) if src is not None and src.k_plane >= 0 else None
    for it in reversed(range(nsteps)):
        s_n, f_n = states[it]
        step_adjoint(grid, s_n, f_n, src, step0 + it, lam, dA)
    return L, lam.lu.copy(), dA, s, f


class _NS:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def _copy_species(sp):
    return _NS(cell=sp.cell.copy(), off=sp.off.copy(), u=sp.u.copy(),
               w=None if sp.w is None else sp.w.copy(), w0=sp.w0, q=sp.q, m=sp.m)


def _copy_fields(f):
    return _NS(E=f.E.copy(), B=f.B.copy(), J=f.J.copy())
