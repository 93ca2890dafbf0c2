"""Seeded synthetic workloads shared by the HIP path, the oracle and the tests.

This module holds no arithmetic of the PIC method: it only draws particles and
builds grid/source descriptions.  The shapes follow the paper's own workloads
(Sec. 4.1: uniform plasma, 8 particles per cell, order-3 shapes, Yee and
Esirkepov; Sec. 4.2: about 2 particles per cell for laser-wakefield runs).

Normalised units: c = eps0 = 1, electrons q = -1, m = 1.  Uniform-plasma
workloads use n0 = 1 (so omega_p = 1) and omega_p dt = 0.1 with cubic cells at
0.99 of the Yee CFL limit.  The laser workload uses omega_L = 1 (lambda = 2 pi)
and n_crit = 1.

Containers hold torch tensors; ``numpy()`` returns FP64 host copies in the
duck-typed layout the oracle takes.  Random streams come from a seeded
``torch.Generator`` on the device the tensors are created on.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np
import torch


@dataclass
class Grid:
    n: tuple            # cells (nx, ny, nz), periodic
    d: tuple            # spacing (dx, dy, dz)
    dt: float
    c: float = 1.0
    eps0: float = 1.0
    order: int = 3      # shape-function order: 1 or 3
    tile: tuple = (0, 0, 0)   # sort/LDS tile edge per direction (0: library default)
    slack: int = -1     # halo slack of the tiled particle kernel (-1: automatic)
    pusher: int = 0     # momentum update: 0 Boris, 1 Vay
    solver: int = 0     # field solver: 0 Yee, 1 Cole-Karkkainen-Cowan
    gather_filter: Optional[tuple] = None   # 6 x 4 z taps per field component, or None

    @property
    def ncells(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def dV(self) -> float:
        return float(self.d[0]) * float(self.d[1]) * float(self.d[2])


@dataclass
class Species:
    cell: torch.Tensor              # (3, N) int32
    off: torch.Tensor               # (3, N) offset in [0, 1), cell units
    u: torch.Tensor                 # (3, N) gamma * v
    w: Optional[torch.Tensor]       # (N,) or None (constant w0)
    w0: float
    q: float = -1.0
    m: float = 1.0

    @property
    def n(self) -> int:
        return int(self.cell.shape[1])

    def to(self, device=None, dtype=None) -> "Species":
        dtype = dtype or self.off.dtype
        off = self.off.to(device=device, dtype=dtype)
        if dtype == torch.float32:
            off = _below_one(off)
        return Species(self.cell.to(device=device).contiguous(), off.contiguous(),
                       self.u.to(device=device, dtype=dtype).contiguous(),
                       None if self.w is None else self.w.to(device=device, dtype=dtype).contiguous(),
                       self.w0, self.q, self.m)

    def clone(self) -> "Species":
        return Species(self.cell.clone(), self.off.clone(), self.u.clone(),
                       None if self.w is None else self.w.clone(), self.w0, self.q, self.m)

    def numpy(self) -> "Species":
        """FP64 host copy (exact upcast of FP32 values) for the oracle."""
        def f(t):
            return np.ascontiguousarray(t.detach().cpu().to(torch.float64).numpy())
        return Species(np.ascontiguousarray(self.cell.detach().cpu().numpy().astype(np.int32)),
                       f(self.off), f(self.u), None if self.w is None else f(self.w),
                       float(self.w0), float(self.q), float(self.m))


@dataclass
class Fields:
    E: torch.Tensor   # (3, nz, ny, nx)
    B: torch.Tensor
    J: torch.Tensor

    @staticmethod
    def zeros(grid: Grid, dtype=torch.float64, device="cpu") -> "Fields":
        shape = (3, int(grid.n[2]), int(grid.n[1]), int(grid.n[0]))
        return Fields(*(torch.zeros(shape, dtype=dtype, device=device) for _ in range(3)))

    def to(self, device=None, dtype=None) -> "Fields":
        return Fields(*(t.to(device=device, dtype=dtype or t.dtype).contiguous() for t in (self.E, self.B, self.J)))

    def clone(self) -> "Fields":
        return Fields(self.E.clone(), self.B.clone(), self.J.clone())

    def numpy(self) -> "Fields":
        def f(t):
            return np.ascontiguousarray(t.detach().cpu().to(torch.float64).numpy())
        return Fields(f(self.E), f(self.B), f(self.J))


@dataclass
class Source:
    """Soft E_x source on the plane k = k_plane: E_x[k_plane] += amp * g[step]."""
    k_plane: int
    amp: torch.Tensor          # (ny, nx)
    g: np.ndarray              # (nsteps,) float64, host

    def to(self, device=None, dtype=None) -> "Source":
        return Source(self.k_plane, self.amp.to(device=device, dtype=dtype or self.amp.dtype).contiguous(),
                      self.g)

    def numpy(self) -> "Source":
        return Source(self.k_plane, np.ascontiguousarray(self.amp.detach().cpu().to(torch.float64).numpy()),
                      np.ascontiguousarray(self.g, dtype=np.float64))


@dataclass
class Workload:
    name: str
    grid: Grid
    species: Species
    fields: Fields
    source: Optional[Source]
    nsteps: int
    sort_every: int
    dtype: str                 # "f64" or "f32"
    seed: int
    description: str = ""
    checkpoint_every: int = 0
    meta: dict = field(default_factory=dict)

    def torch_dtype(self):
        return torch.float64 if self.dtype == "f64" else torch.float32


# ---------------------------------------------------------------------------
# drawing helpers

def _below_one(off: torch.Tensor) -> torch.Tensor:
    """Rounding an FP64 offset to FP32 can give exactly 1.0; keep it in [0,1)."""
    one_minus = torch.nextafter(torch.ones((), dtype=off.dtype, device=off.device),
                                torch.zeros((), dtype=off.dtype, device=off.device))
    return torch.where(off >= 1, one_minus, off)


def _generator(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def uniform_cells(n, ppc, k_min=0, device="cpu"):
    """(3, N) int32 cell indices, exactly ppc particles per cell with k >= k_min,
    listed cell by cell (x fastest)."""
    nx, ny, nz = (int(v) for v in n)
    lin = torch.arange(nx * ny * k_min, nx * ny * nz, device=device, dtype=torch.int64)
    lin = lin.repeat_interleave(int(ppc))
    cell = torch.stack([lin % nx, (lin // nx) % ny, lin // (nx * ny)]).to(torch.int32)
    return cell.contiguous()


def draw_species(cell, u_th, w0, seed, dtype=torch.float64, device="cpu", w=None, shuffle=False,
                 q=-1.0, m=1.0) -> Species:
    """Offsets i.i.d. U[0,1)^3 and momenta u ~ N(0, u_th^2) per component
    (u_th = 0 gives a cold species)."""
    gen = _generator(seed, device)
    nparticles = int(cell.shape[1])
    if shuffle:
        perm = torch.randperm(nparticles, generator=gen, device=device)
        cell = cell[:, perm].contiguous()
        if w is not None:
            w = w[perm].contiguous()
    off = torch.rand((3, nparticles), generator=gen, dtype=dtype, device=device)
    off = _below_one(off)
    if u_th > 0:
        u = torch.randn((3, nparticles), generator=gen, dtype=dtype, device=device) * u_th
    else:
        u = torch.zeros((3, nparticles), dtype=dtype, device=device)
    return Species(cell.contiguous(), off.contiguous(), u.contiguous(),
                   None if w is None else w.to(dtype).contiguous(), float(w0), q, m)


def plasma_grid(n, order, omega_p_dt=0.1, cfl=0.99, tile=(0, 0, 0)) -> Grid:
    """Cubic cells sized so that dt sits at `cfl` of the 3D Yee limit."""
    dt = float(omega_p_dt)
    dx = math.sqrt(3.0) * dt / cfl
    return Grid(tuple(int(v) for v in n), (dx, dx, dx), dt, 1.0, 1.0, int(order), tuple(tile))


# ---------------------------------------------------------------------------
# named workloads

def uniform_plasma(n=(32, 32, 32), ppc=8, u_th=0.01, order=1, nsteps=10, dtype="f64", seed=1001,
                   sort_every=4, device="cpu", shuffle=False, name=None, tile=(0, 0, 0)) -> Workload:
    """Periodic uniform electron plasma (n0 = 1) over an immobile ion background."""
    grid = plasma_grid(n, order, tile=tile)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    cell = uniform_cells(n, ppc, device=device)
    sp = draw_species(cell, u_th, grid.dV / ppc, seed, dtype=torch.float64 if device == "cpu" else tdt,
                      device=device, shuffle=shuffle).to(dtype=tdt)
    f = Fields.zeros(grid, tdt, device)
    nm = name or f"uniform_{n[0]}x{n[1]}x{n[2]}_ppc{ppc}_o{order}_{dtype}"
    return Workload(nm, grid, sp, f, None, nsteps, sort_every, dtype, seed,
                    f"uniform plasma {n[0]}x{n[1]}x{n[2]}, {ppc} ppc, u_th={u_th}c, order {order}, {dtype}",
                    meta={"ppc": ppc, "u_th": u_th})


def laser_plasma(n=(128, 128, 1024), ppc=2, order=3, nsteps=500, dtype="f32", seed=1003, sort_every=4,
                 device="cpu", a0=2.0, waist_lambda=20.0, fwhm_periods=10.0, n0=0.01, ramp=(32, 132),
                 k_source=2, cells_per_lambda=16, width_lambda=80.0, name=None, tile=(0, 0, 0)) -> Workload:
    """Laser wakefield stage: x-polarised Gaussian pulse from a soft source near
    z-min into a plasma with a linear up-ramp; cold electrons, immobile ions.
    omega_L = 1, lambda = 2 pi, n_crit = 1."""
    nx, ny, nz = (int(v) for v in n)
    lam = 2.0 * math.pi
    dz = lam / cells_per_lambda
    dx = width_lambda * lam / nx
    dy = width_lambda * lam / ny
    dt = 0.99 / math.sqrt(1.0 / dx ** 2 + 1.0 / dy ** 2 + 1.0 / dz ** 2)
    grid = Grid((nx, ny, nz), (dx, dy, dz), dt, 1.0, 1.0, order, tuple(tile))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    k0, k1 = int(ramp[0]), int(ramp[1])
    cell = uniform_cells(n, ppc, k_min=k0, device=device)
    gen_dtype = torch.float64 if device == "cpu" else tdt
    sp = draw_species(cell, 0.0, 0.0, seed, dtype=gen_dtype, device=device)
    # density profile n(z) sampled at each particle: linear ramp over [k0, k1) then flat
    z = (sp.cell[2].to(gen_dtype) + sp.off[2]) * dz
    prof = torch.clamp((z - k0 * dz) / ((k1 - k0) * dz), 0.0, 1.0) * n0
    sp.w = (prof * grid.dV / ppc).to(gen_dtype).contiguous()
    sp = sp.to(dtype=tdt)
    f = Fields.zeros(grid, tdt, device)
    # soft source calibrated so that each direction radiates amplitude E0
    E0 = a0  # a0 * m c omega_L / |q| in these units
    w0 = waist_lambda * lam
    x = (torch.arange(nx, dtype=torch.float64) + 0.5) * dx - 0.5 * nx * dx
    y = torch.arange(ny, dtype=torch.float64) * dy - 0.5 * ny * dy
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    amp = 2.0 * (dt / dz) * E0 * torch.exp(-r2 / w0 ** 2)
    tau = fwhm_periods * lam / math.sqrt(2.0 * math.log(2.0))
    t0 = 2.0 * tau
    t = np.arange(nsteps, dtype=np.float64) * dt
    g = np.exp(-((t - t0) / tau) ** 2) * np.sin(t)
    src = Source(int(k_source), amp.to(device=device, dtype=tdt), g)
    nm = name or f"laser_{nx}x{ny}x{nz}_ppc{ppc}_o{order}_{dtype}"
    return Workload(nm, grid, sp, f, src, nsteps, sort_every, dtype, seed,
                    f"laser-plasma {nx}x{ny}x{nz}, {ppc} ppc cold, a0={a0}, ramp k in [{k0},{k1}), {dtype}",
                    meta={"ppc": ppc, "u_th": 0.0})


def differentiable(n=(64, 64, 64), ppc=4, u_th=0.05, order=3, nsteps=20, dtype="f64", seed=1004,
                   checkpoint_every=5, amp0=1e-3, period=16, device="cpu", name=None, tile=(0, 0, 0)) -> Workload:
    """Periodic plasma with a transverse E_x amplitude map on the plane k = 0,
    driven as sin(2 pi n / period); the loss is the final field energy."""
    grid = plasma_grid(n, order, tile=tile)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    cell = uniform_cells(n, ppc, device=device)
    sp = draw_species(cell, u_th, grid.dV / ppc, seed, dtype=torch.float64 if device == "cpu" else tdt,
                      device=device).to(dtype=tdt)
    f = Fields.zeros(grid, tdt, device)
    nx, ny = int(n[0]), int(n[1])
    Lx, Ly = nx * grid.d[0], ny * grid.d[1]
    x = (torch.arange(nx, dtype=torch.float64) + 0.5) * grid.d[0]
    y = torch.arange(ny, dtype=torch.float64) * grid.d[1]
    r2 = (y[:, None] - Ly / 2) ** 2 + (x[None, :] - Lx / 2) ** 2
    amp = amp0 * torch.exp(-r2 / (Lx / 4) ** 2)
    g = np.sin(2.0 * math.pi * np.arange(nsteps, dtype=np.float64) / period)
    src = Source(0, amp.to(device=device, dtype=tdt), g)
    nm = name or f"diff_{n[0]}x{n[1]}x{n[2]}_ppc{ppc}_o{order}_{dtype}"
    return Workload(nm, grid, sp, f, src, nsteps, 0, dtype, seed,
                    f"differentiable plasma {n[0]}x{n[1]}x{n[2]}, {ppc} ppc, u_th={u_th}c, loss=field energy",
                    checkpoint_every=checkpoint_every, meta={"ppc": ppc, "u_th": u_th})


def named(name: str, device="cpu") -> Workload:
    """The five workload shapes the throughput and parity study uses."""
    if name == "uniform32_o1_f64":
        return uniform_plasma((32, 32, 32), 8, 0.01, 1, 10, "f64", 1001, 4, device, name=name)
    if name == "uniform256_o3_f64":
        return uniform_plasma((256, 256, 256), 8, 0.05, 3, 100, "f64", 1002, 4, device, name=name)
    if name == "uniform256_o3_f32":
        return uniform_plasma((256, 256, 256), 8, 0.05, 3, 100, "f32", 1002, 4, device, name=name)
    if name == "laser128x128x1024_o3_f32":
        return laser_plasma(device=device, name=name)
    if name == "diff64_o3_f64":
        return differentiable(device=device, name=name)
    if name == "stress512_o3_f32":
        return uniform_plasma((512, 512, 512), 2, 0.1, 3, 200, "f32", 1005, 20, device, name=name)
    raise KeyError(name)


NAMES = ("uniform32_o1_f64", "uniform256_o3_f64", "uniform256_o3_f32", "laser128x128x1024_o3_f32",
         "diff64_o3_f64", "stress512_o3_f32")
