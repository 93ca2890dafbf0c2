"""Parity at the full workload sizes, in the launch configuration bench.py
times (tiles and slack chosen by the library, a sort at the first step and
none at the next, as in the sort-every-4 / every-20 cycles), on outputs the
oracle computes one by one.

Two GPU steps run from the workload's initial state.  In a few boxes of
cells, the oracle then takes the GPU's own state after the first step on a
local, non-periodic copy of the box plus a margin, and recomputes from it:
the push and move of every particle whose cell lies in the box, the current
of the second step in the box from every particle that can reach it (its
old and new positions from the GPU), and the field update of the second
step in the box from the GPU's fields and current.  FP64 must agree to
1e-12, FP32 (split precision) within the stated bounds (momenta and offsets
2e-6 relative, J, E, B rel-L2 1e-5).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2101_12149_amd import _lib
from paper_2101_12149_amd import workloads as wl
from pic_cases import NS, max_rel, rel_l2

pytestmark = pytest.mark.gpu

BOX = 12      # cells per box edge
MARGIN = 8    # local cells around a box: old cells within 4 of the box, their windows and one field step


def _local_grid(g, margin=MARGIN):
    return NS(n=(BOX + 2 * margin,) * 3, d=tuple(g.d), dt=g.dt, c=g.c, eps0=g.eps0, order=g.order,
              pusher=getattr(g, "pusher", 0), solver=getattr(g, "solver", 0))


def _slice(a, lo, margin=MARGIN):
    """(3, nz, ny, nx) device array -> local (3, L, L, L) float64 host copy
    of cells lo - margin .. lo + BOX + margin (the box is away from the
    periodic boundary)."""
    L = BOX + 2 * margin
    z0, y0, x0 = lo[2] - margin, lo[1] - margin, lo[0] - margin
    return np.ascontiguousarray(a[:, z0:z0 + L, y0:y0 + L, x0:x0 + L].to(torch.float64).cpu().numpy())


def _select(cell, lo, pad):
    """Indices of the particles whose cell lies in [lo - pad, lo + BOX + pad) per axis."""
    m = torch.ones(cell.shape[1], dtype=torch.bool, device=cell.device)
    for d in range(3):
        m &= (cell[d] >= lo[d] - pad) & (cell[d] < lo[d] + BOX + pad)
    return torch.nonzero(m).flatten()


def _local_species(sp, idx, lo, cell=None, off=None, margin=MARGIN):
    """Host FP64 copy of particles idx with cells in the local frame."""
    cell = sp.cell if cell is None else cell
    off = sp.off if off is None else off
    c = cell[:, idx].cpu().numpy().astype(np.int64) - (np.array(lo)[:, None] - margin)
    assert c.min() >= 0 and c.max() < BOX + 2 * margin
    w = None if sp.w is None else np.ascontiguousarray(sp.w[idx].to(torch.float64).cpu().numpy())
    return NS(cell=np.ascontiguousarray(c.astype(np.int32)),
              off=np.ascontiguousarray(off[:, idx].to(torch.float64).cpu().numpy()),
              u=np.ascontiguousarray(sp.u[:, idx].to(torch.float64).cpu().numpy()),
              w=w, w0=sp.w0, q=sp.q, m=sp.m)


def _boxes(w, rng, nbox, margin=MARGIN):
    n = np.array(w.grid.n)
    lo_min = np.full(3, margin)
    if w.source is not None:     # keep the boxes clear of the source plane and inside the plasma
        lo_min[2] = max(lo_min[2], w.source.k_plane + margin + 40)
    return [tuple(int(rng.integers(lo_min[d], n[d] - BOX - margin)) for d in range(3)) for _ in range(nbox)]


@pytest.mark.parametrize("name", ["uniform256_o3_f32", "uniform256_o3_f64", "laser128x128x1024_o3_f32",
                                  "stress512_o3_f32"])
def test_full_size_two_steps_match_oracle_in_sampled_boxes(name):
    w = wl.named(name, device="cuda")
    g, sp, f = w.grid, w.species, w.fields
    src = w.source.to(device="cuda") if w.source is not None else None
    f64 = w.dtype == "f64"
    print(f"[fullsize] {name}: {sp.n} particles, grid {g.n}", flush=True)
    ws = _lib.workspace(g, w.dtype, sp.n)
    ts = torch.zeros(_lib.pic_tile_count(g, w.dtype) + 1, dtype=torch.int32, device="cuda")
    _lib.pic_step(g, sp, f, src, 0, 1, w.sort_every, ts, ws)   # step 0, sorted first
    torch.cuda.synchronize()
    rng = np.random.default_rng(sum(map(ord, name)))
    boxes = _boxes(w, rng, 3)
    # state 1 of every particle that matters for a box, and the box fields
    keep = []
    for lo in boxes:
        near = _select(sp.cell, lo, 4)
        inner = _select(sp.cell, lo, 0)
        keep.append(dict(lo=lo, near=near, inner=inner,
                         s_near=_local_species(sp, near, lo), s_inner=_local_species(sp, inner, lo),
                         E1=_slice(f.E, lo), B1=_slice(f.B, lo)))
    _lib.pic_step(g, sp, f, src, 1, 1, 0, ts, ws)               # step 1 on the same binning
    torch.cuda.synchronize()
    lg = _local_grid(g)
    L = BOX + 2 * MARGIN
    inner_sl = (slice(None), slice(MARGIN, MARGIN + BOX), slice(MARGIN, MARGIN + BOX), slice(MARGIN, MARGIN + BOX))
    tol_p = 1e-12 if f64 else 2e-6
    tol_f = 1e-12 if f64 else 1e-5
    checked = 0
    for k in keep:
        lo = k["lo"]
        # push and move of the box's particles from the GPU's state 1 and fields
        o = k["s_inner"]
        lf = NS(E=k["E1"], B=k["B1"], J=np.zeros_like(k["E1"]))
        Ep, Bp = oracle.gather(lg, o, lf)
        oracle.push(lg, o, Ep, Bp)
        gpu = _local_species(sp, k["inner"], lo)
        assert max_rel(gpu.u, o.u) < tol_p, (name, lo, "u")
        dx = (gpu.cell - o.cell) + (gpu.off - o.off)
        assert np.abs(dx).max() < tol_p * 4, (name, lo, "x")
        # the current of step 1 in the box from every particle that can reach it
        before, after = k["s_near"], _local_species(sp, k["near"], lo)
        Jf = NS(E=np.zeros((3, L, L, L)), B=np.zeros((3, L, L, L)), J=np.zeros((3, L, L, L)))
        oracle.deposit(lg, before, after, Jf)
        J2 = _slice(f.J, lo)
        assert rel_l2(J2[inner_sl], Jf.J[inner_sl]) < tol_f, (name, lo, "J")
        # the field update of step 1 in the box from the GPU's E1, B1 and J2
        ff = NS(E=k["E1"].copy(), B=k["B1"].copy(), J=J2)
        oracle.yee(lg, ff, None, 1)
        assert rel_l2(_slice(f.E, lo)[inner_sl], ff.E[inner_sl]) < tol_f, (name, lo, "E")
        assert rel_l2(_slice(f.B, lo)[inner_sl], ff.B[inner_sl]) < tol_f, (name, lo, "B")
        checked += len(k["inner"])
    assert checked > 1000
    print(f"[fullsize] {name}: {checked} particles checked in {len(boxes)} boxes", flush=True)


AMARGIN = 10   # local cells around a box for the adjoint: its stencils chain to about 8 cells


def _local_lambda(lam, idx, lo):
    """Oracle adjoint state on the local box: particle adjoints of particles
    idx, field adjoints of the local cells (FP64 host copies)."""
    L = BOX + 2 * AMARGIN
    a = oracle.Adjoint(NS(n=(L, L, L)), int(idx.numel()))
    a.lx[:] = lam.lx[:, idx].to(torch.float64).cpu().numpy()
    a.lu[:] = lam.lu[:, idx].to(torch.float64).cpu().numpy()
    a.lE[:] = _slice(lam.lE, lo, AMARGIN)
    a.lB[:] = _slice(lam.lB, lo, AMARGIN)
    return a


@pytest.mark.parametrize("name", ["uniform256_o3_f32", "stress512_o3_f32", "laser128x128x1024_o3_f32"])
def test_full_size_adjoint_step_matches_oracle_in_sampled_boxes(name):
    """The tiled FP32 reverse step as the benchmark times it (particles
    re-binned, two steps on that binning, then one adjoint step with seeded
    random adjoint inputs), checked in a few boxes of cells: the oracle's
    adjoint step on a local copy of the box plus a margin (the GPU's state,
    fields and adjoint inputs there) gives the field adjoints of the box and
    the particle adjoints of the particles in it.  A value in the box depends
    only on data within the field-solve, deposit and gather stencils, chained
    to about 8 cells, so a margin of 10 keeps the local copy's wrap out of it.  8 ppc runs
    most scatter waves on fixed windows, 2 ppc most on per-component runs; the
    laser box has weighted particles of a cold beam (its boxes lie in the
    plasma, away from the source plane)."""
    w = wl.named(name, device="cuda")
    g, sp, f = w.grid, w.species, w.fields
    dt = w.dtype
    print(f"[fullsize-adjoint] {name}: {sp.n} particles, grid {g.n}", flush=True)
    ws = _lib.workspace(g, dt, sp.n)
    ts = torch.zeros(_lib.pic_tile_count(g, dt) + 1, dtype=torch.int32, device="cuda")
    _lib.pic_sort_tiles(g, sp, ts, ws)
    _lib.pic_step(g, sp, f, None, 0, 2, 0, ts, ws)
    gen = torch.Generator(device="cuda").manual_seed(sum(map(ord, name)))
    tdt = sp.off.dtype
    lam = NS(lx=torch.randn(sp.off.shape, generator=gen, device="cuda", dtype=tdt),
             lu=torch.randn(sp.u.shape, generator=gen, device="cuda", dtype=tdt),
             lE=torch.randn(f.E.shape, generator=gen, device="cuda", dtype=tdt),
             lB=torch.randn(f.B.shape, generator=gen, device="cuda", dtype=tdt))
    torch.cuda.synchronize()
    rng = np.random.default_rng(sum(map(ord, name)) + 1)
    boxes = _boxes(w, rng, 3, AMARGIN)
    lg = _local_grid(g, AMARGIN)
    keep = []
    for lo in boxes:
        near = _select(sp.cell, lo, AMARGIN)    # every particle of the local box
        inner = _select(sp.cell, lo, 0)
        keep.append(dict(lo=lo, near=near, inner=inner, sp=_local_species(sp, near, lo, margin=AMARGIN),
                         E=_slice(f.E, lo, AMARGIN), B=_slice(f.B, lo, AMARGIN), lam=_local_lambda(lam, near, lo)))
    _lib.pic_step_adjoint(g, sp, f, None, 2, lam, None, ws, tile_start=ts)
    torch.cuda.synchronize()
    m = AMARGIN
    inner_sl = (slice(None), slice(m, m + BOX), slice(m, m + BOX), slice(m, m + BOX))
    tol = 1e-4
    checked = 0
    for k in keep:
        lo = k["lo"]
        lf = NS(E=k["E"], B=k["B"], J=np.zeros_like(k["E"]))
        ol = k["lam"]
        oracle.step_adjoint(lg, k["sp"], lf, None, 2, ol, None)
        assert rel_l2(_slice(lam.lE, lo, m)[inner_sl], ol.lE[inner_sl]) < tol, (name, lo, "lE")
        assert rel_l2(_slice(lam.lB, lo, m)[inner_sl], ol.lB[inner_sl]) < tol, (name, lo, "lB")
        # the particles of the box, found in the local list
        pos = {int(p): i for i, p in enumerate(k["near"].tolist())}
        sel = np.array([pos[int(p)] for p in k["inner"].tolist()])
        for nm in ("lx", "lu"):
            gpu = getattr(lam, nm)[:, k["inner"]].to(torch.float64).cpu().numpy()
            assert rel_l2(gpu, getattr(ol, nm)[:, sel]) < tol, (name, lo, nm)
        checked += len(k["inner"])
    assert checked > 1000
    print(f"[fullsize-adjoint] {name}: {checked} particles checked in {len(boxes)} boxes", flush=True)
