"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64: results within 1e-12 relative (rel-L2 over the compared array, or max
error over the array's scale).  FP32 split precision: rel-L2 of E, B, J
<= 1e-5 after one step and a charge-conservation residual <= 1e-6, the oracle
starting from the FP32 state upcast exactly to FP64.  Sizes span several
tiles with a ragged last tile where the grid allows it.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2101_12149_amd import _lib
from paper_2101_12149_amd import workloads as wl
from pic_cases import (NS, dev, max_rel, particle_table, random_fields, random_species, rel_l2, tdtype)

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def _grid(n=(12, 16, 20), order=3):
    return wl.plasma_grid(n, order)


def _cpu(t):
    return t.detach().cpu().to(torch.float64).numpy()


# ---------------------------------------------------------------------------
# separate operations

@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gather_matches_oracle(order, dtype):
    g = _grid(order=order)
    sp = random_species(g, 5000, 11, dtype=dtype)
    f = random_fields(g, 12, dtype=dtype)
    Ep, Bp = _lib.pic_gather(g, dev(sp), dev(f))
    torch.cuda.synchronize()
    oE, oB = oracle.gather(g, sp.numpy(), f.numpy())
    tol = F64_TOL if dtype == "f64" else 2e-6
    assert max_rel(_cpu(Ep), oE) < tol
    assert max_rel(_cpu(Bp), oB) < tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_push_matches_oracle(dtype):
    g = _grid()
    sp = random_species(g, 5000, 21, u_th=0.3, dtype=dtype)
    rng = np.random.default_rng(22)
    Ep = torch.tensor(rng.normal(0, 2.0, (3, 5000)), dtype=tdtype(dtype))
    Bp = torch.tensor(rng.normal(0, 5.0, (3, 5000)), dtype=tdtype(dtype))
    d_sp = dev(sp)
    _lib.pic_push(g, d_sp, dev(Ep), dev(Bp))
    torch.cuda.synchronize()
    o = sp.numpy()
    oracle.push(g, o, np.ascontiguousarray(_cpu(Ep)), np.ascontiguousarray(_cpu(Bp)))
    tol = F64_TOL if dtype == "f64" else 2e-6
    assert max_rel(_cpu(d_sp.u), o.u) < tol
    # positions: compare unwrapped (cell + offset) differences
    gx = d_sp.cell.cpu().numpy() + _cpu(d_sp.off)
    ox = o.cell + o.off
    dxy = np.abs(gx - ox)
    dxy = np.minimum(dxy, np.abs(dxy - np.array(g.n)[:, None]))
    assert dxy.max() < (1e-13 if dtype == "f64" else 2e-6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_push_offset_that_rounds_to_one_stays_in_the_cell(dtype):
    """Offset 0 moved by a tiny negative displacement: offset + 1 rounds to 1
    in the working precision, and the position update keeps the particle in
    its cell with offset 0 (FP64: the oracle's result bit for bit, including
    the representable case 1 - 2^-53 one cell down; FP32: the same point as
    the oracle's to 1e-7 of a cell, offsets in [0, 1))."""
    g = wl.plasma_grid((8, 8, 8), 3)
    disp = np.array([-1e-17, -2.0 ** -54, -2.0 ** -53, -1e-300, -1e-9, -2.0 ** -25])
    n = disp.size
    u = np.zeros((3, n))
    u[0] = disp * g.d[0] / g.dt
    sp = wl.Species(torch.full((3, n), 3, dtype=torch.int32), torch.zeros((3, n), dtype=torch.float64),
                    torch.tensor(u), None, 1.0).to(dtype=tdtype(dtype))
    d_sp = dev(sp)
    z = torch.zeros((3, n), dtype=tdtype(dtype), device="cuda")
    _lib.pic_push(g, d_sp, z, z)
    torch.cuda.synchronize()
    o = sp.numpy()
    zo = np.zeros((3, n))
    oracle.push(g, o, zo, zo)
    off = _cpu(d_sp.off)
    cell = d_sp.cell.cpu().numpy()
    assert np.all((off >= 0) & (off < 1))
    if dtype == "f64":
        assert np.array_equal(cell, o.cell)
        assert np.array_equal(off, o.off)
        assert list(cell[0, :4]) == [3, 3, 2, 3]
    else:
        x, ox = cell + off, o.cell + o.off
        assert np.abs(x - ox).max() < 1e-7
        assert list(cell[0, :2]) == [3, 3] and off[0, 0] == 0.0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vay_push_matches_oracle(dtype):
    """Vay's momentum update in strong fields (|q B dt / 2m| up to ~1): the
    oracle's Vay result within the tolerances of the Boris test, and far from
    what Boris gives on the same input (the grid's pusher field is honoured)."""
    g = dataclasses.replace(_grid(), pusher=1)
    sp = random_species(g, 5000, 23, u_th=0.8, dtype=dtype)
    rng = np.random.default_rng(24)
    Ep = torch.tensor(rng.normal(0, 2.0, (3, 5000)), dtype=tdtype(dtype))
    Bp = torch.tensor(rng.normal(0, 8.0, (3, 5000)), dtype=tdtype(dtype))
    d_sp = dev(sp)
    _lib.pic_push(g, d_sp, dev(Ep), dev(Bp))
    torch.cuda.synchronize()
    o = sp.numpy()
    E64, B64 = np.ascontiguousarray(_cpu(Ep)), np.ascontiguousarray(_cpu(Bp))
    oracle.push(g, o, E64, B64)
    tol = F64_TOL if dtype == "f64" else 2e-6
    assert max_rel(_cpu(d_sp.u), o.u) < tol
    ob = sp.numpy()
    oracle.push(dataclasses.replace(g, pusher=0), ob, E64, B64)
    assert max_rel(_cpu(d_sp.u), ob.u) > 1e-3


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vay_push_with_magnetic_rotation_beyond_gamma(dtype):
    """|q B dt / 2m| well above the new gamma (the quadratic's sigma < 0,
    where the root is taken in its cancellation-free form): still the
    oracle's result."""
    g = dataclasses.replace(_grid(), pusher=1)
    sp = random_species(g, 4000, 28, u_th=0.3, dtype=dtype)
    rng = np.random.default_rng(29)
    Ep = torch.tensor(rng.normal(0, 1.0, (3, 4000)), dtype=tdtype(dtype))
    Bp = torch.tensor(rng.normal(0, 200.0, (3, 4000)), dtype=tdtype(dtype))
    tau2 = (0.5 * g.dt) ** 2 * (Bp.double() ** 2).sum(0)
    d_sp = dev(sp)
    _lib.pic_push(g, d_sp, dev(Ep), dev(Bp))
    torch.cuda.synchronize()
    o = sp.numpy()
    oracle.push(g, o, np.ascontiguousarray(_cpu(Ep)), np.ascontiguousarray(_cpu(Bp)))
    gam = np.sqrt(1 + np.sum(o.u ** 2, axis=0))
    assert np.mean(tau2.numpy() > gam ** 2) > 0.9
    tol = F64_TOL if dtype == "f64" else 2e-6
    assert max_rel(_cpu(d_sp.u), o.u) < tol


def test_unknown_pusher_is_rejected():
    g = dataclasses.replace(_grid(), pusher=2)
    sp = dev(random_species(g, 10, 25))
    E = torch.zeros((3, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.PicError, match="pusher"):
        _lib.pic_push(g, sp, E, E)


def _displaced(g, sp, seed, amp=0.9):
    """Copy of sp moved by a random displacement below one cell."""
    rng = np.random.default_rng(seed)
    o = sp.numpy()
    xi = o.off + rng.uniform(-amp, amp, o.off.shape)
    k = np.floor(xi)
    off = xi - k
    off = np.where(off >= 1, 0.0, off)
    cell = (o.cell + k.astype(np.int32)) % np.array(g.n, dtype=np.int32)[:, None]
    after = wl.Species(torch.tensor(cell.astype(np.int32)), torch.tensor(off), sp.u.to(torch.float64),
                       None if sp.w is None else sp.w.to(torch.float64), sp.w0, sp.q, sp.m)
    return after.to(dtype=sp.off.dtype)


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_deposit_matches_oracle_and_conserves_charge(order, dtype):
    g = _grid(order=order)
    before = random_species(g, 4000, 31, dtype=dtype)
    after = _displaced(g, before, 32)
    f = random_fields(g, 33, dtype=dtype)
    f.J.zero_()
    df = dev(f)
    _lib.pic_deposit(g, dev(before), dev(after), df)
    torch.cuda.synchronize()
    of = f.numpy()
    ob, oa = before.numpy(), after.numpy()
    oracle.deposit(g, ob, oa, of)
    J = _cpu(df.J)
    assert rel_l2(J, of.J) < (F64_TOL if dtype == "f64" else 1e-5)
    # continuity with an FP64 charge density of the same positions
    rho0, rho1 = oracle.rho(g, ob), oracle.rho(g, oa)
    drho = (rho1 - rho0) / g.dt
    divJ = sum((J[m] - np.roll(J[m], 1, axis=2 - m)) / g.d[m] for m in range(3))
    assert np.linalg.norm(drho + divJ) / np.linalg.norm(drho) < (1e-13 if dtype == "f64" else 1e-6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_yee_matches_oracle_with_source(dtype):
    g = _grid((16, 12, 20))
    f = random_fields(g, 41, dtype=dtype, with_j=True)
    amp = torch.randn((12, 16), dtype=torch.float64, generator=torch.Generator().manual_seed(42))
    src = wl.Source(5, amp.to(tdtype(dtype)), np.array([0.3, -1.2, 0.7]))
    df = dev(f)
    for step in range(3):
        _lib.pic_yee(g, df, src.to(device="cuda"), step)
    torch.cuda.synchronize()
    of = f.numpy()
    osrc = src.numpy()
    for step in range(3):
        oracle.yee(g, of, osrc, step)
    tol = F64_TOL if dtype == "f64" else 1e-5
    assert rel_l2(_cpu(df.E), of.E) < tol
    assert rel_l2(_cpu(df.B), of.B) < tol
    assert np.array_equal(_cpu(df.J), of.J)   # J is read-only in pic_yee


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ckc_field_solve_matches_oracle(dtype):
    """CKC solver on unequal cells at c dt = 0.99 min d (beyond Yee's limit),
    with J and the plane source, several steps."""
    g = _grid((16, 12, 20))
    g = dataclasses.replace(g, d=(0.2, 0.25, 0.3), dt=0.99 * 0.2, solver=1)
    f = random_fields(g, 43, dtype=dtype, with_j=True)
    amp = torch.randn((12, 16), dtype=torch.float64, generator=torch.Generator().manual_seed(44))
    src = wl.Source(5, amp.to(tdtype(dtype)), np.array([0.3, -1.2, 0.7, 0.1]))
    df = dev(f)
    for step in range(4):
        _lib.pic_yee(g, df, src.to(device="cuda"), step)
    torch.cuda.synchronize()
    of = f.numpy()
    osrc = src.numpy()
    for step in range(4):
        oracle.yee(g, of, osrc, step)
    tol = F64_TOL if dtype == "f64" else 1e-5
    assert rel_l2(_cpu(df.E), of.E) < tol
    assert rel_l2(_cpu(df.B), of.B) < tol
    # the same fields (a fresh copy: numpy() views the tensors that the
    # oracle has just advanced) under Yee's stencil end far from this
    fy = random_fields(g, 43, dtype=dtype, with_j=True).numpy()
    for step in range(4):
        oracle.yee(dataclasses.replace(g, solver=0, dt=0.5 * 0.2), fy, osrc, step)
    assert rel_l2(of.B, fy.B) > 1e-2


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_reduce_matches_oracle(dtype):
    g = _grid()
    sp = random_species(g, 7000, 51, u_th=0.4, dtype=dtype)
    f = random_fields(g, 52, dtype=dtype)
    ws = _lib.workspace(g, dtype, sp.n)
    out = _lib.pic_reduce(g, dev(sp), dev(f), ws)
    torch.cuda.synchronize()
    want = oracle.reduce(g, sp.numpy(), f.numpy())
    np.testing.assert_allclose(out.cpu().numpy(), want, rtol=1e-13, atol=0)


# ---------------------------------------------------------------------------
# sort

def test_sort_tiles_is_a_binning_permutation():
    g = wl.plasma_grid((16, 24, 8), 3)
    sp = random_species(g, 20000, 61, dtype="f32")
    d = dev(sp)
    nt = _lib.pic_tile_count(g, "f32")
    ts = torch.empty(nt + 1, dtype=torch.int32, device="cuda")
    perm = torch.empty(sp.n, dtype=torch.int32, device="cuda")
    ws = _lib.workspace(g, "f32", sp.n)
    _lib.pic_sort_tiles(g, d, ts, ws, perm=perm)
    torch.cuda.synchronize()
    p = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(p), np.arange(sp.n))
    # data moved with the permutation
    assert torch.equal(d.cell.cpu(), sp.cell[:, p])
    assert torch.equal(d.off.cpu(), sp.off[:, p])
    assert torch.equal(d.u.cpu(), sp.u[:, p])
    assert torch.equal(d.w.cpu(), sp.w[p])
    # tiles are contiguous and in order; inside a tile the order is rank-major:
    # (occurrence of the particle's cell so far, local cell) strictly increases
    (tx, ty, tz), _ = _lib.pic_tile_shape(g, "f32")
    c = d.cell.cpu().numpy().astype(np.int64)
    tile = (c[0] // tx) + (g.n[0] // tx) * ((c[1] // ty) + (g.n[1] // ty) * (c[2] // tz))
    local = (c[0] % tx) + tx * ((c[1] % ty) + ty * (c[2] % tz))
    assert np.all(np.diff(tile) >= 0)
    seen = {}
    occ = np.empty(sp.n, dtype=np.int64)
    for j in range(sp.n):
        k = (tile[j], local[j])
        occ[j] = seen.get(k, 0)
        seen[k] = occ[j] + 1
    key2 = tile * (1 << 40) + occ * (1 << 20) + local
    assert np.all(np.diff(key2) > 0)
    hist = np.bincount(tile, minlength=nt)
    assert nt == (g.n[0] // tx) * (g.n[1] // ty) * (g.n[2] // tz)
    want = np.concatenate([[0], np.cumsum(hist)])
    assert np.array_equal(ts.cpu().numpy(), want)


def test_sort_rejects_corrupt_state_without_touching_it():
    g = wl.plasma_grid((16, 16, 16), 3)
    sp = random_species(g, 1000, 62, dtype="f64")
    sp.off[1, 17] = 1.0            # an offset outside [0,1)
    d = dev(sp)
    ts = torch.empty(_lib.pic_tile_count(g, "f64") + 1, dtype=torch.int32, device="cuda")
    ws = _lib.workspace(g, "f64", sp.n)
    with pytest.raises(_lib.PicError) as ei:
        _lib.pic_sort_tiles(g, d, ts, ws)
    assert ei.value.name == "PIC_E_STATE"
    assert torch.equal(d.off.cpu(), sp.off)


# ---------------------------------------------------------------------------
# full steps

def _run_gpu_steps(w, nsteps, sort_every, tiled=True, tile_start=None, diag=False):
    g = w.grid
    sp, f = dev(w.species), dev(w.fields)
    src = w.source.to(device="cuda") if w.source is not None else None
    ws = _lib.workspace(g, w.dtype, sp.n)
    ts = None
    if tiled:
        ts = tile_start if tile_start is not None else torch.zeros(_lib.pic_tile_count(g, w.dtype) + 1,
                                                                   dtype=torch.int32, device="cuda")
    dg = torch.zeros((nsteps, 5), dtype=torch.float64, device="cuda") if diag else None
    _lib.pic_step(g, sp, f, src, 0, nsteps, sort_every, ts, ws, dg)
    torch.cuda.synchronize()
    return sp, f, dg


def _run_oracle(w, nsteps):
    sp, f = w.species.numpy(), w.fields.numpy()
    src = w.source.numpy() if w.source is not None else None
    diag = oracle.step(w.grid, sp, f, src, 0, nsteps)
    return sp, f, diag


def test_uniform32_order1_f64_ten_steps_matches_oracle():
    """32^3 periodic uniform plasma, 8 ppc, u_th = 0.01c, CIC, FP64, 10 steps,
    sorted every 4 steps: fields and the particle set within 1e-12."""
    w = wl.named("uniform32_o1_f64")
    gsp, gf, gdiag = _run_gpu_steps(w, w.nsteps, w.sort_every, diag=True)
    osp, of, odiag = _run_oracle(w, w.nsteps)
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < F64_TOL, name
    gt, ot = particle_table(gsp), particle_table(osp)
    assert np.array_equal(gt[:, :3], ot[:, :3])
    assert rel_l2(gt[:, 3:6], ot[:, 3:6]) < F64_TOL
    assert rel_l2(gt[:, 6:], ot[:, 6:]) < F64_TOL
    np.testing.assert_allclose(gdiag.cpu().numpy(), odiag, rtol=1e-10)


@pytest.mark.parametrize("sort_every", [1, 3])
def test_order3_tiled_f64_matches_oracle(sort_every):
    """Order 3 with a random initial field: tiles of 8 with a ragged grid
    (24 = 3 tiles, 20 -> tile 5), several sorts, LDS and fallback paths."""
    w = wl.uniform_plasma((16, 24, 20), 3, 0.1, 3, 6, "f64", 71, sort_every, shuffle=True)
    f0 = random_fields(w.grid, 72, scale=0.05)
    w.fields = f0
    gsp, gf, _ = _run_gpu_steps(w, w.nsteps, sort_every)
    osp, of, _ = _run_oracle(w, w.nsteps)
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < F64_TOL, name
    gt, ot = particle_table(gsp), particle_table(osp)
    assert np.array_equal(gt[:, :3], ot[:, :3])
    assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_per_cell_deposit_at_8ppc_matches_oracle(dtype, order):
    """8 particles per cell (at order 3 in FP32 the tile step sums the
    current of the particles that stay in their cells per cell, two threads
    per cell; the other cases take the one-pass kernel), random initial fields, u_th = 0.1c so that some particles
    cross cells every step, a ragged grid (20 -> tiles of 5), sorts every 4
    steps (FP64: 5 steps, fields and particles within 1e-12; FP32: one step,
    E, B, J within rel-L2 1e-5 and charge conservation within 1e-6 with rho
    in FP64)."""
    nsteps = 5 if dtype == "f64" else 1
    w = wl.uniform_plasma((16, 24, 20), 8, 0.1, order, nsteps, dtype, 97, 4, shuffle=True)
    w.fields = random_fields(w.grid, 98, scale=0.05, dtype=dtype)
    before = w.species.numpy()
    gsp, gf, _ = _run_gpu_steps(w, nsteps, 4)
    osp, of, _ = _run_oracle(w, nsteps)
    tol = F64_TOL if dtype == "f64" else 1e-5
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < tol, name
    if dtype == "f64":
        gt, ot = particle_table(gsp), particle_table(osp)
        assert np.array_equal(gt[:, :3], ot[:, :3])
        assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL
    else:
        g = w.grid
        drho = (oracle.rho(g, gsp.numpy()) - oracle.rho(g, before)) / g.dt
        J = _cpu(gf.J)
        divJ = sum((J[m] - np.roll(J[m], 1, axis=2 - m)) / g.d[m] for m in range(3))
        assert np.linalg.norm(drho + divJ) / np.linalg.norm(drho) < 1e-6


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vay_steps_match_oracle(dtype):
    """Relativistic plasma (u_th = 0.5c) in strong random fields, order 3,
    Vay's pusher, tiled with re-sorting (FP64: 4 steps, fields and particles
    within 1e-12; FP32: one step, E, B, J within rel-L2 1e-5)."""
    nsteps = 4 if dtype == "f64" else 1
    w = wl.uniform_plasma((16, 24, 20), 3, 0.5, 3, nsteps, dtype, 75, 2, shuffle=True)
    w.grid = dataclasses.replace(w.grid, pusher=1)
    w.fields = random_fields(w.grid, 76, scale=0.5, dtype=dtype)
    gsp, gf, _ = _run_gpu_steps(w, nsteps, 2)
    osp, of, _ = _run_oracle(w, nsteps)
    tol = F64_TOL if dtype == "f64" else 1e-5
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < tol, name
    if dtype == "f64":
        gt, ot = particle_table(gsp), particle_table(osp)
        assert np.array_equal(gt[:, :3], ot[:, :3])
        assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_accelerator_stage_options_steps_match_oracle(dtype):
    """The field and push options of the paper's accelerator stage together:
    Vay's pusher and the CKC solver at c dt = 0.95 min d, order-3 shapes,
    relativistic particles in strong fields, tiled with re-sorting (FP64:
    3 steps, fields and particles within 1e-12; FP32: one step, E, B, J
    within rel-L2 1e-5)."""
    nsteps = 3 if dtype == "f64" else 1
    w = wl.uniform_plasma((16, 24, 20), 3, 0.5, 3, nsteps, dtype, 77, 2, shuffle=True)
    dmin = min(w.grid.d)
    w.grid = dataclasses.replace(w.grid, pusher=1, solver=1, dt=0.95 * dmin / w.grid.c)
    w.fields = random_fields(w.grid, 78, scale=0.5, dtype=dtype)
    gsp, gf, _ = _run_gpu_steps(w, nsteps, 2)
    osp, of, _ = _run_oracle(w, nsteps)
    tol = F64_TOL if dtype == "f64" else 1e-5
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < tol, name
    if dtype == "f64":
        gt, ot = particle_table(gsp), particle_table(osp)
        assert np.array_equal(gt[:, :3], ot[:, :3])
        assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL


GATHER_TAPS = np.array([[0.5, 0.25, 0.0, 0.0], [0.6, 0.25, -0.05, 0.0], [0.4, 0.2, 0.1, 0.0],
                        [0.7, 0.1, 0.05, 0.0], [0.55, 0.2, 0.05, -0.025], [0.5, 0.15, 0.05, 0.05]])


@pytest.mark.parametrize("tiled", [True, False])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gather_filter_steps_match_oracle(dtype, tiled):
    """Vay + CKC + a z filter of E and B before the gather (per-component
    taps up to three cells away), tiled with re-sorting or per particle
    (FP64: 3 steps within 1e-12; FP32: one step within rel-L2 1e-5)."""
    nsteps = 3 if dtype == "f64" else 1
    w = wl.uniform_plasma((16, 24, 20), 3, 0.3, 3, nsteps, dtype, 79, 2 if tiled else 0, shuffle=True)
    dmin = min(w.grid.d)
    w.grid = dataclasses.replace(w.grid, pusher=1, solver=1, dt=0.9 * dmin / w.grid.c, gather_filter=GATHER_TAPS)
    w.fields = random_fields(w.grid, 80, scale=0.5, dtype=dtype)
    gsp, gf, _ = _run_gpu_steps(w, nsteps, 2 if tiled else 0, tiled=tiled)
    osp, of, _ = _run_oracle(w, nsteps)
    tol = F64_TOL if dtype == "f64" else 1e-5
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < tol, name
    if dtype == "f64":
        gt, ot = particle_table(gsp), particle_table(osp)
        assert np.array_equal(gt[:, :3], ot[:, :3])
        assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL
    # the filter changes the result
    w2 = wl.uniform_plasma((16, 24, 20), 3, 0.3, 3, nsteps, dtype, 79, 2 if tiled else 0, shuffle=True)
    w2.grid = dataclasses.replace(w.grid, gather_filter=None)
    w2.fields = random_fields(w.grid, 80, scale=0.5, dtype=dtype)
    _, of2, _ = _run_oracle(w2, nsteps)
    assert rel_l2(of2.J, of.J) > 1e-3


def test_gather_refuses_a_filter():
    g = dataclasses.replace(_grid(), gather_filter=GATHER_TAPS)
    sp = dev(random_species(g, 10, 26))
    f = dev(random_fields(g, 27))
    with pytest.raises(_lib.PicError, match="filter"):
        _lib.pic_gather(g, sp, f)


@pytest.mark.parametrize("tiled", [True, False])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_smallest_grid_with_every_option_matches_oracle(dtype, tiled):
    """4 x 5 x 7 cells, the smallest the library takes along x: the LDS
    regions of a tile (10 cells and more with the halo), the CKC blocks and
    the z filter all wrap around the periodic box more than once.  Vay, CKC
    at 0.95 min d, the filter, order 3 (FP64: 3 steps within 1e-12; FP32:
    one step within rel-L2 1e-5)."""
    nsteps = 3 if dtype == "f64" else 1
    w = wl.uniform_plasma((4, 5, 7), 4, 0.3, 3, nsteps, dtype, 85, 1 if tiled else 0, shuffle=True)
    dmin = min(w.grid.d)
    w.grid = dataclasses.replace(w.grid, pusher=1, solver=1, dt=0.95 * dmin / w.grid.c, gather_filter=GATHER_TAPS)
    w.fields = random_fields(w.grid, 86, scale=0.5, dtype=dtype)
    gsp, gf, _ = _run_gpu_steps(w, nsteps, 1 if tiled else 0, tiled=tiled)
    osp, of, _ = _run_oracle(w, nsteps)
    tol = F64_TOL if dtype == "f64" else 1e-5
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < tol, name
    if dtype == "f64":
        gt, ot = particle_table(gsp), particle_table(osp)
        assert np.array_equal(gt[:, :3], ot[:, :3])
        assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL


def test_untiled_step_matches_oracle_particle_by_particle():
    w = wl.uniform_plasma((16, 16, 16), 2, 0.1, 3, 4, "f64", 73, 0, shuffle=True)
    w.fields = random_fields(w.grid, 74, scale=0.05)
    gsp, gf, _ = _run_gpu_steps(w, w.nsteps, 0, tiled=False)
    osp, of, _ = _run_oracle(w, w.nsteps)
    assert np.array_equal(gsp.cell.cpu().numpy(), osp.cell)
    assert max_rel(_cpu(gsp.off), osp.off) < 1e-13
    assert max_rel(_cpu(gsp.u), osp.u) < F64_TOL
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < F64_TOL, name


def test_stale_binning_uses_the_fallback_path_correctly():
    """Sort once, then step many times without re-sorting at a high thermal
    speed: particles leave their tile's LDS region and are moved as guests of
    the tile that holds their cell (or, the first step after the sort, on the
    global path)."""
    w = wl.uniform_plasma((16, 16, 16), 2, 0.3, 3, 8, "f64", 75, 0, shuffle=True)
    g = w.grid
    sp = dev(w.species)
    ts = torch.zeros(_lib.pic_tile_count(g, "f64") + 1, dtype=torch.int32, device="cuda")
    ws = _lib.workspace(g, "f64", sp.n)
    _lib.pic_sort_tiles(g, sp, ts, ws)
    torch.cuda.synchronize()
    w2 = wl.Workload(w.name, g, wl.Species(sp.cell.cpu(), sp.off.cpu(), sp.u.cpu(), None, sp.w0, sp.q, sp.m),
                     w.fields, None, 8, 0, "f64", 75)
    gsp, gf, _ = _run_gpu_steps(w2, 8, 0, tiled=True, tile_start=ts)
    osp, of, _ = _run_oracle(w2, 8)
    assert np.array_equal(gsp.cell.cpu().numpy(), osp.cell)
    assert max_rel(_cpu(gsp.u), osp.u) < F64_TOL
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < F64_TOL, name


def test_step_rejects_a_binning_that_does_not_span_the_particles():
    """sort_every = 0 with a tile_start that was never filled (all zeros)
    would leave every tile empty: the call fails before any launch."""
    g = _grid()
    sp, f = dev(random_species(g, 1000, 91)), dev(random_fields(g, 92))
    E0 = f.E.clone()
    ts = torch.zeros(_lib.pic_tile_count(g, "f64") + 1, dtype=torch.int32, device="cuda")
    ws = _lib.workspace(g, "f64", sp.n)
    with pytest.raises(_lib.PicError) as ei:
        _lib.pic_step(g, sp, f, None, 0, 1, 0, ts, ws)
    assert ei.value.name == "PIC_E_INVALID"
    assert torch.equal(f.E, E0)


def test_f32_split_precision_one_step_bounds():
    """FP32 fields/momenta with int32 cell + FP32 offset: rel-L2 of E, B, J
    <= 1e-5 after one step against the oracle started from the same FP32
    state, and charge-conservation residual <= 1e-6 with rho in FP64."""
    w = wl.uniform_plasma((32, 32, 32), 8, 0.05, 3, 1, "f32", 81, 1)
    w.fields = random_fields(w.grid, 82, scale=0.02, dtype="f32")
    before = w.species.numpy()
    gsp, gf, _ = _run_gpu_steps(w, 1, 1)
    osp, of, _ = _run_oracle(w, 1)
    for name in ("E", "B", "J"):
        r = rel_l2(_cpu(getattr(gf, name)), getattr(of, name))
        assert r < 1e-5, (name, r)
    g = w.grid
    after = gsp.numpy()
    rho0, rho1 = oracle.rho(g, before), oracle.rho(g, after)
    drho = (rho1 - rho0) / g.dt
    J = _cpu(gf.J)
    divJ = sum((J[m] - np.roll(J[m], 1, axis=2 - m)) / g.d[m] for m in range(3))
    res = np.linalg.norm(drho + divJ) / np.linalg.norm(drho)
    assert res < 1e-6, res


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dense_hot_tiles_overflow_the_crossing_queue(dtype):
    """64 ppc at u_th = 0.9c on 16^3: tens of thousands of particles per tile,
    most of them crossing a cell face each step, far more than the tile
    kernel's LDS queue holds, so the overflow deposits inline.  FP64 within
    1e-12 over two steps (sorted every step); FP32 within 1e-5 after one step
    with the charge-conservation residual <= 1e-6."""
    nsteps = 2 if dtype == "f64" else 1
    w = wl.uniform_plasma((16, 16, 16), 64, 0.9, 3, nsteps, dtype, 83, 1)
    before = w.species.numpy()
    gsp, gf, _ = _run_gpu_steps(w, nsteps, 1)
    osp, of, _ = _run_oracle(w, nsteps)
    tol = F64_TOL if dtype == "f64" else 1e-5
    for name in ("E", "B", "J"):
        r = rel_l2(_cpu(getattr(gf, name)), getattr(of, name))
        assert r < tol, (name, r)
    if dtype == "f64":
        gt, ot = particle_table(gsp), particle_table(osp)
        assert np.array_equal(gt[:, :3], ot[:, :3])
        assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL
    else:
        g = w.grid
        rho0, rho1 = oracle.rho(g, before), oracle.rho(g, gsp.numpy())
        drho = (rho1 - rho0) / g.dt
        J = _cpu(gf.J)
        divJ = sum((J[m] - np.roll(J[m], 1, axis=2 - m)) / g.d[m] for m in range(3))
        assert np.linalg.norm(drho + divJ) / np.linalg.norm(drho) < 1e-6


def test_guest_lists_overflow_to_the_stray_path():
    """64 ppc at u_th = 0.9c on 16^3, sorted once and then stepped without
    re-sorting: thousands of particles per tile leave their home region each
    step, more than a tile's guest list holds, so the rest take the stray
    kernel.  FP64 within 1e-12 over three steps."""
    w = wl.uniform_plasma((16, 16, 16), 64, 0.9, 3, 3, "f64", 87, 0)
    g = w.grid
    sp = dev(w.species)
    ts = torch.zeros(_lib.pic_tile_count(g, "f64") + 1, dtype=torch.int32, device="cuda")
    ws = _lib.workspace(g, "f64", sp.n)
    _lib.pic_sort_tiles(g, sp, ts, ws)
    torch.cuda.synchronize()
    w2 = wl.Workload(w.name, g, wl.Species(sp.cell.cpu(), sp.off.cpu(), sp.u.cpu(), None, sp.w0, sp.q, sp.m),
                     w.fields, None, 3, 0, "f64", 87)
    gsp, gf, _ = _run_gpu_steps(w2, 3, 0, tiled=True, tile_start=ts)
    osp, of, _ = _run_oracle(w2, 3)
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < F64_TOL, name
    assert np.array_equal(gsp.cell.cpu().numpy(), osp.cell)
    assert max_rel(_cpu(gsp.u), osp.u) < F64_TOL
    assert max_rel(_cpu(gsp.off), osp.off) < 1e-13


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_guests_across_a_sort_inside_one_call(dtype):
    """Sorting every 10 steps turns the guest lists on: 12 steps in one call
    at u_th = 0.3c build and read lists on steps 1-9, drop them at the sort
    on step 10 (which renumbers the particles) and build them again there
    for step 11.  FP64 within 1e-12; FP32 within rel-L2 1e-4 after the same
    12 steps (fields) against the oracle started from the same state: the
    one-step bound 1e-5 accumulated over 12 steps, at most linearly on a
    horizon of 3.6 / omega_p (the FP32 tolerance readings of the design)."""
    w = wl.uniform_plasma((16, 16, 24), 2, 0.3, 3, 12, dtype, 89, 10, shuffle=True)
    w.fields = random_fields(w.grid, 90, scale=0.05, dtype=dtype)
    gsp, gf, _ = _run_gpu_steps(w, 12, 10)
    osp, of, _ = _run_oracle(w, 12)
    tol = F64_TOL if dtype == "f64" else 1e-4
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < tol, name
    if dtype == "f64":
        gt, ot = particle_table(gsp), particle_table(osp)
        assert np.array_equal(gt[:, :3], ot[:, :3])
        assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL


def test_guests_that_step_back_home_on_many_tiles():
    """Regression test of the in-place guest step: a particle listed as a
    guest of another tile must be skipped by its home tile even when the host
    tile has already moved it back inside the home region.  64^3 FP64 order 3
    (8x8x4 tiles, 1024 of them, so a tile and its lower z neighbour run 512
    workgroups apart), 1 ppc at u_th = 0.4c gyrating in a uniform B_x = 3
    (gyro-diameter ~2.4 cells across z), sorted at the first step only
    (sort_every 20) and stepped 12 times in one call.  The oracle's
    trajectory shows thousands of particles re-entering their home region
    from outside; the GPU state matches the oracle within 1e-12."""
    n = (64, 64, 64)
    w = wl.uniform_plasma(n, 1, 0.4, 3, 12, "f64", 95, 20, shuffle=True)
    w.fields.B[0].fill_(3.0)
    g = w.grid
    tile, slack = _lib.pic_tile_shape(g, "f64")
    assert tuple(tile) == (8, 8, 4) and slack == 1
    gsp, gf, _ = _run_gpu_steps(w, 12, 20)
    # the oracle one step at a time, counting re-entries into the home region
    # (home: the tile of the cell at the sort of step 0)
    osp, of = w.species.numpy(), w.fields.numpy()
    t = np.array(tile)[:, None]
    nn = np.array(n)[:, None]
    t0 = (osp.cell // t) * t

    def inside(cell):
        v = cell - t0
        v = np.where(v < -slack, v + nn, np.where(v >= t + slack, v - nn, v))
        return np.all((v >= -slack) & (v < t + slack), axis=0)

    prev, back = inside(osp.cell), 0
    for s in range(12):
        oracle.step(g, osp, of, None, s, 1)
        cur = inside(osp.cell)
        back += int(np.sum(~prev & cur))
        prev = cur
    assert back > 1000, back
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < F64_TOL, name
    gt, ot = particle_table(gsp), particle_table(osp)
    assert np.array_equal(gt[:, :3], ot[:, :3])
    assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL


def test_resort_of_a_tile_holding_over_a_million_particles():
    """The re-sort's counting pass packs each particle's region cell and
    local rank into one word while a tile's segment holds at most 2^20
    particles (8^3 tiles: 2^11 region cells); beyond that it keeps the rank
    alone and reads the cell again.  One fixed 8^3 tile holding 1,100,000
    particles (FP64, order 3), two steps with a sort at each (the second a
    re-sort of the binned particles), against the oracle within 1e-12."""
    w = wl.uniform_plasma((8, 8, 8), 2149, 0.02, 3, 2, "f64", 97, 1)
    w.grid.tile = (8, 8, 8)
    assert w.species.n > (1 << 20)
    assert _lib.pic_tile_count(w.grid, "f64") == 1
    gsp, gf, _ = _run_gpu_steps(w, 2, 1)
    osp, of, _ = _run_oracle(w, 2)
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < F64_TOL, name
    gt, ot = particle_table(gsp), particle_table(osp)
    assert np.array_equal(gt[:, :3], ot[:, :3])
    assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL


def test_regions_that_wrap_more_than_once_with_two_cells_of_slack():
    """A 4-cell axis with two cells of slack: the current region (4 + 2 * 2 +
    5 = 13 cells) wraps the axis more than once, so the tile kernels' region
    walks take the general wrap; order 3, FP64, six steps sorted every 3,
    against the oracle within 1e-12."""
    w = wl.uniform_plasma((4, 8, 12), 6, 0.1, 3, 6, "f64", 98, 3)
    w.grid.slack = 2
    tile, slack = _lib.pic_tile_shape(w.grid, "f64")
    assert slack == 2 and tile[0] == 4
    gsp, gf, _ = _run_gpu_steps(w, w.nsteps, w.sort_every)
    osp, of, _ = _run_oracle(w, w.nsteps)
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < F64_TOL, name
    gt, ot = particle_table(gsp), particle_table(osp)
    assert np.array_equal(gt[:, :3], ot[:, :3])
    assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL


def test_laser_plasma_reduced_with_empty_tiles_and_source():
    """Laser workload shape at reduced size: vacuum tiles without particles,
    a density up-ramp with per-particle weights, the soft source."""
    w = wl.laser_plasma((16, 16, 96), 2, 3, 40, "f64", 91, 4, ramp=(32, 60), k_source=2, cells_per_lambda=16,
                        width_lambda=4.0)
    gsp, gf, _ = _run_gpu_steps(w, w.nsteps, w.sort_every)
    osp, of, _ = _run_oracle(w, w.nsteps)
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < F64_TOL, name
    gt, ot = particle_table(gsp), particle_table(osp)
    assert np.array_equal(gt[:, :3], ot[:, :3])
    assert rel_l2(gt[:, 3:], ot[:, 3:]) < F64_TOL


def test_zero_particles_and_edge_offsets():
    g = wl.plasma_grid((8, 8, 8), 3)
    # no particles: the step is a pure field solve
    empty = wl.Species(torch.zeros((3, 0), dtype=torch.int32), torch.zeros((3, 0), dtype=torch.float64),
                       torch.zeros((3, 0), dtype=torch.float64), None, 1.0)
    f = random_fields(g, 92)
    w = wl.Workload("empty", g, empty, f, None, 2, 1, "f64", 0)
    _, gf, _ = _run_gpu_steps(w, 2, 1)
    _, of, _ = _run_oracle(w, 2)
    assert rel_l2(_cpu(gf.E), of.E) < F64_TOL
    # offsets at 0 and just below 1, crossing the periodic seam
    n = 6
    cell = torch.tensor([[0, 7, 7, 0, 3, 7], [0, 7, 0, 7, 3, 7], [7, 0, 7, 0, 3, 7]], dtype=torch.int32)
    one_m = float(np.nextafter(1.0, 0.0))
    off = torch.tensor([[0.0, one_m, one_m, 0.0, 0.5, one_m]] * 3, dtype=torch.float64)
    u = torch.tensor([[-0.5, 0.5, 0.5, -0.5, 0.0, 0.9], [0.4, 0.3, -0.4, 0.2, 0.0, 0.1],
                      [0.1, -0.2, 0.3, -0.6, 0.0, 0.2]], dtype=torch.float64)
    sp = wl.Species(cell, off, u, None, 0.3)
    w = wl.Workload("edges", g, sp, random_fields(g, 93), None, 3, 1, "f64", 0)
    gsp, gf, _ = _run_gpu_steps(w, 3, 1)
    osp, of, _ = _run_oracle(w, 3)
    for name in ("E", "B", "J"):
        assert rel_l2(_cpu(getattr(gf, name)), getattr(of, name)) < F64_TOL, name
    gt, ot = particle_table(gsp), particle_table(osp)
    assert np.array_equal(gt[:, :3], ot[:, :3])
    assert np.abs(gt[:, 3:] - ot[:, 3:]).max() < 1e-13


def test_corrupt_momentum_reports_state_error():
    w = wl.uniform_plasma((8, 8, 8), 1, 0.05, 3, 1, "f64", 94, 1)
    w.species.u[0, 5] = float("nan")
    with pytest.raises(_lib.PicError) as ei:
        _run_gpu_steps(w, 1, 1)
    assert ei.value.name == "PIC_E_STATE"


def test_unit_calls_report_corrupt_state():
    """pic_gather, pic_push and pic_deposit read their device error word back:
    a corrupt particle gives PIC_E_STATE, the other particles are processed,
    and the next clean call returns OK (the word is cleared per call)."""
    g = _grid()
    sp = random_species(g, 2000, 31, u_th=0.2)
    f = random_fields(g, 32)
    bad = sp.clone()
    bad.cell[1, 7] = int(g.n[1])            # cell outside the grid
    d_bad, d_f = dev(bad), dev(f)
    Ep = torch.zeros((3, sp.n), dtype=torch.float64, device="cuda")
    Bp = torch.zeros_like(Ep)
    with pytest.raises(_lib.PicError) as ei:
        _lib.pic_gather(g, d_bad, d_f, Ep, Bp)
    assert ei.value.name == "PIC_E_STATE"
    oE, oB = oracle.gather(g, sp.numpy(), f.numpy())
    keep = np.arange(sp.n) != 7
    assert max_rel(_cpu(Ep)[:, keep], oE[:, keep]) < F64_TOL
    assert np.all(_cpu(Ep)[:, 7] == 0.0) and np.all(_cpu(Bp)[:, 7] == 0.0)
    _lib.pic_gather(g, dev(sp), d_f, Ep, Bp)   # clean call after an error: OK
    # push: a non-finite momentum leaves that particle unchanged
    nanp = sp.clone()
    nanp.u[2, 11] = float("nan")
    d_nan = dev(nanp)
    with pytest.raises(_lib.PicError) as ei:
        _lib.pic_push(g, d_nan, Ep, Bp)
    assert ei.value.name == "PIC_E_STATE"
    assert torch.equal(d_nan.cell[:, 11].cpu(), nanp.cell[:, 11])
    o = sp.numpy()
    oracle.push(g, o, np.ascontiguousarray(_cpu(Ep)), np.ascontiguousarray(_cpu(Bp)))
    keep = np.arange(sp.n) != 11
    assert max_rel(_cpu(d_nan.u)[:, keep], o.u[:, keep]) < F64_TOL
    # deposit: a particle that moved two cells deposits nothing
    before = sp.clone()
    after = sp.clone()
    after.cell[0, 3] = (after.cell[0, 3] + 2) % int(g.n[0])
    fj = dev(wl.Fields.zeros(g))
    with pytest.raises(_lib.PicError) as ei:
        _lib.pic_deposit(g, dev(before), dev(after), fj)
    assert ei.value.name == "PIC_E_STATE"
    keep = torch.arange(sp.n) != 3
    b2 = wl.Species(before.cell[:, keep].contiguous(), before.off[:, keep].contiguous(),
                    before.u[:, keep].contiguous(), before.w[keep].contiguous(), before.w0)
    a2 = wl.Species(after.cell[:, keep].contiguous(), after.off[:, keep].contiguous(),
                    after.u[:, keep].contiguous(), after.w[keep].contiguous(), after.w0)
    of = wl.Fields.zeros(g).numpy()
    oracle.deposit(g, b2.numpy(), a2.numpy(), of)
    assert rel_l2(_cpu(fj.J), of.J) < F64_TOL
