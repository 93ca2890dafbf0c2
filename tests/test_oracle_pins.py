"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test targets a plausible mistake: a wrong shape polynomial, a wrong
staggering, a sign error in the curl or the current, a missing factor in the
Esirkepov coefficient, a wrong Boris rotation angle.  None of them re-types
an oracle formula: they check closed forms, invariants, brute force and
textbook values.
"""
import dataclasses
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2101_12149_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class NS:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def grid(n=(8, 8, 8), d=(0.3, 0.25, 0.35), dt=0.05, order=3):
    return NS(n=n, d=d, dt=dt, c=1.0, eps0=1.0, order=order)


def species(cell, off, u, w=None, w0=1.0, q=-1.0, m=1.0):
    return NS(cell=np.ascontiguousarray(cell, dtype=np.int32), off=np.ascontiguousarray(off, dtype=np.float64),
              u=np.ascontiguousarray(u, dtype=np.float64), w=w, w0=w0, q=q, m=m)


def zero_fields(g):
    shape = (3, g.n[2], g.n[1], g.n[0])
    return NS(E=np.zeros(shape), B=np.zeros(shape), J=np.zeros(shape))


def random_species(g, n, rng, u_scale=0.1):
    cell = np.stack([rng.integers(0, g.n[d], n) for d in range(3)])
    off = rng.random((3, n))
    u = rng.normal(0, u_scale, (3, n))
    return species(cell, off, u, w=rng.random(n) + 0.5)


# --------------------------------------------------------------------------
# shapes

def test_bspline_golden_values():
    path = os.path.join(GOLDEN, "bspline_values.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 10
    for order, r, frac in rows:
        want = float(Fraction(frac))
        got = oracle.shape(int(order), float(r))
        assert abs(got - want) < 1e-15, (order, r, got, want)


@pytest.mark.parametrize("order", [1, 3])
def test_shape_partition_of_unity_and_first_moment(order):
    rng = np.random.default_rng(1)
    for x in rng.random(200) * 10 - 5:
        nodes = np.arange(math.floor(x) - 3, math.floor(x) + 4)
        s = oracle.shape(order, x - nodes)
        assert abs(s.sum() - 1.0) < 1e-14
        assert abs((s * nodes).sum() - x) < 1e-13     # linear reproduction


@pytest.mark.parametrize("order", [1, 3])
def test_shape_is_convolution_of_boxes(order):
    """S_order = box * box * ... (order+1 boxes); brute-force quadrature of the
    repeated convolution on a fine grid."""
    h = 1.0 / 2000
    xs = np.arange(-0.5 + h / 2, 0.5, h)      # midpoint samples of the unit box
    dens = np.ones_like(xs) * h
    conv = dens.copy()
    for _ in range(order):
        conv = np.convolve(conv, dens)
    # the support of the (order+1)-fold convolution, centred
    grid_x = (np.arange(conv.size) - (conv.size - 1) / 2) * h
    pdf = conv / h
    for r in [-1.7, -1.2, -0.6, 0.0, 0.3, 0.9, 1.4, 1.95]:
        want = np.interp(r, grid_x, pdf, left=0.0, right=0.0)
        assert abs(oracle.shape(order, r) - want) < 2e-5, (order, r)


@pytest.mark.parametrize("order", [1, 3])
def test_dshape_matches_central_difference(order):
    rng = np.random.default_rng(2)
    eps = 1e-6
    for r in rng.random(100) * 4.4 - 2.2:
        if order == 1 and min(abs(r - k) for k in (-1, 0, 1)) < 1e-3:
            continue
        fd = (oracle.shape(order, r + eps) - oracle.shape(order, r - eps)) / (2 * eps)
        assert abs(oracle.dshape(order, r) - fd) < 1e-8


# --------------------------------------------------------------------------
# gather

STAG_E = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5)]
STAG_B = [(0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]


def _linear_field(g, coef, stag):
    nz, ny, nx = g.n[2], g.n[1], g.n[0]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = (i + stag[0]) * g.d[0]
    y = (j + stag[1]) * g.d[1]
    z = (k + stag[2]) * g.d[2]
    return coef[0] + coef[1] * x + coef[2] * y + coef[3] * z


@pytest.mark.parametrize("order", [1, 3])
def test_gather_reproduces_uniform_and_linear_fields(order):
    """B-splines reproduce linear functions, so a linear field sampled at its
    staggered points is gathered exactly, for every component (a wrong
    staggering offset or a transposed weight fails this)."""
    g = grid(n=(16, 16, 16), order=order)
    rng = np.random.default_rng(3)
    # keep particles away from the periodic seam where the field is not linear
    n = 300
    cell = np.stack([rng.integers(4, 12, n) for _ in range(3)])
    sp = species(cell, rng.random((3, n)), np.zeros((3, n)))
    f = zero_fields(g)
    coefs = []
    for m in range(3):
        ce = rng.normal(size=4)
        cb = rng.normal(size=4)
        f.E[m] = _linear_field(g, ce, STAG_E[m])
        f.B[m] = _linear_field(g, cb, STAG_B[m])
        coefs.append((ce, cb))
    Ep, Bp = oracle.gather(g, sp, f)
    xp = (sp.cell + sp.off) * np.array(g.d)[:, None]
    for m in range(3):
        ce, cb = coefs[m]
        want_e = ce[0] + ce[1] * xp[0] + ce[2] * xp[1] + ce[3] * xp[2]
        want_b = cb[0] + cb[1] * xp[0] + cb[2] * xp[1] + cb[3] * xp[2]
        np.testing.assert_allclose(Ep[m], want_e, rtol=0, atol=1e-12)
        np.testing.assert_allclose(Bp[m], want_b, rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# Boris + position

def _unwrapped(cell_hist, off_hist, n, d):
    """Unwrap a periodic trajectory of one particle (cell units -> length)."""
    x = []
    acc = cell_hist[0] + off_hist[0]
    x.append(acc.copy())
    for a in range(1, len(cell_hist)):
        step = (cell_hist[a] - cell_hist[a - 1]) + (off_hist[a] - off_hist[a - 1])
        step = np.where(step > n / 2, step - n, step)
        step = np.where(step < -n / 2, step + n, step)
        acc = acc + step
        x.append(acc.copy())
    return np.array(x) * np.array(d)


def _run_uniform(g, E, B, u0, nsteps, cell0=(4, 4, 4), off0=(0.5, 0.5, 0.5)):
    f = zero_fields(g)
    for m in range(3):
        f.E[m][...] = E[m]
        f.B[m][...] = B[m]
    sp = species(np.array(cell0)[:, None], np.array(off0)[:, None], np.array(u0, dtype=float)[:, None])
    us, cells, offs = [sp.u[:, 0].copy()], [sp.cell[:, 0].copy()], [sp.off[:, 0].copy()]
    for _ in range(nsteps):
        Ep, Bp = oracle.gather(g, sp, f)
        oracle.push(g, sp, Ep, Bp)
        us.append(sp.u[:, 0].copy())
        cells.append(sp.cell[:, 0].copy())
        offs.append(sp.off[:, 0].copy())
    return np.array(us), _unwrapped(cells, offs, np.array(g.n), g.d)


def test_boris_uniform_E_is_exact_and_converges_to_hyperbolic_motion():
    """Uniform E, B = 0: u^{n+1/2} = u^{n-1/2} + (q/m) E dt exactly, and the
    position converges at second order to the hyperbolic trajectory
    x(t) = (c^2/a) (sqrt(1 + (a t / c)^2) - 1)."""
    qm, Ex = -1.0, -0.8          # electron accelerated along +x, a = 0.8
    a = qm * Ex
    T = 3.0
    errs = []
    for nst in (30, 60, 120):
        dt = T / nst
        g = grid(n=(64, 8, 8), d=(0.2, 0.2, 0.2), dt=dt)
        u0 = (-0.5 * a * dt, 0.0, 0.0)   # u(0) = 0, staggered back by dt/2
        us, xs = _run_uniform(g, (Ex, 0, 0), (0, 0, 0), u0, nst)
        n = np.arange(nst + 1)
        np.testing.assert_allclose(us[:, 0], u0[0] + a * dt * n, rtol=0, atol=1e-13)
        assert np.all(us[:, 1:] == 0)
        x_exact = (1.0 / a) * (math.sqrt(1 + (a * T) ** 2) - 1)
        errs.append(abs((xs[-1, 0] - xs[0, 0]) - x_exact))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.05)


def test_boris_uniform_B_energy_angle_and_gyroradius():
    """Uniform B, E = 0: |u| and gamma are invariant, each step rotates u by
    2 atan(omega_c dt / 2), and the positions lie on a circle of radius
    r_L sqrt(1 + (omega_c dt/2)^2)."""
    g = grid(n=(64, 64, 8), d=(0.1, 0.1, 0.1), dt=0.3)
    Bz = 2.0
    u0 = (0.5, 0.0, 0.0)
    us, xs = _run_uniform(g, (0, 0, 0), (0, 0, Bz), u0, 60, cell0=(32, 32, 4))
    umag = np.linalg.norm(us, axis=1)
    np.testing.assert_allclose(umag, 0.5, rtol=1e-14)
    gam = math.sqrt(1 + 0.25)
    wc = abs(-1.0) * Bz / (1.0 * gam)
    theta = 2 * math.atan(wc * g.dt / 2)
    ang = np.arctan2(us[1:, 1], us[1:, 0]) - np.arctan2(us[:-1, 1], us[:-1, 0])
    ang = (ang + np.pi) % (2 * np.pi) - np.pi
    np.testing.assert_allclose(np.abs(ang), theta, rtol=1e-12)
    # circumcentre of three vertices, then every vertex at radius R
    p = xs[:, :2]
    (ax, ay), (bx, by), (cx, cy) = p[0], p[5], p[11]
    dd = 2 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    ux = ((ax ** 2 + ay ** 2) * (by - cy) + (bx ** 2 + by ** 2) * (cy - ay) + (cx ** 2 + cy ** 2) * (ay - by)) / dd
    uy = ((ax ** 2 + ay ** 2) * (cx - bx) + (bx ** 2 + by ** 2) * (ax - cx) + (cx ** 2 + cy ** 2) * (bx - ax)) / dd
    r = np.hypot(p[:, 0] - ux, p[:, 1] - uy)
    v = 0.5 / gam
    R = (v / wc) * math.sqrt(1 + (wc * g.dt / 2) ** 2)
    np.testing.assert_allclose(r, R, rtol=1e-11)
    assert np.ptp(xs[:, 2]) == 0


def _push_once(g, u0, E, B, q=-1.0):
    """Momentum after one push of particles at rest in the middle of a large
    cell (positions do not matter here); u0, E, B are (3, N)."""
    n = u0.shape[1]
    sp = species(np.full((3, n), 1), np.full((3, n), 0.5), np.array(u0, dtype=float), q=q)
    oracle.push(g, sp, np.ascontiguousarray(E, dtype=float), np.ascontiguousarray(B, dtype=float))
    return sp.u


def _tiny_moves(g, disp):
    """Particles at offset 0 of cell 3 (all axes) moved by the given tiny
    displacements (cell units) along x: E = B = 0, u chosen so that
    dt u / (gamma d_x) is disp (gamma = 1 to rounding at these speeds)."""
    disp = np.asarray(disp, dtype=float)
    n = disp.size
    u = np.zeros((3, n))
    u[0] = disp * g.d[0] / g.dt
    sp = species(np.full((3, n), 3), np.zeros((3, n)), u)
    z = np.zeros((3, n))
    oracle.push(g, sp, z, z)
    return sp


def test_position_update_offset_that_rounds_to_one_moves_to_the_next_cell():
    """A position just below a cell face seen from the cell above: offset 0
    moved by -1e-17 or by -2^-54 gives xi + 1 that rounds to exactly 1 in
    FP64 (the second a tie, rounded to even), so the offset would be 1; the
    update keeps the particle in its cell with offset 0 (the same point to
    rounding).  At -2^-53 the sum 1 - 2^-53 is representable: the particle
    moves down one cell with that offset.  The offset stays in [0, 1)."""
    g = grid(n=(8, 8, 8), d=(0.3, 0.25, 0.35), dt=0.05)
    sp = _tiny_moves(g, [-1e-17, -2.0 ** -54, -2.0 ** -53, -1e-300])
    assert np.all((sp.off >= 0) & (sp.off < 1))
    assert list(sp.cell[0]) == [3, 3, 2, 3]
    assert sp.off[0, 0] == 0.0 and sp.off[0, 1] == 0.0 and sp.off[0, 3] == 0.0
    assert sp.off[0, 2] == 1.0 - 2.0 ** -53
    assert np.all(sp.cell[1:] == 3) and np.all(sp.off[1:] == 0.0)


def _vay_grid(dt, pusher=1):
    g = grid(n=(4, 4, 4), d=(1e3, 1e3, 1e3), dt=dt)
    g.pusher = pusher
    return g


def test_vay_reduces_to_boris_without_magnetic_or_electric_field():
    """With B = 0 both pushers are the plain kick u0 + (q/m) E dt; with E = 0
    the mean-velocity force of Vay's pusher is the implicit-midpoint rotation
    by the tangent-half-angle vector, the same map as Boris's rotation."""
    rng = np.random.default_rng(21)
    n = 64
    u0 = rng.normal(0, 2.0, (3, n))
    E = rng.normal(0, 1.0, (3, n))
    B = rng.normal(0, 3.0, (3, n))
    Z = np.zeros((3, n))
    dt = 0.4
    kick = u0 + (-1.0) * E * dt
    np.testing.assert_allclose(_push_once(_vay_grid(dt), u0, E, Z), kick, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(_push_once(_vay_grid(dt), u0, Z, B), _push_once(_vay_grid(dt, 0), u0, Z, B),
                               rtol=1e-13, atol=1e-13)


def test_vay_keeps_the_force_free_drift_exactly():
    """E = -v x B makes the Lorentz force vanish: a particle moving with v
    keeps its momentum.  Vay's pusher reproduces this for any dt and gamma
    (the property it was designed for); Boris's half kicks do not."""
    rng = np.random.default_rng(22)
    n = 64
    v = rng.normal(0, 1.0, (3, n))
    v *= rng.uniform(0.5, 0.995, n) / np.linalg.norm(v, axis=0)
    gam = 1.0 / np.sqrt(1.0 - np.sum(v * v, axis=0))
    u0 = gam * v
    B = rng.normal(0, 2.0, (3, n))
    E = -np.cross(v, B, axis=0)
    dt = 0.5
    u_vay = _push_once(_vay_grid(dt), u0, E, B)
    np.testing.assert_allclose(u_vay, u0, rtol=0, atol=1e-12 * np.max(np.abs(u0)))
    u_boris = _push_once(_vay_grid(dt, 0), u0, E, B)
    assert np.max(np.abs(u_boris - u0)) > 1e-2


def test_vay_solves_its_implicit_equation():
    """The result satisfies the defining equation
    u1 - u0 = (q dt/m) E + (q dt/2m) (u0/gamma0 + u1/gamma1) x B
    to rounding, also where |q B dt / 2m| exceeds the new gamma (the
    quadratic's coefficient sigma is negative there)."""
    rng = np.random.default_rng(23)
    n = 200
    u0 = rng.normal(0, 1.5, (3, n))
    E = rng.normal(0, 2.0, (3, n))
    B = rng.normal(0, 1.0, (3, n)) * rng.choice([0.1, 1.0, 30.0], n)
    dt = 0.6
    u1 = _push_once(_vay_grid(dt), u0, E, B)
    h = -1.0 * dt / 2
    g0 = np.sqrt(1 + np.sum(u0 * u0, axis=0))
    g1 = np.sqrt(1 + np.sum(u1 * u1, axis=0))
    res = u1 - u0 - 2 * h * E - h * np.cross(u0 / g0 + u1 / g1, B, axis=0)
    scale = np.abs(u0) + np.abs(u1) + np.abs(2 * h * E) + np.abs(h) * np.linalg.norm(B, axis=0) * 2
    assert np.max(np.abs(res) / scale) < 1e-13
    tau2 = h * h * np.sum(B * B, axis=0)
    assert np.any(tau2 > g1 ** 2)   # the sigma < 0 branch was taken


# --------------------------------------------------------------------------
# Esirkepov

def _div_edges(g, J):
    """Backward-difference divergence of an edge vector field (nodes)."""
    out = np.zeros(J.shape[1:])
    for m, ax in ((0, 2), (1, 1), (2, 0)):
        out += (J[m] - np.roll(J[m], 1, axis=ax)) / g.d[m]
    return out


@pytest.mark.parametrize("order", [1, 3])
def test_esirkepov_discrete_continuity_and_total_current(order):
    g = grid(n=(8, 8, 8), order=order)
    rng = np.random.default_rng(4)
    before = random_species(g, 200, rng)
    after = species(before.cell.copy(), before.off.copy(), before.u, w=before.w)
    disp = rng.uniform(-0.9, 0.9, (3, 200))
    xi = before.off + disp
    k = np.floor(xi)
    after.off[:] = xi - k
    after.cell[:] = (before.cell + k.astype(np.int32)) % np.array(g.n)[:, None]
    f = zero_fields(g)
    oracle.deposit(g, before, after, f)
    rho0 = oracle.rho(g, before)
    rho1 = oracle.rho(g, after)
    res = (rho1 - rho0) / g.dt + _div_edges(g, f.J)
    assert np.abs(res).max() < 1e-12 * np.abs((rho1 - rho0) / g.dt).max()
    # total current = sum q w v
    dV = np.prod(g.d)
    for m in range(3):
        want = np.sum(before.q * before.w * disp[m] * g.d[m] / g.dt)
        assert abs(f.J[m].sum() * dV - want) < 1e-12 * abs(want) + 1e-13


def test_esirkepov_stationary_and_one_dimensional_motion():
    g = grid(order=3)
    rng = np.random.default_rng(5)
    sp = random_species(g, 50, rng)
    f = zero_fields(g)
    oracle.deposit(g, sp, sp, f)
    assert np.all(f.J == 0)
    after = species(sp.cell.copy(), sp.off.copy(), sp.u, w=sp.w)
    after.off[0] = np.clip(sp.off[0] + 0.3, 0, 0.999)
    f = zero_fields(g)
    oracle.deposit(g, sp, after, f)
    assert np.abs(f.J[0]).max() > 0
    assert np.all(f.J[1] == 0) and np.all(f.J[2] == 0)


# --------------------------------------------------------------------------
# Yee

def _mode(g, kvec, amp, stag, phase=0.0):
    nz, ny, nx = g.n[2], g.n[1], g.n[0]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = (i + stag[0]) * g.d[0]
    y = (j + stag[1]) * g.d[1]
    z = (k + stag[2]) * g.d[2]
    return amp * np.cos(kvec[0] * x + kvec[1] * y + kvec[2] * z - phase)


def test_yee_discrete_plane_wave_eigenmode():
    """A plane wave with K_d = (2/dx_d) sin(k_d dx_d / 2) and
    sin(omega dt/2) = (c dt/2)|K| is an exact eigenmode of the staggered
    leapfrog: E^n = E cos(k.x - omega t_n), B^n = cos(omega dt/2) (K x E / W)
    cos(k.x - omega t_n) with W = 2 sin(omega dt/2)/dt."""
    g = grid(n=(16, 12, 20), d=(0.2, 0.25, 0.15), dt=0.08)
    L = np.array(g.n) * np.array(g.d)
    kvec = 2 * np.pi * np.array([2, -1, 3]) / L
    K = 2 / np.array(g.d) * np.sin(kvec * np.array(g.d) / 2)
    E0 = np.cross(K, [0.3, 1.0, -0.4])
    E0 /= np.linalg.norm(E0)
    assert abs(E0 @ K) < 1e-12
    s = g.c * g.dt * np.linalg.norm(K) / 2
    omega = 2 * math.asin(s) / g.dt
    W = 2 * math.sin(omega * g.dt / 2) / g.dt
    B0 = np.cross(K, E0) / W * math.cos(omega * g.dt / 2)
    f = zero_fields(g)
    for m in range(3):
        f.E[m] = _mode(g, kvec, E0[m], STAG_E[m])
        f.B[m] = _mode(g, kvec, B0[m], STAG_B[m])
    nst = 40
    for n in range(nst):
        oracle.yee(g, f, None, n)
    t = nst * g.dt
    for m in range(3):
        np.testing.assert_allclose(f.E[m], _mode(g, kvec, E0[m], STAG_E[m], omega * t), atol=1e-12)
        np.testing.assert_allclose(f.B[m], _mode(g, kvec, B0[m], STAG_B[m], omega * t), atol=1e-12)
    # the wrong dispersion (continuous omega = c|k|) is far off
    assert abs(omega - np.linalg.norm(kvec)) * t > 1e-3


def _ckc_grid(d, dt=None):
    g = grid(n=(8, 8, 8), d=d, dt=dt if dt is not None else 0.5 * min(d))
    g.solver = 1
    return g


def test_ckc_coefficients_for_cubic_cells_are_the_published_values():
    """The oracle's own CKC weights for cubic cells are the published ones
    (Cole; Karkkainen et al.): centre 7/12, each edge neighbour 1/12, each
    corner 1/48, for the differences along every axis."""
    for d in ((0.2, 0.2, 0.2), (1.0, 1.0, 1.0)):
        co = oracle.ckc_coeffs(_ckc_grid(d))
        for a in range(3):
            assert tuple(co[a]) == pytest.approx((7 / 12, 1 / 12, 1 / 12, 1 / 48), rel=1e-14, abs=1e-16)


def _ckc_symbol(co, kd):
    """Transverse average of the difference along each axis for the wave
    vector kd = k * d (per axis), from the given weights."""
    A = []
    for a in range(3):
        p, q = (a + 1) % 3, (a + 2) % 3
        al, bp, bq, gm = co[a]
        A.append(al + 2 * bp * np.cos(kd[p]) + 2 * bq * np.cos(kd[q]) + 4 * gm * np.cos(kd[p]) * np.cos(kd[q]))
    return A


@pytest.mark.parametrize("d", [(0.2, 0.25, 0.3), (0.3, 0.2, 0.25), (0.1, 0.3, 0.3), (0.5, 1.0, 1.0)])
def test_ckc_coefficients_make_the_smallest_cell_the_exact_stability_limit(d):
    """What the CKC weights are built for, on unequal cells: they sum to one
    per axis (a transversely uniform difference is unchanged), and at
    c dt = min d the amplification symbol (c dt)^2 sum_a sin^2(k_a d_a/2)
    A_a(k) / d_a^2 stays at or below 1 over the whole Brillouin zone and
    reaches 1 (marginal stability: c dt = min d is the exact limit).  Weights
    with the two edge neighbours swapped, or the corner term's S dependence
    dropped, exceed 1 (by 5-26 %) on these cells."""
    co = oracle.ckc_coeffs(_ckc_grid(d))
    for a in range(3):
        assert co[a][0] + 2 * co[a][1] + 2 * co[a][2] + 4 * co[a][3] == pytest.approx(1.0, abs=1e-15)
    dl = min(d)
    k = np.linspace(0.0, np.pi, 65)
    kd = np.meshgrid(k, k, k, indexing="ij")
    A = _ckc_symbol(co, kd)
    amp = sum((dl / d[a]) ** 2 * np.sin(kd[a] / 2) ** 2 * A[a] for a in range(3))
    assert amp.max() <= 1.0 + 1e-12
    assert amp.max() >= 1.0 - 1e-12
    assert amp.min() >= -1e-15


def _ckc_eigenmode(g, kvec, co, nst=40):
    """Propagate the discrete CKC eigenmode for wave vector kvec with the
    oracle's field solve and compare with its analytic phase; co gives the
    weights of the expected dispersion."""
    dd = np.array(g.d)
    K = 2 / dd * np.sin(kvec * dd / 2)
    A = np.array(_ckc_symbol(co, kvec * dd))
    Kp = K * A
    E0 = np.cross(K, [0.3, 1.0, -0.4])
    E0 /= np.linalg.norm(E0)
    s = g.c * g.dt * math.sqrt(K @ Kp) / 2
    assert s < 1
    omega = 2 * math.asin(s) / g.dt
    W = 2 * math.sin(omega * g.dt / 2) / g.dt
    B0 = np.cross(Kp, E0) / W * math.cos(omega * g.dt / 2)
    f = zero_fields(g)
    for m in range(3):
        f.E[m] = _mode(g, kvec, E0[m], STAG_E[m])
        f.B[m] = _mode(g, kvec, B0[m], STAG_B[m])
    for n in range(nst):
        oracle.yee(g, f, None, n)
    t = nst * g.dt
    for m in range(3):
        np.testing.assert_allclose(f.E[m], _mode(g, kvec, E0[m], STAG_E[m], omega * t), atol=1e-12)
        np.testing.assert_allclose(f.B[m], _mode(g, kvec, B0[m], STAG_B[m], omega * t), atol=1e-12)
    omega_yee = 2 * math.asin(g.c * g.dt * np.linalg.norm(K) / 2) / g.dt
    return omega, omega_yee, t


def test_ckc_discrete_plane_wave_eigenmode_cubic_cells():
    """Cubic cells, with the expected dispersion from the published weights
    7/12, 1/12, 1/48 (not from the oracle): the difference along a carries
    the transverse average A_a(k) = alpha + 2 beta (cos k_p d + cos k_q d)
    + 4 gamma cos k_p d cos k_q d, so a divergence-free E0 with
    B0 = cos(omega dt/2) (K' x E0 / W), K'_a = K_a A_a, is an eigenmode with
    sin(omega dt/2) = (c dt/2) sqrt(K . K'), at c dt = 0.9 d (beyond Yee's
    limit d/sqrt(3)); Yee's frequency for the same k is far off."""
    g = grid(n=(16, 12, 20), d=(0.2, 0.2, 0.2), dt=0.9 * 0.2)
    g.solver = 1
    L = np.array(g.n) * np.array(g.d)
    kvec = 2 * np.pi * np.array([3, -2, 4]) / L
    co = [(7 / 12, 1 / 12, 1 / 12, 1 / 48)] * 3
    omega, omega_yee, t = _ckc_eigenmode(g, kvec, co)
    assert abs(omega - omega_yee) * t > 1e-2


def test_ckc_discrete_plane_wave_eigenmode_unequal_cells():
    """The same eigenmode on unequal cells with the oracle's weights (held by
    the stability-limit test above): the field solve applies each weight to
    the right neighbours of the right difference."""
    g = grid(n=(16, 12, 20), d=(0.2, 0.25, 0.15), dt=0.12)
    g.solver = 1
    L = np.array(g.n) * np.array(g.d)
    kvec = 2 * np.pi * np.array([3, -2, 4]) / L
    omega, omega_yee, t = _ckc_eigenmode(g, kvec, oracle.ckc_coeffs(g))
    assert abs(omega - omega_yee) * t > 1e-2


def test_ckc_axis_wave_has_no_dispersion_at_the_magic_time_step():
    """Along the axis with the smallest cell and c dt equal to that cell, a
    wave of any wavelength moves at exactly c (the transverse average of a
    transversely uniform wave is the identity: the coefficients sum to 1)."""
    g = grid(n=(16, 8, 8), d=(0.2, 0.25, 0.3), dt=0.2)
    g.solver = 1
    for kx in (1, 5, 7):
        kvec = np.array([2 * np.pi * kx / (16 * 0.2), 0.0, 0.0])
        E0 = np.array([0.0, 1.0, 0.0])
        omega = np.linalg.norm(kvec)      # exact, c = 1
        W = 2 * math.sin(omega * g.dt / 2) / g.dt
        K = np.array([2 / 0.2 * math.sin(kvec[0] * 0.2 / 2), 0, 0])
        B0 = np.cross(K, E0) / W * math.cos(omega * g.dt / 2)
        f = zero_fields(g)
        for m in range(3):
            f.E[m] = _mode(g, kvec, E0[m], STAG_E[m])
            f.B[m] = _mode(g, kvec, B0[m], STAG_B[m])
        for n in range(24):
            oracle.yee(g, f, None, n)
        np.testing.assert_allclose(f.E[1], _mode(g, kvec, 1.0, STAG_E[1], omega * 24 * g.dt), atol=1e-12)


def _energy_after(g, nsteps, seed):
    f = zero_fields(g)
    rng = np.random.default_rng(seed)
    f.E[:] = rng.normal(size=f.E.shape)
    f.B[:] = rng.normal(size=f.B.shape)
    e0 = np.sum(f.E ** 2) + np.sum(f.B ** 2)
    for n in range(nsteps):
        oracle.yee(g, f, None, n)
    return (np.sum(f.E ** 2) + np.sum(f.B ** 2)) / e0


def test_ckc_is_stable_up_to_the_smallest_cell_and_yee_is_not():
    """The CKC step is stable up to c dt = min d (its extended stencil makes
    the highest mode exactly marginal there), unstable just beyond; Yee's
    limit is 1/sqrt(sum 1/d^2), well below.  Near the limit the plain field
    energy of random fields oscillates by several times (the leapfrog keeps
    a modified energy), so "stable" is a bound far below the growth."""
    d = (0.3, 0.25, 0.35)
    ckc_ok = grid(n=(8, 8, 8), d=d, dt=0.995 * 0.25)
    ckc_ok.solver = 1
    assert _energy_after(ckc_ok, 400, 31) < 20
    ckc_bad = grid(n=(8, 8, 8), d=d, dt=1.03 * 0.25)
    ckc_bad.solver = 1
    assert _energy_after(ckc_bad, 60, 31) > 1e6
    yee = grid(n=(8, 8, 8), d=d, dt=0.995 * 0.25)
    assert _energy_after(yee, 60, 31) > 1e6


FILTER_TAPS = np.array([[0.5, 0.25, 0.0, 0.0], [0.6, 0.25, -0.05, 0.0], [0.4, 0.2, 0.1, 0.0],
                        [0.7, 0.1, 0.05, 0.0], [0.55, 0.2, 0.05, -0.025], [0.5, 0.15, 0.05, 0.05]])


def test_gather_filter_identity_taps_change_nothing():
    g = grid(n=(8, 6, 10))
    rng = np.random.default_rng(41)
    f = zero_fields(g)
    f.E[:] = rng.normal(size=f.E.shape)
    f.B[:] = rng.normal(size=f.B.shape)
    sp = random_species(g, 200, rng)
    E0, B0 = oracle.gather(g, sp, f)
    g.gather_filter = np.tile([1.0, 0.0, 0.0, 0.0], (6, 1))
    E1, B1 = oracle.gather(g, sp, f)
    assert np.array_equal(E0, E1) and np.array_equal(B0, B1)


def test_gather_filter_transfer_function_on_a_z_mode():
    """Fields that vary only along z as cos(2 pi q k / n_z) are eigenfunctions
    of a symmetric z stencil: the filtered gather is the plain one times
    H(q) = w0 + 2 sum_s w_s cos(2 pi q s / n_z), per component."""
    g = grid(n=(6, 6, 16))
    nz = g.n[2]
    q = 3
    f = zero_fields(g)
    kz = np.arange(nz)
    mode = np.cos(2 * np.pi * q * kz / nz + 0.4)[:, None, None] * np.ones((nz, g.n[1], g.n[0]))
    for m in range(3):
        f.E[m] = mode * (m + 1)
        f.B[m] = mode * (m - 2.5)
    rng = np.random.default_rng(42)
    sp = random_species(g, 100, rng)
    E0, B0 = oracle.gather(g, sp, f)
    g.gather_filter = FILTER_TAPS
    E1, B1 = oracle.gather(g, sp, f)
    H = FILTER_TAPS[:, 0] + 2 * sum(FILTER_TAPS[:, s] * np.cos(2 * np.pi * q * s / nz) for s in (1, 2, 3))
    for m in range(3):
        np.testing.assert_allclose(E1[m], H[m] * E0[m], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(B1[m], H[3 + m] * B0[m], rtol=1e-12, atol=1e-13)
    assert np.ptp(H) > 0.1      # the components really are filtered differently


def test_yee_source_adds_on_plane_and_keeps_divB():
    g = grid(n=(8, 8, 8))
    f = zero_fields(g)
    amp = np.random.default_rng(6).normal(size=(8, 8))
    src = NS(k_plane=3, amp=amp, g=np.array([0.0, 2.0]))
    oracle.yee(g, f, src, 1)
    # after one step from zero the source plane carries 2*amp before the last B half-step
    assert np.allclose(f.E[0][3], 2 * amp)
    assert np.all(f.E[0][np.arange(8) != 3] == 0)
    divB = ((np.roll(f.B[0], -1, 2) - f.B[0]) / g.d[0] + (np.roll(f.B[1], -1, 1) - f.B[1]) / g.d[1]
            + (np.roll(f.B[2], -1, 0) - f.B[2]) / g.d[2])
    assert np.abs(divB).max() < 1e-13


# --------------------------------------------------------------------------
# full step

def test_laser_source_radiates_a0_after_the_discrete_dispersion_correction():
    """The laser workload's soft source in vacuum (a plane wave: its waist
    made huge) radiates a pulse of peak amplitude a0 m c omega_L / |q| (= a0
    in these units) each way.  For a sheet that adds S g(n) to E_x every
    step, the discrete Yee wave equation gives the exact ratio of radiated to
    continuum amplitude 1 / cos(kappa dz / 2), with kappa from
    sin(omega dt / 2) = (c dt / dz) sin(kappa dz / 2) (about 1.02 at 16
    cells per wavelength).  The envelope peaks (analytic signal of E_x along
    z) of the forward and the backward pulse match a0 / cos(kappa dz / 2)
    within 0.2 %, and differ from the uncorrected a0 by more than 1 %."""
    from scipy.signal import hilbert
    nz, nsteps, a0 = 1536, 650, 2.0
    w = wl.laser_plasma((4, 4, nz), ppc=2, order=3, nsteps=nsteps, dtype="f64", ramp=(nz, nz), k_source=2,
                        waist_lambda=1e7, a0=a0)
    assert w.species.n == 0
    g = w.grid
    f, src = w.fields.numpy(), w.source.numpy()
    for n in range(nsteps):
        oracle.yee(g, f, src, n)
    env = np.abs(hilbert(f.E[0][:, 0, 0]))
    omega = 1.0   # the workload's laser frequency (omega_L = 1)
    dz, dt = g.d[2], g.dt
    kappa = 2 * math.asin(dz / (g.c * dt) * math.sin(omega * dt / 2)) / dz
    want = a0 / math.cos(kappa * dz / 2)
    fwd, bwd = env[: nz // 2].max(), env[nz // 2:].max()
    assert abs(fwd / want - 1) < 2e-3 and abs(bwd / want - 1) < 2e-3, (fwd, bwd, want)
    assert abs(fwd / a0 - 1) > 1e-2
    # the transverse field is uniform (a plane wave) and only E_x, B_y carry it
    assert np.allclose(f.E[0], f.E[0][:, :1, :1], atol=1e-12)
    assert np.abs(f.E[1]).max() < 1e-12 and np.abs(f.E[2]).max() < 1e-12


def test_full_step_gauss_residual_is_invariant():
    """Esirkepov's current and the Yee update keep div E - rho/eps0 fixed
    node by node (no Poisson solve: the initial residual is thermal noise)."""
    w = wl.uniform_plasma((8, 8, 8), 2, 0.05, 3, 4, "f64", 77)
    g = w.grid
    sp, f = w.species.numpy(), w.fields.numpy()
    r0, s0 = oracle.gauss(g, sp, f)
    assert np.abs(r0).max() > 1e-3
    for n in range(4):
        oracle.step(g, sp, f, None, n, 1)
        r, s = oracle.gauss(g, sp, f)
        np.testing.assert_allclose(r, r0, rtol=0, atol=1e-12 * np.abs(r0).max())
        assert abs(s[0] - s0[0]) < 1e-12 * s0[0]


def test_gauss_residual_of_a_lattice_potential_and_of_one_particle():
    """Without particles, E = -grad phi on the edges of a cosine mode phi
    gives div E = sum_d K_d^2 phi with K_d = (2/d_d) sin(k_d d_d/2), the
    discrete Laplacian's eigenvalue (a wrong sign, index or axis in the
    divergence fails); with E = 0 and one particle, the residual is minus
    its nodal density over eps0 less the mean, which sums to zero, and the
    species' charge is q w (partition of unity)."""
    g = grid(n=(8, 10, 12), order=3)
    k = [2 * math.pi * m / (n * d) for m, n, d in zip((1, 2, 3), g.n, g.d)]
    z, y, x = np.meshgrid(*(np.arange(n) * d for n, d in zip(g.n[::-1], g.d[::-1])), indexing="ij")
    phi = np.cos(k[0] * x + k[1] * y + k[2] * z)
    f = zero_fields(g)
    for m, ax in ((0, 2), (1, 1), (2, 0)):
        f.E[m] = -(np.roll(phi, -1, axis=ax) - phi) / g.d[m]
    none = species(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros((3, 0)))
    res, out = oracle.gauss(g, none, f)
    lam = sum((2.0 / d * math.sin(kd * d / 2)) ** 2 for kd, d in zip(k, g.d))
    np.testing.assert_allclose(res, lam * phi, rtol=0, atol=1e-12 * lam)
    assert abs(out[0] - lam * np.linalg.norm(phi)) < 1e-12 * out[0] and out[1] == 0 and out[2] == 0
    one = species([[3], [4], [5]], [[0.3], [0.6], [0.9]], np.zeros((3, 1)), w=np.array([2.5]), q=-1.5)
    res, out = oracle.gauss(g, one, zero_fields(g))
    dV = float(np.prod(g.d))
    assert abs(out[2] - (-1.5 * 2.5)) < 1e-14
    assert abs(res.sum()) < 1e-12 * np.abs(res).max()
    # the particle's own node (3, 4, 5) carries S(0.3) S(0.6) S(0.9)
    s3 = oracle.shape(3, 0.3) * oracle.shape(3, 0.6) * oracle.shape(3, 0.9)
    rt = ((-1.5 * 2.5 / dV) * s3 - (-1.5 * 2.5 / dV) / res.size) / g.eps0
    assert abs(res[5, 4, 3] + rt) < 1e-12 * abs(rt)


def test_step_does_not_depend_on_the_thread_count_beyond_rounding():
    """The oracle's parallel loops (particles split over threads, private
    current buffers summed afterwards) give the same step on 1 and on 4
    threads up to the summation order of the buffers: a race or a lost
    buffer would show as an O(1) difference."""
    outs = []
    nt0 = oracle.num_threads()
    try:
        for nt in (1, 4):
            oracle.set_num_threads(nt)
            w = wl.uniform_plasma((8, 8, 8), 4, 0.05, 3, 3, "f64", 91)
            sp, f = w.species.numpy(), w.fields.numpy()
            oracle.step(w.grid, sp, f, None, 0, 3)
            outs.append((sp.cell.copy(), sp.off.copy(), sp.u.copy(), f.E.copy(), f.B.copy(), f.J.copy()))
    finally:
        oracle.set_num_threads(nt0)
    (c1, o1, u1, E1, B1, J1), (c4, o4, u4, E4, B4, J4) = outs
    np.testing.assert_array_equal(c1, c4)
    for a, b in ((o1, o4), (u1, u4), (E1, E4), (B1, B4), (J1, J4)):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(a).max())


def test_cold_plasma_oscillation_frequency():
    """Regular cold plasma, all electrons given the same tiny velocity: J and E
    stay uniform and E obeys the leapfrog oscillator
    E^{n+1} + E^{n-1} = (2 - omega_p^2 dt^2) E^n, omega_p^2 = n0 q^2/(eps0 m)."""
    n = (4, 4, 4)
    ppc = 1
    g0 = wl.plasma_grid(n, 3)
    g = NS(n=n, d=g0.d, dt=g0.dt, c=1.0, eps0=1.0, order=3)
    N = 64
    cell = wl.uniform_cells(n, ppc).numpy()
    off = np.full((3, N), 0.3)
    u = np.zeros((3, N))
    u[0] = 1e-5      # small enough that gamma-1 ~ 5e-11, large enough that
                     # offset rounding (1e-16) is tiny against the step (6e-6)
    dV = np.prod(g.d)
    n0 = 1.0
    sp = species(cell, off, u, w0=n0 * dV / ppc)
    f = zero_fields(g)
    Ex = []
    for it in range(40):
        oracle.step(g, sp, f, None, it, 1)
        assert np.ptp(f.E[0]) < 1e-12 * np.abs(f.E[0]).max()
        Ex.append(f.E[0].mean())
    Ex = np.array(Ex)
    lhs = Ex[2:] + Ex[:-2]
    rhs = (2 - (n0 * g.dt ** 2)) * Ex[1:-1]
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-9 * np.abs(Ex).max())


def test_reductions_closed_forms():
    g = grid(n=(4, 4, 4))
    f = zero_fields(g)
    f.E[0][:] = 2.0
    f.B[2][:] = 3.0
    u = np.array([[0.0, 3.0 / 4.0], [0.0, 0.0], [0.0, 0.0]])
    sp = species(np.zeros((3, 2)), np.zeros((3, 2)), u, w=np.array([1.0, 2.0]))
    out = oracle.reduce(g, sp, f)
    dV = np.prod(g.d)
    assert out[0] == pytest.approx(0.5 * dV * 64 * 4.0, rel=1e-14)
    assert out[1] == pytest.approx(0.5 * dV * 64 * 9.0, rel=1e-14)
    assert out[2] == pytest.approx(2.0 * (1.25 - 1.0), rel=1e-14)   # gamma = 5/4
    assert out[3] == pytest.approx(-3.0, rel=1e-14)
    assert out[4] == 0.0


# --------------------------------------------------------------------------
# adjoint

@pytest.mark.parametrize("solver", [0, 1])
def test_adjoint_field_solve_dot_product(solver):
    """With no particles the step is linear in (E, B): <M x, y> = <x, M^T y>
    (Yee, and CKC whose B update carries the transverse average)."""
    g = grid(n=(6, 5, 7))
    g.solver = solver
    rng = np.random.default_rng(8)
    f = zero_fields(g)
    f.E[:] = rng.normal(size=f.E.shape)
    f.B[:] = rng.normal(size=f.B.shape)
    x = (f.E.copy(), f.B.copy())
    oracle.yee(g, f, None, 0)
    lam = oracle.Adjoint(g, 0)
    lam.lE[:] = rng.normal(size=lam.lE.shape)
    lam.lB[:] = rng.normal(size=lam.lB.shape)
    y = (lam.lE.copy(), lam.lB.copy())
    empty = species(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros((3, 0)))
    oracle.step_adjoint(g, empty, zero_fields(g), None, 0, lam, None)
    lhs = np.sum(f.E * y[0]) + np.sum(f.B * y[1])
    rhs = np.sum(x[0] * lam.lE) + np.sum(x[1] * lam.lB)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _rollout_loss(g, sp, f, src, nsteps):
    s = oracle._copy_species(sp)
    ff = oracle._copy_fields(f)
    oracle.step(g, s, ff, src, 0, nsteps)
    L, _ = oracle.loss(g, ff, 0)
    return L


def _fd_tol(an, L, eps):
    """1e-6 relative, plus the rounding noise of a central difference of a
    loss of size L (a few ulps of L divided by eps)."""
    return 1e-6 * abs(an) + 10 * np.finfo(float).eps * abs(L) / eps


@pytest.mark.parametrize("pusher", [0, 1])
@pytest.mark.parametrize("order", [3])
def test_adjoint_matches_central_finite_differences(order, pusher):
    """Gradient of the final field energy w.r.t. the initial momenta and the
    source amplitude map, against central differences with eps = 1e-6 along
    seeded random directions and single coordinates.  Fields start at zero,
    so the loss is made by the particles' own currents and the source and
    every checked derivative is far above the difference's rounding noise."""
    w = wl.differentiable((8, 8, 8), 1, 0.05, order, 3, "f64", 1234, amp0=2e-2, period=4)
    g = dataclasses.replace(w.grid, pusher=pusher)
    sp, f, src = w.species.numpy(), w.fields.numpy(), w.source.numpy()
    rng = np.random.default_rng(9)
    L, gu, gA, _, _ = oracle.rollout_grad(g, sp, f, src, 0, w.nsteps)
    eps = 1e-6
    checks = []
    for t in range(4):
        v = rng.normal(size=sp.u.shape)
        v /= np.linalg.norm(v)
        sp_p, sp_m = oracle._copy_species(sp), oracle._copy_species(sp)
        sp_p.u += eps * v
        sp_m.u -= eps * v
        fd = (_rollout_loss(g, sp_p, f, src, w.nsteps) - _rollout_loss(g, sp_m, f, src, w.nsteps)) / (2 * eps)
        checks.append((fd, np.sum(gu * v)))
    for t in range(3):
        v = rng.normal(size=src.amp.shape)
        v /= np.linalg.norm(v)
        sp_ = NS(k_plane=src.k_plane, amp=src.amp + eps * v, g=src.g)
        sm_ = NS(k_plane=src.k_plane, amp=src.amp - eps * v, g=src.g)
        fd = (_rollout_loss(g, sp, f, sp_, w.nsteps) - _rollout_loss(g, sp, f, sm_, w.nsteps)) / (2 * eps)
        checks.append((fd, np.sum(gA * v)))
    for p in (0, 100, 311):
        for d in range(3):
            sp_p, sp_m = oracle._copy_species(sp), oracle._copy_species(sp)
            sp_p.u[d, p] += eps
            sp_m.u[d, p] -= eps
            fd = (_rollout_loss(g, sp_p, f, src, w.nsteps) - _rollout_loss(g, sp_m, f, src, w.nsteps)) / (2 * eps)
            checks.append((fd, gu[d, p]))
    for fd, an in checks:
        assert abs(fd - an) <= _fd_tol(an, L, eps), (fd, an)
        assert 10 * np.finfo(float).eps * abs(L) / eps < 1e-6 * abs(an)   # noise below the bar


@pytest.mark.parametrize("pusher,solver,filt", [(0, 0, False), (1, 0, False), (0, 1, False), (1, 1, True)])
def test_adjoint_position_and_field_gradients_by_finite_differences(pusher, solver, filt):
    """dL/dx0 and dL/dE0, dL/dB0 from the reverse sweep against central
    differences (pins the deposit transpose in both positions, the gather
    transpose and the transpose of either momentum update, of the CKC field
    solve and of the filter before the gather)."""
    w = wl.differentiable((8, 8, 8), 1, 0.08, 3, 2, "f64", 4321, amp0=0.0)
    g = dataclasses.replace(w.grid, pusher=pusher, solver=solver,
                            gather_filter=FILTER_TAPS if filt else None)
    sp, f = w.species.numpy(), w.fields.numpy()
    rng = np.random.default_rng(10)
    f.E[:] = rng.normal(0, 0.1, f.E.shape)
    f.B[:] = rng.normal(0, 0.1, f.B.shape)
    # reverse sweep keeping lam for x, E, B
    states = []
    s = oracle._copy_species(sp)
    ff = oracle._copy_fields(f)
    for it in range(w.nsteps):
        states.append((oracle._copy_species(s), oracle._copy_fields(ff)))
        oracle.step(g, s, ff, None, it, 1)
    L, lam = oracle.loss(g, ff, sp.cell.shape[1])
    for it in reversed(range(w.nsteps)):
        oracle.step_adjoint(g, states[it][0], states[it][1], None, it, lam, None)
    eps = 1e-6
    for p in (3, 200, 500):
        for d in range(3):
            if not (1e-4 < sp.off[d, p] < 1 - 1e-4):
                continue
            sp_p, sp_m = oracle._copy_species(sp), oracle._copy_species(sp)
            sp_p.off[d, p] += eps
            sp_m.off[d, p] -= eps
            fd = (_rollout_loss(g, sp_p, f, None, w.nsteps) - _rollout_loss(g, sp_m, f, None, w.nsteps)) / (2 * eps)
            assert abs(fd - lam.lx[d, p]) <= _fd_tol(fd, L, eps), (p, d, fd, lam.lx[d, p])
    for name, arr, lamarr in (("E", f.E, lam.lE), ("B", f.B, lam.lB)):
        for t in range(6):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            fp, fm = oracle._copy_fields(f), oracle._copy_fields(f)
            getattr(fp, name)[idx] += eps
            getattr(fm, name)[idx] -= eps
            fd = (_rollout_loss(g, sp, fp, None, w.nsteps) - _rollout_loss(g, sp, fm, None, w.nsteps)) / (2 * eps)
            assert abs(fd - lamarr[idx]) <= _fd_tol(fd, L, eps), (name, idx, fd, lamarr[idx])
