"""Device diagnostics against the FP64 oracle: the Gauss-law residual
(pic_gauss_residual) and the FP64 diagnostics history of a long run.

Tolerances: the Gauss residual is computed in FP64 on both sides from the
same state (FP32 values upcast exactly), so it matches within 1e-12 in both
precisions.  Its invariance over steps holds to rounding in FP64 (1e-12);
in FP32 the residual field drifts by the per-step charge-conservation error
and the FP32 rounding of the E update, a few 1e-8 of its norm per step,
bounded here by 1e-5 over 12 steps.  The long FP64 history (100 steps) is
compared at 1e-9 relative: round-off differences between the two summation
orders grow along chaotic trajectories, and the summed diagnostics stay far
below that bound.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2101_12149_amd import _lib
from paper_2101_12149_amd import workloads as wl
from pic_cases import dev, random_fields, random_species

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("order", [1, 3])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gauss_residual_matches_oracle(order, dtype):
    g = wl.plasma_grid((12, 16, 20), order)
    sp = random_species(g, 6000, 31, dtype=dtype)
    f = random_fields(g, 32, dtype=dtype)
    ws = _lib.workspace(g, dtype, sp.n)
    out = _lib.pic_gauss_residual(g, dev(sp), dev(f), ws).cpu().numpy()
    _, want = oracle.gauss(g, sp.numpy(), f.numpy())
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gauss_residual_is_invariant_on_the_device(dtype):
    """Twelve steps (sorts every 4), the residual after each: its norm stays
    at the initial thermal-noise level, and the last state's value matches
    the oracle's evaluation of the same state."""
    w = wl.uniform_plasma((16, 16, 16), 4, 0.05, 3, 12, dtype, 2301, 4)
    g = w.grid
    sp, f = dev(w.species), dev(w.fields)
    ws = _lib.workspace(g, dtype, sp.n)
    ts = torch.zeros(_lib.pic_tile_count(g, dtype) + 1, dtype=torch.int32, device="cuda")
    r0 = _lib.pic_gauss_residual(g, sp, f, ws).cpu().numpy()
    assert r0[0] > 1.0   # thermal noise: no Poisson solve at the start
    tol = 1e-12 if dtype == "f64" else 1e-5
    for n in range(w.nsteps):
        _lib.pic_step(g, sp, f, None, n, 1, w.sort_every, ts, ws)
        r = _lib.pic_gauss_residual(g, sp, f, ws).cpu().numpy()
        assert abs(r[0] - r0[0]) <= tol * r0[0], (n, r[0], r0[0])
        assert abs(r[2] - r0[2]) <= 1e-12 * abs(r0[2])
    _, want = oracle.gauss(g, sp.numpy(), f.numpy())
    np.testing.assert_allclose(r, want, rtol=1e-12, atol=0)


def test_gauss_residual_reports_corrupt_state():
    g = wl.plasma_grid((8, 8, 8), 3)
    sp = random_species(g, 100, 33)
    sp.cell[1, 7] = 8
    ws = _lib.workspace(g, "f64", sp.n)
    with pytest.raises(_lib.PicError) as e:
        _lib.pic_gauss_residual(g, dev(sp), dev(random_fields(g, 34)), ws)
    assert e.value.status == 5


def test_long_fp64_diagnostics_history_matches_oracle():
    """100 steps of a 32^3 order-3 plasma (4 ppc, u_th = 0.05 c, sorts every
    4): the five FP64 diagnostics after every step against the oracle's."""
    w = wl.uniform_plasma((32, 32, 32), 4, 0.05, 3, 100, "f64", 2201, 4)
    g = w.grid
    sp, f = dev(w.species), dev(w.fields)
    ws = _lib.workspace(g, "f64", sp.n)
    ts = torch.zeros(_lib.pic_tile_count(g, "f64") + 1, dtype=torch.int32, device="cuda")
    diag = torch.zeros((w.nsteps, 5), dtype=torch.float64, device="cuda")
    _lib.pic_step(g, sp, f, None, 0, w.nsteps, w.sort_every, ts, ws, diag)
    got = diag.cpu().numpy()
    want = oracle.step(g, w.species.numpy(), w.fields.numpy(), None, 0, w.nsteps)
    assert np.all(want[:, 0] > 0) and np.all(want[:, 1] > 0)
    rel = np.abs(got - want) / np.abs(want)
    assert rel.max() < 1e-9, (rel.max(axis=0), rel.argmax(axis=0))
