"""pic_step_noalloc (the entry point for callers that cannot allocate) against
pic_step with a caller's workspace, through the C ABI.

Both run the same kernels on the same seeded state; they differ only in
where the scratch lives (the library's static device array instead of the
workspace) and in the order of floating-point atomics.  FP64 results agree
within 1e-12 (rel-L2 of E, B, J, the diagnostics history and the particle
set), FP32 within 1e-5 (the one-step FP32 bound on E, B, J).  Two calls in
a row, the second on a smaller grid with fewer particles, so that the
second call starts from the scratch contents the first left behind; the
second also runs the guest lists (sorts more than 8 steps apart), whose
buffers live in the scratch.
"""
import numpy as np
import pytest
import torch

from paper_2101_12149_amd import _lib
from paper_2101_12149_amd import workloads as wl
from pic_cases import dev, particle_table, rel_l2

pytestmark = pytest.mark.gpu


def _run(w, noalloc):
    g = w.grid
    dtype = "f64" if w.species.off.dtype == torch.float64 else "f32"
    sp, f = dev(w.species), dev(w.fields)
    ts = torch.zeros(_lib.pic_tile_count(g, dtype) + 1, dtype=torch.int32, device="cuda")
    diag = torch.zeros((w.nsteps, 5), dtype=torch.float64, device="cuda")
    if noalloc:
        _lib.pic_step_noalloc(g, sp, f, None, 0, w.nsteps, w.sort_every, ts, diag)
    else:
        ws = _lib.workspace(g, dtype, sp.n)
        _lib.pic_step(g, sp, f, None, 0, w.nsteps, w.sort_every, ts, ws, diag)
    torch.cuda.synchronize()
    return sp.numpy(), f.numpy(), diag.cpu().numpy()


def _compare(w, tol):
    sa, fa, da = _run(w, noalloc=False)
    sb, fb, db = _run(w, noalloc=True)
    for name in ("E", "B", "J"):
        assert rel_l2(getattr(fb, name), getattr(fa, name)) < tol, name
    assert rel_l2(db, da) < tol
    assert rel_l2(particle_table(sb), particle_table(sa)) < tol


def test_noalloc_step_matches_the_workspace_step_on_two_calls_in_a_row():
    # first call: 24x16x20 cells (8x8x5 tiles), 4 ppc, order 3, FP64, sorts every 4
    big = wl.uniform_plasma((24, 16, 20), 4, 0.05, 3, 6, "f64", 2101, 4)
    assert _lib.pic_workspace_bytes(big.grid, "f64", big.species.n) <= _lib.NOALLOC_SCRATCH_BYTES
    _compare(big, 1e-12)
    # second call, smaller: 12^3 cells, 2 ppc, order 1, sorts every 10 over
    # 12 steps (guest lists read from the scratch between the sorts)
    small = wl.uniform_plasma((12, 12, 12), 2, 0.1, 1, 12, "f64", 2102, 10)
    assert small.species.n < big.species.n
    _compare(small, 1e-12)


def test_noalloc_step_in_fp32_after_the_fp64_calls():
    w = wl.uniform_plasma((16, 16, 16), 4, 0.05, 3, 1, "f32", 2103, 4)
    _compare(w, 1e-5)


def test_noalloc_step_refuses_a_grid_beyond_its_scratch():
    """A 256^3 grid needs more than the 128 MiB static scratch: refused
    before any launch, the fields untouched."""
    g = wl.plasma_grid((256, 256, 256), 3)
    assert _lib.pic_workspace_bytes(g, "f32", 0) > _lib.NOALLOC_SCRATCH_BYTES
    sp = wl.Species(torch.zeros((3, 0), dtype=torch.int32), torch.zeros((3, 0)), torch.zeros((3, 0)), None,
                    1.0, -1.0, 1.0).to(dtype=torch.float32)
    shape = (3, 4, 4, 4)   # never read: the size check comes first
    f = wl.Fields(torch.ones(shape), torch.ones(shape), torch.ones(shape)).to(dtype=torch.float32)
    dsp, df = dev(sp), dev(f)
    with pytest.raises(_lib.PicError) as e:
        _lib.pic_step_noalloc(g, dsp, df, None, 0, 1, 0, None)
    assert e.value.status == 4 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert float(df.E.sum()) == 3 * 64
