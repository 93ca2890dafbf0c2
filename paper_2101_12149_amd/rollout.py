"""Differentiable PIC rollout: a torch.autograd.Function over pic_step with a
hand-written reverse sweep (pic_step_adjoint) and checkpointing every k steps.

Forward: nsteps PIC steps from the initial momenta u0 with the source map
`amp` on the plane k_plane; the state is stored every k steps.  The loss is
the field energy U_E + U_B after the last step (pic_energy_loss).
Backward: for each checkpoint segment, last first, the segment is replayed
from its checkpoint keeping every step's input state, then the steps are
reversed with pic_step_adjoint.  Returns dL/du0 and dL/damp.

With `tiled` (the default) the particles are binned by tile once, before the
first step (pic_sort_tiles, keeping the permutation), and the forward steps
run the tile kernels on that binning.  Each replay segment of the reverse
sweep bins its checkpoint afresh, so that the adjoint steps never run on a
binning more than k steps old: the particle adjoints are gathered into the
segment's order before its steps and scattered back after them, and dL/du0
is scattered back to the order of u0 at the end.  All arithmetic runs in the
library's kernels; this module only orders the calls and holds device
buffers.
"""
import torch

from . import _lib
from . import workloads as wl


class Problem:
    """Static inputs of a rollout: grid, the particles' positions/weights,
    initial fields, the source time series, step count and checkpoint
    interval.  Tensors live on the device in the working precision."""

    def __init__(self, grid, species, fields, source, nsteps, checkpoint_every, dtype, tiled=True):
        self.grid = grid
        self.species = species
        self.fields = fields
        self.source = source
        self.nsteps = int(nsteps)
        self.k = max(1, int(checkpoint_every or nsteps))
        self.dtype = dtype
        self.ws = _lib.workspace(grid, dtype, species.n)
        self.tiled = bool(tiled) and species.n > 0
        self.tile_start = None
        if self.tiled:
            self.tile_start = torch.zeros(_lib.pic_tile_count(grid, dtype) + 1, dtype=torch.int32,
                                          device=species.off.device)

    def source_with(self, amp):
        if self.source is None:
            return None
        return wl.Source(self.source.k_plane, amp.detach().contiguous(), self.source.g)


class _Adjoint:
    def __init__(self, n, fields):
        self.lx = torch.zeros((3, n), dtype=fields.E.dtype, device=fields.E.device)
        self.lu = torch.zeros((3, n), dtype=fields.E.dtype, device=fields.E.device)
        self.lE = torch.zeros_like(fields.E)
        self.lB = torch.zeros_like(fields.B)


def _advance(pb, sp, f, src, step0, nsteps):
    if nsteps > 0:
        _lib.pic_step(pb.grid, sp, f, src, step0, nsteps, 0, pb.tile_start, pb.ws)


class PICRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, amp, pb):
        sp = pb.species.clone()
        sp.u = u0.detach().clone().contiguous()
        perm = None
        if pb.tiled:
            perm = torch.empty(sp.n, dtype=torch.int32, device=sp.off.device)
            _lib.pic_sort_tiles(pb.grid, sp, pb.tile_start, pb.ws, perm=perm)
        f = pb.fields.clone()
        src = pb.source_with(amp) if amp is not None else None
        checkpoints = []
        s = 0
        while s < pb.nsteps:
            checkpoints.append((s, sp.clone(), f.clone()))
            n = min(pb.k, pb.nsteps - s)
            _advance(pb, sp, f, src, s, n)
            s += n
        lam = _Adjoint(sp.n, f)
        loss = _lib.pic_energy_loss(pb.grid, f, lam, pb.ws)
        ctx.pb = pb
        ctx.src = src
        ctx.checkpoints = checkpoints
        ctx.final_fields = f
        ctx.has_amp = amp is not None
        ctx.perm = perm
        return loss[0].clone()

    @staticmethod
    def backward(ctx, grad_loss):
        pb, src = ctx.pb, ctx.src
        seed = float(grad_loss.detach().cpu())
        lam = _Adjoint(pb.species.n, ctx.final_fields)
        _lib.pic_energy_loss(pb.grid, ctx.final_fields, lam, pb.ws, seed=seed)
        dA = None
        if ctx.has_amp and src is not None:
            dA = torch.zeros(src.amp.shape, dtype=torch.float64, device=src.amp.device)
        for (s0, sp0, f0) in reversed(ctx.checkpoints):
            n = min(pb.k, pb.nsteps - s0)
            sp, f = sp0.clone(), f0.clone()
            seg = None
            if pb.tiled:
                # a fresh binning for the segment; the particle adjoints follow
                # the particles into its order (new j <- old seg[j])
                seg = torch.empty(sp.n, dtype=torch.int32, device=sp.off.device)
                _lib.pic_sort_tiles(pb.grid, sp, pb.tile_start, pb.ws, perm=seg)
                seg = seg.long()
                lam.lx = lam.lx[:, seg].contiguous()
                lam.lu = lam.lu[:, seg].contiguous()
            # replay the segment, keeping the input state of every step
            states = []
            for i in range(n):
                states.append((sp.clone(), f.clone()))
                _advance(pb, sp, f, src, s0 + i, 1)
            for i in reversed(range(n)):
                sp_n, f_n = states[i]
                _lib.pic_step_adjoint(pb.grid, sp_n, f_n, src, s0 + i, lam, dA, pb.ws, tile_start=pb.tile_start)
            if seg is not None:
                for name in ("lx", "lu"):
                    back = torch.empty_like(getattr(lam, name))
                    back[:, seg] = getattr(lam, name)
                    setattr(lam, name, back)
        ctx.checkpoints = None
        if ctx.perm is not None:
            du0 = torch.empty_like(lam.lu)
            du0[:, ctx.perm.long()] = lam.lu      # back to the order of u0
        else:
            du0 = lam.lu.clone()
        damp = dA.to(src.amp.dtype) if dA is not None else None
        return du0, damp, None


def rollout_loss(u0, amp, pb):
    """Field energy after pb.nsteps steps, differentiable in u0 and amp."""
    return PICRollout.apply(u0, amp, pb)
