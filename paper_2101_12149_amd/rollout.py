"""Differentiable PIC rollout: a torch.autograd.Function over pic_step with a
hand-written reverse sweep (pic_step_adjoint) and checkpointing every k steps.

Forward: nsteps PIC steps from the initial momenta u0 with the source map
`amp` on the plane k_plane; the loss is the field energy U_E + U_B after the
last step (pic_energy_loss).  The steps run in segments of k: each segment
stores its input state (the checkpoint), bins the particles by tile
(pic_sort_tiles, keeping the permutation and the binning) and takes its k
steps on that binning, so that no step runs on a binning more than k steps
old.
Backward: for each segment, last first, the checkpoint is put in the
segment's binned order with the stored permutation and replayed keeping
every step's input state, then the steps are reversed with
pic_step_adjoint on the same binning.  The particle adjoints arrive in the
binned order of the segment (its steps do not reorder particles) and leave
in the order of its checkpoint, which is the order at the end of the
previous segment.  Returns dL/du0 and dL/damp.

With `tiled` False the particles are never binned and every kernel runs per
particle.  All arithmetic runs in the library's kernels; this module only
orders the calls and holds device buffers.
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
        self.ntiles = _lib.pic_tile_count(grid, dtype) if self.tiled else 0

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


def _permute(sp, perm):
    """The species with particle j taken from index perm[j]."""
    return wl.Species(sp.cell[:, perm].contiguous(), sp.off[:, perm].contiguous(), sp.u[:, perm].contiguous(),
                      None if sp.w is None else sp.w[perm].contiguous(), sp.w0, sp.q, sp.m)


class PICRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, amp, pb):
        sp = pb.species.clone()
        sp.u = u0.detach().clone().contiguous()
        f = pb.fields.clone()
        src = pb.source_with(amp) if amp is not None else None
        segments = []   # (first step, checkpoint species, fields, permutation, binning)
        s = 0
        while s < pb.nsteps:
            n = min(pb.k, pb.nsteps - s)
            cp = (sp.clone(), f.clone())
            perm = ts = None
            if pb.tiled:
                perm = torch.empty(sp.n, dtype=torch.int32, device=sp.off.device)
                ts = torch.zeros(pb.ntiles + 1, dtype=torch.int32, device=sp.off.device)
                _lib.pic_sort_tiles(pb.grid, sp, ts, pb.ws, perm=perm)
            segments.append((s, cp[0], cp[1], perm, ts))
            _lib.pic_step(pb.grid, sp, f, src, s, n, 0, ts, pb.ws)
            s += n
        lam = _Adjoint(sp.n, f)
        loss = _lib.pic_energy_loss(pb.grid, f, lam, pb.ws)
        ctx.pb = pb
        ctx.src = src
        ctx.segments = segments
        ctx.final_fields = f
        ctx.has_amp = amp is not None
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
        for (s0, sp0, f0, perm, ts) in reversed(ctx.segments):
            n = min(pb.k, pb.nsteps - s0)
            # the segment's state in its binned order; lam is in that order
            pl = perm.long() if perm is not None else None
            sp = _permute(sp0, pl) if pl is not None else sp0.clone()
            f = f0.clone()
            # replay the segment, keeping the input state of every step
            states = []
            for i in range(n):
                states.append((sp.clone(), f.clone()))
                _lib.pic_step(pb.grid, sp, f, src, s0 + i, 1, 0, ts, pb.ws)
            for i in reversed(range(n)):
                sp_n, f_n = states[i]
                _lib.pic_step_adjoint(pb.grid, sp_n, f_n, src, s0 + i, lam, dA, pb.ws, tile_start=ts)
            if pl is not None:
                # back to the checkpoint's order (new j <- old perm[j])
                for name in ("lx", "lu"):
                    back = torch.empty_like(getattr(lam, name))
                    back[:, pl] = getattr(lam, name)
                    setattr(lam, name, back)
        ctx.segments = None
        du0 = lam.lu.clone()
        damp = dA.to(src.amp.dtype) if dA is not None else None
        return du0, damp, None


def rollout_loss(u0, amp, pb):
    """Field energy after pb.nsteps steps, differentiable in u0 and amp."""
    return PICRollout.apply(u0, amp, pb)
