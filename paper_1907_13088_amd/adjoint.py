"""Differentiable field stepping: a torch.autograd.Function over the C-ABI.

Forward: J0 = sum_s a_s g_s (mx_sources_assemble), then nsteps field steps
(mx_step), keeping a checkpoint of (E, B) every `checkpoint_every` steps.
Backward: for each checkpoint segment, last first, the forward segment is
recomputed from its checkpoint (which also re-derives the per-step sweep
counts of a tolerance solve and checks that recomputation reproduces the
next checkpoint bit for bit), then the transposed steps run (mx_adjoint)
and the current gradient is projected on the source shapes
(mx_sources_project).  Every arithmetic step runs in the HIP library.

The step is linear with coefficients independent of the state, so the
transposed step needs only the sweep counts; the recomputation is what a
state-dependent (particle-coupled) step would need and is kept so that this
path exercises it.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch

from . import mx


class SourceSet:
    """Localised current shapes g_s on a 2D grid (device tensors)."""

    def __init__(self, origins, shapes):
        self.origins = origins          # int64 (nsrc, 2) on the device
        self.shapes = shapes            # (nsrc, 3, W, W) in the grid dtype

    @property
    def nsrc(self) -> int:
        return int(self.shapes.shape[0])


class _FieldSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, amps, E0x, E0y, E0z, B0x, B0y, B0z, grid: mx.Grid, sources: SourceSet,
                env: Sequence[float], nsteps: int, checkpoint_every: int, verify: bool):
        g = grid
        shape = g.shape
        E = [t.detach().clone().contiguous() for t in (E0x, E0y, E0z)]
        B = [t.detach().clone().contiguous() for t in (B0x, B0y, B0z)]
        J0 = [torch.empty(shape, dtype=g.torch_dtype, device=g.device) for _ in range(3)]
        g.sources_assemble(sources.origins, sources.shapes, amps.detach().contiguous(), J0)
        g.bind(E, B)
        g.set_current(J0)
        ckpts = []
        counts: List[tuple] = []
        K = max(1, int(checkpoint_every))
        s = 0
        while s < nsteps:
            ckpts.append((s, [t.clone() for t in E], [t.clone() for t in B]))
            n = min(K, nsteps - s)
            st = g.step(n, env=list(env[s:s + n]), stats=True)
            counts += [x.sweeps for x in st]
            s += n
        ctx.grid, ctx.sources, ctx.env, ctx.nsteps = g, sources, list(env), nsteps
        ctx.ckpts, ctx.counts, ctx.J0, ctx.verify, ctx.K = ckpts, counts, J0, verify, K
        ctx.final = ([t.clone() for t in E], [t.clone() for t in B])
        return tuple(E) + tuple(B)

    @staticmethod
    def backward(ctx, gEx, gEy, gEz, gBx, gBy, gBz):
        g = ctx.grid
        shape = g.shape
        zeros = lambda: torch.zeros(shape, dtype=g.torch_dtype, device=g.device)
        Eb = [(x if x is not None else zeros()).detach().clone().contiguous() for x in (gEx, gEy, gEz)]
        Bb = [(x if x is not None else zeros()).detach().clone().contiguous() for x in (gBx, gBy, gBz)]
        dJ = [zeros() for _ in range(3)]
        ends = [c[0] for c in ctx.ckpts[1:]] + [ctx.nsteps]
        for (s0, Ec, Bc), s1 in reversed(list(zip(ctx.ckpts, ends))):
            n = s1 - s0
            counts = ctx.counts[s0:s1]
            if ctx.verify:
                # recompute the segment from its checkpoint with the same counts
                E = [t.clone() for t in Ec]
                B = [t.clone() for t in Bc]
                g.bind(E, B)
                g.set_current(ctx.J0)
                g.step(n, env=ctx.env[s0:s1], replay=counts)
                nxt = ctx.final if s1 == ctx.nsteps else next((c[1], c[2]) for c in ctx.ckpts if c[0] == s1)
                for a, b in zip(E + B, nxt[0] + nxt[1]):
                    if not torch.equal(a, b):
                        raise RuntimeError(f"recomputed segment [{s0}, {s1}) differs from its checkpoint")
            g.adjoint(n, ctx.env[s0:s1], counts, Eb, Bb, dJ)
        grad_amps = torch.empty(ctx.sources.nsrc, dtype=g.torch_dtype, device=g.device)
        g.sources_project(ctx.sources.origins, ctx.sources.shapes, dJ, grad_amps)
        return (grad_amps, *Eb, *Bb, None, None, None, None, None, None)


def field_steps(amps, E0, B0, grid: mx.Grid, sources: SourceSet, env: Sequence[float], nsteps: int,
                checkpoint_every: int = 50, verify: bool = True):
    """Differentiable nsteps of the field step; returns (E[3], B[3]) after the
    steps, with gradients flowing to amps, E0 and B0."""
    out = _FieldSteps.apply(amps, *E0, *B0, grid, sources, env, nsteps, checkpoint_every, verify)
    return list(out[:3]), list(out[3:])
