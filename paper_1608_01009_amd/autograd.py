"""``torch.autograd.Function`` over a recorded PIC run (FP64).

``run(sim, EB0, particles, nsteps, checkpoint_every)`` loads the initial
fields ``EB0`` (a (6, n_cells) float64 tensor: Ex, Ey, Ez, Bx, By, Bz) and per
species the initial particles (an (n_s, 6) float64 tensor: x, y, z, ux, uy,
uz in the caller's order), records ``nsteps`` steps and returns the final
fields (6, n_cells) and the final particles, again (n_s, 6) in the caller's
order.  Its backward calls the library's reverse sweep (``pic_backward``:
transposed Yee update, particle vector-Jacobian products, re-sort transposes,
forward recomputation from checkpoints every ``checkpoint_every`` steps) and
returns the gradients with respect to ``EB0`` and the initial particles.

The library keeps particles in its own sorted order; the caller's order is
restored through the particle ids (0 .. n_s - 1 in the caller's order), with
PyTorch indexing on the device.  Positions are in cell units and their
gradients per cell unit.
"""
from __future__ import annotations

from typing import List, Sequence

import torch

from . import pic

KEYS = ("x", "y", "z", "ux", "uy", "uz")


def _stored(sim: pic.Simulation, s: int, n: int, dev):
    out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in KEYS}
    out["id"] = torch.empty(n, dtype=torch.int64, device=dev)
    pic.pic_get_particles(sim.ctx, s, capacity=n, out=out)
    return out


class _PicRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim, nsteps, every, EB0, *parts):
        dev = EB0.device
        ncell = sim.ncell
        if EB0.dtype != torch.float64 or tuple(EB0.shape) != (6, ncell):
            raise ValueError(f"EB0 must be a float64 tensor of shape (6, {ncell})")
        fields = [EB0[k].detach().contiguous() for k in range(6)]
        counts = []
        cols = []
        for P in parts:
            if P.dtype != torch.float64 or P.dim() != 2 or P.shape[1] != 6:
                raise ValueError("particles must be float64 tensors of shape (n, 6)")
            n = int(P.shape[0])
            counts.append(n)
            Pc = P.detach()
            cols.append([Pc[:, k].contiguous() for k in range(6)] +
                        [torch.arange(n, dtype=torch.int64, device=dev)])
        # the library works on its own stream: finish torch's work on the inputs
        torch.cuda.current_stream(dev).synchronize()
        sim.set_fields(fields)
        for s, c in enumerate(cols):
            sim.load_particles(s, *c)
        sim.record(every)
        start_ids = [_stored(sim, s, n, dev)["id"] for s, n in enumerate(counts)]
        sim.step(nsteps)
        EB = torch.empty(6, ncell, dtype=torch.float64, device=dev)
        pic.pic_get_fields(sim.ctx, ncell, out=[EB[k] for k in range(6)] + [None] * 3)
        outs = []
        final_ids = []
        for s, n in enumerate(counts):
            st = _stored(sim, s, n, dev)
            P = torch.empty(n, 6, dtype=torch.float64, device=dev)
            for k, key in enumerate(KEYS):
                P[st["id"], k] = st[key]
            outs.append(P)
            final_ids.append(st["id"])
        ctx.sim = sim
        ctx.counts = counts
        ctx.start_ids = start_ids
        ctx.final_ids = final_ids
        return (EB, *outs)

    @staticmethod
    def backward(ctx, gEB, *gparts):
        sim = ctx.sim
        dev = ctx.start_ids[0].device if ctx.start_ids else gEB.device
        ncell = sim.ncell
        seed_fields = None
        if gEB is not None:
            g = gEB.to(torch.float64).contiguous()
            seed_fields = [g[k] for k in range(6)]
        seed_particles = []
        for s, n in enumerate(ctx.counts):
            gp = gparts[s] if s < len(gparts) else None
            if gp is None:
                seed_particles.append(None)
                continue
            gs = gp.to(torch.float64)[ctx.final_ids[s]]       # caller order -> stored order
            seed_particles.append([gs[:, k].contiguous() for k in range(6)])
        grad_fields = [torch.empty(ncell, dtype=torch.float64, device=dev) for _ in range(6)]
        grad_parts = [[torch.empty(n, dtype=torch.float64, device=dev) for _ in range(6)]
                      for n in ctx.counts]
        torch.cuda.current_stream(dev).synchronize()
        pic.pic_backward(sim.ctx, ncell, ctx.counts, seed_fields, seed_particles, grad_fields,
                         grad_parts)
        gEB0 = torch.stack(grad_fields)
        gP0 = []
        for s, n in enumerate(ctx.counts):
            G = torch.empty(n, 6, dtype=torch.float64, device=dev)
            for k in range(6):
                G[ctx.start_ids[s], k] = grad_parts[s][k]   # stored order -> caller order
            gP0.append(G)
        return (None, None, None, gEB0, *gP0)


def run(sim: pic.Simulation, EB0: torch.Tensor, particles: Sequence[torch.Tensor], nsteps: int,
        checkpoint_every: int = 20) -> List[torch.Tensor]:
    """Differentiable ``nsteps`` steps of ``sim`` from (EB0, particles);
    returns [EB (6, n_cells), P_0 (n_0, 6), P_1, ...]."""
    return list(_PicRun.apply(sim, int(nsteps), int(checkpoint_every), EB0, *particles))
