"""torch.autograd wrapper of the all-DG IMEX step and its adjoint.

GRFFEStep.apply(u0, dom, n_steps, dt, checkpoint_every) advances the DG state u0
((9, E, (N+1)^3) float64 on the device) by n_steps steps of `dom` (a Domain
created with hybrid = HYBRID_DG_ONLY, so no element leaves DG and the
representation is the same in the forward and the backward pass).  The forward
pass keeps the state every `checkpoint_every` steps; the backward pass recomputes
each segment from its checkpoint, keeping the segment's step-start states, and
runs the library's step adjoint back through them.  Every step and adjoint runs
in the HIP library; this module only orders the calls and holds the checkpoints.
"""
from __future__ import annotations

import torch

from . import grffe


def _set_dg(dom, u):
    fd = torch.zeros(dom.fd_shape(), dtype=torch.float64, device=u.device)
    rep = torch.zeros((dom.E,), dtype=torch.int32, device=u.device)
    dom.set_state(u.contiguous(), fd, rep)


def _advance(dom, u, n, dt):
    """States at the start of each of n steps from u, and the state after them."""
    starts = []
    _set_dg(dom, u)
    for _ in range(n):
        starts.append(dom.get_state()[0])
        dom.step(1, dt)
    return starts, dom.get_state()[0]


class GRFFEStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, dom, n_steps, dt=0.0, checkpoint_every=20):
        if dom.params.hybrid != grffe.HYBRID_DG_ONLY:
            raise grffe.GrffeError("GRFFEStep differentiates all-DG steps: create the domain with hybrid = 0")
        every = max(1, int(checkpoint_every))
        dt = float(dt) if dt and dt > 0 else dom.dt()
        ckpts = []
        u = u0.detach().contiguous()
        done = 0
        while done < n_steps:
            k = min(every, n_steps - done)
            ckpts.append((u.clone(), k))
            _set_dg(dom, u)
            dom.step(k, dt)
            u = dom.get_state()[0]
            done += k
        ctx.dom, ctx.dt, ctx.ckpts = dom, dt, ckpts
        return u.clone()

    @staticmethod
    def backward(ctx, grad):
        lam = grad.contiguous().clone()
        for u_start, k in reversed(ctx.ckpts):
            starts, _ = _advance(ctx.dom, u_start, k, ctx.dt)
            for u in reversed(starts):
                lam = ctx.dom.step_adjoint(u, lam, ctx.dt)
        return lam, None, None, None, None
