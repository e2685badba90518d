"""torch.autograd wrappers of the IMEX step and its adjoint.

GRFFEStep.apply(u0, dom, n_steps, dt, checkpoint_every) advances the DG state u0
((9, E, (N+1)^3) float64 on the device) by n_steps steps of `dom` (a Domain
created with hybrid = HYBRID_DG_ONLY, so no element leaves DG and the
representation is the same in the forward and the backward pass).  The forward
pass keeps the state every `checkpoint_every` steps; the backward pass recomputes
each segment from its checkpoint, keeping the segment's step-start states and
stage values, and runs the library's step adjoint back through them.  Every step
and adjoint runs in the HIP library; this module only orders the calls and holds
the checkpoints.

GRFFEStepFrozen.apply(u_dg, u_fd, rep, dom, n_steps, dt, checkpoint_every) does
the same for a state of DG and FD elements (rep: the representation of each), in
the domain's hybrid mode: forced (the partition held) or adaptive (the indicator
decides; its decisions are frozen from the forward pass and the adjoint follows
the same rollbacks and switches).  It returns (u_dg, u_fd, rep) after the steps,
each element's state in its own representation (the other's entries zero).
"""
from __future__ import annotations

import torch

from . import grffe


def _set_dg(dom, u):
    fd = torch.zeros(dom.fd_shape(), dtype=torch.float64, device=u.device)
    rep = torch.zeros((dom.E,), dtype=torch.int32, device=u.device)
    dom.set_state(u.contiguous(), fd, rep)


def _advance(dom, u, n, dt):
    """States at the start of each of n steps from u with each step's stage values
    (U_3, U_4), and the state after them."""
    starts, stages = [], []
    _set_dg(dom, u)
    for _ in range(n):
        starts.append(dom.get_dg())
        dom.step(1, dt)
        stages.append(dom.get_stages())
    return starts, stages, dom.get_dg()


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
            starts, stages, _ = _advance(ctx.dom, u_start, k, ctx.dt)
            for u, (u3, u4) in zip(reversed(starts), reversed(stages)):
                lam = ctx.dom.step_adjoint_stages(u, u3, u4, lam, ctx.dt)
        return lam, None, None, None, None


def _advance_frozen(dom, dg, fd, rep, n, dt):
    starts = []
    dom.set_state(dg.contiguous(), fd.contiguous(), rep)
    for _ in range(n):
        starts.append(dom.get_state())
        dom.step(1, dt)
    return starts


def _own(dg, fd, rep):
    """The state with the entries of each element's other representation zeroed."""
    on_fd = (rep == 1).view(1, -1, 1)
    return torch.where(on_fd, torch.zeros_like(dg), dg), torch.where(on_fd, fd, torch.zeros_like(fd))


class GRFFEStepFrozen(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u_dg, u_fd, rep, dom, n_steps, dt=0.0, checkpoint_every=20):
        if dom.params.hybrid not in (grffe.HYBRID_FORCED, grffe.HYBRID_ADAPTIVE):
            raise grffe.GrffeError("GRFFEStepFrozen differentiates hybrid steps: create the domain with hybrid = 1 "
                                   "(adaptive, decisions frozen from the forward pass) or 2 (forced partition)")
        every = max(1, int(checkpoint_every))
        dt = float(dt) if dt and dt > 0 else dom.dt()
        r = rep.detach().to(torch.int32).contiguous()
        ckpts = []
        g, f = u_dg.detach().contiguous(), u_fd.detach().contiguous()
        done = 0
        while done < n_steps:
            k = min(every, n_steps - done)
            ckpts.append((g.clone(), f.clone(), r.clone(), k))
            dom.set_state(g, f, r)
            dom.step(k, dt)
            g, f, r = dom.get_state()
            done += k
        ctx.dom, ctx.dt, ctx.ckpts, ctx.rep_out = dom, dt, ckpts, r
        gz, fz = _own(g, f, r)
        ctx.mark_non_differentiable(r)
        return gz, fz, r

    @staticmethod
    def backward(ctx, grad_dg, grad_fd, _grad_rep):
        dom = ctx.dom
        lam_dg = grad_dg.contiguous().clone() if grad_dg is not None else torch.zeros(
            dom.dg_shape(), dtype=torch.float64, device="cuda")
        lam_fd = grad_fd.contiguous().clone() if grad_fd is not None else torch.zeros(
            dom.fd_shape(), dtype=torch.float64, device="cuda")
        lam_dg, lam_fd = _own(lam_dg, lam_fd, ctx.rep_out)
        for g0, f0, r0, k in reversed(ctx.ckpts):
            starts = _advance_frozen(dom, g0, f0, r0, k, ctx.dt)
            for g, f, r in reversed(starts):
                lam_dg, lam_fd = dom.step_adjoint_frozen(g, f, r, lam_dg, lam_fd, ctx.dt)
        return lam_dg, lam_fd, None, None, None, None, None
