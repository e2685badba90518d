"""The objective of the adjoint workload and the checkpointed gradient of a time
integral of such an objective.

SphereFlux(w) evaluates, for a DG state U of workload w (every live element on DG),
the outgoing Poynting flux through the Euclidean sphere of radius R,
    L(U) = sum_q w_q sqrt(gamma) S^i x_i / R,   S^i = eps^{ijk} E_j B_k,
eps^{ijk} = [ijk] / sqrt(gamma), E = E~ / sqrt(gamma), B = B~ / sqrt(gamma)
(Sec. II A; the flux through a coordinate sphere as in the paper's magnetosphere
diagnostics), with the fields taken from the DG polynomial of the element that
contains each quadrature point and the background metric evaluated there.  It is a
small torch function of the state (a user's objective, differentiated by
torch.autograd), not part of the solver.

time_integral_gradient(dom, u0, steps, dt, every, L) returns
    Phi = sum_{n=1..steps} dt L(U^n)
and dPhi/dU^0, by the adjoint recursion
    lam_steps = dt dL/dU^steps,  lam_n = (dU^{n+1}/dU^n)^T lam_{n+1} + dt dL/dU^n,
with the states kept every `every` steps and each segment recomputed from its
checkpoint (keeping each step's stage values, so the step adjoints need no
forward re-run); every step and step adjoint runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import grffe
from . import inputs as I


def _lagrange(nodes, xi):
    """Values (len(xi), n) of the Lagrange basis on `nodes` at the points xi."""
    n = len(nodes)
    out = np.ones((xi.size, n))
    for j in range(n):
        for k in range(n):
            if k != j:
                out[:, j] *= (xi - nodes[k]) / (nodes[j] - nodes[k])
    return out


class SphereFlux:
    def __init__(self, w, R=20.0, n_theta=32, n_phi=64, device="cuda"):
        N = w["degree"]
        n = N + 1
        nodes = grffe.operator(N, 0)
        pts, wq = I.sphere_quadrature(R, n_theta, n_phi)
        lower = np.asarray(w["lower"], np.float64)
        upper = np.asarray(w["upper"], np.float64)
        ne = np.asarray(w["n_elem"])
        h = (upper - lower) / ne
        idx = np.clip(np.floor((pts.T - lower) / h).astype(np.int64), 0, ne - 1)
        xi = 2.0 * (pts.T - lower - idx * h) / h - 1.0
        Lx, Ly, Lz = (_lagrange(nodes, xi[:, d]) for d in range(3))
        # node index i + n (j + n k): flatten (k, j, i)
        W = np.einsum("qi,qj,qk->qkji", Lx, Ly, Lz).reshape(-1, n ** 3)
        elem = idx[:, 0] + ne[0] * (idx[:, 1] + ne[1] * idx[:, 2])
        # interpolation grouped by element: the elements holding points, each with its
        # points' weights (zero-padded), as one batched product
        Q, n3 = W.shape
        uniq, uidx = np.unique(elem, return_inverse=True)
        counts = np.bincount(uidx)
        slot = np.zeros(Q, np.int64)
        seen = np.zeros(len(uniq), np.int64)
        for q in range(Q):
            slot[q] = seen[uidx[q]]
            seen[uidx[q]] += 1
        Wp = np.zeros((len(uniq), int(counts.max()), n3))
        Wp[uidx, slot] = W
        self.uniq = torch.from_numpy(uniq).to(device)
        self.uidx = torch.from_numpy(uidx).to(device)
        self.slot = torch.from_numpy(slot).to(device)
        self.Wp = torch.from_numpy(Wp).to(device)
        self.WpT = self.Wp.transpose(1, 2).contiguous()
        if w.get("curved"):
            bg = I.background(w, pts[0], pts[1], pts[2])
            gl = bg[4:10]
        else:
            gl = np.zeros((6, pts.shape[1]))
            gl[0] = gl[3] = gl[5] = 1.0
        g = np.array([[gl[0], gl[1], gl[2]], [gl[1], gl[3], gl[4]], [gl[2], gl[4], gl[5]]])  # (3, 3, Q)
        sg = np.sqrt(np.linalg.det(np.moveaxis(g, -1, 0)))
        self.R = float(R)
        self.elem = torch.from_numpy(elem).to(device)
        self.W = torch.from_numpy(np.ascontiguousarray(W)).to(device)
        self.g = torch.from_numpy(np.ascontiguousarray(g)).to(device)
        self.sg = torch.from_numpy(sg).to(device)
        self.x = torch.from_numpy(np.ascontiguousarray(pts)).to(device)
        self.wq = torch.from_numpy(wq).to(device)

    def __call__(self, u):
        """L(U) for the DG state u, (9, E, (N+1)^3) float64 on the device."""
        v = self._at_points(u)  # (9, Q) at the sphere points
        E = v[0:3] / self.sg
        B = v[3:6] / self.sg
        El = (self.g * E[None]).sum(1)
        Bl = (self.g * B[None]).sum(1)
        # sqrt(gamma) eps^{ijk} E_j B_k x_i = x . (E_lo x B_lo)
        flux = (self.x * torch.linalg.cross(El, Bl, dim=0)).sum(0) / self.R
        return (self.wq * flux).sum()

    def grad(self, u):
        """dL/dU, written out: with x . (E_lo x B_lo) = E_lo . (B_lo x x) = B_lo . (x x E_lo),
        dL/dE~ = g (B_lo x x) w / (R sqrt(gamma)), dL/dB~ = g (x x E_lo) w / (R sqrt(gamma)) at
        the points, spread to the nodes of the containing elements with the
        interpolation weights."""
        v = self._at_points(u)
        El = (self.g * (v[0:3] / self.sg)[None]).sum(1)
        Bl = (self.g * (v[3:6] / self.sg)[None]).sum(1)
        c = self.wq / (self.R * self.sg)
        gE = (self.g * torch.linalg.cross(Bl, self.x, dim=0)[None]).sum(1) * c
        gB = (self.g * torch.linalg.cross(self.x, El, dim=0)[None]).sum(1) * c
        dv = torch.zeros_like(v)
        dv[0:3] = gE
        dv[3:6] = gB
        dvp = torch.zeros((self.Wp.shape[0], self.Wp.shape[1], 6), dtype=u.dtype, device=u.device)
        dvp[self.uidx, self.slot] = dv[0:6].t()
        ge = torch.bmm(self.WpT, dvp)  # (elements, nodes, 6)
        out = torch.zeros_like(u)
        out[0:6, self.uniq, :] = ge.permute(2, 0, 1)
        return out

    def _at_points(self, u):
        """The DG interpolants at the points, (9, Q); only the six field rows are
        formed (the other three are zero)."""
        if u.requires_grad:
            return (u[:, self.elem, :] * self.W).sum(-1)
        ue = u[0:6, self.uniq, :].permute(1, 2, 0).contiguous()  # (elements, nodes, 6)
        vq = torch.bmm(self.Wp, ue)  # (elements, points, 6)
        v = torch.zeros((9, self.W.shape[0]), dtype=u.dtype, device=u.device)
        v[0:6] = vq[self.uidx, self.slot].t()
        return v


def _set_dg(dom, u):
    if getattr(dom, "_zero_fd", None) is None:
        dom._zero_fd = torch.zeros(dom.fd_shape(), dtype=torch.float64, device=u.device)
        dom._zero_rep = torch.zeros((dom.E,), dtype=torch.int32, device=u.device)
    dom.set_state(u.contiguous(), dom._zero_fd, dom._zero_rep)


def time_integral(dom, u0, steps, dt, L):
    """Phi = sum_{n=1..steps} dt L(U^n) from U^0 = u0 (all DG)."""
    _set_dg(dom, u0)
    phi = torch.zeros((), dtype=torch.float64, device=u0.device)
    with torch.no_grad():
        for _ in range(steps):
            dom.step(1, dt)
            phi = phi + dt * L(dom.get_dg())
    return float(phi)


def time_integral_gradient(dom, u0, steps, dt, every, L):
    """(Phi, dPhi/dU^0) with checkpoints every `every` steps (see the module docstring)."""
    if dom.params.hybrid != grffe.HYBRID_DG_ONLY:
        raise grffe.GrffeError("the time-integral gradient differentiates all-DG steps: use hybrid = 0")
    every = max(1, int(every))
    ckpts = []
    phi = torch.zeros((), dtype=torch.float64, device=u0.device)
    _set_dg(dom, u0)
    with torch.no_grad():
        for n in range(steps):
            if n % every == 0:
                ckpts.append((n, dom.get_dg()))
            dom.step(1, dt)
            phi = phi + dt * L(dom.get_dg())
    lam = torch.zeros_like(u0)
    for n0, uc in reversed(ckpts):
        k = min(every, steps - n0)
        # the segment recomputed, with each step's stage values kept for its adjoint
        states, stages = [uc], []
        _set_dg(dom, uc)
        for _ in range(k):
            dom.step(1, dt)
            stages.append(dom.get_stages())
            states.append(dom.get_dg())
        for j in range(k - 1, -1, -1):
            lam = lam + dt * L.grad(states[j + 1])
            lam = dom.step_adjoint_stages(states[j], stages[j][0], stages[j][1], lam, dt)
    return float(phi), lam


class AdjointWorkload:
    """The black-hole adjoint workload: Kerr-Schild background of workload w (all
    elements on DG, elements meeting the excision radius removed), initial data
    kerr_schild_parametrised_field(parameters), objective SphereFlux at radius R."""

    PARAMS = ("B0", "tilt", "m", "d")

    def __init__(self, w, R=20.0, device="cuda"):
        N = w["degree"]
        self.w = w
        x, y, z = I.points(w["n_elem"], w["lower"], w["upper"], grffe.operator(N, 0))
        self.xyz = (x, y, z)
        E, n3 = int(np.prod(w["n_elem"])), (N + 1) ** 3
        with np.errstate(all="ignore"):
            bg = I.background(w, x, y, z).reshape(26, E, n3)
        self.exc = I.excision_mask(w).astype(bool)
        bg[:, self.exc] = I.flat_background((int(self.exc.sum()), n3))
        p = grffe.default_params(eta=w["eta"], cfl=w["cfl"], hybrid=grffe.HYBRID_DG_ONLY)
        self.dom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], N, w["bc"], params=p,
                                bg=torch.from_numpy(np.ascontiguousarray(bg)).to(device),
                                excised=self.exc.astype(np.uint8))
        self.dt = self.dom.dt()
        self.L = SphereFlux(w, R, device=device)
        self.E, self.n3, self.device = E, n3, device

    def initial(self, params):
        """U^0 (9, E, n^3) on the device for the parameter dict `params`."""
        with np.errstate(all="ignore"):
            u = I.kerr_schild_parametrised_field(*self.xyz, self.w["M"], self.w["spin"], **params)
        u = u.reshape(9, self.E, self.n3)
        u[:, self.exc] = 0.0
        return torch.from_numpy(np.ascontiguousarray(u)).to(self.device)

    def initial_derivatives(self, params, rel=1e-6):
        """dU^0/dp for every parameter p, by central differences of the analytic data."""
        out = {}
        for k in self.PARAMS:
            h = rel * max(1.0, abs(params[k]))
            up = self.initial(dict(params, **{k: params[k] + h}))
            um = self.initial(dict(params, **{k: params[k] - h}))
            out[k] = (up - um) / (2.0 * h)
        return out

    def phi(self, params, steps):
        return time_integral(self.dom, self.initial(params), steps, self.dt, self.L)

    def gradient(self, params, steps, every):
        """(Phi, {p: dPhi/dp}) through the checkpointed adjoint."""
        phi, lam = time_integral_gradient(self.dom, self.initial(params), steps, self.dt, every, self.L)
        du = self.initial_derivatives(params)
        return phi, {k: float((lam * du[k]).sum()) for k in self.PARAMS}

    def close(self):
        self.dom.close()
