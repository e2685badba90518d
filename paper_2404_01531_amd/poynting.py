"""The objective of the adjoint workload and the checkpointed gradient of a time
integral of such an objective.

SphereFlux(w) evaluates, for a state U of workload w, the outgoing Poynting flux
through the Euclidean sphere of radius R,
    L(U) = sum_q w_q sqrt(gamma) S^i x_i / R,   S^i = eps^{ijk} E_j B_k,
eps^{ijk} = [ijk] / sqrt(gamma), E = E~ / sqrt(gamma), B = B~ / sqrt(gamma)
(Sec. II A; the flux through a coordinate sphere as in the paper's magnetosphere
diagnostics), with the fields taken from the DG polynomial of the element that
contains each quadrature point (for an element on FD, the polynomial R U_FD of its
subcell values, R the FD-to-DG reconstruction of Sec. III C 1) and the background
metric evaluated there.  It is a small torch function of the state (a user's
objective), not part of the solver.

time_integral_gradient(dom, u0, steps, dt, every, L) returns
    Phi = sum_{n=1..steps} dt L(U^n)
and dPhi/dU^0, by the adjoint recursion
    lam_steps = dt dL/dU^steps,  lam_n = (dU^{n+1}/dU^n)^T lam_{n+1} + dt dL/dU^n,
with the states kept every `every` steps and each segment recomputed from its
checkpoint; every step and step adjoint runs in the HIP library.  All-DG domains
keep each recomputed step's stage values, so their step adjoints need no forward
re-run.  Domains with the hybrid control (adaptive or forced) carry the state as
(U_DG, U_FD, representation), and each step adjoint re-runs its step to take the
decisions (rollbacks, switches back) of the forward pass as fixed
(grffe_step_adjoint_frozen): the gradient is that of the piecewise-smooth map on
the branch the forward pass took.
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
        self.n, self.m = n, 2 * N + 1
        self.Rm = torch.from_numpy(np.ascontiguousarray(grffe.operator(N, 6).reshape(n, 2 * N + 1))).to(device)
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

    def _recon(self, f):
        """R (x) R (x) R of FD values f (c, k, m^3) -> (c, k, n^3); axes (z, y, x)."""
        c, k = f.shape[0], f.shape[1]
        n, m, R = self.n, self.m, self.Rm
        x = f.reshape(-1, m) @ R.t()                                       # x axis
        x = x.reshape(c, k, m, m, n).transpose(3, 4).contiguous()          # (z, x, y)
        x = (x.reshape(-1, m) @ R.t()).reshape(c, k, m, n, n)              # y axis
        x = x.permute(0, 1, 3, 4, 2).contiguous()                          # (x, y, z)
        x = (x.reshape(-1, m) @ R.t()).reshape(c, k, n, n, n)              # z axis
        return x.permute(0, 1, 4, 3, 2).contiguous().reshape(c, k, n ** 3)  # (z, y, x)

    def _recon_t(self, g):
        """The transpose of _recon: (c, k, n^3) -> (c, k, m^3)."""
        c, k = g.shape[0], g.shape[1]
        n, m, R = self.n, self.m, self.Rm
        x = g.reshape(-1, n) @ R                                           # x axis
        x = x.reshape(c, k, n, n, m).transpose(3, 4).contiguous()          # (z, x, y)
        x = (x.reshape(-1, n) @ R).reshape(c, k, n, m, m)                  # y axis
        x = x.permute(0, 1, 3, 4, 2).contiguous()                          # (x, y, z)
        x = (x.reshape(-1, n) @ R).reshape(c, k, m, m, m)                  # z axis
        return x.permute(0, 1, 4, 3, 2).contiguous().reshape(c, k, m ** 3)  # (z, y, x)

    def _nodal(self, u, fd, rep):
        """(elements holding points, n^3, 6): the six field rows of the point-holding
        elements at their DG nodes, from fd through R where rep says FD."""
        ue = u[0:6, self.uniq, :]
        if fd is not None:
            # formed for every point-holding element (a few hundred small products),
            # so that no host synchronisation decides which
            onfd = (rep[self.uniq] == 1).view(1, -1, 1)
            ue = torch.where(onfd, self._recon(fd[0:6, self.uniq, :]), ue)
        return ue.permute(1, 2, 0).contiguous()

    def __call__(self, u, fd=None, rep=None):
        """L(U) for the state u, (9, E, (N+1)^3) float64 on the device; with fd and rep
        (the FD state and the representation), elements on FD are read from fd."""
        v = self._at_points(u, fd, rep)  # (9, Q) at the sphere points
        E = v[0:3] / self.sg
        B = v[3:6] / self.sg
        El = (self.g * E[None]).sum(1)
        Bl = (self.g * B[None]).sum(1)
        # sqrt(gamma) eps^{ijk} E_j B_k x_i = x . (E_lo x B_lo)
        flux = (self.x * torch.linalg.cross(El, Bl, dim=0)).sum(0) / self.R
        return (self.wq * flux).sum()

    def grad(self, u, fd=None, rep=None):
        """dL/dU, written out: with x . (E_lo x B_lo) = E_lo . (B_lo x x) = B_lo . (x x E_lo),
        dL/dE~ = g (B_lo x x) w / (R sqrt(gamma)), dL/dB~ = g (x x E_lo) w / (R sqrt(gamma)) at
        the points, spread to the nodes of the containing elements with the
        interpolation weights.  With fd and rep: (dL/dU_DG, dL/dU_FD), the nodes'
        gradient of an element on FD taken to its cells through R^T."""
        v = self._at_points(u, fd, rep)
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
        ge = torch.bmm(self.WpT, dvp).permute(2, 0, 1)  # (6, elements, nodes)
        out = torch.zeros_like(u)
        if fd is None:
            out[0:6, self.uniq, :] = ge
            return out
        out_fd = torch.zeros_like(fd)
        onfd = (rep[self.uniq] == 1).view(1, -1, 1)
        zero = torch.zeros((), dtype=ge.dtype, device=ge.device)
        out[0:6, self.uniq, :] = torch.where(onfd, zero, ge)
        out_fd[0:6, self.uniq, :] = torch.where(onfd, self._recon_t(ge.contiguous()), zero)
        return out, out_fd

    def _at_points(self, u, fd=None, rep=None):
        """The interpolants at the points, (9, Q); only the six field rows are formed
        (the other three are zero)."""
        if u.requires_grad:
            return (u[:, self.elem, :] * self.W).sum(-1)
        ue = self._nodal(u, fd, rep)  # (elements, nodes, 6)
        vq = torch.bmm(self.Wp, ue)  # (elements, points, 6)
        v = torch.zeros((9, self.W.shape[0]), dtype=u.dtype, device=u.device)
        v[0:6] = vq[self.uidx, self.slot].t()
        return v


def _set_dg(dom, u):
    if getattr(dom, "_zero_fd", None) is None:
        dom._zero_fd = torch.zeros(dom.fd_shape(), dtype=torch.float64, device=u.device)
        dom._zero_rep = torch.zeros((dom.E,), dtype=torch.int32, device=u.device)
    dom.set_state(u.contiguous(), dom._zero_fd, dom._zero_rep)


def _dg_only(dom):
    return dom.params.hybrid == grffe.HYBRID_DG_ONLY


def time_integral(dom, u0, steps, dt, L, log=None):
    """Phi = sum_{n=1..steps} dt L(U^n) from U^0 = u0 (every element starting on DG).
    log (a list, hybrid domains only) receives the representation after every step."""
    _set_dg(dom, u0)
    phi = torch.zeros((), dtype=torch.float64, device=u0.device)
    with torch.no_grad():
        for _ in range(steps):
            dom.step(1, dt)
            if _dg_only(dom):
                phi = phi + dt * L(dom.get_dg())
                continue
            st = dom.get_state()
            phi = phi + dt * L(*st)
            if log is not None:
                log.append(st[2].clone())
    return float(phi)


def time_integral_gradient(dom, u0, steps, dt, every, L, log=None):
    """(Phi, dPhi/dU^0) with checkpoints every `every` steps (see the module docstring).
    U^0 = u0 has every element on DG, so dPhi/dU^0 is a DG array.  log (a list, hybrid
    domains only) receives the representation after every step of the forward pass."""
    if _dg_only(dom):
        return _gradient_dg(dom, u0, steps, dt, every, L)
    return _gradient_hybrid(dom, u0, steps, dt, every, L, log)


def _gradient_dg(dom, u0, steps, dt, every, L):
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


def _gradient_hybrid(dom, u0, steps, dt, every, L, log):
    # the forward pass keeps the checkpoints and every state of the last segment, so
    # that segment needs no recomputation (with every >= steps, none does: one state
    # per step is held, (9 (n^3 + m^3) E + E) values each)
    every = max(1, int(every))
    ckpts, last = [], []
    last_start = ((steps - 1) // every) * every if steps > 0 else 0
    phi = torch.zeros((), dtype=torch.float64, device=u0.device)
    _set_dg(dom, u0)
    with torch.no_grad():
        for n in range(steps):
            if n % every == 0 and n < last_start:
                ckpts.append((n, dom.get_state()))
            if n == last_start:
                last.append(dom.get_state())
            dom.step(1, dt)
            st = dom.get_state()
            phi = phi + dt * L(*st)
            if n >= last_start:
                last.append(st)
            if log is not None:
                log.append(st[2].clone())
    lam_dg = torch.zeros_like(u0)
    lam_fd = torch.zeros(dom.fd_shape(), dtype=torch.float64, device=u0.device)
    segments = [(last_start, None)] + [(n0, sc) for n0, sc in reversed(ckpts)]
    for n0, sc in segments:
        k = min(every, steps - n0)
        if sc is None:
            states = last
        else:
            states = [sc]
            dom.set_state(*sc)
            for _ in range(k):
                dom.step(1, dt)
                states.append(dom.get_state())
        for j in range(k - 1, -1, -1):
            g_dg, g_fd = L.grad(*states[j + 1])
            lam_dg = lam_dg + dt * g_dg
            lam_fd = lam_fd + dt * g_fd
            lam_dg, lam_fd = dom.step_adjoint_frozen(*states[j], lam_dg, lam_fd, dt)
    return float(phi), lam_dg


class AdjointWorkload:
    """The black-hole adjoint workload: Kerr-Schild background of workload w (elements
    meeting the excision radius removed), initial data
    kerr_schild_parametrised_field(parameters) on DG, objective SphereFlux at radius R;
    hybrid = HYBRID_DG_ONLY keeps every element on DG, HYBRID_ADAPTIVE runs the
    indicator and differentiates with its decisions frozen."""

    PARAMS = ("B0", "tilt", "m", "d")

    def __init__(self, w, R=20.0, device="cuda", hybrid=grffe.HYBRID_DG_ONLY):
        N = w["degree"]
        self.w = w
        x, y, z = I.points(w["n_elem"], w["lower"], w["upper"], grffe.operator(N, 0))
        self.xyz = (x, y, z)
        E, n3 = int(np.prod(w["n_elem"])), (N + 1) ** 3
        with np.errstate(all="ignore"):
            bg = I.background(w, x, y, z).reshape(26, E, n3)
        self.exc = I.excision_mask(w).astype(bool)
        bg[:, self.exc] = I.flat_background((int(self.exc.sum()), n3))
        p = grffe.default_params(eta=w["eta"], cfl=w["cfl"], hybrid=hybrid)
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

    def phi(self, params, steps, log=None):
        return time_integral(self.dom, self.initial(params), steps, self.dt, self.L, log)

    def gradient(self, params, steps, every, log=None):
        """(Phi, {p: dPhi/dp}) through the checkpointed adjoint."""
        phi, lam = time_integral_gradient(self.dom, self.initial(params), steps, self.dt, every, self.L, log)
        du = self.initial_derivatives(params)
        return phi, {k: float((lam * du[k]).sum()) for k in self.PARAMS}

    def close(self):
        self.dom.close()
