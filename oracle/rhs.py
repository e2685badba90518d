"""Semi-discrete right-hand side on DG elements and on FD subcell elements.

TEST INFRASTRUCTURE ONLY (see oracle/operators.py).

DG (Sec. III A): nodal DG-SEM in strong form on GLL points with a lumped
mass matrix; with a Rusanov numerical flux F* at element faces (Sec. III C 2
names Rusanov for the FD grid; the same flux is used at DG faces):

    dU/dt = -sum_d (2/h_d) [ D_d F^d + W^-1 (e_N (F*_R - F_N) - e_0 (F*_L - F_0)) ] + S.

FD (Sec. III C 2, Eq. (fd time derivative)): conservative finite
differences on 2N+1 uniform subcells per axis, dimension by dimension:
WENO5-Z (exponent q = 2) reconstruction of the point values of U and of J~
to the subcell faces,
Rusanov flux F*, fourth-order corrector built from cell-centred fluxes
(Eq. (higher order flux correction)):

    Fhat_{i+1/2} = F*_{i+1/2} - (1/6) (F_i - 2 F*_{i+1/2} + F_{i+1}),
    dU_i/dt = -sum_d (2N+1)/h_d (Fhat_{i+1/2} - Fhat_{i-1/2}) + S(U_i).

Neighbour data across element faces: a DG neighbour's nodal trace; an FD
neighbour seen from a DG element is reconstructed with R (x) R (x) R; a DG
neighbour seen from an FD element is projected with P (x) P (x) P into three
ghost layers; at domain boundaries the no-incoming-Poynting state (Sec. III D)
is the external state / fills the ghost layers, except on Dirichlet faces
(Sec. IV A), whose fixed exterior state plays that role.

The densitized current J~ travels with U across DG<->FD interfaces: the
state handed over is W = (U, J~(U)) with J~ evaluated where U lives, and the
interpolation (R or P) acts on all 12 components.  Recomputing J~ from an
interpolated U would multiply the interpolation error of E.B by eta (this is
why the FD scheme reconstructs J~ rather than recomputing it at faces,
Sec. III C 2).
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from . import physics as ph
from .domain import DG, FD, axis_of, geo_take


def _take_slice(a, axis, idx):
    return np.take(a, idx, axis=axis)


def _slice_geo(geo, axis, idx):
    """Geometry at one index along a point axis (negative axis numbering)."""
    g = ph.Geometry.__new__(ph.Geometry)
    for k, v in vars(geo).items():
        setattr(g, k, np.take(v, idx, axis=axis))
    return g


def exterior(dom, elems, f, Ui, gi, layer=None):
    """External state at the boundary face f of each element of `elems` from its
    interior values Ui (9, len(elems), ...): the stored state on Dirichlet faces
    (the face's uniform row, or the point's entry of the per-point field: at the
    face nodes for a DG face, layer `layer` of the ghost cells for an FD face), the
    no-incoming-Poynting state of Ui elsewhere."""
    d, s = divmod(f, 2)
    Ub = ph.boundary_state(Ui, gi, d, +1 if s else -1)
    mask = dom.dirichlet_faces(elems, f)
    if np.any(mask):
        if dom.boundary_field is not None:
            if layer is None:
                n = dom.n
                fixed = dom.boundary_field[0][:, elems, f].reshape(9, len(elems), n, n)
            else:
                m = dom.m
                fixed = np.expand_dims(dom.boundary_field[1][:, elems, f, layer].reshape(9, len(elems), m, m),
                                       axis_of(d))
        else:
            fixed = np.broadcast_to(dom.boundary_state[f].reshape((9, 1) + (1,) * (Ui.ndim - 2)), Ui.shape)
        sel = mask.reshape((1, -1) + (1,) * (Ui.ndim - 2))
        Ub = np.where(sel, fixed, Ub)
    return Ub


def with_current(dom, U, geo):
    """W = (U, J~(U)): the 12 transported components at a set of points."""
    jd, je = ph.split_current(U, geo, dom.params["eta"])
    return np.concatenate([U, jd + je], axis=0)


def dg_rhs(dom, elems, W_dg, W_fd, rep, parts=3):
    """RHS of the DG elements ``elems``.

    W_dg (12, E, n, n, n) holds (U, J~) at the DG nodes of every element whose
    ``rep`` is DG, W_fd (12, E, m, m, m) that of every FD element.  Returns
    (9, len, n, n, n).  parts: 1 explicit operator only, 2 stiff source only,
    3 both.
    """
    p = dom.params
    elems = np.asarray(elems, np.int64)
    N = dom.N
    x, w = ops.gll(N)
    D = ops.diff_matrix(N)
    R = ops.reconstruction_matrix(N)
    U = W_dg[:9, elems]
    J = W_dg[9:, elems]
    geo = geo_take(dom.geo_dg, elems)
    out = np.zeros_like(U)
    if parts & 2:
        out += ph.source_stiff(U, geo, p["eta"], p["kappa_psi"], p["kappa_phi"])
    if not parts & 1:
        return out
    out += ph.source_explicit(U, geo, p["eta"])
    # neighbour DG views: FD neighbours reconstructed (U and J~) to DG nodes
    nbr_dg = W_dg.copy()
    fd_e = np.nonzero(rep == FD)[0]
    if fd_e.size:
        nbr_dg[:, fd_e] = ops.apply_3d(R, W_fd[:, fd_e])
    for d in range(3):
        ax = axis_of(d)
        scale = 2.0 / dom.h[d]
        F = ph.flux(U, geo, d, J)
        out -= scale * ops.apply_1d(D, F, ax)
        for s in (0, 1):
            f = 2 * d + s
            i_own = 0 if s == 0 else N
            i_nbr = N if s == 0 else 0
            Ui = _take_slice(U, ax, i_own)
            Ji = _take_slice(J, ax, i_own)
            gi = _slice_geo(geo, ax, i_own)
            Fi = _take_slice(F, ax, i_own)
            o = dom.nbr[elems, f]
            has = o >= 0
            oo = np.where(has, o, 0)
            Wx = _take_slice(nbr_dg[:, oo], ax, i_nbr)
            gx = _slice_geo(geo_take(dom.geo_dg, oo), ax, i_nbr)
            Ub = exterior(dom, elems, f, Ui, gi)
            Wb = with_current(dom, Ub, gi)
            Wx = np.where(has[None, :, None, None], Wx, Wb)
            # metric of the external side: the neighbour's face node, or the interior node at a boundary
            gx = _blend_geo(gx, gi, has)
            Ux, Jx = Wx[:9], Wx[9:]
            if s == 0:
                Fs = ph.rusanov(Ux, Ui, gx, gi, d, Jx, Ji)
                corr = scale * (Fs - Fi) / w[0]
            else:
                Fs = ph.rusanov(Ui, Ux, gi, gx, d, Ji, Jx)
                corr = -scale * (Fs - Fi) / w[N]
            sl = [slice(None)] * out.ndim
            sl[ax] = i_own
            out[tuple(sl)] += corr
    return out


def _blend_geo(gx, gi, has):
    """Per element: gx where ``has`` else gi (``has`` runs over the element axis)."""
    g = ph.Geometry.__new__(ph.Geometry)
    for k, v in vars(gx).items():
        vi = getattr(gi, k)
        nc = _n_comp_axes(k)
        mask = has.reshape((1,) * nc + has.shape + (1,) * (v.ndim - nc - 1))
        setattr(g, k, np.where(mask, v, vi))
    return g


def _n_comp_axes(k):
    if k in ("alpha", "sqrtg", "K"):
        return 0
    if k in ("beta", "dalpha", "Gam"):
        return 1
    return 2


def weno5z(vm2, vm1, v0, vp1, vp2, eps, q=2):
    """WENO5-Z value at face i+1/2 from the point values at cells i-2..i+2.

    The FD scheme holds point values, so the three candidate values are the
    quadratic Lagrange interpolants of the point values evaluated at the face
    (weights 3/8, -10/8, 15/8 etc.), combined with the optimal weights
    (1/16, 10/16, 5/16) of the fifth-order interpolant; the nonlinear weights
    are the Z weights of Borges et al. (2008) with tau5 = |beta0 - beta2|,
    Jiang-Shu smoothness indicators and exponent q (Sec. III C 2).
    """
    q0 = (3.0 * vm2 - 10.0 * vm1 + 15.0 * v0) / 8.0
    q1 = (-vm1 + 6.0 * v0 + 3.0 * vp1) / 8.0
    q2 = (3.0 * v0 + 6.0 * vp1 - vp2) / 8.0
    b0 = 13.0 / 12.0 * (vm2 - 2.0 * vm1 + v0) ** 2 + 0.25 * (vm2 - 4.0 * vm1 + 3.0 * v0) ** 2
    b1 = 13.0 / 12.0 * (vm1 - 2.0 * v0 + vp1) ** 2 + 0.25 * (vm1 - vp1) ** 2
    b2 = 13.0 / 12.0 * (v0 - 2.0 * vp1 + vp2) ** 2 + 0.25 * (3.0 * v0 - 4.0 * vp1 + vp2) ** 2
    tau = np.abs(b0 - b2)
    a0 = (1.0 / 16.0) * (1.0 + (tau / (b0 + eps)) ** q)
    a1 = (10.0 / 16.0) * (1.0 + (tau / (b1 + eps)) ** q)
    a2 = (5.0 / 16.0) * (1.0 + (tau / (b2 + eps)) ** q)
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


def ghost_extended(dom, elems, W_own, geo_own, W_dg, W_fd, rep, d):
    """Own FD (U, J~) plus 3 ghost layers on each side along direction d.

    Returns (W_ext, geo_ext) with 2N+7 cells along axis d.  Ghost values come
    from the neighbour's FD cells, from P (x) P (x) P of a DG neighbour, or
    from the no-incoming-Poynting state of the outermost own cell.
    """
    m = dom.m
    ax = axis_of(d)
    P = ops.projection_matrix(dom.N)
    parts, gparts = {}, {}
    for s in (0, 1):
        f = 2 * d + s
        o = dom.nbr[elems, f]
        has = o >= 0
        oo = np.where(has, o, 0)
        nbr_fd = W_fd[:, oo].copy()
        isdg = has & (rep[oo] == DG)
        if np.any(isdg):
            nbr_fd[:, isdg] = ops.apply_3d(P, W_dg[:, oo[isdg]])
        idx = np.arange(m - 3, m) if s == 0 else np.arange(0, 3)
        G = np.take(nbr_fd, idx, axis=ax)
        gG = _take_geo_idx(geo_take(dom.geo_fd, oo), ax, idx)
        i_out = 0 if s == 0 else m - 1
        Ui = np.take(W_own[:9], [i_out], axis=ax)
        gi = _take_geo_idx(geo_own, ax, [i_out])
        # ghost layers l = 0, 1, 2 counted outwards from the face, in their order
        # along the axis
        layers = [with_current(dom, exterior(dom, elems, f, Ui, gi, layer=l), gi) for l in range(3)]
        Wb = np.concatenate(layers[::-1] if s == 0 else layers, axis=ax)
        gb = _take_geo_idx(geo_own, ax, [i_out, i_out, i_out])
        mask = has[None, :, None, None, None]
        parts[s] = np.where(mask, G, Wb)
        gparts[s] = _blend_geo(gG, gb, has)
    W_ext = np.concatenate([parts[0], W_own, parts[1]], axis=ax)
    geo_ext = _concat_geo([gparts[0], geo_own, gparts[1]], ax)
    return W_ext, geo_ext


def _take_geo_idx(geo, ax, idx):
    g = ph.Geometry.__new__(ph.Geometry)
    for k, v in vars(geo).items():
        setattr(g, k, np.take(v, idx, axis=ax))
    return g


def _concat_geo(gs, ax):
    g = ph.Geometry.__new__(ph.Geometry)
    for k in vars(gs[0]):
        setattr(g, k, np.concatenate([getattr(x, k) for x in gs], axis=ax))
    return g


def fd_rhs(dom, elems, W_own, W_dg, W_fd, rep, parts=3):
    """RHS of FD elements ``elems`` whose own subcell (U, J~) is W_own (12, len, m, m, m).

    Neighbour data comes from W_dg / W_fd according to ``rep``.
    """
    p = dom.params
    elems = np.asarray(elems, np.int64)
    m = dom.m
    geo = geo_take(dom.geo_fd, elems)
    V = W_own[:9]
    out = np.zeros_like(V)
    if parts & 2:
        out += ph.source_stiff(V, geo, p["eta"], p["kappa_psi"], p["kappa_phi"])
    if not parts & 1:
        return out
    out += ph.source_explicit(V, geo, p["eta"])
    eps = p["weno_eps"]
    for d in range(3):
        ax = axis_of(d)
        W, ge = ghost_extended(dom, elems, W_own, geo, W_dg, W_fd, rep, d)

        def c(k0, count):  # cells k0 .. k0+count-1 of the extended array
            return np.take(W, np.arange(k0, k0 + count), axis=ax)

        nf = m + 1
        # face i+1/2 for i = -1..m-1  <->  extended cell index i+3 = 2..m+2
        left = weno5z(c(0, nf), c(1, nf), c(2, nf), c(3, nf), c(4, nf), eps)
        right = weno5z(c(5, nf), c(4, nf), c(3, nf), c(2, nf), c(1, nf), eps)
        gf = geo_take(dom.geo_face[d], elems)
        Fs = ph.rusanov(left[:9], right[:9], gf, gf, d, left[9:], right[9:])
        if p["fd_order"] == 4:
            Fc = ph.flux(W[:9], ge, d, W[9:])  # cell-centred fluxes on the extended cells
            Fm = np.take(Fc, np.arange(2, 2 + nf), axis=ax)  # F_i for i = -1..m-1
            Fp = np.take(Fc, np.arange(3, 3 + nf), axis=ax)  # F_{i+1}
            Fh = Fs - (Fm - 2.0 * Fs + Fp) / 6.0
        else:
            Fh = Fs
        dF = np.take(Fh, np.arange(1, m + 1), axis=ax) - np.take(Fh, np.arange(0, m), axis=ax)
        out -= (m / dom.h[d]) * dF
    return out


def rhs(dom, U_dg, U_fd, rep, parts=3):
    """Semi-discrete dU/dt of every active element in its representation."""
    out_dg = np.zeros_like(U_dg)
    out_fd = np.zeros_like(U_fd)
    act = dom.active
    dg_e = np.nonzero(act & (rep == DG))[0]
    fd_e = np.nonzero(act & (rep == FD))[0]
    W_dg = with_current(dom, U_dg, dom.geo_dg)
    W_fd = with_current(dom, U_fd, dom.geo_fd)
    if dg_e.size:
        out_dg[:, dg_e] = dg_rhs(dom, dg_e, W_dg, W_fd, rep, parts)
    if fd_e.size:
        out_fd[:, fd_e] = fd_rhs(dom, fd_e, W_fd[:, fd_e], W_dg, W_fd, rep, parts)
    return out_dg, out_fd
