"""Spherical shell of cubed-sphere wedges with curved element maps; the DG
right-hand side and the DG step on it.

TEST INFRASTRUCTURE ONLY (see oracle/operators.py).

Grid (Sec. IV B, the black-hole grid; Sec. III A, the map x(xi) of each element):
the shell r_in <= r <= r_out is cut into six wedges, one about each of the
directions +x, -x, +y, -y, +z, -z.  A wedge has coordinates (A, B, Z) in
[-1, 1]^3 with the equiangular map along the two angular directions and the
logarithmic map along the radial one,

    X = tan(pi A / 4),  Y = tan(pi B / 4),  r = r_in (r_out / r_in)^((Z + 1) / 2),
    local point  r (X, Y, 1) / sqrt(1 + X^2 + Y^2),

and the local axes (1, 2, 3) are turned onto (s e_{k+1}, e_{k+2}, s e_k) for the
wedge about s e_k (s = +-1, indices mod 3; a proper rotation).  Wedge w = 2 k +
(0 for s = +1, 1 for s = -1) is cut into n_radial x n_angular x n_angular
elements of equal extent in (A, B, Z); element e = w n_r n_a^2 + ir n_a^2 +
ib n_a + ia, with its reference coordinates (xi^1, xi^2, xi^3) along (A, B, Z),
node (i, j, k) along them, arrays over nodes with axes (..., k, j, i) as on the
Cartesian grid.

DG on curved elements (Sec. III A): nodal DG-SEM in strong form with a lumped
GLL mass matrix.  The divergence of the flux is the logical derivative of every
Cartesian flux component contracted with the inverse Jacobian at the node,

    dU/dt = S - sum_{i, j} (d xi^i / d x^j) D_i F^j - sum_faces lift,

the same placement of the inverse Jacobian as in the paper's FD time derivative
(Eq. (fd time derivative)).  At a node of the face xi^i = +-1 with outward
covector m = +-grad xi^i (the row i of the inverse Jacobian, unnormalised) the
lift is (1 / w_end) (G*(m) - m_j F^j(U_int)), with the Rusanov flux along m

    G*(m) = (m_j F^j(U_int) + m_j F^j(U_ext)) / 2 - lambda(m) (U_ext - U_int) / 2,
    lambda(m) = alpha sqrt(gamma^{jk} m_j m_k) + |beta^j m_j|,

the largest characteristic speed along m times |m| (both homogeneous of degree
one in m, so no normalisation enters).  On an axis-aligned affine element this
is the Cartesian operator term by term.  Neighbours across wedge faces have
their own orientation; the exterior state of a face node is the neighbour's
node at the same point, found by matching coordinates.

Boundaries: the inner and outer spheres take one of: Dirichlet (a given
exterior state at every face node), outflow (no boundary condition, the
exterior state is the interior one, so the face adds nothing: the inner
boundary of the exact-Wald test inside the horizon, Sec. IV B 1), or the
no-incoming-Poynting state along the face normal (Sec. III D).

FD subcells on curved elements (Sec. III C 2, Eq. (fd time derivative), with the
second-order flux F-hat = F* since the fourth-order corrector is Cartesian only):
the (2N+1)^3 cells are uniform in the reference coordinates; along each reference
direction xi^d the point values of U and of the three components of J~ are
reconstructed to the cell faces with WENO5-Z (the Cartesian flux of every direction
needs its component of J~).  At a face the Rusanov flux is formed for each
Cartesian component j with the dissipation along the face's unit covector
nu = grad xi^d / |grad xi^d| (Euclidean norm, closed form at the face),

    F-hat^j = (F^j(U_L) + F^j(U_R)) / 2 - lambda(nu) (U_R - U_L) nu_j / 2,

so that nu_j F-hat^j is the Rusanov flux along nu, and the time derivative is the
paper's contraction with the inverse Jacobian at the cell centre,

    dU/dt = S - sum_{d, j} (d xi^d / d x^j) (F-hat^j_{i+1/2} - F-hat^j_{i-1/2}) / dxi,

dxi = 2 / (2N+1).  On an axis-aligned box cell this is the Cartesian scheme term
by term.  Ghost cells (three layers per face) are the neighbour's cells next to
the shared face, in the neighbour's own orientation (faces between wedges are
matched by the positions of the face-cell centres), from its FD state or from P
(x) P (x) P of a DG neighbour's (U, J~); on the spheres the outermost own cell
(outflow), its no-incoming-Poynting state along the outward covector, or a given
exterior state per ghost cell (Dirichlet).  The metric at the cells and faces is
the nodal background evaluated there as a polynomial (as on the Cartesian grid).
A DG element next to an FD element takes the exterior (U, J~) of a face node from R
(x) R (x) R of the neighbour's cells at the matched node.  The hybrid control
(indicator, rollback, switch back) is the Cartesian grid's step with these two
right-hand sides.

Time step (Eq. (spectre DG CFL condition)): (dx)_min is the smallest distance
between neighbouring DG nodes along a reference line, lambda_max the largest
alpha + |beta|_gamma over the nodes (the largest characteristic speed over all
directions); this reading gives the exact-Wald table's nine time steps.
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from . import physics as ph
from .domain import DG, FD, axis_of, default_params, face_shape, geo_take
from .rhs import weno5z as ph_weno
from .rhs import with_current
from .step import _candidate, _filter_fn, derived_stages

SHELL_DIRICHLET = 2
SHELL_NO_INCOMING_POYNTING = 1
SHELL_OUTFLOW = 3


def wedge_axes(w):
    """Columns: the images of the wedge's local axes 1, 2, 3 (a rotation)."""
    k, s = w // 2, (1.0 if w % 2 == 0 else -1.0)
    R = np.zeros((3, 3))
    R[(k + 1) % 3, 0] = s
    R[(k + 2) % 3, 1] = 1.0
    R[k, 2] = s
    return R


class Shell:
    def __init__(self, degree, n_radial, n_angular, r_in, r_out, bc_inner=SHELL_OUTFLOW, bc_outer=SHELL_DIRICHLET,
                 bg=None, params=None, boundary_field=None):
        self.N = int(degree)
        self.n = self.N + 1
        self.m = 2 * self.N + 1
        self.nr, self.na = int(n_radial), int(n_angular)
        self.r_in, self.r_out = float(r_in), float(r_out)
        self.bc_inner, self.bc_outer = int(bc_inner), int(bc_outer)
        self.E = 6 * self.nr * self.na * self.na
        self.params = default_params() if params is None else {**default_params(), **params}
        self.x_dg = self.points(fd=False)
        self.dxdxi = self.jacobian(fd=False)  # [a][i] = d x^a / d xi^i
        jm = np.moveaxis(self.dxdxi, (0, 1), (-2, -1))
        self.invJ = np.moveaxis(np.linalg.inv(jm), (-2, -1), (0, 1))  # [i][a] = d xi^i / d x^a
        self.detJ = np.linalg.det(jm)
        shape = (self.E, self.n, self.n, self.n)
        self.bg = None if bg is None else np.asarray(bg, np.float64)
        self.geo = ph.Geometry(self.bg, shape)
        # exterior states of Dirichlet spheres at every face node (9, E, 6, n^2); may be
        # set after construction (it is usually computed from the node coordinates)
        self.boundary_field = None if boundary_field is None else np.asarray(boundary_field, np.float64)
        # exterior states of Dirichlet spheres at the FD ghost cells (9, E, 6, 3, m^2): layer l
        # counted outwards from the face, face cell t1 + m t2; needed only where an FD
        # element touches a Dirichlet sphere
        self.boundary_field_fd = None
        self._connect()
        self._fd_geometry()
        # what the hybrid step of the Cartesian grid reads
        self.geo_dg = self.geo
        self.active = np.ones(self.E, bool)
        self.conductor = None
        self.rhs_pair = (shell_dg_rhs, shell_fd_rhs)

    # ------------------------------------------------------------------ map
    def element_index(self, w, ir, ib, ia):
        return ((w * self.nr + ir) * self.na + ib) * self.na + ia

    def _wedge_coords(self, e, refs):
        """Wedge coordinates (A, B, Z) of element e on the tensor grid of the 1D
        reference points refs = (along xi^1, xi^2, xi^3), each with axes (Z, B, A)."""
        na, nr = self.na, self.nr
        ia, ib = e % na, (e // na) % na
        ir, w = (e // (na * na)) % nr, e // (na * na * nr)
        A = -1.0 + (ia + 0.5 * (refs[0] + 1.0)) * 2.0 / na
        B = -1.0 + (ib + 0.5 * (refs[1] + 1.0)) * 2.0 / na
        Z = -1.0 + (ir + 0.5 * (refs[2] + 1.0)) * 2.0 / nr
        ZZ, BB, AA = np.meshgrid(Z, B, A, indexing="ij")
        return w, AA, BB, ZZ

    def _ref(self, fd):
        return ops.fd_centres(self.N) if fd else ops.gll(self.N)[0]

    def map_points(self, e, ref1, ref2, ref3):
        """x(xi) of element e at the reference points (ref3, ref2, ref1) (arrays of one
        shape; complex arguments are carried through, for derivative checks)."""
        na, nr = self.na, self.nr
        ia, ib = e % na, (e // na) % na
        ir, w = (e // (na * na)) % nr, e // (na * na * nr)
        A = -1.0 + (ia + 0.5 * (ref1 + 1.0)) * 2.0 / na
        B = -1.0 + (ib + 0.5 * (ref2 + 1.0)) * 2.0 / na
        Z = -1.0 + (ir + 0.5 * (ref3 + 1.0)) * 2.0 / nr
        X, Y = np.tan(0.25 * np.pi * A), np.tan(0.25 * np.pi * B)
        r = self.r_in * (self.r_out / self.r_in) ** (0.5 * (Z + 1.0))
        s = r / np.sqrt(1.0 + X * X + Y * Y)
        return np.einsum("al,l...->a...", wedge_axes(w), np.stack([s * X, s * Y, s]))

    def _refs(self, fd, face_dir=None):
        """Reference points per axis: DG nodes, FD cell centres, or (face_dir = d) the FD
        faces along xi^d and the cell centres along the other two axes."""
        r = self._ref(fd)
        refs = [r, r, r]
        if face_dir is not None:
            refs[face_dir] = ops.fd_faces(self.N)
        return refs

    def points(self, fd=False, face_dir=None):
        """Cartesian coordinates (3, E, k3, k2, k1) of the DG nodes, the FD cell centres,
        or the FD faces normal to xi^face_dir."""
        refs = self._refs(fd, face_dir)
        R3, R2, R1 = np.meshgrid(refs[2], refs[1], refs[0], indexing="ij")
        out = np.empty((3, self.E) + R1.shape)
        for e in range(self.E):
            out[:, e] = self.map_points(e, R1, R2, R3)
        return out

    def jacobian(self, fd=False, face_dir=None):
        """d x^a / d xi^i (3, 3, E, k3, k2, k1) in closed form (chain rule through X, Y, r)."""
        refs = self._refs(fd, face_dir)
        out = np.empty((3, 3, self.E, refs[2].size, refs[1].size, refs[0].size))
        for e in range(self.E):
            w, A, B, Z = self._wedge_coords(e, refs)
            X, Y = np.tan(0.25 * np.pi * A), np.tan(0.25 * np.pi * B)
            r = self.r_in * (self.r_out / self.r_in) ** (0.5 * (Z + 1.0))
            rho = np.sqrt(1.0 + X * X + Y * Y)
            v = np.stack([X, Y, np.ones_like(X)])
            dL_dX = r * (np.stack([np.ones_like(X), 0 * X, 0 * X]) / rho - X * v / rho ** 3)
            dL_dY = r * (np.stack([0 * X, np.ones_like(X), 0 * X]) / rho - Y * v / rho ** 3)
            dL_dr = v / rho
            dX_dxi = 0.25 * np.pi * (1.0 + X * X) / self.na
            dY_dxi = 0.25 * np.pi * (1.0 + Y * Y) / self.na
            dr_dxi = 0.5 * r * np.log(self.r_out / self.r_in) / self.nr
            local = np.stack([dL_dX * dX_dxi, dL_dY * dY_dxi, dL_dr * dr_dxi], axis=1)  # [l][i]
            out[:, :, e] = np.einsum("al,li...->ai...", wedge_axes(w), local)
        return out

    # ---------------------------------------------------------- connectivity
    def face_nodes(self, x, f):
        """Values (..., E, n^2) of x (..., E, n, n, n) at the nodes of face f = 2 i + s,
        node t1 + n t2 with t1 along the lower tangential reference axis."""
        i, s = divmod(f, 2)
        a = np.take(x, self.N if s else 0, axis=axis_of(i))
        return a.reshape(a.shape[:-2] + (self.n * self.n,))

    def _face_volume_index(self, f):
        """Flat node index i + n (j + n k) of each node of face f, in face order."""
        idx = np.arange(self.n ** 3).reshape(self.n, self.n, self.n)
        return self.face_nodes(idx, f)

    def _connect(self):
        """nbr[e, f]: neighbour across face f (-1 on the inner sphere, -2 on the outer);
        nbr_node[e, f, t]: flat node index, in the neighbour, of the point of face node t."""
        E, n = self.E, self.n
        self.nbr = np.full((E, 6), -1, np.int64)
        self.nface = np.full((E, 6), -1, np.int64)  # the neighbour's face towards e
        self.nbr_node = np.full((E, 6, n * n), -1, np.int64)
        fx = [np.moveaxis(self.face_nodes(self.x_dg, f), 0, -1) for f in range(6)]  # (E, n^2, 3)
        scale = 1e-9 * self.r_out
        table = {}
        for e in range(E):
            for f in range(6):
                key = tuple(np.round(fx[f][e].mean(axis=0) / scale).astype(np.int64))
                table.setdefault(key, []).append((e, f))
        vidx = [self._face_volume_index(f) for f in range(6)]
        for pair in table.values():
            if len(pair) == 1:
                e, f = pair[0]
                if f not in (4, 5):
                    raise RuntimeError("an angular face without a neighbour")
                ir = (e // (self.na * self.na)) % self.nr
                if (f == 4 and ir != 0) or (f == 5 and ir != self.nr - 1):
                    raise RuntimeError("a radial face inside the shell without a neighbour")
                self.nbr[e, f] = -1 if f == 4 else -2
                continue
            if len(pair) != 2:
                raise RuntimeError("a face shared by more than two elements")
            for (e, f), (o, fo) in (pair, pair[::-1]):
                self.nbr[e, f] = o
                self.nface[e, f] = fo
                d = np.linalg.norm(fx[f][e][:, None, :] - fx[fo][o][None, :, :], axis=-1)
                t = np.argmin(d, axis=1)
                if np.max(d[np.arange(n * n), t]) > scale or len(set(t.tolist())) != n * n:
                    raise RuntimeError("face nodes of neighbours do not coincide")
                self.nbr_node[e, f] = vidx[fo][t]

    def _fd_geometry(self):
        """FD subcells: the metric at the cell centres and faces (the nodal background
        evaluated there as a polynomial), the inverse Jacobian at the cell centres, the
        unit covectors grad xi^d / |grad xi^d| at the faces normal to xi^d (both in
        closed form), and the ghost-cell table."""
        E, m = self.E, self.m
        jc = np.moveaxis(self.jacobian(fd=True), (0, 1), (-2, -1))
        self.invJ_fd = np.moveaxis(np.linalg.inv(jc), (-2, -1), (0, 1))  # [d][j] at the cells
        self.nu_face = []
        for d in range(3):
            jf = np.moveaxis(self.jacobian(fd=True, face_dir=d), (0, 1), (-2, -1))
            row = np.moveaxis(np.linalg.inv(jf), (-2, -1), (0, 1))[d]  # grad xi^d, (3, E, faces)
            self.nu_face.append(row / np.sqrt((row * row).sum(axis=0)))
        if self.bg is None:
            self.geo_fd = ph.Geometry(None, (E, m, m, m))
            self.geo_face = [ph.Geometry(None, face_shape(E, m, d)) for d in range(3)]
        else:
            P, Q = ops.projection_matrix(self.N), ops.face_eval_matrix(self.N)
            self.geo_fd = ph.Geometry(ops.apply_3d(P, self.bg))
            self.geo_face = []
            for d in range(3):
                b = self.bg
                for dd in range(3):
                    b = ops.apply_1d(Q if dd == d else P, b, axis_of(dd))
                self.geo_face.append(ph.Geometry(b))
        # nbr_cell[e, f, l, t]: flat cell index, in the neighbour across face f, of ghost
        # layer l (0 next to the face) at face cell t = t1 + m t2; the face-cell centres
        # of the two sides of a face are matched by position
        self.nbr_cell = np.full((E, 6, 3, m * m), -1, np.int64)
        fc = []
        for f in range(6):
            d, s = divmod(f, 2)
            a = np.take(self.points(fd=True, face_dir=d), m if s else 0, axis=axis_of(d))
            fc.append(np.moveaxis(a.reshape(3, E, m * m), 0, -1))  # (E, m^2, 3)
        scale = 1e-9 * self.r_out
        for e in range(E):
            for f in range(6):
                o, fo = self.nbr[e, f], self.nface[e, f]
                if o < 0:
                    continue
                dist = np.linalg.norm(fc[f][e][:, None, :] - fc[fo][o][None, :, :], axis=-1)
                t = np.argmin(dist, axis=1)
                if np.max(dist[np.arange(m * m), t]) > scale or len(set(t.tolist())) != m * m:
                    raise RuntimeError("face cells of neighbours do not coincide")
                for l in range(3):
                    self.nbr_cell[e, f, l] = self.cell_index(fo, l, t)

    def cell_index(self, f, l, t):
        """Flat cell index i + m j + m^2 k of the cell in layer l (0 next to the face) under
        face f = 2 d + s at face cell t = t1 + m t2 (t1 along the lower tangential axis)."""
        m = self.m
        d, s = divmod(f, 2)
        t = np.asarray(t)
        idx = [None, None, None]
        idx[d] = np.full(t.shape, (m - 1 - l) if s else l)
        lo, hi = [a for a in range(3) if a != d]
        idx[lo], idx[hi] = t % m, t // m
        return idx[0] + m * idx[1] + m * m * idx[2]

    # -------------------------------------------------------------- geometry
    def dx_min(self):
        """Smallest distance between neighbouring DG nodes along a reference line."""
        best = np.inf
        for i in range(3):
            dx = np.diff(self.x_dg, axis=axis_of(i))
            best = min(best, float(np.sqrt((dx * dx).sum(axis=0)).min()))
        return best

    def lambda_max(self):
        """max over nodes of alpha + |beta|_gamma."""
        g = self.geo
        return float((g.alpha + np.sqrt(ph.dot(g.beta, g.beta, g))).max())

    def dt(self):
        p = self.params
        c = p["stab_c"] if p.get("stab_c") else ops.ssp_rk3_c()
        return p["cfl"] * self.dx_min() / self.lambda_max() * c / 3.0

    def volume(self):
        """sum over nodes of w_i w_j w_k |det J|: the shell's volume up to quadrature error."""
        _, w = ops.gll(self.N)
        W = w[:, None, None] * w[None, :, None] * w[None, None, :]
        return float((np.abs(self.detJ) * W[None]).sum())


def _face_geo(sh, f):
    """Geometry at the nodes of face f (point shape (E, n^2))."""
    g = ph.Geometry.__new__(ph.Geometry)
    for k, v in vars(sh.geo).items():
        setattr(g, k, sh.face_nodes(v, f))
    return g


def char_speed_normal(geo, m):
    """lambda(m) = alpha sqrt(gamma^{jk} m_j m_k) + |beta^j m_j| for a covector m."""
    mm = np.einsum("ij...,i...,j...->...", geo.ginv, m, m)
    return geo.alpha * np.sqrt(mm) + np.abs(np.einsum("i...,i...->...", geo.beta, m))


def normal_flux(U, geo, J, m):
    """m_j F^j(U)."""
    return sum(m[j] * ph.flux(U, geo, j, J) for j in range(3))


def boundary_state_normal(U, geo, m):
    """No-incoming-Poynting state (Sec. III D) for the outward covector m: copy E~, B~,
    q~, set psi~ = phi~ = 0, and E~ = 0 where m_i [ijk] E~_j B~_k < 0 (the Poynting
    flux points into the domain)."""
    Ub = U.copy()
    Ub[6] = 0.0
    Ub[7] = 0.0
    El, Bl = ph.lower(U[0:3], geo), ph.lower(U[3:6], geo)
    cross = np.einsum("ijk,j...,k...->i...", ph.LEVI, El, Bl)
    inward = np.einsum("i...,i...->...", m, cross) < 0.0
    Ub[0:3] = np.where(inward, 0.0, U[0:3])
    return Ub


def _geo_sel(geo, fn):
    """Geometry with fn applied to every field (point axes last)."""
    g = ph.Geometry.__new__(ph.Geometry)
    for k, v in vars(geo).items():
        setattr(g, k, fn(v))
    return g


def shell_dg_rhs(sh, elems, W_dg, W_fd, rep, parts=3):
    """Right-hand side (9, len(elems), n, n, n) of the DG elements ``elems``.

    W_dg (12, E, n, n, n) holds (U, J~) at the nodes of every DG element, W_fd
    (12, E, m, m, m) that of every FD element (rep: 0 DG, 1 FD).  An FD neighbour's
    face state is R (x) R (x) R of its (U, J~) at the matched node; a DG neighbour's
    J~ is that of its U at the shared point."""
    p = sh.params
    N, n = sh.N, sh.n
    elems = np.asarray(elems, np.int64)
    _, w = ops.gll(N)
    D = ops.diff_matrix(N)
    geo = geo_take(sh.geo, elems)
    U = W_dg[:9, elems]
    invJ = sh.invJ[:, :, elems]
    out = np.zeros_like(U)
    if parts & 2:
        out += ph.source_stiff(U, geo, p["eta"], p["kappa_psi"], p["kappa_phi"])
    if not parts & 1:
        return out
    jd, je = ph.split_current(U, geo, p["eta"])
    J = jd + je
    out += ph.source_explicit(U, geo, p["eta"])
    F = [ph.flux(U, geo, j, J) for j in range(3)]
    for i in range(3):
        for j in range(3):
            out -= invJ[i, j] * ops.apply_1d(D, F[j], axis_of(i))
    # the neighbours' (U, J~) at their nodes: FD neighbours reconstructed to DG
    nb = W_dg.copy()
    fd_e = np.nonzero(np.asarray(rep) == FD)[0]
    if fd_e.size:
        nb[:, fd_e] = ops.apply_3d(ops.reconstruction_matrix(N), W_fd[:, fd_e])
    nb = nb.reshape(12, sh.E, n ** 3)
    L = len(elems)
    lift = np.zeros((6, 9, L, n * n))
    for f in range(6):
        i, s = divmod(f, 2)
        gf = _geo_sel(geo, lambda v: sh.face_nodes(v, f))
        Ui = sh.face_nodes(U, f)
        Ji = sh.face_nodes(J, f)
        mvec = (1.0 if s else -1.0) * sh.face_nodes(invJ[i], f)  # (3, L, n^2)
        Ue = np.empty_like(Ui)
        Je = np.empty_like(Ji)
        o_all = sh.nbr[elems, f]
        inner = o_all >= 0
        o = o_all[inner]
        Wx = nb[:, o[:, None], sh.nbr_node[elems[inner], f]]
        Ue[:, inner] = Wx[:9]
        Je[:, inner] = Wx[9:]
        for code, bc in ((-1, sh.bc_inner), (-2, sh.bc_outer)):
            sel = o_all == code
            if not np.any(sel):
                continue
            if bc == SHELL_OUTFLOW:
                Ue[:, sel] = Ui[:, sel]
            elif bc == SHELL_DIRICHLET:
                if sh.boundary_field is None:
                    raise ValueError("Dirichlet spheres need boundary_field (9, E, 6, n^2)")
                Ue[:, sel] = sh.boundary_field[:, elems[sel], f]
            else:
                gsel = _geo_sel(gf, lambda v: v[..., sel, :])
                Ue[:, sel] = boundary_state_normal(Ui[:, sel], gsel, mvec[:, sel])
        # J~ of the exterior state: the reconstructed one for an FD neighbour, else that
        # of the state at the shared point
        jde, jee = ph.split_current(Ue, gf, p["eta"])
        from_fd = np.zeros(L, bool)
        from_fd[inner] = np.asarray(rep)[o] == FD
        Je = np.where(from_fd[None, :, None], Je, jde + jee)
        Fi = normal_flux(Ui, gf, Ji, mvec)
        Fe = normal_flux(Ue, gf, Je, mvec)
        lam = char_speed_normal(gf, mvec)
        G = 0.5 * (Fi + Fe) - 0.5 * lam * (Ue - Ui)
        lift[f] = (G - Fi) / w[N if s else 0]
    for f in range(6):
        i, s = divmod(f, 2)
        ax = axis_of(i)
        sl = [slice(None)] * 5
        sl[ax] = N if s else 0
        out[tuple(sl)] -= lift[f].reshape(9, L, n, n)
    return out


def _ghosts(sh, e, f, W_own, nbr_fd):
    """Three ghost layers (12, 3, m, m) [component][layer][t2][t1] of FD element e across
    face f, from the neighbour's FD-grid (U, J~) ``nbr_fd`` (12, m^3) or, on a sphere,
    from the own outermost cells of W_own (12, m, m, m)."""
    m = sh.m
    d, s = divmod(f, 2)
    o = sh.nbr[e, f]
    if o >= 0:
        g = np.stack([nbr_fd[:, sh.nbr_cell[e, f, l]] for l in range(3)], axis=1)
        return g.reshape(12, 3, m, m)
    ax = axis_of(d)
    Wi = np.take(W_own, m - 1 if s else 0, axis=ax)  # (12, m, m): [t2][t1]
    bc = sh.bc_inner if o == -1 else sh.bc_outer
    if bc == SHELL_OUTFLOW:
        return np.repeat(Wi[:, None], 3, axis=1)
    gi = _geo_sel(geo_take(sh.geo_fd, [e]), lambda v: np.take(v, m - 1 if s else 0, axis=ax)[..., 0, :, :])
    if bc == SHELL_DIRICHLET:
        if sh.boundary_field_fd is None:
            raise ValueError("FD elements on a Dirichlet sphere need boundary_field_fd (9, E, 6, 3, m^2)")
        layers = []
        for l in range(3):
            Ub = sh.boundary_field_fd[:, e, f, l].reshape(9, m, m)
            layers.append(with_current(sh, Ub, gi))
        return np.stack(layers, axis=1)
    mvec = (1.0 if s else -1.0) * np.take(sh.invJ_fd[d, :, e], m - 1 if s else 0, axis=ax)
    Ub = boundary_state_normal(Wi[:9], gi, mvec)
    return np.repeat(with_current(sh, Ub, gi)[:, None], 3, axis=1)


def shell_fd_rhs(sh, elems, W_own, W_dg, W_fd, rep, parts=3):
    """Right-hand side (9, len(elems), m, m, m) of the FD elements ``elems`` whose own
    (U, J~) is W_own (12, len, m, m, m); neighbour data from W_dg / W_fd by ``rep``."""
    p = sh.params
    m = sh.m
    elems = np.asarray(elems, np.int64)
    geo = geo_take(sh.geo_fd, elems)
    V = W_own[:9]
    out = np.zeros_like(V)
    if parts & 2:
        out += ph.source_stiff(V, geo, p["eta"], p["kappa_psi"], p["kappa_phi"])
    if not parts & 1:
        return out
    out += ph.source_explicit(V, geo, p["eta"])
    Pm = ops.projection_matrix(sh.N)
    rep = np.asarray(rep)

    def nbr_view(o):
        if o < 0:
            return None
        v = W_fd[:, o] if rep[o] == FD else ops.apply_3d(Pm, W_dg[:, o])
        return v.reshape(12, m ** 3)

    eps = p["weno_eps"]
    for q, e in enumerate(elems):
        for d in range(3):
            ax = axis_of(d)
            # the element's cells with the direction d first: [component][c][t2][t1]
            own = np.moveaxis(W_own[:, q], ax, -3)
            lo = _ghosts(sh, e, 2 * d, W_own[:, q], nbr_view(sh.nbr[e, 2 * d]))
            hi = _ghosts(sh, e, 2 * d + 1, W_own[:, q], nbr_view(sh.nbr[e, 2 * d + 1]))
            ext = np.concatenate([lo[:, ::-1], own, hi], axis=1)  # cells -3 .. m+2

            def c(k0):
                return ext[:, k0:k0 + m + 1]

            left = ph_weno(c(0), c(1), c(2), c(3), c(4), eps)
            right = ph_weno(c(5), c(4), c(3), c(2), c(1), eps)
            gf = _geo_sel(geo_take(sh.geo_face[d], [e]), lambda v: np.moveaxis(v, ax, -3)[..., 0, :, :, :])
            nu = np.moveaxis(sh.nu_face[d][:, e], ax, -3)  # (3, m+1, m, m)
            lam = char_speed_normal(gf, nu)
            jinv = np.moveaxis(sh.invJ_fd[d, :, e], ax, -3)  # (3, m, m, m): d xi^d / d x^j
            acc = np.zeros((9, m, m, m))
            for j in range(3):
                FL = ph.flux(left[:9], gf, j, left[9:])
                FR = ph.flux(right[:9], gf, j, right[9:])
                Fh = 0.5 * (FL + FR) - 0.5 * lam * (right[:9] - left[:9]) * nu[j]
                acc += jinv[j] * (Fh[:, 1:] - Fh[:, :-1])
            out[:, q] -= (m / 2.0) * np.moveaxis(acc, -3, ax)
    return out


def shell_rhs(sh, U, parts=3):
    """Right-hand side (9, E, n, n, n) of the all-DG state U on the shell."""
    W = with_current(sh, U, sh.geo)
    rep = np.zeros(sh.E, np.int64)
    return shell_dg_rhs(sh, np.arange(sh.E), W, None, rep, parts)


def shell_step(sh, Un, dt):
    """One IMEX-SSP3(4,3,3) step of the all-DG shell: the implicit pre-stages, then the
    three substeps with the filtered explicit update (the stage algebra of the
    Cartesian oracle's step, with every element on DG)."""
    geo = sh.geo
    _, U2, _, _ = derived_stages(sh, Un, geo, dt)
    filt = _filter_fn(sh)
    H = {"Un": Un}
    X = U2
    for k in (1, 2, 3):
        Lk = shell_rhs(sh, X, parts=1)
        X, upd = _candidate(sh, k, H, X, Lk, geo, dt, filt)
        H.update(upd)
    return X


def initial_dg(sh, u_fd):
    """DG nodal data from FD cell-centre data (the start-up of Sec. III C 1, every
    element kept on DG): the reconstruction R (x) R (x) R."""
    return ops.apply_3d(ops.reconstruction_matrix(sh.N), u_fd)


def l2_error(a, b):
    """sqrt(mean over nodes of |a - b|^2) over the three components given (Sec. IV B 1)."""
    d = a - b
    return float(np.sqrt((d * d).sum(axis=0).mean()))
