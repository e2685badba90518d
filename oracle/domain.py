"""Element grid, neighbours and per-point geometry for the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/operators.py).

Sec. III A: the domain is a set of non-overlapping cubes, each mapped from
the reference cube [-1, 1]^3; here every map is affine and axis-aligned.
Elements are numbered e = ex + nx (ey + ny ez).  Faces are numbered
f = 2 d + (0 for the lower side, 1 for the upper side) along direction d.
Arrays over points have axes (..., z, y, x), so direction d lives on array
axis -1 - d.
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from .physics import Geometry

BC_PERIODIC = 0
BC_NO_INCOMING_POYNTING = 1
BC_DIRICHLET = 2

DG = 0
FD = 1


def axis_of(d):
    return -1 - d


class Domain:
    def __init__(self, n_elem, lower, upper, degree, bc, excised=None, bg=None, params=None, boundary_state=None,
                 boundary_field=None, conductor=None):
        self.n_elem = tuple(int(v) for v in n_elem)
        self.lower = np.asarray(lower, np.float64)
        self.upper = np.asarray(upper, np.float64)
        self.N = int(degree)
        self.n = self.N + 1
        self.m = 2 * self.N + 1
        self.bc = tuple(int(b) for b in bc)
        self.E = int(np.prod(self.n_elem))
        self.h = (self.upper - self.lower) / np.asarray(self.n_elem)
        self.excised = np.zeros(self.E, bool) if excised is None else np.asarray(excised).astype(bool)
        self.active = ~self.excised
        self.params = default_params() if params is None else {**default_params(), **params}
        # Dirichlet faces (Sec. IV A, the 1D problems): a fixed exterior state per
        # outer face f = 2 d + s, uniform over the face
        self.boundary_state = None if boundary_state is None else np.asarray(boundary_state, np.float64).reshape(6, 9)
        # or point by point (an analytic state varying along the face): the state at
        # every DG face node (9, E, 6, n^2) and at every FD ghost cell (9, E, 6, 3, m^2),
        # node or cell t1 + n t2 (t1 along the lower tangential axis), layer l counted
        # outwards from the face
        self.boundary_field = None
        if boundary_field is not None:
            bd, bf = boundary_field
            self.boundary_field = (np.asarray(bd, np.float64), np.asarray(bf, np.float64))
        if any(b == BC_DIRICHLET for b in self.bc) and self.boundary_state is None and self.boundary_field is None:
            raise ValueError("Dirichlet faces need boundary_state (6, 9) or boundary_field")
        # rotating perfect conductor (Sec. IV C): dict(centre=(3,), radius=R, omega=W),
        # rotation about the z axis through the centre at W relative to the grid (on
        # a background, e.g. the rotating frame, the shift adds to that motion)
        self.conductor = None
        if conductor is not None:
            self.conductor = dict(centre=np.asarray(conductor["centre"], np.float64),
                                  radius=float(conductor["radius"]), omega=float(conductor["omega"]))
        self._build_neighbours()
        self._build_geometry(bg)

    # ------------------------------------------------------------------ grid
    def coords(self, e):
        nx, ny, _ = self.n_elem
        return e % nx, (e // nx) % ny, e // (nx * ny)

    def point_coords(self, elems, fd):
        """Coordinates x, y, z (len(elems), k, k, k), axes (z, y, x), of the DG nodes
        (GLL points of each element, k = N + 1) or of the FD cell centres (k = 2N + 1
        uniform subcells) of the listed elements."""
        elems = np.asarray(elems, np.int64)
        if fd:
            ref = -1.0 + (2.0 * np.arange(self.m) + 1.0) / self.m
        else:
            ref = ops.gll(self.N)[0]
        k = ref.size
        out = []
        for d in range(3):
            idx = np.array([self.coords(e)[d] for e in elems], np.float64)
            lo = self.lower[d] + idx * self.h[d]
            c = lo[:, None] + 0.5 * self.h[d] * (ref[None, :] + 1.0)
            shape = [len(elems), 1, 1, 1]
            shape[3 - d] = k
            out.append(np.broadcast_to(c.reshape(shape), (len(elems), k, k, k)).copy())
        return out

    def index(self, ex, ey, ez):
        nx, ny, _ = self.n_elem
        return ex + nx * (ey + ny * ez)

    def _build_neighbours(self):
        """nbr[e, f] = neighbour element across face f, or -1 for a domain boundary."""
        nbr = -np.ones((self.E, 6), np.int64)
        for e in range(self.E):
            c = list(self.coords(e))
            for d in range(3):
                for s in (0, 1):
                    cc = list(c)
                    cc[d] += 1 if s else -1
                    if cc[d] < 0 or cc[d] >= self.n_elem[d]:
                        if self.bc[2 * d + s] != BC_PERIODIC:
                            continue
                        cc[d] %= self.n_elem[d]
                    o = self.index(*cc)
                    if self.excised[o]:
                        continue
                    nbr[e, 2 * d + s] = o
        self.nbr = nbr

    def dirichlet_faces(self, elems, f):
        """Mask over `elems`: face f of the element is an outer face of Dirichlet kind
        (faces towards excised elements keep the no-incoming-Poynting state)."""
        if self.bc[f] != BC_DIRICHLET:
            return np.zeros(len(elems), bool)
        d, s = divmod(f, 2)
        c = np.array([self.coords(int(e))[d] for e in elems])
        return c == (self.n_elem[d] - 1 if s else 0)

    # -------------------------------------------------------------- geometry
    def _build_geometry(self, bg):
        """Metric at DG nodes (given), at FD cell centres and at FD faces (polynomial evaluation)."""
        self.bg = None if bg is None else np.asarray(bg, np.float64)
        shape_dg = (self.E, self.n, self.n, self.n)
        shape_fd = (self.E, self.m, self.m, self.m)
        if self.bg is None:
            self.geo_dg = Geometry(None, shape_dg)
            self.geo_fd = Geometry(None, shape_fd)
            self.geo_face = [Geometry(None, face_shape(self.E, self.m, d)) for d in range(3)]
            self.bg_fd = None
            return
        P = ops.projection_matrix(self.N)
        Q = ops.face_eval_matrix(self.N)
        self.geo_dg = Geometry(self.bg)
        self.bg_fd = ops.apply_3d(P, self.bg)
        self.geo_fd = Geometry(self.bg_fd)
        self.geo_face = []
        for d in range(3):
            b = self.bg
            for dd in range(3):
                b = ops.apply_1d(Q if dd == d else P, b, axis_of(dd))
            self.geo_face.append(Geometry(b))

    def dx_min(self):
        x, _ = ops.gll(self.N)
        return np.min(np.diff(x)) * np.min(self.h) / 2.0

    def lambda_max(self):
        """max over active nodes and directions of alpha sqrt(gamma^dd) + |beta^d|."""
        from .physics import char_speed
        lam = 0.0
        for d in range(3):
            v = char_speed(self.geo_dg, d)
            v = np.broadcast_to(v, (self.E, self.n, self.n, self.n))
            lam = max(lam, float(v[self.active].max()))
        return lam

    def dt(self):
        """Eq. (spectre DG CFL condition): f (dx)_min / lambda_max * c / D with D = 3."""
        p = self.params
        c = p["stab_c"] if p.get("stab_c") else ops.ssp_rk3_c()
        return p["cfl"] * self.dx_min() / self.lambda_max() * c / 3.0


def face_shape(E, m, d):
    """Shape of an FD face array for direction d: m+1 faces along axis d, m cells on the others."""
    s = [E, m, m, m]
    s[3 - d] = m + 1
    return tuple(s)


def default_params():
    return dict(
        eta=1e6, kappa_psi=1.0, kappa_phi=1.0,
        cfl=0.25, stab_c=0.0,
        tci_M=0, tci_alpha=4.0, tci_alpha_fd=5.0, tci_mode=2,
        filter_a=36.0, filter_b=50.0, filter_on=1, filter_after_solve=0,
        weno_eps=1e-40, fd_order=4,
        ff_clamp=0, ff_margin=1e-12,
        hybrid=1,
    )


def geo_take(geo, e_idx):
    """Geometry restricted to a subset of elements (axis 0 of the point axes)."""
    g = Geometry.__new__(Geometry)
    for k, v in vars(geo).items():
        if k in ("alpha", "sqrtg", "K"):
            setattr(g, k, v[e_idx])
        elif k in ("beta", "dalpha", "Gam"):
            setattr(g, k, v[:, e_idx])
        else:  # g, ginv, dbeta
            setattr(g, k, v[:, :, e_idx])
    return g
