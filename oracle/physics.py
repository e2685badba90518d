"""Pointwise GRFFE physics (FP64): current closure, fluxes, sources, implicit solve.

TEST INFRASTRUCTURE ONLY (see oracle/operators.py).

Variables are the densitized U = sqrt(gamma) (E^i, B^i, psi, phi, q), stored
as arrays of shape (9, ...) in the order (E~x, E~y, E~z, B~x, B~y, B~z,
psi~, phi~, q~).  All formulas are written in the densitized variables:

* spatial Levi-Civita epsilon^{ijk} = [ijk] / sqrt(gamma), from the sign
  convention eps_abcd = sqrt(-g) [abcd], [0123] = +1 and eps^{ijk} =
  n_d eps^{dijk} (Sec. I and Sec. II A);
* electric current, Eq. (electric current density), densitized as
  J~^i = alpha sqrt(gamma) J^i;
* fluxes, Eq. (fluxes); sources, Eq. (sources);
* IMEX split (Sec. III B): the eta part of the current and the kappa
  damping of psi, phi are stiff; everything else is explicit.
"""
from __future__ import annotations

import numpy as np

LEVI = np.zeros((3, 3, 3))
for (i, j, k), s in {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}.items():
    LEVI[i, j, k] = s


class Geometry:
    """3+1 background quantities at a set of points (shape ``shape``)."""

    def __init__(self, bg, shape=None):
        if bg is None:
            one = np.ones(shape)
            zero = np.zeros(shape)
            self.alpha = one
            self.beta = np.zeros((3,) + tuple(shape))
            self.g = np.zeros((3, 3) + tuple(shape))
            for i in range(3):
                self.g[i, i] = 1.0
            self.ginv = self.g.copy()
            self.sqrtg = one
            self.dalpha = np.zeros((3,) + tuple(shape))
            self.dbeta = np.zeros((3, 3) + tuple(shape))
            self.K = zero
            self.Gam = np.zeros((3,) + tuple(shape))
            return
        bg = np.asarray(bg, np.float64)
        self.alpha = bg[0]
        self.beta = bg[1:4]
        g = np.empty((3, 3) + bg.shape[1:])
        for (i, j), k in {(0, 0): 4, (0, 1): 5, (0, 2): 6, (1, 1): 7, (1, 2): 8, (2, 2): 9}.items():
            g[i, j] = bg[k]
            g[j, i] = bg[k]
        self.g = g
        gm = np.moveaxis(g, (0, 1), (-2, -1))
        # (a background may hold NaN at points no kernel reads: the Kerr-Schild
        # fields on the singular disc inside an excision ball)
        with np.errstate(invalid="ignore"):
            self.ginv = np.moveaxis(np.linalg.inv(gm), (-2, -1), (0, 1))
            self.sqrtg = np.sqrt(np.linalg.det(gm))
        self.dalpha = bg[10:13]
        self.dbeta = bg[13:22].reshape((3, 3) + bg.shape[1:])  # [j][i] = d_j beta^i
        self.K = bg[22]
        self.Gam = bg[23:26]


def lower(v, geo):
    return np.einsum("ij...,j...->i...", geo.g, v)


def dot(u, v, geo):
    return np.einsum("ij...,i...,j...->...", geo.g, u, v)


def split_current(U, geo, eta):
    """Densitized current J~ = alpha sqrt(gamma) J split into drift and eta parts.

    J^i = q eps^{ijk} E_j B_k / B^2 + eta [(E.B / B^2) B^i + R(E^2 - B^2)/B^2 E^i]
    with R(x) = max(x, 0).  Where B~^2 = 0 the current is set to zero.
    """
    Et, Bt, qt = U[0:3], U[3:6], U[8]
    B2 = dot(Bt, Bt, geo)
    E2 = dot(Et, Et, geo)
    EB = dot(Et, Bt, geo)
    safe = np.where(B2 > 0.0, B2, 1.0)
    live = B2 > 0.0
    El, Bl = lower(Et, geo), lower(Bt, geo)
    cross = np.einsum("ijk,j...,k...->i...", LEVI, El, Bl)  # [ijk] E~_j B~_k
    j_drift = geo.alpha * qt * cross / (geo.sqrtg * safe)
    j_eta = geo.alpha * eta * ((EB / safe) * Bt + (np.maximum(E2 - B2, 0.0) / safe) * Et)
    j_drift = np.where(live, j_drift, 0.0)
    j_eta = np.where(live, j_eta, 0.0)
    return j_drift, j_eta


def flux(U, geo, d, Jt=None, eta=0.0):
    """F^d(U), Eq. (fluxes), for spatial direction d.  ``Jt`` is the full J~ (or computed)."""
    if Jt is None:
        jd, je = split_current(U, geo, eta)
        Jt = jd + je
    Et, Bt, psi, phi, qt = U[0:3], U[3:6], U[6], U[7], U[8]
    a, bd = geo.alpha, geo.beta[d]
    El, Bl = lower(Et, geo), lower(Bt, geo)
    F = np.empty_like(U)
    for i in range(3):
        epsB = sum(LEVI[i, d, k] * Bl[k] for k in range(3)) / geo.sqrtg
        epsE = sum(LEVI[i, d, k] * El[k] for k in range(3)) / geo.sqrtg
        F[i] = -bd * Et[i] + a * (geo.ginv[i, d] * psi - epsB)
        F[3 + i] = -bd * Bt[i] + a * (geo.ginv[i, d] * phi + epsE)
    F[6] = -bd * psi + a * Et[d]
    F[7] = -bd * phi + a * Bt[d]
    F[8] = Jt[d] - bd * qt
    return F


def source_explicit(U, geo, eta):
    """Non-stiff part of Eq. (sources): everything except the eta current and kappa damping."""
    jd, _ = split_current(U, geo, eta)
    Et, Bt, psi, phi, qt = U[0:3], U[3:6], U[6], U[7], U[8]
    a = geo.alpha
    S = np.zeros_like(U)
    grad_a_up = np.einsum("ij...,j...->i...", geo.ginv, geo.dalpha)
    for i in range(3):
        S[i] = -jd[i] - sum(Et[j] * geo.dbeta[j, i] for j in range(3)) + psi * (grad_a_up[i] - a * geo.Gam[i])
        S[3 + i] = -sum(Bt[j] * geo.dbeta[j, i] for j in range(3)) + phi * (grad_a_up[i] - a * geo.Gam[i])
    S[6] = sum(Et[k] * geo.dalpha[k] for k in range(3)) + a * qt - a * psi * geo.K
    S[7] = sum(Bt[k] * geo.dalpha[k] for k in range(3)) - a * phi * geo.K
    S[8] = 0.0
    return S


def source_stiff(U, geo, eta, kpsi, kphi):
    """Stiff part of Eq. (sources): -alpha sqrt(gamma) J_eta and -alpha kappa (psi, phi)."""
    _, je = split_current(U, geo, eta)
    S = np.zeros_like(U)
    S[0:3] = -je
    S[6] = -geo.alpha * kpsi * U[6]
    S[7] = -geo.alpha * kphi * U[7]
    return S


def implicit_solve(Y, geo, eta, kpsi, kphi, h):
    """Solve U = Y + h S_stiff(U) pointwise (Sec. III B, the IMEX stage equation).

    B~ and q~ have no stiff source.  psi~ and phi~ follow from the linear
    equation.  For E~, with c = alpha eta h the equation reads
        E = E* - c [ (E.B/B^2) B + R(E^2 - B^2)/B^2 E ].
    Split E* into parts parallel and perpendicular to B~ (gamma inner
    product).  With s = R(E^2 - B^2)/B^2 >= 0 the solution is
        E = E*_perp / (1 + c s) + E*_par / (1 + c + c s),
    where s = 0 if that gives E^2 <= B^2, and otherwise s > 0 is the unique
    root of |E*_perp|^2/(1+cs)^2 + |E*_par|^2/(1+c+cs)^2 = (1+s) B^2,
    found here by bisection to full precision.
    """
    U = Y.copy()
    a = geo.alpha
    U[6] = Y[6] / (1.0 + a * kpsi * h)
    U[7] = Y[7] / (1.0 + a * kphi * h)
    Es, Bt = Y[0:3], Y[3:6]
    B2 = dot(Bt, Bt, geo)
    live = B2 > 0.0
    safe = np.where(live, B2, 1.0)
    c = a * eta * h
    par = (dot(Es, Bt, geo) / safe) * Bt
    perp = Es - par
    P2 = dot(perp, perp, geo)
    Q2 = dot(par, par, geo)
    cand = perp + par / (1.0 + c)
    need = live & (dot(cand, cand, geo) > B2)
    s = np.zeros(B2.shape)
    if np.any(need):
        lo = np.zeros(B2.shape)
        hi = np.where(need, dot(Es, Es, geo) / safe, 0.0)

        def g(sv):
            return P2 / (1.0 + c * sv) ** 2 + Q2 / (1.0 + c + c * sv) ** 2 - (1.0 + sv) * B2

        for _ in range(200):
            mid = 0.5 * (lo + hi)
            pos = g(mid) > 0.0
            lo = np.where(need & pos, mid, lo)
            hi = np.where(need & ~pos, mid, hi)
        s = np.where(need, 0.5 * (lo + hi), 0.0)
    E = perp / (1.0 + c * s) + par / (1.0 + c + c * s)
    U[0:3] = np.where(live, E, Es)
    return U


def constraint_clamp(U, geo, margin):
    """Algebraic force-free fix (Sec. II B): remove E parallel to B, then enforce E^2 <= (1-margin) B^2."""
    U = U.copy()
    Et, Bt = U[0:3], U[3:6]
    B2 = dot(Bt, Bt, geo)
    live = B2 > 0.0
    safe = np.where(live, B2, 1.0)
    E = Et - (dot(Et, Bt, geo) / safe) * Bt
    E2 = dot(E, E, geo)
    lim = (1.0 - margin) * B2
    scale = np.where(E2 > lim, np.sqrt(lim / np.where(E2 > 0, E2, 1.0)), 1.0)
    U[0:3] = np.where(live, E * scale, Et)
    return U


def corotating_conductor(U, x, y, z, centre, radius, omega, geo=None):
    """Rotating perfect conductor (Sec. IV C, pulsar magnetospheres): at every point
    with |x - centre| <= radius, E is replaced by the value the ideal condition
    E + v x B = 0 gives for the conductor's rigid rotation, and psi~ and q~ are set
    to zero there.  B and phi~ are left to the evolution.  Points outside are
    returned unchanged.

    Flat space, grid at rest (geo None): v = omega z^ x (x - centre) =
    omega (-(y - c_y), x - c_x, 0), E = -(v x B).

    With a 3+1 background geo (e.g. flat space in coordinates that rotate with the
    star, whose shift is beta = Omega z^ x x): the conductor moves through the grid
    with coordinate velocity omega z^ x (x - centre) (omega its rotation relative to
    the grid, 0 for a grid that rotates with it), so its velocity relative to the
    normal observers is v^i = (omega (z^ x (x - centre))^i + beta^i) / alpha; the
    condition E_i = -eps_ijk v^j B^k with eps_ijk = sqrt(gamma) [ijk] and
    B^k = B~^k / sqrt(gamma) gives E_i = -[ijk] v^j B~^k, and E~^i =
    sqrt(gamma) gamma^{ij} E_j."""
    U = U.copy()
    rx, ry, rz = x - centre[0], y - centre[1], z - centre[2]
    inside = rx * rx + ry * ry + rz * rz <= radius * radius
    v = np.array([-omega * ry, omega * rx, np.zeros_like(rx)])
    B = U[3:6]
    if geo is None:
        Et = -np.einsum("ijk,j...,k...->i...", LEVI, v, B)
    else:
        v = (v + geo.beta) / geo.alpha
        El = -np.einsum("ijk,j...,k...->i...", LEVI, v, B)
        Et = geo.sqrtg * np.einsum("ij...,j...->i...", geo.ginv, El)
    for i in range(3):
        U[i] = np.where(inside, Et[i], U[i])
    U[6] = np.where(inside, 0.0, U[6])
    U[8] = np.where(inside, 0.0, U[8])
    return U


def char_speed(geo, d):
    """Coordinate speed alpha sqrt(gamma^dd) + |beta^d| bounding the light cone along x^d."""
    return geo.alpha * np.sqrt(geo.ginv[d, d]) + np.abs(geo.beta[d])


def boundary_state(U, geo, d, side):
    """No-incoming-Poynting external state (Sec. III D).

    Copy E~, B~, q~ from the interior; psi~ = phi~ = 0; E~ = 0 where the
    Poynting flux eps^{ijk} E_j B_k points into the domain.  ``side`` is the
    sign of the outward normal along x^d.
    """
    Ub = U.copy()
    Ub[6] = 0.0
    Ub[7] = 0.0
    El, Bl = lower(U[0:3], geo), lower(U[3:6], geo)
    Sd = sum(LEVI[d, j, k] * El[j] * Bl[k] for j in range(3) for k in range(3))
    inward = side * Sd < 0.0
    Ub[0:3] = np.where(inward, 0.0, U[0:3])
    return Ub


def rusanov(UL, UR, geoL, geoR, d, JL, JR):
    """Rusanov flux at a face normal to x^d with speed max(lambda_L, lambda_R)."""
    FL = flux(UL, geoL, d, JL)
    FR = flux(UR, geoR, d, JR)
    lam = np.maximum(char_speed(geoL, d), char_speed(geoR, d))
    return 0.5 * (FL + FR) - 0.5 * lam * (UR - UL)
