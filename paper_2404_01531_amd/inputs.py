"""Seeded synthetic inputs for the GRFFE DG-FD hot path.

This module is shared by the CPU oracle tests, the GPU parity tests, the
smoke entry point and the benchmark.  It only *samples* analytic data:
element boxes, point coordinates, initial fields, Gaussian noise and the
Kerr-Schild background metric with its first derivatives.  It contains none
of the scheme's arithmetic (no collocation points, no derivative or
interpolation operators, no fluxes, no time stepping).  Callers that need
values at DG collocation points pass in their own 1D reference points.

Array conventions
-----------------
* Elements are numbered e = ex + nx*(ey + ny*ez).
* Point arrays have shape (E, n, n, n) with axes (z, y, x): the x (xi^1)
  index runs fastest in memory, matching the library's node ordering.
* Field arrays have a leading component axis: (ncomp, E, n, n, n).

Physical content
----------------
* Evolved variables U = sqrt(gamma) (E^i, B^i, psi, phi, q) (Sec. II A, the
  conservative-form variables).
* The Kerr-Schild line element in Cartesian form (Appendix B): g = eta +
  2 H l l with H = M r^3 / (r^4 + a^2 z^2) and the quartic relation for r.
* Background field order (26 fields): alpha; beta^x, beta^y, beta^z;
  gamma_xx, gamma_xy, gamma_xz, gamma_yy, gamma_yz, gamma_zz; d_x alpha,
  d_y alpha, d_z alpha; d_j beta^i for j = x,y,z (outer) and i = x,y,z
  (inner); K (trace of the extrinsic curvature, sign convention
  d_t gamma_ij = -2 alpha K_ij + L_beta gamma_ij); Gamma^i = gamma^jk
  Gamma^i_jk for i = x,y,z.
"""
from __future__ import annotations

import numpy as np

N_BG = 26

# ----------------------------------------------------------------------------
# element geometry and point sets


def element_boxes(n_elem, lower, upper):
    """Lower corners (E,3) and widths (3,) of an affine Cartesian element grid."""
    n_elem = np.asarray(n_elem, dtype=np.int64)
    lower = np.asarray(lower, dtype=np.float64)
    upper = np.asarray(upper, dtype=np.float64)
    h = (upper - lower) / n_elem
    E = int(np.prod(n_elem))
    e = np.arange(E)
    ex = e % n_elem[0]
    ey = (e // n_elem[0]) % n_elem[1]
    ez = e // (n_elem[0] * n_elem[1])
    corner = np.stack([lower[0] + ex * h[0], lower[1] + ey * h[1], lower[2] + ez * h[2]], axis=1)
    return corner, h


def points(n_elem, lower, upper, ref_1d):
    """Physical coordinates of a tensor-product point set in every element.

    ``ref_1d`` holds reference coordinates in [-1, 1] (used for all three
    axes).  Returns x, y, z each of shape (E, n, n, n) with axes (z, y, x).
    """
    ref_1d = np.asarray(ref_1d, dtype=np.float64)
    corner, h = element_boxes(n_elem, lower, upper)
    t = 0.5 * (ref_1d + 1.0)
    n = ref_1d.size
    E = corner.shape[0]
    x = corner[:, 0, None, None, None] + h[0] * t[None, None, None, :]
    y = corner[:, 1, None, None, None] + h[1] * t[None, None, :, None]
    z = corner[:, 2, None, None, None] + h[2] * t[None, :, None, None]
    shape = (E, n, n, n)
    return np.broadcast_to(x, shape).copy(), np.broadcast_to(y, shape).copy(), np.broadcast_to(z, shape).copy()


def fd_cell_centres_1d(degree):
    """Reference centres of the 2N+1 uniform subcells of [-1, 1]."""
    m = 2 * degree + 1
    return -1.0 + (2.0 * np.arange(m) + 1.0) / m


def fd_points(n_elem, lower, upper, degree):
    return points(n_elem, lower, upper, fd_cell_centres_1d(degree))


# ----------------------------------------------------------------------------
# Kerr-Schild background (Appendix B, Cartesian Kerr-Schild line element)


def _at_singularity_nan(fun):
    """Evaluate ``fun`` with numpy's divide/invalid warnings off: on the disc
    r = 0 (z = 0, x^2 + y^2 <= a^2, bounded by the ring singularity; the origin
    alone when a = 0) the Kerr-Schild fields are 0/0 and come out NaN.  The disc
    lies inside every excision ball (r_excise > a), and the excised elements are
    neither updated nor read by their neighbours."""
    import functools

    @functools.wraps(fun)
    def wrapped(*args, **kwargs):
        with np.errstate(divide="ignore", invalid="ignore"):
            return fun(*args, **kwargs)
    return wrapped


def _ks_radius(x, y, z, a):
    rho2 = x * x + y * y + z * z
    t = rho2 - a * a
    r2 = 0.5 * (t + np.sqrt(t * t + 4.0 * a * a * z * z))
    return np.sqrt(r2)


def ks_radius(x, y, z, a):
    """Kerr-Schild radial coordinate r(x, y, z) from the quartic relation."""
    return _ks_radius(np.asarray(x, np.float64), np.asarray(y, np.float64), np.asarray(z, np.float64), a)


def _ks_3p1(x, y, z, M, a):
    """alpha, beta^i (3), gamma_ij (3,3), gamma^ij (3,3), sqrt(gamma) (complex-safe)."""
    r = _ks_radius(x, y, z, a)
    H = M * r ** 3 / (r ** 4 + a * a * z * z)
    ra = r * r + a * a
    l = [(r * x + a * y) / ra, (r * y - a * x) / ra, z / r]  # spatial part of the null covector, l_t = 1
    ll = sum(li * li for li in l)  # equals 1 for the Kerr-Schild null vector
    g = [[(1.0 if i == j else 0.0) + 2.0 * H * l[i] * l[j] for j in range(3)] for i in range(3)]
    ginv = [[(1.0 if i == j else 0.0) - 2.0 * H * l[i] * l[j] / (1.0 + 2.0 * H * ll) for j in range(3)]
            for i in range(3)]
    beta_lo = [2.0 * H * l[i] for i in range(3)]
    beta = [sum(ginv[i][j] * beta_lo[j] for j in range(3)) for i in range(3)]
    g00 = -1.0 + 2.0 * H
    alpha = np.sqrt(sum(beta_lo[i] * beta[i] for i in range(3)) - g00)
    sqrtg = np.sqrt(1.0 + 2.0 * H * ll)
    return alpha, beta, g, ginv, sqrtg


def _cstep(fun, x, y, z, h=1e-30):
    """Complex-step partial derivatives of ``fun`` (which returns a list of arrays)."""
    out = []
    for d in range(3):
        xs = [x.astype(np.complex128), y.astype(np.complex128), z.astype(np.complex128)]
        xs[d] = xs[d] + 1j * h
        vals = fun(*xs)
        out.append([np.imag(v) / h for v in vals])
    return out  # out[d][k] = d_d of value k


def _sks_map(xb, yb, zb, a):
    """Kerr-Schild Cartesian coordinates (x, y, z) of the point with Cartesian projection
    (xb, yb, zb) of the spherical Kerr-Schild coordinates (r, theta, phi) (Appendix B:
    x = (r cos phi - a sin phi) sin theta, y = (r sin phi + a cos phi) sin theta,
    z = r cos theta, with xb = r sin theta cos phi, ...): x = xb - a yb / r,
    y = yb + a xb / r, z = zb, r = |xb|; and the Jacobian J[p][i] = d x^p / d xb^i
    (complex-safe)."""
    r = np.sqrt(xb * xb + yb * yb + zb * zb)
    r3 = r * r * r
    x = xb - a * yb / r
    y = yb + a * xb / r
    one, zero = 1.0 + 0.0 * r, 0.0 * r
    J = [[one + a * yb * xb / r3, -a / r + a * yb * yb / r3, a * yb * zb / r3],
         [a / r - a * xb * xb / r3, one - a * xb * yb / r3, -a * xb * zb / r3],
         [zero, zero, one]]
    return x, y, zb, J


def _inv3(m):
    """Inverse of a 3x3 matrix of arrays (nested lists), by cofactors."""
    c = [[m[(j + 1) % 3][(i + 1) % 3] * m[(j + 2) % 3][(i + 2) % 3]
          - m[(j + 1) % 3][(i + 2) % 3] * m[(j + 2) % 3][(i + 1) % 3] for j in range(3)] for i in range(3)]
    det = m[0][0] * c[0][0] + m[0][1] * c[1][0] + m[0][2] * c[2][0]
    return [[c[i][j] / det for j in range(3)] for i in range(3)], det


def _sks_3p1(xb, yb, zb, M, a):
    """alpha, beta^i, gamma_ij, gamma^ij, sqrt(gamma) of the Kerr metric in the
    Cartesian projection of spherical Kerr-Schild coordinates: the Kerr-Schild
    fields pulled back through _sks_map (a time-independent change of the spatial
    coordinates: the lapse is a scalar, the shift a vector, gamma a tensor)."""
    x, y, z, J = _sks_map(xb, yb, zb, a)
    alpha, beta, g, ginv, sqrtg = _ks_3p1(x, y, z, M, a)
    Ji, detJ = _inv3(J)  # Ji[i][p] = d xb^i / d x^p
    gb = [[sum(J[p][i] * J[q][j] * g[p][q] for p in range(3) for q in range(3)) for j in range(3)] for i in range(3)]
    gib = [[sum(Ji[i][p] * Ji[j][q] * ginv[p][q] for p in range(3) for q in range(3)) for j in range(3)]
           for i in range(3)]
    bb = [sum(Ji[i][p] * beta[p] for p in range(3)) for i in range(3)]
    return alpha, bb, gb, gib, sqrtg * detJ


def _background_26(f3p1, x, y, z):
    """The 26 background fields from a complex-safe function of the points returning
    (alpha, beta^i, gamma_ij, gamma^ij, sqrt(gamma)) of a stationary metric."""
    alpha, beta, g, ginv, sqrtg = f3p1(x, y, z)

    def flat_vals(x_, y_, z_):
        al, be, gg, _, sg = f3p1(x_, y_, z_)
        vals = [al] + list(be) + [gg[i][j] for i in range(3) for j in range(3)] + [sg * be[i] for i in range(3)]
        return vals

    der = _cstep(flat_vals, x, y, z)
    # unpack: index 0 alpha, 1..3 beta, 4..12 gamma_ij (row-major), 13..15 sqrtg*beta^i
    dalpha = [der[d][0] for d in range(3)]
    dbeta = [[der[j][1 + i] for i in range(3)] for j in range(3)]  # [j][i] = d_j beta^i
    dg = [[[der[k][4 + 3 * i + j] for j in range(3)] for i in range(3)] for k in range(3)]  # dg[k][i][j]
    div_sgb = sum(der[i][13 + i] for i in range(3))
    K = div_sgb / (sqrtg * alpha)  # K = D_i beta^i / alpha for a stationary slice
    # Gamma^i = gamma^jk Gamma^i_jk, Gamma^i_jk = 1/2 gamma^il (d_j g_lk + d_k g_lj - d_l g_jk)
    Gam = []
    for i in range(3):
        acc = 0.0
        for j in range(3):
            for k in range(3):
                for l_ in range(3):
                    acc = acc + 0.5 * ginv[j][k] * ginv[i][l_] * (dg[j][l_][k] + dg[k][l_][j] - dg[l_][j][k])
        Gam.append(acc)
    fields = [alpha, beta[0], beta[1], beta[2],
              g[0][0], g[0][1], g[0][2], g[1][1], g[1][2], g[2][2],
              dalpha[0], dalpha[1], dalpha[2]]
    for j in range(3):
        for i in range(3):
            fields.append(dbeta[j][i])
    fields.append(K)
    fields.extend(Gam)
    out = np.stack([np.broadcast_to(np.real(f), x.shape) for f in fields], axis=0).astype(np.float64)
    return out


@_at_singularity_nan
def kerr_schild_background(x, y, z, M=1.0, a=0.0):
    """The 26 background fields at the given points (see module docstring)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    return _background_26(lambda x_, y_, z_: _ks_3p1(x_, y_, z_, M, a), x, y, z)


@_at_singularity_nan
def spherical_kerr_schild_background(xb, yb, zb, M=1.0, a=0.0):
    """The 26 background fields of the Kerr metric in the Cartesian projection of
    spherical Kerr-Schild coordinates (Appendix B), where the horizons are the
    spheres r = M (1 +- sqrt(1 - a^2)); equal to kerr_schild_background at a = 0."""
    xb = np.asarray(xb, np.float64)
    yb = np.asarray(yb, np.float64)
    zb = np.asarray(zb, np.float64)
    return _background_26(lambda x_, y_, z_: _sks_3p1(x_, y_, z_, M, a), xb, yb, zb)


def flat_background(shape):
    """The 26 background fields of flat space in Cartesian coordinates."""
    bg = np.zeros((N_BG,) + tuple(shape))
    bg[0] = 1.0
    bg[4] = bg[7] = bg[9] = 1.0
    return bg


def rotating_frame_background(x, y, z, omega, centre=(0.0, 0.0, 0.0)):
    """The 26 background fields of flat space in Cartesian coordinates that rotate
    at omega about the z axis through `centre` (the rotating grid of the pulsar
    runs, Sec. IV C): with phi' = phi - omega t the line element is
    -dt^2 + dr^2 + r^2 (dphi' + omega dt)^2 + dz^2, so alpha = 1, gamma_ij = delta_ij
    and the shift is beta = omega z^ x (x - centre) = omega (-(y - c_y), x - c_x, 0);
    d_y beta^x = -omega, d_x beta^y = omega, the lapse is constant, and K = 0 (a
    rigid rotation is a Killing motion)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    bg = flat_background(np.broadcast(x, y, z).shape)
    bg[1] = -omega * (y - centre[1])
    bg[2] = omega * (x - centre[0])
    bg[13 + 3 * 1 + 0] = -omega  # d_y beta^x
    bg[13 + 3 * 0 + 1] = omega   # d_x beta^y
    return bg


# ----------------------------------------------------------------------------
# initial data (all returned as densitized evolved variables, shape (9, ...))


def noise(seed, shape, sigma=1e-3):
    """Seeded N(0, sigma^2) samples (PCG64)."""
    rng = np.random.default_rng(seed)
    return sigma * rng.standard_normal(shape)


def fast_wave_sine(x, amplitude=0.1, k=np.pi):
    """Flat-space fast wave moving in +x: B = (1, -A sin kx, 0), E = (0, 0, A sin kx)."""
    U = np.zeros((9,) + x.shape)
    s = amplitude * np.sin(k * x)
    U[3] = 1.0
    U[4] = -s
    U[2] = s
    return U


def current_sheet(x, width=0.05, half_length=1.0):
    """Flat-space current sheet across x = 0: B = (1, tanh(x/w) - x tanh(L/w)/L, 0), E = 0.

    The linear term makes B_y (and its first derivative) continuous across
    the periodic wrap at x = +-L, so the box holds a single sheet.
    """
    U = np.zeros((9,) + x.shape)
    U[3] = 1.0
    U[4] = np.tanh(x / width) - x * np.tanh(half_length / width) / half_length
    return U


def fast_wave_1d(x):
    """Fast-wave problem (Appendix A): B = (1, B_y, 0), E = (0, 0, -B_y) with B_y = 1
    for x < -0.1, 0.85 - 1.5 x for |x| < 0.1, 0.7 for x > 0.1 (flat space, so the
    densitized and plain fields agree; div E = 0).  Exact solution Q(x - t)."""
    x = np.asarray(x, np.float64)
    by = np.where(x < -0.1, 1.0, np.where(x > 0.1, 0.7, 0.85 - 1.5 * x))
    U = np.zeros((9,) + x.shape)
    U[3] = 1.0
    U[4] = by
    U[2] = -by
    return U


def alfven_stationary_1d(x):
    """Stationary Alfven wave (Appendix A): B = (1, 1, B_z), E = (-B_z, 0, 1) with
    B_z = 1 for x < -0.1, 1.15 + 0.15 sin(5 pi x) for |x| < 0.1, 1.3 for x > 0.1;
    q = d_x E_x = -dB_z/dx."""
    x = np.asarray(x, np.float64)
    inner = np.abs(x) < 0.1
    bz = np.where(x < -0.1, 1.0, np.where(x > 0.1, 1.3, 1.15 + 0.15 * np.sin(5.0 * np.pi * x)))
    dbz = np.where(inner, 0.75 * np.pi * np.cos(5.0 * np.pi * x), 0.0)
    U = np.zeros((9,) + x.shape)
    U[0] = -bz
    U[2] = 1.0
    U[3] = 1.0
    U[4] = 1.0
    U[5] = bz
    U[8] = -dbz
    return U


def ffe_breakdown_1d(x):
    """FFE breakdown problem (Appendix A): B = (1, b, b) with b = 1 for x < -0.1,
    -10 x for |x| < 0.1, -1 for x > 0.1; E = (0, 0.5, -0.5); div E = 0."""
    x = np.asarray(x, np.float64)
    b = np.where(x < -0.1, 1.0, np.where(x > 0.1, -1.0, -10.0 * x))
    U = np.zeros((9,) + x.shape)
    U[1] = 0.5
    U[2] = -0.5
    U[3] = 1.0
    U[4] = b
    U[5] = b
    return U


def smooth_fast_wave(x, wavelength=2.0):
    """The fast wave made smooth (Sec. IV D 1, accuracy comparison): B = (1, -s, 0),
    E = (0, 0, s) with s = sin(2 pi x / wavelength); a vacuum mode moving towards +x
    at the speed of light, exact solution Q(x - t) (periodic)."""
    x = np.asarray(x, np.float64)
    sn = np.sin(2.0 * np.pi * x / wavelength)
    U = np.zeros((9,) + x.shape)
    U[3] = 1.0
    U[4] = -sn
    U[2] = sn
    return U


def smooth_pulses_1d(x, amplitude=0.1, centres=(0.7, 0.3), half_width=0.2):
    """Two vacuum fast-wave pulses on B = (1, 0, 0): B_y = A g(x - c0) + A g(x - c1),
    E_z = -A g(x - c0) + A g(x - c1) (the first moves towards +x, the second towards
    -x, both at the speed of light), g(s) = cos^8(pi s / (2 w)) for |s| < w."""
    x = np.asarray(x, np.float64)

    def g(s):
        return np.where(np.abs(s) < half_width, np.cos(0.5 * np.pi * s / half_width) ** 8, 0.0)

    gr, gl = amplitude * g(x - centres[0]), amplitude * g(x - centres[1])
    U = np.zeros((9,) + x.shape)
    U[3] = 1.0
    U[4] = gr + gl
    U[2] = -gr + gl
    return U


def add_noise_by_and_ez(U, seed, sigma=1e-3):
    """Independent noise on B_y and E_z at every point (drawn B_y first, then E_z)."""
    U = U.copy()
    nz = noise(seed, (2,) + U.shape[1:], sigma)
    U[4] += nz[0]
    U[2] += nz[1]
    return U


@_at_singularity_nan
def wald_a0(x, y, z, M=1.0, B0=1.0):
    """Exact Wald field for a = 0 in Kerr-Schild coordinates (densitized; Sec. IV B)."""
    r2 = x * x + y * y + z * z
    U = np.zeros((9,) + np.shape(x))
    U[5] = B0
    U[0] = -2.0 * M * B0 * y / r2
    U[1] = 2.0 * M * B0 * x / r2
    return U


def _wald_potential(x, y, z, M, a, B0):
    """Spatial covariant components A_k of Wald's potential A = (B0 / 2) (d_phi + 2 a d_t)
    (Eq. exact wald solution) in Cartesian Kerr-Schild coordinates: with the Killing
    vectors d_phi = -y d_x + x d_y and d_t, A_k = (B0 / 2) (gamma_kj phi^j + 2 a g_k0),
    where g_k0 = gamma_kj beta^j (complex-safe)."""
    _, beta, g, _, _ = _ks_3p1(x, y, z, M, a)
    phi = (-y, x, 0.0 * x)
    return [0.5 * B0 * sum(g[k][j] * (phi[j] + 2.0 * a * beta[j]) for j in range(3)) for k in range(3)]


@_at_singularity_nan
def wald_vacuum(x, y, z, M=1.0, a=0.0, B0=1.0):
    """Initial data of the vacuum Wald problem (Sec. IV B 2): the magnetic field of
    Wald's potential, B~^i = [ijk] d_j A_k (densitized, so divergence-free in
    coordinates), with E~ = psi~ = phi~ = q~ = 0.  At a = 0 it is the uniform
    B~ = (0, 0, B0)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    dA = _cstep(lambda x_, y_, z_: _wald_potential(x_, y_, z_, M, a, B0), x, y, z)  # dA[j][k] = d_j A_k
    U = np.zeros((9,) + x.shape)
    U[3] = dA[1][2] - dA[2][1]
    U[4] = dA[2][0] - dA[0][2]
    U[5] = dA[0][1] - dA[1][0]
    return U


@_at_singularity_nan
def wald_vacuum_spherical(xb, yb, zb, M=1.0, a=0.0, B0=1.0):
    """The vacuum Wald initial data in the Cartesian projection of spherical
    Kerr-Schild coordinates: Wald's potential pulled back, A_bar_i = (d x^p / d xb^i) A_p,
    B~^i = [ijk] d_j A_bar_k (densitized), E~ = psi~ = phi~ = q~ = 0."""
    xb = np.asarray(xb, np.float64)
    yb = np.asarray(yb, np.float64)
    zb = np.asarray(zb, np.float64)

    def potential(x_, y_, z_):
        x, y, z, J = _sks_map(x_, y_, z_, a)
        A = _wald_potential(x, y, z, M, a, B0)
        return [sum(J[p][i] * A[p] for p in range(3)) for i in range(3)]
    dA = _cstep(potential, xb, yb, zb)
    U = np.zeros((9,) + xb.shape)
    U[3] = dA[1][2] - dA[2][1]
    U[4] = dA[2][0] - dA[0][2]
    U[5] = dA[0][1] - dA[1][0]
    return U


def king_flux(a, B0=1.0):
    """Magnetic flux of the stationary vacuum field through the upper half of the outer
    horizon (Eq. vacuum wald magnetic flux), in units M = 1: pi r_+^2 B0 (1 - a^4 / r_+^4)
    with r_+ = 1 + sqrt(1 - a^2) and a the dimensionless spin."""
    rp = 1.0 + np.sqrt(1.0 - a * a)
    return np.pi * rp * rp * B0 * (1.0 - a ** 4 / rp ** 4)


def rotator_dipole(x, y, z, mu=1.0, theta=0.0, delta=0.1):
    """Initial data of the rotating-star tests (Sec. IV C, flat space): the field of
    the regularised dipole A = mu m x r / (r^2 + delta^2)^(3/2) with moment direction
    m = (sin theta, 0, cos theta) (theta = 0: A_phi = mu (x^2 + y^2) / (r^2 +
    delta^2)^(3/2)),
        B = curl A = mu [3 r (m . r) - m (r^2 - 2 delta^2)] / (r^2 + delta^2)^(5/2),
    and E = psi = phi = q = 0."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    m = (np.sin(theta), 0.0, np.cos(theta))
    r2 = x * x + y * y + z * z
    s = r2 + delta * delta
    mr = m[0] * x + m[1] * y + m[2] * z
    f = mu / (s * s * np.sqrt(s))
    U = np.zeros((9,) + x.shape)
    for i, xi in enumerate((x, y, z)):
        U[3 + i] = f * (3.0 * xi * mr - m[i] * (r2 - 2.0 * delta * delta))
    return U


def _ideal_e_tilde(x, y, z, M, a, Bt):
    """E~^i from E_i = -[ijk] v^j B~^k with v = beta/alpha (plasma at rest in KS coordinates)."""
    alpha, beta, g, ginv, sqrtg = _ks_3p1(x, y, z, M, a)
    v = [beta[i] / alpha for i in range(3)]
    E_lo = [-(v[1] * Bt[2] - v[2] * Bt[1]), -(v[2] * Bt[0] - v[0] * Bt[2]), -(v[0] * Bt[1] - v[1] * Bt[0])]
    return [sqrtg * sum(ginv[i][j] * E_lo[j] for j in range(3)) for i in range(3)]


@_at_singularity_nan
def kerr_schild_uniform_field(x, y, z, M=1.0, a=0.0, B0=1.0):
    """Wald-like data: B~ = (0, 0, B0), E~ from the ideal condition, q~ = d_i E~^i."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    Bt = [0.0 * x, 0.0 * x, B0 + 0.0 * x]

    def et(x_, y_, z_):
        return _ideal_e_tilde(x_, y_, z_, M, a, [0.0, 0.0, B0])

    Et = et(x, y, z)
    der = _cstep(et, x, y, z)
    q = der[0][0] + der[1][1] + der[2][2]
    U = np.zeros((9,) + x.shape)
    for i in range(3):
        U[i] = np.real(Et[i])
        U[3 + i] = Bt[i]
    U[8] = q
    return U


def _dipole_field(x, y, z, m, d, delta):
    """B~ = curl A of the regularised dipole A = m (-y, x - d, 0) / (R^2 + delta^2)^(3/2),
    R^2 = (x - d)^2 + y^2 + z^2, written out (complex-step safe):
    B~ = 3 m s u ((x - d) z, y z, 0) + m s (0, 0, 2 - 3 ((x - d)^2 + y^2) u),
    s = (R^2 + delta^2)^(-3/2), u = 1 / (R^2 + delta^2).  Divergence-free exactly."""
    xp = x - d
    u = 1.0 / (xp * xp + y * y + z * z + delta * delta)
    s = u * np.sqrt(u)
    return [3.0 * m * s * u * xp * z, 3.0 * m * s * u * y * z, m * s * (2.0 - 3.0 * (xp * xp + y * y) * u)]


def kerr_schild_parametrised_field(x, y, z, M, a, B0, tilt, m, d, delta=0.1):
    """Initial data of the adjoint workload: a uniform field of strength B0 tilted by
    `tilt` about the x axis, B~ = B0 (0, -sin tilt, cos tilt), plus the regularised
    dipole of amplitude m centred at (d, 0, 0) (off the spin axis by d); E~ from the
    ideal condition (plasma at rest in Kerr-Schild coordinates) and q~ = d_i E~^i."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)

    def bt(x_, y_, z_):
        dip = _dipole_field(x_, y_, z_, m, d, delta)
        zero = 0.0 * x_
        return [dip[0] + zero, dip[1] - B0 * np.sin(tilt) + zero, dip[2] + B0 * np.cos(tilt) + zero]

    def et(x_, y_, z_):
        return _ideal_e_tilde(x_, y_, z_, M, a, bt(x_, y_, z_))

    Bt = bt(x, y, z)
    Et = et(x, y, z)
    der = _cstep(et, x, y, z)
    U = np.zeros((9,) + x.shape)
    for i in range(3):
        U[i] = np.real(Et[i])
        U[3 + i] = np.real(Bt[i])
    U[8] = der[0][0] + der[1][1] + der[2][2]
    return U


def adjoint_parameters(seed=1005):
    """The four seeded initial-field parameters of the adjoint workload:
    B0 ~ 1 + 0.1 N(0,1), tilt ~ U(0, 0.3), dipole amplitude m ~ U(20, 60), offset d ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    return dict(B0=1.0 + 0.1 * rng.standard_normal(), tilt=0.3 * rng.random(), m=20.0 + 40.0 * rng.random(),
                d=-1.0 + 2.0 * rng.random())


def sphere_quadrature(R=20.0, n_theta=32, n_phi=64):
    """Points (3, n_theta * n_phi) on the Euclidean sphere of radius R and weights of
    the surface integral: Gauss-Legendre in cos(theta), uniform midpoints in phi."""
    ct, wt = np.polynomial.legendre.leggauss(n_theta)
    ph = 2.0 * np.pi * (np.arange(n_phi) + 0.5) / n_phi
    st = np.sqrt(1.0 - ct * ct)
    X = R * np.outer(st, np.cos(ph)).ravel()
    Y = R * np.outer(st, np.sin(ph)).ravel()
    Z = R * np.outer(ct, np.ones(n_phi)).ravel()
    W = np.outer(wt, np.full(n_phi, 2.0 * np.pi / n_phi)).ravel() * R * R
    return np.stack([X, Y, Z]), W


# ----------------------------------------------------------------------------
# named workloads (shapes of the paper's flat-space wave tests and
# black-hole magnetospheres)

BC_PERIODIC = 0
BC_NO_INCOMING_POYNTING = 1
BC_DIRICHLET = 2

_ONE_D = {"fast_wave_1d": ((-0.5, 1.5), 9.22e-4, fast_wave_1d),
          "alfven_1d": ((-1.5, 1.5), 1.38e-3, alfven_stationary_1d),
          "ffe_breakdown_1d": ((-0.5, 0.5), 4.61e-4, ffe_breakdown_1d)}


def workload(name, **over):
    """Grid and parameter description of a named synthetic workload."""
    if name == "wave":  # 2^3 elements, periodic [-1,1]^3, smooth sine + noise
        w = dict(n_elem=(2, 2, 2), lower=(-1.0, -1.0, -1.0), upper=(1.0, 1.0, 1.0), degree=5,
                 bc=(BC_PERIODIC,) * 6, eta=1e6, cfl=0.25, steps=10, seed=1001, curved=False,
                 amplitude=0.1, kind="wave")
    elif name == "sheet":  # 8^3 elements, tanh current sheet, mixed DG/FD
        w = dict(n_elem=(8, 8, 8), lower=(-1.0, -1.0, -1.0), upper=(1.0, 1.0, 1.0), degree=5,
                 bc=(BC_PERIODIC,) * 6, eta=1e6, cfl=0.25, steps=200, seed=1002, curved=False,
                 width=0.05, kind="sheet")
    elif name == "kerr_schild":  # black hole a=0.9, 16^3 elements on [-40,40]^3
        w = dict(n_elem=(16, 16, 16), lower=(-40.0,) * 3, upper=(40.0,) * 3, degree=5,
                 bc=(BC_NO_INCOMING_POYNTING,) * 6, eta=1e5, cfl=0.25, steps=1000, seed=1003,
                 curved=True, M=1.0, spin=0.9, B0=1.0, r_excise=1.8, kind="kerr_schild")
    elif name == "rotator":
        # rotating magnetised star (Sec. IV C): R = 1, one element per R, Omega = 1/(5R),
        # eta = 1e5/R, dipole regularised with delta = 0.1R, inclination theta
        w = dict(n_elem=(24, 24, 24), lower=(-12.0,) * 3, upper=(12.0,) * 3, degree=5,
                 bc=(BC_NO_INCOMING_POYNTING,) * 6, eta=1e5, cfl=0.25, curved=False, kind="rotator",
                 mu=1.0, theta=0.0, delta=0.1, radius=1.0, omega=0.2, centre=(0.0, 0.0, 0.0))
    elif name == "smooth_fast_wave":  # Sec. IV D 1: [0, 2]^3, 4^3 P5 elements, periodic
        w = dict(n_elem=(4, 4, 4), lower=(0.0,) * 3, upper=(2.0,) * 3, degree=5, bc=(BC_PERIODIC,) * 6, eta=1e6,
                 cfl=0.3, curved=False, kind="smooth_fast_wave", wavelength=2.0)
    elif name in _ONE_D:
        # one-dimensional problems (Sec. IV A, Table 1): 32 * 2^level elements of P5
        # along x, one along y and z ([-0.1, 0.1], periodic), Dirichlet at both x ends
        (x0, x1), _, _ = _ONE_D[name]
        level = int(over.pop("level", 0))
        w = dict(n_elem=(32 * 2 ** level, 1, 1), lower=(x0, -0.1, -0.1), upper=(x1, 0.1, 0.1), degree=5,
                 bc=(BC_DIRICHLET, BC_DIRICHLET) + (BC_PERIODIC,) * 4, eta=1e6, cfl=0.3, curved=False,
                 kind=name, level=level)
    else:
        raise ValueError(f"unknown workload {name!r}")
    w.update(over)
    return w


def boundary_field(w, fn, ref_dg):
    """Per-point exterior states of Dirichlet faces from an analytic state
    fn(x, y, z) -> (9, ...): at every DG face node ((9, E, 6, n^2), node t1 + n t2 of
    face f = 2 d + s, t1 along the lower tangential axis; ref_dg are the caller's 1D
    DG nodes) and at every FD ghost cell ((9, E, 6, 3, m^2), layer l = 0, 1, 2 counted
    outwards from the face: the boundary cell's centre moved by (l + 1) cell widths)."""
    ne = w["n_elem"]
    N = w["degree"]
    n, m = N + 1, 2 * N + 1
    E = int(np.prod(ne))
    h = (np.asarray(w["upper"], np.float64) - np.asarray(w["lower"], np.float64)) / np.asarray(ne)
    x, y, z = points(ne, w["lower"], w["upper"], ref_dg)
    xf, yf, zf = fd_points(ne, w["lower"], w["upper"], N)
    dg = np.zeros((9, E, 6, n * n))
    fd = np.zeros((9, E, 6, 3, m * m))
    for d in range(3):
        ax = 3 - d  # point arrays are (E, z, y, x)
        for s in (0, 1):
            f = 2 * d + s
            pts = [np.take(c, [0 if s == 0 else N], axis=ax).reshape(E, n * n) for c in (x, y, z)]
            dg[:, :, f] = fn(*pts)
            for l in range(3):
                gp = [np.take(c, [0 if s == 0 else m - 1], axis=ax).reshape(E, m * m).copy() for c in (xf, yf, zf)]
                gp[d] += (1 if s else -1) * (l + 1) * h[d] / m
                fd[:, :, f, l] = fn(*gp)
    return dg, fd


def table1_dt(name, level=0):
    """The time step Table 1 prints for a one-dimensional problem (x 2^-level)."""
    return _ONE_D[name][1] * 2.0 ** -level


def boundary_states(w):
    """(6, 9) exterior states of a workload's Dirichlet faces: its initial data at the
    two ends of the x axis (uniform over each face); rows of other faces are zero."""
    out = np.zeros((6, 9))
    for s, x in ((0, w["lower"][0]), (1, w["upper"][0])):
        if w["bc"][s] == BC_DIRICHLET:
            out[s] = initial_data(w, np.array([x]), np.zeros(1), np.zeros(1), with_noise=False)[:, 0]
    return out


def batch_workloads(count=64, seed=4, n_range=(4, 12), degree_range=(3, 7)):
    """Descriptions of `count` independent flat periodic domains on [-1,1]^3:
    n^3 elements with n ~ U{n_range}, degree N ~ U{degree_range}, kind wave or sheet
    with equal probability; domain j draws its noise from seed 4000 + j."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        N = int(rng.integers(degree_range[0], degree_range[1] + 1))
        kind = "wave" if rng.random() < 0.5 else "sheet"
        out.append(workload(kind, n_elem=(n, n, n), degree=N, seed=4000 + j))
    return out


def excision_mask(w):
    """Elements whose box intersects the Euclidean ball of radius r_excise (uint8, E)."""
    E = int(np.prod(w["n_elem"]))
    if not w.get("curved") or not w.get("r_excise"):
        return np.zeros(E, np.uint8)
    corner, h = element_boxes(w["n_elem"], w["lower"], w["upper"])
    lo = corner
    hi = corner + h[None, :]
    closest = np.clip(0.0, lo, hi)
    d = np.sqrt((closest ** 2).sum(axis=1))
    return (d < w["r_excise"]).astype(np.uint8)


def initial_data(w, x, y, z, with_noise=True):
    """Densitized initial U (9, ...) of workload ``w`` at the given points."""
    kind = w["kind"]
    if kind == "wave":
        U = fast_wave_sine(x, w.get("amplitude", 0.1))
    elif kind == "sheet":
        U = current_sheet(x, w.get("width", 0.05), 0.5 * (w["upper"][0] - w["lower"][0]))
    elif kind == "kerr_schild":
        U = kerr_schild_uniform_field(x, y, z, w.get("M", 1.0), w.get("spin", 0.0), w.get("B0", 1.0))
    elif kind == "wald_a0":
        U = wald_a0(x, y, z, w.get("M", 1.0), w.get("B0", 1.0))
    elif kind == "rotator":
        c = w.get("centre", (0.0, 0.0, 0.0))
        U = rotator_dipole(np.asarray(x) - c[0], np.asarray(y) - c[1], np.asarray(z) - c[2], w.get("mu", 1.0),
                           w.get("theta", 0.0), w.get("delta", 0.1))
    elif kind in _ONE_D:
        U = _ONE_D[kind][2](x)
    elif kind == "pulses_1d":
        U = smooth_pulses_1d(x)
    elif kind == "smooth_fast_wave":
        U = smooth_fast_wave(x, w.get("wavelength", 2.0))
    else:
        raise ValueError(kind)
    if with_noise and kind in ("wave", "sheet"):
        U = add_noise_by_and_ez(U, w["seed"], w.get("noise", 1e-3))
    return U


def background(w, x, y, z):
    """Background fields (26, ...) of workload ``w`` at given points (None when flat
    in coordinates at rest); the rotator with frame = "rotating" runs in the frame
    that rotates with the star."""
    if w.get("kind") == "rotator" and w.get("frame") == "rotating":
        return rotating_frame_background(x, y, z, w["omega"], w.get("centre", (0.0, 0.0, 0.0)))
    if not w.get("curved"):
        return None
    return kerr_schild_background(x, y, z, w.get("M", 1.0), w.get("spin", 0.0))
