"""The oracle's rotating perfect conductor (Sec. IV C, pulsar magnetospheres), pinned
to what the ideal condition and the scheme's locality fix.

* In a uniform field B0 z^ a conductor rotating about z with angular velocity
  Omega is the unipolar inductor: corotation v = Omega z^ x (x - c) demands the
  radial field E = -Omega B0 (x - c_x, y - c_y, 0) inside it (the textbook result,
  whose divergence -2 Omega B0 is the Goldreich-Julian charge of these units).
  With E = 0 and B uniform the fields are otherwise stationary, so after a step the
  points inside the sphere hold that field up to |v| times the small change of B
  (B moves where E jumps at the sphere inside an element), psi~ and q~ are zero there and
  phi~ is not touched; points of the same elements outside the sphere are not
  overwritten but have been driven by it (which they are only if the overwrite
  enters the later substeps' right-hand sides); elements three or more faces away
  from any overwritten point keep their E and B.
* The same holds with the conductor's elements on the FD grid.
* For a rotating dipole the enforced E is perpendicular to both B and v."""
import numpy as np

from oracle import step as S
from oracle.domain import DG, FD, Domain
from paper_2404_01531_amd import inputs as I

NE, LO, HI = (8, 2, 2), (-4.0, -1.0, -1.0), (4.0, 1.0, 1.0)
COND = dict(centre=(0.13, -0.07, 0.05), radius=0.8, omega=0.3)
B0 = 1.7


def _uniform(shape):
    U = np.zeros((9,) + shape)
    U[5] = B0
    U[6] = 0.01   # psi~: forced to zero inside
    U[7] = 0.02   # phi~: evolves
    U[8] = 0.03   # q~: forced to zero inside
    return U


def _run(forced=None, conductor=COND, N=3):
    params = dict(eta=1e5, hybrid=S.HYBRID_FORCED if forced is not None else S.HYBRID_DG_ONLY)
    dom = Domain(NE, LO, HI, N, (0,) * 6, params=params, conductor=conductor)
    m = 2 * N + 1
    st0 = S.initial_state(dom, _uniform((dom.E, m, m, m)), forced=forced)
    st = S.step(dom, st0, dom.dt())
    return dom, st0, st


def _check_unipolar(dom, st, rep):
    c = COND
    el = np.nonzero(st.rep == rep)[0]
    U = st.dg if rep == DG else st.fd
    x, y, z = dom.point_coords(el, rep == FD)
    rx, ry, rz = x - c["centre"][0], y - c["centre"][1], z - c["centre"][2]
    inside = rx ** 2 + ry ** 2 + rz ** 2 <= c["radius"] ** 2
    assert inside.sum() > 10
    u = U[:, el]
    ex, ey = -c["omega"] * B0 * rx, -c["omega"] * B0 * ry
    # E - E_unipolar = -v x (B - B0 z^): bounded by |v| |B - B0 z^| (B itself moves a
    # little where E jumps at the sphere inside an element)
    dB = np.sqrt(u[3] ** 2 + u[4] ** 2 + (u[5] - B0) ** 2)[inside]
    speed = c["omega"] * np.hypot(rx, ry)[inside]
    dE = np.sqrt((u[0][inside] - ex[inside]) ** 2 + (u[1][inside] - ey[inside]) ** 2 + u[2][inside] ** 2)
    assert np.all(dE <= speed * dB * (1 + 1e-9) + 1e-13)
    assert dB.max() < 0.05 * B0
    assert np.all(u[6][inside] == 0.0) and np.all(u[8][inside] == 0.0)
    assert np.abs(u[7][inside]).min() > 0.01
    # outside the sphere, within the conductor's elements: not the corotation value
    # but driven away from E = 0
    hit = inside.reshape(len(el), -1).any(1)
    out = ~inside & hit[:, None, None, None]
    dev = np.hypot(u[0][out] - ex[out], u[1][out] - ey[out])
    assert dev.max() > 0.05
    assert np.abs(u[0:3][:, out]).max() > 1e-4
    return el[hit]


def test_unipolar_inductor_on_dg():
    dom, st0, st = _run()
    assert (st.rep == DG).all()
    held = _check_unipolar(dom, st, DG)
    ex = sorted({dom.coords(e)[0] for e in held})
    assert ex == [3, 4]
    far = np.array([e for e in range(dom.E) if dom.coords(e)[0] in (0, 7)])
    # (psi~ and phi~ decay everywhere by their damping)
    assert np.abs(st.dg[0:6, far] - st0.dg[0:6, far]).max() < 1e-12
    near = np.array([e for e in range(dom.E) if dom.coords(e)[0] in (2, 5)])
    assert np.abs(st.dg[0:3, near]).max() > 1e-6


def test_unipolar_inductor_on_fd():
    forced = np.zeros(16 * 2, bool)
    for e in range(32):
        forced[e] = (e % 8) in (3, 4)
    dom, st0, st = _run(forced=forced)
    assert np.array_equal(st.rep == FD, forced)
    _check_unipolar(dom, st, FD)
    far = np.array([e for e in range(dom.E) if dom.coords(e)[0] in (0, 7)])
    assert np.abs(st.dg[0:6, far] - st0.dg[0:6, far]).max() < 1e-12


def test_no_conductor_is_stationary():
    dom, st0, st = _run(conductor=None)
    assert np.abs(st.dg[0:6] - st0.dg[0:6]).max() < 1e-12


def test_rotating_dipole_field_is_ideal_inside():
    w = dict(kind="rotator", mu=1.0, theta=np.pi / 4, delta=0.3, centre=(0.0, 0.0, 0.0))
    cond = dict(centre=(0.0, 0.0, 0.0), radius=0.9, omega=0.2)
    dom = Domain((4, 2, 2), (-2.0, -1.0, -1.0), (2.0, 1.0, 1.0), 3, (1,) * 6,
                 params=dict(eta=1e5, hybrid=S.HYBRID_DG_ONLY), conductor=cond)
    xf, yf, zf = I.fd_points(dom.n_elem, dom.lower, dom.upper, 3)
    st = S.step(dom, S.initial_state(dom, I.initial_data(w, xf, yf, zf)), dom.dt())
    x, y, z = dom.point_coords(np.arange(dom.E), False)
    inside = x ** 2 + y ** 2 + z ** 2 <= 0.81
    E, B = st.dg[0:3][:, inside], st.dg[3:6][:, inside]
    v = np.array([-0.2 * y[inside], 0.2 * x[inside], 0 * x[inside]])
    scale = np.sqrt((E * E).sum(0) * (B * B).sum(0)).max()
    assert np.abs((E * B).sum(0)).max() < 1e-12 * scale
    assert np.abs((E * v).sum(0)).max() < 1e-12 * scale
    assert np.sqrt((E * E).sum(0)).max() > 0.01


# ------------------------------------------------------------------ rotating frame


def _rotating_domain(N, omega, params=None, conductor=None):
    from oracle import operators as ops
    ne, lo, hi = (4, 4, 2), (-2.0, -2.0, -1.0), (2.0, 2.0, 1.0)
    x, y, z = I.points(ne, lo, hi, ops.gll(N)[0])
    bg = I.rotating_frame_background(x, y, z, omega)
    return Domain(ne, lo, hi, N, (0,) * 6, bg=bg, params=params or dict(eta=0.0), conductor=conductor)


def test_uniform_field_rotates_backwards_in_the_rotating_frame():
    """Sec. IV C's rotating grid: in coordinates rotating at Omega the normal observers
    are the inertial ones, so a field that is uniform and static in the inertial frame
    (E = 0, B uniform) keeps E = 0 and appears to turn at -Omega: dB/dt = -Omega z^ x B
    exactly (the right-hand side of the scheme with the rotating frame's shift,
    every flux divergence of uniform data vanishing), on DG nodes and on FD cells."""
    from oracle import rhs as R
    omega = 0.3
    for N in (3, 5):
        dom = _rotating_domain(N, omega)
        Bv = np.array([0.4, -0.7, 1.1])
        dg = np.zeros((9, dom.E, dom.n, dom.n, dom.n))
        fd = np.zeros((9, dom.E, dom.m, dom.m, dom.m))
        for i in range(3):
            dg[3 + i] = Bv[i]
            fd[3 + i] = Bv[i]
        rep = (np.arange(dom.E) % 2).astype(np.int64)  # DG and FD elements side by side
        ddg, dfd = R.rhs(dom, dg, fd, rep)
        want = np.array([omega * Bv[1], -omega * Bv[0], 0.0])
        # rounding: the fluxes beta^d B^i (up to ~1.3) differentiated by operators of
        # norm ~ N^2 / h leave ~1e-14
        tol = 2e-13
        for r, D in ((0, ddg), (1, dfd)):
            el = np.nonzero(rep == r)[0]
            assert np.abs(D[0:3, el]).max() < tol
            for i in range(3):
                assert np.abs(D[3 + i, el] - want[i]).max() < tol, (N, r, i)
            assert np.abs(D[6:9, el]).max() < tol


def test_conductor_at_rest_in_the_rotating_frame_is_the_corotating_one():
    """The conductor at rest on the rotating grid (omega = 0 relative to it) is moved
    by the frame's shift alone: its E equals the inertial frame's corotation field
    -(Omega z^ x (x - c)) x B at the same points (with c on the axis)."""
    from oracle import physics as ph
    omega = 0.3
    dom = _rotating_domain(3, omega)
    rng = np.random.default_rng(12)
    U = rng.standard_normal((9, dom.E, dom.n, dom.n, dom.n))
    x, y, z = dom.point_coords(np.arange(dom.E), False)
    centre = (0.0, 0.0, 0.1)
    got = ph.corotating_conductor(U, x, y, z, centre, 1.5, 0.0, dom.geo_dg)
    ref = ph.corotating_conductor(U, x, y, z, centre, 1.5, omega)
    inside = x ** 2 + y ** 2 + (z - 0.1) ** 2 <= 1.5 ** 2
    assert inside.sum() > 50
    assert np.abs(got - ref).max() < 1e-14
    assert np.array_equal(got[:, ~inside], U[:, ~inside])
