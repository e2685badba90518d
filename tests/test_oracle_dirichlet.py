"""The oracle's Dirichlet faces and the one-dimensional problems (Sec. IV A, Table 1,
Appendix A), pinned to exact solutions.

* The fast wave is a pure right-moving vacuum mode (E_z = -B_y, J = 0), and the
  Rusanov flux with speed 1 is the exact upwind flux for it: the element next to the
  inflow face sees no left-moving signal and must keep the left state to rounding,
  while the kink travels as Q(x - t).  Swapping the two faces' states, or taking
  the no-incoming-Poynting state there, changes that element at once.
* Two smooth pulses leaving through the Dirichlet faces (whose state is the
  background the pulses move into) must leave nothing behind but the scheme's
  truncation error; a Rusanov flux with the exterior state on the wrong side blocks
  the outgoing characteristic and reflects the pulse.
* The Appendix-A data satisfy what the paper states of them (continuity, the
  stationary Alfven wave's force-free balance, magnetic dominance)."""
import numpy as np
import pytest

from oracle import operators as ops
from oracle import rhs as R
from oracle import step as S
from oracle.domain import DG, FD, Domain
from paper_2404_01531_amd import inputs as I


def _domain(w):
    return Domain(w["n_elem"], w["lower"], w["upper"], w["degree"], w["bc"],
                  params=dict(eta=w["eta"], cfl=w["cfl"]), boundary_state=I.boundary_states(w))


def _run(w, steps):
    dom = _domain(w)
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], w["degree"])
    st = S.initial_state(dom, I.initial_data(w, xf, yf, zf))
    dt = dom.dt()
    for _ in range(steps):
        st = S.step(dom, st, dt)
    return dom, st, steps * dt


def test_fast_wave_inflow_element_exact_and_kink_advected():
    w = I.workload("fast_wave_1d", n_elem=(8, 1, 1))
    dom, st, t = _run(w, 20)
    left, right = I.boundary_states(w)[:2]
    assert st.rep[0] == DG
    assert np.abs(st.dg[:, 0] - left[:, None, None, None]).max() < 1e-12
    assert np.abs(st.dg[:, -1] - right[:, None, None, None]).max() < 1e-5
    x, _, _ = I.points(w["n_elem"], w["lower"], w["upper"], ops.gll(5)[0])
    xf, _, _ = I.fd_points(w["n_elem"], w["lower"], w["upper"], 5)
    exact_dg, exact_fd = I.fast_wave_1d(x - t), I.fast_wave_1d(xf - t)
    for e in range(dom.E):
        got, ref = (st.dg[:, e], exact_dg[:, e]) if st.rep[e] == DG else (st.fd[:, e], exact_fd[:, e])
        # the C0 kinks limit the pointwise error near them (Sec. IV A 1)
        assert np.abs(got - ref).max() < 0.03, e


def test_pulses_leave_through_dirichlet_faces():
    w = I.workload("fast_wave_1d", n_elem=(4, 1, 1), lower=(0.0, -0.125, -0.125), upper=(1.0, 0.125, 0.125),
                   kind="pulses_1d")
    bg = np.zeros(9)
    bg[3] = 1.0
    assert np.allclose(I.boundary_states(w)[:2], bg)
    dom = _domain(w)
    dt = dom.dt()
    steps = int(np.ceil(0.55 / dt))  # both pulses (half width 0.2, 0.3 from the faces) have left
    dom, st, _ = _run(w, steps)
    x, _, _ = I.points(w["n_elem"], w["lower"], w["upper"], ops.gll(5)[0])
    assert np.abs(I.initial_data(w, x, x, x) - bg[:, None, None, None, None]).max() > 0.05
    assert (st.rep == DG).all()
    assert np.abs(st.dg - bg[:, None, None, None, None]).max() < 3e-3


def test_one_d_initial_data():
    x = np.linspace(-1.5, 1.5, 30001)
    fw = I.fast_wave_1d(x)
    assert np.array_equal(fw[2], -fw[4]) and np.all(fw[3] == 1.0)
    for f in (I.fast_wave_1d, I.alfven_stationary_1d, I.ffe_breakdown_1d):
        for xb in (-0.1, 0.1):  # continuous at the layer's edges
            lo, hi = f(np.array([xb - 1e-12])), f(np.array([xb + 1e-12]))
            assert np.abs(lo - hi).max() < 1e-9, f.__name__
        U = f(x)
        E, B = U[0:3], U[3:6]
        assert np.abs((E * B).sum(0)).max() < 1e-14, f.__name__
        assert ((B * B).sum(0) - (E * E).sum(0)).min() > 0.0, f.__name__
    # stationary Alfven wave: q = div E and curl B equals the force-free current
    # rho E x B / B^2 + (B . curl B - E . curl E) B / B^2 (so dE/dt = 0), curl E = 0
    U = I.alfven_stationary_1d(x)
    dx = x[1] - x[0]
    d = lambda f: np.gradient(f, dx)
    E, B = U[0:3], U[3:6]
    # central differences, away from the ends and from the second derivative's jumps at +-0.1
    inner = (np.arange(x.size) > 1) & (np.arange(x.size) < x.size - 2) & (np.abs(np.abs(x) - 0.1) > 3 * dx)
    assert np.abs(U[8] - d(E[0]))[inner].max() < 1e-5
    curlB = np.array([0 * x, -d(B[2]), d(B[1])])
    curlE = np.array([0 * x, -d(E[2]), d(E[1])])
    B2 = (B * B).sum(0)
    J = U[8] * np.cross(E, B, axis=0) / B2 + ((B * curlB).sum(0) - (E * curlE).sum(0)) * B / B2
    assert np.abs(curlB - J)[:, inner].max() < 1e-5
    assert np.abs(curlE).max() == 0.0


def test_boundary_states_and_required():
    w = I.workload("alfven_1d")
    bs = I.boundary_states(w)
    assert np.array_equal(bs[0], I.alfven_stationary_1d(np.array([-1.5]))[:, 0])
    assert np.array_equal(bs[1], I.alfven_stationary_1d(np.array([1.5]))[:, 0])
    assert not bs[2:].any()
    with pytest.raises(ValueError):
        Domain(w["n_elem"], w["lower"], w["upper"], 5, w["bc"])


def test_per_point_dirichlet_keeps_exact_wald_stationary():
    """The a = 0 Wald field (Kerr-Schild background, Sec. IV B) is stationary.  On a
    box away from the hole with every face a Dirichlet face holding the exact field
    point by point, the right-hand side of every element -- boundary elements
    included -- vanishes spectrally as N grows; with no-incoming-Poynting faces it
    does not.  An FD element's residual falls with N too, and is larger when its
    ghost layers are taken in the wrong order."""
    ne, lo, hi = (2, 2, 2), (4.0, -2.0, -2.0), (8.0, 2.0, 2.0)
    res, res_fd, res_fd_rev = [], [], []
    rep_mixed = np.array([1, 0, 0, 0, 0, 0, 0, 1])
    for N in (3, 5, 7):
        w = dict(n_elem=ne, lower=lo, upper=hi, degree=N)
        x, y, z = I.points(ne, lo, hi, ops.gll(N)[0])
        xf, yf, zf = I.fd_points(ne, lo, hi, N)
        bg = I.kerr_schild_background(x, y, z, 1.0, 0.0)
        field = I.boundary_field(w, I.wald_a0, ops.gll(N)[0])
        U, Uf = I.wald_a0(x, y, z), I.wald_a0(xf, yf, zf)
        dom = Domain(ne, lo, hi, N, (2,) * 6, bg=bg, params=dict(eta=1e5), boundary_field=field)
        L, _ = R.rhs(dom, U, Uf, np.zeros(8, np.int64), parts=3)
        res.append(np.abs(L).max())
        _, Lf = R.rhs(dom, U, Uf, rep_mixed, parts=3)
        res_fd.append(np.abs(Lf[:, rep_mixed == 1]).max())
        rev = Domain(ne, lo, hi, N, (2,) * 6, bg=bg, params=dict(eta=1e5),
                     boundary_field=(field[0], field[1][:, :, :, ::-1]))
        _, Lr = R.rhs(rev, U, Uf, rep_mixed, parts=3)
        res_fd_rev.append(np.abs(Lr[:, rep_mixed == 1]).max())
        if N == 7:
            nip = Domain(ne, lo, hi, N, (1,) * 6, bg=bg, params=dict(eta=1e5))
            Ln, _ = R.rhs(nip, U, Uf, np.zeros(8, np.int64), parts=3)
            assert np.abs(Ln).max() > 1.0
    assert res[1] < res[0] / 30 and res[2] < res[1] / 30 and res[2] < 1e-5
    assert res_fd[1] < res_fd[0] / 10 and res_fd[2] < res_fd[1] / 3
    assert res_fd_rev[2] > 5 * res_fd[2]
