"""Pins of the oracle's step, hybrid control, boundary state, current closure and
curved indicator against formulations other than its own.

* The register-form step of ``oracle.step.step`` against the plain Butcher form of
  IMEX-SSP3(4,3,3) (Sec. III B): ``imex_step_generic`` on all-DG and all-FD domains,
  and a Butcher-form step written here that carries the hybrid control of
  Sec. III C 1 (an element redone on FD in substep k, its history moved with P,
  its pre-stages re-derived from the projected U^n) for rollbacks in each of the
  three substeps.
* A substep-1 rollback against a step with the element on FD from the start (the
  two agree exactly when P, R and the stiff solve commute: R P = I, flat space,
  vanishing current).
* The end-of-step switch back (alpha + 1 = 5, Sec. III C 3) on data whose
  indicator ratio is known in closed form.
* The no-incoming-Poynting state (Sec. III D), the drift current (Eq. electric
  current density) and the curved indicator (|B~| with gamma_ij) on hand-built
  cases.
* The reason for the filter placement: the filter applied to the solved stage
  values makes the noisy wave blow up.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import operators as ops
from oracle import physics as ph
from oracle import rhs as R
from oracle import step as S
from oracle import tci
from oracle.domain import DG, FD, Domain, geo_take
from paper_2404_01531_amd import inputs as I

from helpers import GROUPS, state_arrays

# ------------------------------------------------------------------ helpers


def _group_err(got, ref):
    """max |got - ref| over each variable group, relative to the largest |ref| of all nine components."""
    got = np.asarray(got).reshape(9, -1)
    ref = np.asarray(ref).reshape(9, -1)
    sc = max(np.abs(ref).max(), 1e-300)
    return max(np.abs(got[a:b] - ref[a:b]).max() for a, b in GROUPS) / sc


def _periodic(n_elem, N, **params):
    return Domain(n_elem, (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0), N, (0,) * 6, params=params)


def _solve(dom, geo):
    p = dom.params
    return lambda Y, h: ph.implicit_solve(Y, geo, p["eta"], p["kappa_psi"], p["kappa_phi"], h)


def _stiff(dom, geo):
    p = dom.params
    return lambda U: ph.source_stiff(U, geo, p["eta"], p["kappa_psi"], p["kappa_phi"])


# ------------------------------------------- register form vs plain Butcher form


@pytest.mark.parametrize("eta,kappa", [(0.0, 0.0), (1e3, 1.5)])
def test_step_all_dg_equals_butcher_form(eta, kappa):
    """Sec. III B: with the filter off, one step of an all-DG periodic domain is the
    IMEX-SSP3(4,3,3) Butcher step of dU/dt = L(U) + S(U) with the oracle's DG operator."""
    dom = _periodic((2, 2, 2), 3, eta=eta, kappa_psi=kappa, kappa_phi=kappa, filter_on=0, hybrid=S.HYBRID_DG_ONLY)
    dg, _ = state_arrays(dom, np.random.default_rng(11), None)
    zero_fd = np.zeros((9, dom.E, dom.m, dom.m, dom.m))
    rep = np.zeros(dom.E, np.int64)
    dt = dom.dt()
    got = S.step(dom, S.State(dg, zero_fd, rep), dt)
    ref = S.imex_step_generic(dg, dt, lambda U: R.rhs(dom, U, zero_fd, rep, parts=1)[0],
                              _stiff(dom, dom.geo_dg), _solve(dom, dom.geo_dg))
    assert _group_err(got.dg, ref) < 1e-14


@pytest.mark.parametrize("eta,kappa", [(0.0, 0.0), (1e3, 1.5)])
def test_step_all_fd_equals_butcher_form(eta, kappa):
    """The same on an all-FD domain (FD operator of Sec. III C 2)."""
    dom = _periodic((2, 2, 2), 3, eta=eta, kappa_psi=kappa, kappa_phi=kappa, hybrid=S.HYBRID_FORCED)
    _, fd = state_arrays(dom, np.random.default_rng(12), None)
    zero_dg = np.zeros((9, dom.E, dom.n, dom.n, dom.n))
    rep = np.ones(dom.E, np.int64)
    dt = dom.dt()
    got = S.step(dom, S.State(zero_dg, fd, rep), dt)
    ref = S.imex_step_generic(fd, dt, lambda U: R.rhs(dom, zero_dg, U, rep, parts=1)[1],
                              _stiff(dom, dom.geo_fd), _solve(dom, dom.geo_fd))
    assert _group_err(got.fd, ref) < 1e-14


def _butcher_hybrid(dom, st, dt, roll):
    """One IMEX-SSP3(4,3,3) step in Butcher form with the hybrid control of
    Sec. III C 1, for a given set of rollbacks.

    Stage i = 0..3 (U_1..U_4): Y_i = U^n + dt sum_{j<i} (Aex_ij L_j + Aim_ij S_j),
    U_i = solve(Y_i, a dt); substep k = 1, 2, 3 evaluates L at stage k, and the
    output is U^n + dt sum_i w_i (L_i + S_i).  On DG the filter acts on Y_2, Y_3
    before the solve and on the output.  roll[e] = k: the element, on DG at the
    step start, is updated on FD from substep k on; there its neighbours still read
    it on DG (the representation at the substep start).  When it moves, U^n, the
    stage value U_k (k >= 2), the explicit terms L_j (j < k) and, for k = 3, the
    stiff term S_2 (evaluated in substep 2) are projected with P; U_1, U_2, S_1, S_2
    are re-derived from P U^n on the FD grid.  After the step every FD element
    whose reconstruction passes the indicator with alpha + 1 goes back to DG.
    """
    p = dom.params
    N = dom.N
    A, Ah, W = S.AEX, S.AIM, S.BW
    a = Ah[0, 0]
    Pm = ops.projection_matrix(N)
    Fm = ops.filter_matrix(N, p["filter_a"], p["filter_b"]) if p["filter_on"] else None
    filt = (lambda u: ops.apply_3d(Fm, u)) if Fm is not None else (lambda u: u)
    geo = [dom.geo_dg, dom.geo_fd]
    solve = [_solve(dom, g) for g in geo]
    stiff = [_stiff(dom, g) for g in geo]
    roll = np.asarray(roll, np.int64)
    start_fd = (st.rep == FD) & dom.active
    Un = [st.dg.copy(), st.fd.copy()]
    U = [[None, None] for _ in range(4)]
    Sx = [[None, None] for _ in range(4)]
    L = [[None, None] for _ in range(4)]
    for g in (DG, FD):
        U[0][g] = solve[g](Un[g], dt * a)
        Sx[0][g] = stiff[g](U[0][g])
        U[1][g] = solve[g](Un[g] + dt * Ah[1, 0] * Sx[0][g], dt * a)
        Sx[1][g] = stiff[g](U[1][g])
    out = [None, None]
    for k in (1, 2, 3):
        rep0 = np.where(start_fd | ((roll > 0) & (roll < k)), FD, DG)
        moving = np.nonzero((roll == k) & ~start_fd)[0]
        for e in moving:
            ge = geo_take(dom.geo_fd, [e])
            Un[FD][:, e] = ops.apply_3d(Pm, Un[DG][:, e])
            sol, stf = _solve(dom, ge), _stiff(dom, ge)
            u0 = sol(Un[FD][:, [e]], dt * a)
            s0 = stf(u0)
            u1 = sol(Un[FD][:, [e]] + dt * Ah[1, 0] * s0, dt * a)
            s1 = stf(u1)
            U[0][FD][:, e], Sx[0][FD][:, e], U[1][FD][:, e], Sx[1][FD][:, e] = u0[:, 0], s0[:, 0], u1[:, 0], s1[:, 0]
            for j in range(1, k):
                L[j][FD][:, e] = ops.apply_3d(Pm, L[j][DG][:, e])
            if k >= 2:
                U[k][FD][:, e] = ops.apply_3d(Pm, U[k][DG][:, e])
            if k == 3:
                Sx[2][FD][:, e] = ops.apply_3d(Pm, Sx[2][DG][:, e])
        Ld, Lf = R.rhs(dom, U[k][DG], U[k][FD], rep0, parts=1)
        for e in moving:
            r1 = rep0.copy()
            r1[e] = FD
            Lf[:, e] = R.rhs(dom, U[k][DG], U[k][FD], r1, parts=1)[1][:, e]
        L[k] = [Ld, Lf]
        if k >= 2:  # S_k at this substep's input (S_2 of a move in substep 3 stays projected)
            Sx[k] = [stiff[DG](U[k][DG]), stiff[FD](U[k][FD])]
        for g in (DG, FD):
            if k < 3:
                Y = Un[g] + dt * sum(A[k + 1, j] * L[j][g] for j in range(1, k + 1))
                Y = Y + dt * sum(Ah[k + 1, j] * Sx[j][g] for j in range(0, k + 1))
                if g == DG:
                    Y = filt(Y)
                U[k + 1][g] = solve[g](Y, dt * a)
            else:
                o = Un[g] + dt * sum(W[j] * (L[j][g] + Sx[j][g]) for j in range(1, 4))
                out[g] = filt(o) if g == DG else o
    rep = np.where(start_fd | (roll > 0), FD, DG)
    rep[~dom.active] = DG
    dg, fd = out
    M = p["tci_M"] if p["tci_M"] else ops.tci_M(N)
    thr_fd = tci.tci_threshold(N, M, p["tci_alpha_fd"])
    for e in np.nonzero(rep == FD)[0]:
        rec = tci.reconstruct_fd_to_dg(fd[:, [e]], N)
        if tci.tci_ratio(rec, geo_take(dom.geo_dg, [e]), N, M, p["tci_mode"])[0] <= thr_fd:
            dg[:, e] = rec[:, 0]
            rep[e] = DG
    return dg, fd, rep


def _hybrid_case(N=3):
    dom = _periodic((3, 2, 2), N, eta=1e3, kappa_psi=1.0, kappa_phi=1.0, hybrid=S.HYBRID_ADAPTIVE)
    dg, fd = state_arrays(dom, np.random.default_rng(13), None)
    rep = np.zeros(dom.E, np.int64)
    rep[7] = FD  # one element on FD at the step start
    return dom, S.State(dg, fd, rep)


@pytest.mark.parametrize("rolls", [{1: [4]}, {2: [4]}, {3: [4]}, {1: [0], 2: [5], 3: [10, 11]}],
                         ids=["substep1", "substep2", "substep3", "all_three"])
def test_rollbacks_equal_butcher_form_with_switches(rolls):
    """Sec. III C 1 and reading 21: a step whose DG elements are redone on FD in
    substep 1, 2 or 3 (host-forced flags) equals the Butcher-form step with the
    history moved at that substep (filter on, stiff driver current, q~ != 0)."""
    dom, st = _hybrid_case()
    force = np.zeros((3, dom.E), bool)
    roll = np.zeros(dom.E, np.int64)
    for k, els in rolls.items():
        force[k - 1, els] = True
        roll[els] = k
    dt = dom.dt()
    log = []
    got = S.step(dom, st, dt, log=log, force=force)
    # the indicator itself flags nothing on this smooth data: every rollback is a forced one
    for entry in log:
        if entry[0] == "substep":
            _, k, dg_e, ratio, thr = entry
            assert (ratio <= thr).all()
    dg, fd, rep = _butcher_hybrid(dom, st, dt, roll)
    assert np.array_equal(got.rep, rep)
    el_dg, el_fd = np.nonzero(rep == DG)[0], np.nonzero(rep == FD)[0]
    assert _group_err(got.dg[:, el_dg], dg[:, el_dg]) < 1e-13
    if el_fd.size:
        assert _group_err(got.fd[:, el_fd], fd[:, el_fd]) < 1e-13


def test_butcher_hybrid_without_rollbacks_matches_filtered_step():
    """The Butcher-form reference itself with no rollback: the same as the register
    step of a mixed DG/FD domain with the filter on."""
    dom, st = _hybrid_case()
    dt = dom.dt()
    got = S.step(dom, st, dt)
    dg, fd, rep = _butcher_hybrid(dom, st, dt, np.zeros(dom.E, np.int64))
    assert np.array_equal(got.rep, rep)
    el = np.nonzero(rep == DG)[0]
    assert _group_err(got.dg[:, el], dg[:, el]) < 1e-13


def test_substep1_rollback_equals_step_with_element_on_fd():
    """Sec. III C 1 (a flagged DG substep is discarded, the element projected to FD and
    the substep redone there): with N = 5 (R P = I), flat space and
    no current (eta = 0, q~ = 0: the stiff solve is a pointwise linear map that
    commutes with P), an element flagged by the indicator in substep 1 and redone on
    FD gives the same step as the forced partition with that element on FD from
    P U^n at the start."""
    N = 5
    dom = _periodic((3, 2, 2), N, eta=0.0, kappa_psi=1.0, kappa_phi=1.0, hybrid=S.HYBRID_ADAPTIVE)
    x, y, z = I.points(dom.n_elem, dom.lower, dom.upper, ops.gll(N)[0])
    U = I.fast_wave_sine(x, 0.1)
    U[6] = 0.01 * np.sin(np.pi * (y + z))
    U[7] = 0.01 * np.cos(np.pi * (x - y))
    # a bump of B~x centred in element 4 (x in [-1/3, 1/3], y in [0, 1], z in [-1, 0]):
    # indicator ratio 0.021 there (above 1/81), below 1e-3 elsewhere
    e = 4
    cx, cy, cz = 0.0, 0.5, -0.5
    U[3] += 0.5 * np.exp(-((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) / 0.2 ** 2)
    st = S.State(U, np.zeros((9, dom.E, dom.m, dom.m, dom.m)), np.zeros(dom.E, np.int64))
    dt = dom.dt()
    log = []
    got = S.step(dom, st, dt, log=log)
    flagged = {k: set(dg_e[ratio > thr].tolist()) for (tag, k, dg_e, ratio, thr) in
               [l for l in log if l[0] == "substep"]}
    assert flagged == {1: {e}, 2: set(), 3: set()}
    assert got.rep[e] == FD and (got.rep[np.arange(dom.E) != e] == DG).all()
    fdom = _periodic((3, 2, 2), N, eta=0.0, kappa_psi=1.0, kappa_phi=1.0, hybrid=S.HYBRID_FORCED)
    fd0 = np.zeros((9, dom.E, dom.m, dom.m, dom.m))
    fd0[:, e] = tci.project_dg_to_fd(U[:, [e]], N)[:, 0]
    rep0 = np.zeros(dom.E, np.int64)
    rep0[e] = FD
    ref = S.step(fdom, S.State(U, fd0, rep0), dt)
    others = np.arange(dom.E) != e
    assert _group_err(got.dg[:, others], ref.dg[:, others]) < 1e-13
    assert _group_err(got.fd[:, e], ref.fd[:, e]) < 1e-13


# ------------------------------------------------------------------ switch back


def _mode3_fd_state(dom, amps):
    """All-FD state with B~x = 2 + c_e L_3(xi) in element e (xi the element's reference x),
    sampled at the subcell centres; every other component zero."""
    N = dom.N
    xi = np.broadcast_to(ops.fd_centres(N)[None, None, :], (dom.m,) * 3)
    fd = np.zeros((9, dom.E, dom.m, dom.m, dom.m))
    for e, c in enumerate(amps):
        fd[3, e] = 2.0 + c * ops.legendre(3, xi)
    return fd


def _closed_form_ratio(N, c):
    """Indicator ratio of u = 2 + c L_3(xi) on the GLL nodes (reading 9: u minus its
    modes with every index below M = 3 is the L_3 part)."""
    x, _ = ops.gll(N)
    X = np.broadcast_to(x[None, None, :], (N + 1,) * 3)
    u = 2.0 + c * ops.legendre(3, X)
    return np.sqrt(((c * ops.legendre(3, X)) ** 2).sum() / (u ** 2).sum())


def test_switch_back_uses_alpha_plus_one():
    """Sec. III C 3: an FD element goes back to DG after the step only if the
    reconstructed data pass the indicator with alpha + 1 = 5 (1/243 for N = 5).  A
    ratio between 1/243 and 1/81 stays on FD; below 1/243 it switches, and its DG
    values are R of its subcell values (exact here: the data are of degree 3)."""
    N = 5
    dom = _periodic((2, 1, 1), N, eta=0.0, hybrid=S.HYBRID_ADAPTIVE)
    # amplitudes giving ratios 1/150 (inside the window) and 1/400 (below it)
    from scipy.optimize import brentq
    c_in = brentq(lambda c: _closed_form_ratio(N, c) - 1 / 150, 1e-6, 1.0)
    c_out = brentq(lambda c: _closed_form_ratio(N, c) - 1 / 400, 1e-6, 1.0)
    fd = _mode3_fd_state(dom, [c_in, c_out])
    st = S.State(np.zeros((9, dom.E, dom.n, dom.n, dom.n)), fd, np.ones(dom.E, np.int64))
    log = []
    got = S.step(dom, st, 1e-12, log=log)
    (_, fd_e, ratio, thr_fd), = [l for l in log if l[0] == "fd_check"]
    assert abs(thr_fd - 1 / 243) < 1e-16
    assert np.allclose(ratio, [1 / 150, 1 / 400], rtol=1e-9)
    assert got.rep.tolist() == [FD, DG]
    x, _ = ops.gll(N)
    X = np.broadcast_to(x[None, None, :], (N + 1,) * 3)
    assert np.abs(got.dg[3, 1] - (2.0 + c_out * ops.legendre(3, X))).max() < 1e-12


# ------------------------------------------------------------------ boundary state


def test_no_incoming_poynting_state_flat_hand_cases():
    """Sec. III D: psi~ = phi~ = 0; E~ is kept where the Poynting flux E x B leaves
    through the face and set to zero where it enters.  E = z^, B = y^: E x B = -x^."""
    U = np.zeros((9, 1))
    U[2], U[4], U[6], U[7], U[8] = 1.0, 1.0, 0.3, -0.2, 0.7
    geo = ph.Geometry(None, (1,))
    up = ph.boundary_state(U, geo, 0, +1)    # outward normal +x, flux along -x: inward
    lo = ph.boundary_state(U, geo, 0, -1)    # outward normal -x: outward
    assert np.array_equal(up[0:3, 0], [0.0, 0.0, 0.0])
    assert np.array_equal(lo[0:3, 0], [0.0, 0.0, 1.0])
    for Ub in (up, lo):
        assert Ub[6, 0] == 0.0 and Ub[7, 0] == 0.0
        assert np.array_equal(Ub[3:6, 0], U[3:6, 0]) and Ub[8, 0] == U[8, 0]
    # along y the flux has no normal component: never inward, E~ kept on both faces
    for side in (-1, +1):
        assert np.array_equal(ph.boundary_state(U, geo, 1, side)[0:3, 0], [0.0, 0.0, 1.0])


def test_no_incoming_poynting_state_kerr_schild_point():
    """At the Kerr-Schild (a = 0, M = 1) point x = y = 3/sqrt(2), z = 0 the metric is
    gamma = 1 + 2H l l with H = 1/3, l = (1, 1, 0)/sqrt(2).  The Poynting vector
    eps^{ijk} E_j B_k has the direction of gamma^-1 (E~ x B~) (the cross product of
    two lowered vectors is det(gamma) gamma^-1 (E~ x B~)).  With E~ x B~ = (0.1, 1, 0):
    gamma^-1 = 1 - (2/5) l l gives x component 0.1 - 0.2 (0.1 + 1) = -0.12 < 0, so
    through the +x face the flux enters although E~ x B~ itself points outwards."""
    x = np.array([3.0 / np.sqrt(2.0)])
    y = x.copy()
    z = np.zeros(1)
    geo = ph.Geometry(I.kerr_schild_background(x, y, z, 1.0, 0.0))
    assert np.allclose(geo.g[:, :, 0], np.eye(3) + (2.0 / 3.0) * 0.5 * np.array([[1, 1, 0], [1, 1, 0], [0, 0, 0]]))
    U = np.zeros((9, 1))
    U[0:3, 0] = [0.0, 0.0, 1.0]
    U[3:6, 0] = [1.0, -0.1, 0.0]
    assert np.allclose(np.cross(U[0:3, 0], U[3:6, 0]), [0.1, 1.0, 0.0])
    assert np.array_equal(ph.boundary_state(U, geo, 0, +1)[0:3, 0], [0.0, 0.0, 0.0])
    assert np.array_equal(ph.boundary_state(U, geo, 0, -1)[0:3, 0], [0.0, 0.0, 1.0])
    # along y: 1 - 0.2 (1.1) = 0.78 > 0 leaves through +y
    assert np.array_equal(ph.boundary_state(U, geo, 1, +1)[0:3, 0], [0.0, 0.0, 1.0])
    assert np.array_equal(ph.boundary_state(U, geo, 1, -1)[0:3, 0], [0.0, 0.0, 0.0])


# ------------------------------------------------------------------ drift current


def test_drift_current_flat_hand_values():
    """Eq. (electric current density), drift part: J = q E x B / B^2 (the charge moving
    with the drift velocity).  E~ = (0, 0, 0.5), B~ = (0, 2, 0), q~ = 0.3:
    E x B = (-1, 0, 0), B^2 = 4, J~ = (-0.075, 0, 0); the driver part vanishes
    (E.B = 0, E < B)."""
    U = np.zeros((9, 1))
    U[2], U[4], U[8] = 0.5, 2.0, 0.3
    jd, je = ph.split_current(U, ph.Geometry(None, (1,)), 1e6)
    assert np.allclose(jd[:, 0], [-0.075, 0.0, 0.0], rtol=0, atol=1e-17)
    assert np.array_equal(je[:, 0], [0.0, 0.0, 0.0])


def test_drift_current_kerr_schild_closed_form():
    """Densitized: J~ = alpha sqrt(gamma) q eps^{ijk} E_j B_k / B^2 with q = q~/sqrt(gamma),
    E_j = gamma_jk E~^k / sqrt(gamma), B^2 = B~.B~ / gamma, eps^{ijk} = [ijk]/sqrt(gamma).
    Using [ijk] (gE~)_j (gB~)_k = det(gamma) (gamma^-1 (E~ x B~))^i this is
    J~ = alpha q~ sqrt(gamma) gamma^-1 (E~ x B~) / (gamma_ij B~^i B~^j)."""
    rng = np.random.default_rng(21)
    pts = rng.uniform(2.5, 6.0, (3, 40)) * rng.choice([-1.0, 1.0], (3, 40))
    bg = I.kerr_schild_background(*pts, 1.0, 0.9)
    geo = ph.Geometry(bg)
    U = rng.standard_normal((9, 40))
    U[0:3] *= 0.2  # E < B keeps the driver part small; it is not what is checked
    jd, _ = ph.split_current(U, geo, 0.0)
    for q in range(40):
        g = geo.g[:, :, q]
        Et, Bt = U[0:3, q], U[3:6, q]
        expect = geo.alpha[q] * U[8, q] * np.sqrt(np.linalg.det(g)) * np.linalg.solve(g, np.cross(Et, Bt)) \
            / (Bt @ g @ Bt)
        assert np.allclose(jd[:, q], expect, rtol=1e-12, atol=1e-15)


def test_uniform_charged_state_sources():
    """Flat space, uniform fields (every flux divergence vanishes, Eq. sources):
    dE~/dt = -J~_drift, dpsi~/dt = q~ (alpha q~), dB~/dt = 0, dq~/dt = 0 (eta = 0)."""
    dom = _periodic((2, 1, 1), 3, eta=0.0)
    U = np.zeros((9, dom.E, dom.n, dom.n, dom.n))
    U[2], U[4], U[8] = 0.5, 2.0, 0.3
    L, _ = R.rhs(dom, U, np.zeros((9, dom.E, dom.m, dom.m, dom.m)), np.zeros(dom.E, np.int64), parts=3)
    assert np.allclose(L[0], 0.075, atol=1e-14) and np.allclose(L[1:3], 0.0, atol=1e-14)
    assert np.allclose(L[3:6], 0.0, atol=1e-14) and np.allclose(L[7:9], 0.0, atol=1e-14)
    assert np.allclose(L[6], 0.3, atol=1e-14)


# ------------------------------------------------------------------ curved indicator


def test_indicator_uses_the_metric_norm_of_b():
    """Sec. III C 3 on u = |B~| = sqrt(gamma_ij B~^i B~^j) at Kerr-Schild nodes, against a
    brute-force evaluation: the norm node by node, then the modes of u from a least-
    squares fit in the tensor Legendre basis (exact: n^3 nodes, n^3 modes), removing
    those with every index below M (reading 9)."""
    N = 5
    M = ops.tci_M(N)
    n = N + 1
    dom_args = ((1, 1, 1), (3.0, 2.0, -1.0), (6.0, 5.0, 2.0))
    x, y, z = I.points(*dom_args, ops.gll(N)[0])
    bg = I.kerr_schild_background(x, y, z, 1.0, 0.9)
    dom = Domain(*dom_args, N, (1,) * 6, bg=bg)
    U = np.zeros((9, 1, n, n, n))
    U[3] = 1.0 + 0.3 * np.sin(x)
    U[4] = -0.7 + 0.2 * np.cos(y * z)
    U[5] = 0.4 * x * y / 10.0
    got = tci.tci_ratio(U, dom.geo_dg, N, M)[0]
    u = np.zeros((n, n, n))
    for k in range(n):
        for j in range(n):
            for i in range(n):
                g = dom.geo_dg.g[:, :, 0, k, j, i]
                b = U[3:6, 0, k, j, i]
                u[k, j, i] = np.sqrt(b @ g @ b)
    xi = ops.gll(N)[0]
    Zr, Yr, Xr = np.meshgrid(xi, xi, xi, indexing="ij")
    V = npleg.legvander3d(Xr.ravel(), Yr.ravel(), Zr.ravel(), [N, N, N])  # columns: (i_x, i_y, i_z) index order
    coef = np.linalg.lstsq(V, u.ravel(), rcond=None)[0].reshape(n, n, n)  # [px][py][pz]
    low = np.zeros_like(coef)
    low[:M, :M, :M] = coef[:M, :M, :M]
    uh = u.ravel() - V @ low.ravel()
    brute = np.sqrt((uh ** 2).sum() / (u ** 2).sum())
    assert abs(got - brute) < 1e-12 * brute
    # the flat norm would give a different value: the metric matters here
    flat = np.sqrt((U[3:6, 0] ** 2).sum(axis=0))
    assert abs(np.sqrt(((flat.ravel() - V @ _low(V, flat, n, M)) ** 2).sum() / (flat ** 2).sum()) - brute) > 1e-3 * brute


def _low(V, u, n, M):
    coef = np.linalg.lstsq(V, u.ravel(), rcond=None)[0].reshape(n, n, n)
    low = np.zeros_like(coef)
    low[:M, :M, :M] = coef[:M, :M, :M]
    return low.ravel()


# ------------------------------------------------------------------ filter placement


def test_filter_after_the_solve_is_unstable_on_the_noisy_wave():
    """Reading 13 (Sec. III A's filter, applied at every substep, with Sec. III B's stiff
    solve): filtering the solved stage values changes E parallel to B after the
    relaxation, and the next stiff source multiplies that change by eta dt ~ 10^3.
    On the noisy wave (eta = 10^6) that placement grows the field tenfold per step
    within a few steps; filtering the explicit update before the solve keeps it
    bounded."""
    w = I.workload("wave")
    N = w["degree"]
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], N)
    u0 = I.initial_data(w, xf, yf, zf)
    peak = {}
    for post in (0, 1):
        dom = Domain(w["n_elem"], w["lower"], w["upper"], N, w["bc"],
                     params=dict(eta=w["eta"], cfl=w["cfl"], hybrid=S.HYBRID_DG_ONLY, filter_after_solve=post))
        st = S.initial_state(dom, u0)
        dt = dom.dt()
        for _ in range(5):
            st = S.step(dom, st, dt)
        peak[post] = np.abs(st.dg[0:3]).max()
    assert peak[0] < 0.11
    assert peak[1] > 1e3
