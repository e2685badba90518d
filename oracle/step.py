"""IMEX-SSP3(4,3,3) step with the DG-FD hybrid control (Sec. III B, Sec. III C 1).

TEST INFRASTRUCTURE ONLY (see oracle/operators.py).

Time stepper: IMEX-SSP3(4,3,3) of Pareschi & Russo (2005), cited in
Sec. III B.  Its tableaux (not printed in the paper; taken from that
reference) are, with a = 0.24169426078821, b = 0.06042356519705,
e = 0.12915286960590:

    explicit  c=(0, 0, 1, 1/2)        implicit
    0   0   0   0                     a    0      0            0
    0   0   0   0                     -a   a      0            0
    0   1   0   0                     0    1-a    a            0
    0  1/4 1/4  0                     b    e   1/2-b-e-a       a
    weights (0, 1/6, 1/6, 2/3) for both.

Stage i: Y_i = U^n + dt sum_j<i (Aex_ij L(U_j) + Aim_ij S(U_j)), then
U_i = Y_i + dt Aim_ii S(U_i) solved pointwise.  L is the explicit operator
(fluxes + non-stiff sources), S the stiff sources.  L is needed at U_2,
U_3, U_4: the three "substeps" of the step.

Hybrid control (Sec. III C 1): in each DG substep the explicit update is
filtered (Eq. (exponential filter)) -- before the pointwise implicit solve in
substeps 1 and 2, so that the stage values stay exact solutions of the stiff
relaxation -- and the resulting candidate (U_3, U_4, U^{n+1}) is checked by the
indicator with alpha; a troubled element discards its candidate, moves its
stepper history to the FD grid with P and redoes the substep there, with its
neighbours' data as they were at the start of the substep.  After the full
step every FD element is reconstructed with R and checked with alpha + 1; if
it passes it continues on DG.

History moved by a switch: U^n, the substep's input stage value (U_3 or
U_4), and the explicit increments L(U_j) and stiff increment S(U_3)
evaluated in earlier substeps.  U_1, U_2, S(U_1) and S(U_2) are functions of
U^n alone and are re-derived from the (projected) U^n wherever needed.
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from . import physics as ph
from .domain import DG, FD, geo_take
from .rhs import dg_rhs, fd_rhs, with_current
from .tci import project_dg_to_fd, reconstruct_fd_to_dg, tci_ratio, tci_threshold

IMEX_A = 0.24169426078821
IMEX_B = 0.06042356519705
IMEX_E = 0.12915286960590
AEX = np.array([[0, 0, 0, 0], [0, 0, 0, 0], [0, 1, 0, 0], [0, 0.25, 0.25, 0]], dtype=np.float64)
AIM = np.array([[IMEX_A, 0, 0, 0], [-IMEX_A, IMEX_A, 0, 0], [0, 1 - IMEX_A, IMEX_A, 0],
                [IMEX_B, IMEX_E, 0.5 - IMEX_B - IMEX_E - IMEX_A, IMEX_A]], dtype=np.float64)
BW = np.array([0.0, 1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0])

HYBRID_DG_ONLY = 0
HYBRID_ADAPTIVE = 1
HYBRID_FORCED = 2


def imex_step_generic(y, dt, L, S, solve):
    """One IMEX-SSP3(4,3,3) step of y' = L(y) + S(y) in Butcher form (for ODE tests)."""
    Ls, Ss = [None] * 4, [None] * 4
    for i in range(4):
        Y = y.copy() if hasattr(y, "copy") else y
        for j in range(i):
            if AEX[i, j] != 0.0:
                Y = Y + dt * AEX[i, j] * Ls[j]
            if AIM[i, j] != 0.0:
                Y = Y + dt * AIM[i, j] * Ss[j]
        U = solve(Y, dt * AIM[i, i])
        Ss[i] = S(U)
        Ls[i] = L(U)
    out = y
    for i in range(4):
        out = out + dt * BW[i] * (Ls[i] + Ss[i])
    return out


class State:
    """Domain state: DG nodal data, FD subcell data, representation per element."""

    def __init__(self, dg, fd, rep):
        self.dg = np.array(dg, np.float64)
        self.fd = np.array(fd, np.float64)
        self.rep = np.array(rep, np.int64)

    def copy(self):
        return State(self.dg, self.fd, self.rep)


def _pair_zeros(dom):
    return [np.zeros((9, dom.E, dom.n, dom.n, dom.n)), np.zeros((9, dom.E, dom.m, dom.m, dom.m))]


def _geos(dom):
    return [dom.geo_dg, dom.geo_fd]


def _solve(dom, Y, geo, h):
    p = dom.params
    return ph.implicit_solve(Y, geo, p["eta"], p["kappa_psi"], p["kappa_phi"], h)


def _stiff(dom, U, geo):
    p = dom.params
    return ph.source_stiff(U, geo, p["eta"], p["kappa_psi"], p["kappa_phi"])


def derived_stages(dom, Un, geo, dt):
    """U_1, U_2, S(U_1), S(U_2): the implicit pre-stages, functions of U^n only."""
    U1 = _solve(dom, Un, geo, dt * AIM[0, 0])
    S1 = _stiff(dom, U1, geo)
    Y2 = Un + dt * AIM[1, 0] * S1
    U2 = _solve(dom, Y2, geo, dt * AIM[1, 1])
    S2 = _stiff(dom, U2, geo)
    return U1, U2, S1, S2


def _candidate(dom, k, H, X, Lk, geo, dt, filt):
    """Candidate output of substep k (1, 2, 3) for one representation (arrays over points).

    ``filt`` is applied to the explicit update of the substep: before the
    pointwise implicit solve in substeps 1 and 2, to the final combination in
    substep 3 (which has no solve).  The parameter ``filter_after_solve`` = 1
    moves it behind the solve in substeps 1 and 2 (the other reading of "filter
    after every substep"; kept only to show that it is unstable with a stiff
    driver current).
    """
    Un = H["Un"]
    _, _, S1, S2 = derived_stages(dom, Un, geo, dt)
    post = bool(dom.params.get("filter_after_solve", 0))

    def solve_filtered(Y, h):
        return filt(_solve(dom, Y, geo, h)) if post else _solve(dom, filt(Y), geo, h)

    if k == 1:
        Y = Un + dt * AEX[2, 1] * Lk + dt * (AIM[2, 0] * S1 + AIM[2, 1] * S2)
        return solve_filtered(Y, dt * AIM[2, 2]), {"L1": Lk}
    if k == 2:
        S3 = _stiff(dom, X, geo)
        Y = (Un + dt * (AEX[3, 1] * H["L1"] + AEX[3, 2] * Lk)
             + dt * (AIM[3, 0] * S1 + AIM[3, 1] * S2 + AIM[3, 2] * S3))
        return solve_filtered(Y, dt * AIM[3, 3]), {"L2": Lk, "S3": S3}
    S4 = _stiff(dom, X, geo)
    out = (Un + dt * (BW[1] * H["L1"] + BW[2] * H["L2"] + BW[3] * Lk)
           + dt * (BW[1] * S2 + BW[2] * H["S3"] + BW[3] * S4))
    return filt(out), {}


def _filter_fn(dom):
    p = dom.params
    if not p["filter_on"]:
        return lambda u: u
    Fm = ops.filter_matrix(dom.N, p["filter_a"], p["filter_b"])
    return lambda u: ops.apply_3d(Fm, u)


def _identity(u):
    return u


def _rhs_pair(dom):
    """The DG and FD right-hand sides of the domain's grid: the Cartesian box's, or
    those a grid of curved elements provides (attribute ``rhs_pair``)."""
    return getattr(dom, "rhs_pair", (dg_rhs, fd_rhs))


def _post(dom, C, geo, el, fd):
    """What follows the update of every substep: the optional algebraic clamp, then
    the rotating conductor's E, psi~, q~ inside its sphere (Sec. IV C: enforced at
    every substep; here on the three substep results U_3, U_4, U^{n+1}, before the
    indicator looks at them -- it sees only B~, which neither changes)."""
    p = dom.params
    if p["ff_clamp"]:
        C = ph.constraint_clamp(C, geo, p["ff_margin"])
    if dom.conductor is not None:
        c = dom.conductor
        x, y, z = dom.point_coords(el, fd)
        C = ph.corotating_conductor(C, x, y, z, c["centre"], c["radius"], c["omega"],
                                    geo if dom.bg is not None else None)
    return C


def _post_dg(dom, C, geo, el):
    return _post(dom, C, geo, el, False)


def _post_fd(dom, C, geo, el):
    return _post(dom, C, geo, el, True)


def _M(dom):
    p = dom.params
    return p["tci_M"] if p["tci_M"] else ops.tci_M(dom.N)


def _replay(decided, ratio, thr, theirs, tol, events, where, elems):
    """Parity harness (not part of the method): where an indicator ratio lies within
    ``tol`` (relative) of its threshold, rounding alone can decide the comparison, so
    the other implementation's decision ``theirs`` is taken instead of ``decided``;
    every such event is appended to ``events`` as (where, element, ratio, threshold,
    own decision, taken decision)."""
    near = np.abs(ratio / thr - 1.0) <= tol
    out = decided.copy()
    out[near] = theirs[near]
    if events is not None:
        for i in np.nonzero(near)[0]:
            events.append((where, int(elems[i]), float(ratio[i]), float(thr), bool(decided[i]), bool(out[i])))
    return out


def step(dom, st, dt, log=None, force=None, replay=None, replay_tol=1e-10, replay_events=None):
    """Advance State ``st`` by one step of size dt; returns a new State.

    ``force`` (test instrument, nullable): boolean array (3, E); in the adaptive
    mode an element on DG with force[k - 1] set is treated as troubled in
    substep k whatever its indicator ratio (a host-forced flag, so that rollbacks
    can be made to happen in any substep).

    ``replay`` (parity harness, nullable): the other implementation's
    representation log of the same step, integer array (5, E): before the step,
    after substeps 1, 2, 3 and after the step.  A decision whose ratio lies within
    ``replay_tol`` of its threshold follows that log (an element flagged in substep
    k is FD in row k; an element switched back at the end is DG in row 4) and is
    recorded in ``replay_events``."""
    p = dom.params
    act = dom.active
    N, M = dom.N, _M(dom)
    thr = tci_threshold(N, M, p["tci_alpha"])
    thr_fd = tci_threshold(N, M, p["tci_alpha_fd"])
    rep = st.rep.copy()
    # history per representation: index 0 = DG arrays, 1 = FD arrays
    H = {"Un": [st.dg.copy(), st.fd.copy()]}
    for k in (1, 2, 3):
        rep0 = rep.copy()
        dg_e = np.nonzero(act & (rep0 == DG))[0]
        fd_e = np.nonzero(act & (rep0 == FD))[0]
        # substep input per representation
        X = _pair_zeros(dom)
        for r, el in ((0, dg_e), (1, fd_e)):
            if el.size == 0:
                continue
            geo = geo_take(_geos(dom)[r], el)
            if k == 1:
                X[r][:, el] = derived_stages(dom, H["Un"][r][:, el], geo, dt)[1]
            else:
                X[r][:, el] = H["U%d" % (k + 1)][r][:, el]
        W = [with_current(dom, X[0], dom.geo_dg), with_current(dom, X[1], dom.geo_fd)]
        newH = {key: [v[0].copy(), v[1].copy()] for key, v in H.items()}
        cand = _pair_zeros(dom)
        for r, el in ((0, dg_e), (1, fd_e)):
            if el.size == 0:
                continue
            geo = geo_take(_geos(dom)[r], el)
            if r == 0:
                Lk = _rhs_pair(dom)[0](dom, el, W[0], W[1], rep0, parts=1)
            else:
                Lk = _rhs_pair(dom)[1](dom, el, W[1][:, el], W[0], W[1], rep0, parts=1)
            Hs = {key: v[r][:, el] for key, v in H.items()}
            C, upd = _candidate(dom, k, Hs, X[r][:, el], Lk, geo, dt, _filter_fn(dom) if r == 0 else _identity)
            C = _post_dg(dom, C, geo, el) if r == 0 else _post_fd(dom, C, geo, el)
            cand[r][:, el] = C
            for key, v in upd.items():
                newH.setdefault(key, _pair_zeros(dom))
                newH[key][r][:, el] = v
        # indicator on DG candidates
        bad = np.zeros(0, np.int64)
        if p["hybrid"] == HYBRID_ADAPTIVE and dg_e.size:
            ratio = tci_ratio(cand[0][:, dg_e], geo_take(dom.geo_dg, dg_e), N, M, p["tci_mode"])
            hit = ratio > thr
            if replay is not None:
                hit = _replay(hit, ratio, thr, np.asarray(replay)[k][dg_e] == FD, replay_tol, replay_events,
                              ("substep", k), dg_e)
            if force is not None:
                hit = hit | np.asarray(force, bool)[k - 1][dg_e]
            bad = dg_e[hit]
            if log is not None:
                log.append(("substep", k, dg_e.copy(), ratio.copy(), thr))
        if bad.size:
            geo = geo_take(dom.geo_fd, bad)
            # move the history of the troubled elements to the FD grid
            for key, v in H.items():
                v_fd = project_dg_to_fd(v[0][:, bad], N)
                newH[key][1][:, bad] = v_fd
            Hs = {key: newH[key][1][:, bad] for key in H}
            if k == 1:
                Xb = derived_stages(dom, Hs["Un"], geo, dt)[1]
            else:
                Xb = Hs["U%d" % (k + 1)]
            Lk = _rhs_pair(dom)[1](dom, bad, with_current(dom, Xb, geo), W[0], W[1], rep0, parts=1)
            C, upd = _candidate(dom, k, Hs, Xb, Lk, geo, dt, _identity)
            cand[1][:, bad] = _post_fd(dom, C, geo, bad)
            for key, v in upd.items():
                newH.setdefault(key, _pair_zeros(dom))
                newH[key][1][:, bad] = v
            rep[bad] = FD
        H = newH
        if k < 3:
            H["U%d" % (k + 2)] = cand
        else:
            H["Un"] = cand
    out = State(H["Un"][0], H["Un"][1], rep)
    # end of step: FD elements that look smooth on the DG grid go back to DG
    if p["hybrid"] == HYBRID_ADAPTIVE:
        fd_e = np.nonzero(act & (rep == FD))[0]
        if fd_e.size:
            rec = reconstruct_fd_to_dg(out.fd[:, fd_e], N)
            ratio = tci_ratio(rec, geo_take(dom.geo_dg, fd_e), N, M, p["tci_mode"])
            ok = ratio <= thr_fd
            if replay is not None:
                ok = ~_replay(~ok, ratio, thr_fd, np.asarray(replay)[4][fd_e] == FD, replay_tol, replay_events,
                              ("fd_check",), fd_e)
            if log is not None:
                log.append(("fd_check", fd_e.copy(), ratio.copy(), thr_fd))
            back = fd_e[ok]
            out.dg[:, back] = rec[:, ok]
            out.rep[back] = DG
    return out


def initial_state(dom, u_fd, forced=None, replay=None, replay_tol=1e-10, replay_events=None):
    """Sec. III C 1: data given on the FD grid is reconstructed to DG; the indicator
    (alpha + 1) decides which elements start on DG.  ``forced`` (bool, E) pins
    elements to FD in the forced-partition mode.  ``replay`` (nullable, integer E):
    the other implementation's start-up representation, taken for ratios within
    ``replay_tol`` of the threshold (see step)."""
    p = dom.params
    N, M = dom.N, _M(dom)
    dg = reconstruct_fd_to_dg(u_fd, N)
    rep = np.full(dom.E, DG, np.int64)
    if p["hybrid"] == HYBRID_ADAPTIVE:
        ratio = tci_ratio(dg, dom.geo_dg, N, M, p["tci_mode"])
        thr_fd = tci_threshold(N, M, p["tci_alpha_fd"])
        hit = ratio > thr_fd
        if replay is not None:
            hit = _replay(hit, ratio, thr_fd, np.asarray(replay) == FD, replay_tol, replay_events, ("start",),
                          np.arange(dom.E))
        rep[hit] = FD
    elif p["hybrid"] == HYBRID_FORCED and forced is not None:
        rep[np.asarray(forced, bool)] = FD
    rep[~dom.active] = DG
    fd = np.where((rep == FD)[None, :, None, None, None], u_fd, 0.0)
    dg = np.where((rep == DG)[None, :, None, None, None], dg, 0.0)
    dg[:, ~dom.active] = 0.0
    return State(dg, fd, rep)
