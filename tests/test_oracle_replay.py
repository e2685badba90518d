"""The parity harness's decision replay in the oracle (CPU): where an indicator ratio
lies within a tolerance of its threshold, the oracle takes the other implementation's
decision from its representation log and records the event.  Checked on steps of
the sheet with rollbacks and switches back, and at start-up with a ratio placed at
the threshold."""
import numpy as np

from oracle import operators as ops
from oracle import step as S
from oracle.domain import DG, FD, Domain
from paper_2404_01531_amd import inputs as I


def _sheet():
    """The sheet on 4 x 2 x 2 P3 elements: the elements at the sheet start on DG (and
    are rolled back in substep 1), those of the first column on FD (and switch back)."""
    w = I.workload("sheet", n_elem=(4, 2, 2), degree=3)
    dom = Domain(w["n_elem"], w["lower"], w["upper"], 3, w["bc"], params=dict(eta=300.0, cfl=0.25))
    rng = np.random.default_rng(78)
    x, y, z = I.points(w["n_elem"], w["lower"], w["upper"], ops.gll(3)[0])
    dg = I.initial_data(w, x, y, z) + 1e-4 * rng.standard_normal((9,) + x.shape)
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], 3)
    fd = I.initial_data(w, xf, yf, zf) + 1e-4 * rng.standard_normal((9,) + xf.shape)
    rep = ((np.arange(dom.E) % w["n_elem"][0]) == 0).astype(np.int64)
    dg[:, rep == 1] = 0.0
    fd[:, rep == 0] = 0.0
    return dom, S.State(dg, fd, rep)


def _own_log(st, log, rep_after):
    """The representation log (5, E) of a step from its decision log."""
    rows = [st.rep.copy()]
    for k in (1, 2, 3):
        r = rows[-1].copy()
        for entry in log:
            if entry[0] == "substep" and entry[1] == k:
                _, _, el, ratio, thr = entry
                r[el[ratio > thr]] = FD
        rows.append(r)
    rows.append(rep_after.copy())
    return np.array(rows)


def test_replay_of_own_decisions_changes_nothing():
    dom, st = _sheet()
    dt = dom.dt()
    log = []
    ref = S.step(dom, st, dt, log=log)
    own = _own_log(st, log, ref.rep)
    assert (own[1] != own[0]).any() and (own[4] != own[3]).any(), "the step needs rollbacks and switches back"
    ev = []
    got = S.step(dom, st, dt, replay=own, replay_tol=np.inf, replay_events=ev)
    assert np.array_equal(got.rep, ref.rep) and np.array_equal(got.dg, ref.dg) and np.array_equal(got.fd, ref.fd)
    assert len(ev) > 0 and all(e[4] == e[5] for e in ev)


def test_replayed_decision_is_taken_and_logged():
    """A log that adds a rollback in substep 2 is followed when its ratio counts as
    near (tolerance infinite here): the result is the forced step with that element
    flagged in substep 2; with the 1e-10 tolerance the same log is ignored there."""
    dom, st = _sheet()
    dt = dom.dt()
    log = []
    ref = S.step(dom, st, dt, log=log)
    other = _own_log(st, log, ref.rep)
    e = int(np.nonzero(other[1] == DG)[0][0])
    other[2:4, e] = FD
    other[4, e] = ref.rep[e]
    ev = []
    got = S.step(dom, st, dt, replay=other, replay_tol=np.inf, replay_events=ev)
    force = np.zeros((3, dom.E), bool)
    force[1, e] = True
    forced = S.step(dom, st, dt, force=force)
    assert np.array_equal(got.rep, forced.rep)
    assert np.array_equal(got.dg, forced.dg) and np.array_equal(got.fd, forced.fd)
    assert [x for x in ev if x[0] == ("substep", 2) and x[1] == e and x[4] != x[5]]
    ev = []
    plain = S.step(dom, st, dt, replay=other, replay_events=ev)
    assert np.array_equal(plain.rep, ref.rep) and np.array_equal(plain.dg, ref.dg)
    assert ev == []


def test_replay_at_start_up_near_the_threshold():
    """A start-up ratio placed within 1e-13 of the threshold (alpha + 1): the other
    side's decision is taken in either direction and the event is recorded."""
    from scipy.optimize import brentq
    N = 5
    dom = Domain((2, 1, 1), (-1.0,) * 3, (1.0,) * 3, N, (0,) * 6, params=dict(eta=0.0, hybrid=S.HYBRID_ADAPTIVE))
    thr = S.tci_threshold(N, 3, dom.params["tci_alpha_fd"])
    x, _ = ops.gll(N)
    X = np.broadcast_to(x[None, None, :], (N + 1,) * 3)

    def ratio(c):
        u = 2.0 + c * ops.legendre(3, X)
        return np.sqrt(((c * ops.legendre(3, X)) ** 2).sum() / (u ** 2).sum())

    c = brentq(lambda c: ratio(c) / thr - 1.0, 1e-6, 1.0, xtol=1e-18, rtol=1e-15)
    xi = np.broadcast_to(ops.fd_centres(N)[None, None, :], (dom.m,) * 3)
    fd = np.zeros((9, dom.E, dom.m, dom.m, dom.m))
    fd[3, 0] = 2.0 + c * ops.legendre(3, xi)
    fd[3, 1] = 2.0
    for theirs in (DG, FD):
        ev = []
        st = S.initial_state(dom, fd, replay=np.array([theirs, DG]), replay_events=ev)
        assert st.rep[0] == theirs and st.rep[1] == DG
        assert len(ev) == 1 and ev[0][0] == ("start",) and ev[0][1] == 0 and abs(ev[0][2] / thr - 1.0) < 1e-10
