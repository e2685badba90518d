"""The decision log of a library step (grffe_step_logged) and the oracle's replay of
it: the log's rows must be the oracle's own decisions where those are clear, and where
an indicator ratio lies within 1e-10 of its threshold the oracle takes the library's
decision (recorded as an event), so the two runs stay comparable element by element.
Cases: start-up with a ratio placed at the threshold (alpha + 1), and steps of the
sheet with rollbacks in substep 1 and switches back."""
import sys

import numpy as np
import pytest

from oracle import operators as ops
from oracle import step as OS
from oracle.domain import DG, FD
from oracle.domain import Domain as ODomain
from paper_2404_01531_amd import inputs as I

from helpers import from_dev, group_err, oracle_params, to_dev

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _own_log(st, log, rep_after):
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


def _compare(ldom, st, label):
    gdg, gfd, grep = ldom.get_state()
    assert np.array_equal(grep.cpu().numpy(), st.rep), f"{label}: representation differs"
    for r, G, R in ((DG, from_dev(gdg, st.dg.shape), st.dg), (FD, from_dev(gfd, st.fd.shape), st.fd)):
        el = np.nonzero(st.rep == r)[0]
        if el.size:
            e = group_err(G[:, el], R[:, el])
            _say(f"  {label} rep {r}: group err {np.array2string(e, precision=2)}")
            assert np.all(e <= 1e-12), (label, r, e.tolist())


def test_logged_steps_of_the_sheet_match_the_oracle_decisions():
    torch = _torch()
    from paper_2404_01531_amd import grffe
    w = I.workload("sheet", n_elem=(4, 2, 2), degree=3)
    p = grffe.default_params(eta=300.0, cfl=0.25)
    odom = ODomain(w["n_elem"], w["lower"], w["upper"], 3, w["bc"], params=oracle_params(p))
    ldom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], 3, w["bc"], params=p)
    rng = np.random.default_rng(78)
    x, y, z = I.points(w["n_elem"], w["lower"], w["upper"], ops.gll(3)[0])
    dg = I.initial_data(w, x, y, z) + 1e-4 * rng.standard_normal((9,) + x.shape)
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], 3)
    fd = I.initial_data(w, xf, yf, zf) + 1e-4 * rng.standard_normal((9,) + xf.shape)
    rep = ((np.arange(odom.E) % w["n_elem"][0]) == 0).astype(np.int64)
    dg[:, rep == 1] = 0.0
    fd[:, rep == 0] = 0.0
    st = OS.State(dg, fd, rep)
    ldom.set_state(to_dev(dg), to_dev(fd), torch.from_numpy(rep.astype(np.int32)).cuda())
    dt = ldom.dt()
    changes = 0
    for k in range(2):
        glog = ldom.step_logged(dt).cpu().numpy()
        olog, ev = [], []
        nst = OS.step(odom, st, dt, log=olog, replay=glog, replay_events=ev)
        own = _own_log(st, olog, nst.rep)
        changes += int((glog[1:] != glog[:-1]).sum())
        assert np.array_equal(glog, own), f"step {k + 1}: the library's decision log differs from the oracle's"
        assert ev == [], f"step {k + 1}: a decision lies within 1e-10 of its threshold: {ev}"
        st = nst
        _compare(ldom, st, f"logged step {k + 1}")
    assert changes > 0, "the steps must roll elements back or switch them"


def test_start_up_at_the_threshold_is_replayed():
    """Element 0's start-up ratio is placed within 1e-13 of the threshold 1/243:
    whatever the library decides, the oracle takes it (one recorded event), and two
    logged steps stay in parity.  (Measured: the oracle's ratio fell 1.5e-14 below
    the threshold and the library's above it; the library's FD start was taken.)"""
    torch = _torch()
    from scipy.optimize import brentq

    from paper_2404_01531_amd import grffe
    N = 5
    p = grffe.default_params(eta=0.0, cfl=0.25)
    odom = ODomain((2, 1, 1), (-1.0,) * 3, (1.0,) * 3, N, (0,) * 6, params=oracle_params(p))
    ldom = grffe.Domain((2, 1, 1), (-1.0,) * 3, (1.0,) * 3, N, (0,) * 6, params=p)
    thr = OS.tci_threshold(N, 3, odom.params["tci_alpha_fd"])
    xg, _ = ops.gll(N)
    X = np.broadcast_to(xg[None, None, :], (N + 1,) * 3)

    def ratio(c):
        u = 2.0 + c * ops.legendre(3, X)
        return np.sqrt(((c * ops.legendre(3, X)) ** 2).sum() / (u ** 2).sum())

    c = brentq(lambda c: ratio(c) / thr - 1.0, 1e-6, 1.0, xtol=1e-18, rtol=1e-15)
    xi = np.broadcast_to(ops.fd_centres(N)[None, None, :], (odom.m,) * 3)
    fd = np.zeros((9, odom.E, odom.m, odom.m, odom.m))
    fd[3, 0] = 2.0 + c * ops.legendre(3, xi)
    fd[3, 1] = 2.0
    ldom.init_from_fd(to_dev(fd))
    _, _, grep = ldom.get_state()
    grep = grep.cpu().numpy()
    ev = []
    st = OS.initial_state(odom, fd, replay=grep, replay_events=ev)
    _say(f"start-up: library representation {grep.tolist()}, replay events {ev}")
    assert np.array_equal(st.rep, grep)
    assert [x for x in ev if x[1] == 0 and abs(x[2] / x[3] - 1.0) < 1e-10]
    _compare(ldom, st, "start-up")
    dt = ldom.dt()
    for k in range(2):
        glog = ldom.step_logged(dt).cpu().numpy()
        ev = []
        st = OS.step(odom, st, dt, replay=glog, replay_events=ev)
        if ev:
            _say(f"  step {k + 1}: replayed {ev}")
        _compare(ldom, st, f"step {k + 1} after a replayed start-up")


def test_step_logged_errors():
    torch = _torch()
    from paper_2404_01531_amd import grffe
    w = I.workload("sheet", n_elem=(2, 1, 1), degree=3)
    d = grffe.Domain(w["n_elem"], w["lower"], w["upper"], 3, w["bc"], params=grffe.default_params())
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], 3)
    d.init_from_fd(to_dev(I.initial_data(w, xf, yf, zf)))
    log = d.step_logged()
    assert tuple(log.shape) == (5, d.E) and log.dtype == torch.int32
    from paper_2404_01531_amd.grffe import lib
    assert lib().grffe_step_logged(d._h, 0.0, None, None) != 0
