"""Adjoint of the right-hand side and of the IMEX step (all elements on DG).

Each adjoint is checked through the dot-product identity
    <ubar, delta> = <lambda, J delta>
where J delta is the directional derivative of the FP64 oracle's right-hand side
(or step), taken by central differences on the CPU.  The finite difference has
a truncation error O(eps^2) and a rounding error O(1e-16/eps); with eps = 1e-6
relative to the state the two sides agree to ~1e-7, and the bound is 1e-6.  The
same identity is checked against central differences of the library's own
forward path, and the checkpointed torch.autograd gradient of a multi-step
objective against finite differences of the objective.
"""
import sys

import numpy as np
import pytest

from oracle import rhs as OR
from oracle import step as OS
from oracle.domain import DG, FD
from paper_2404_01531_amd import inputs as I

from helpers import curved_state, make_pair, node_coords, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-6


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wave_state(odom, w, rng):
    x, y, z = node_coords(w)
    U = I.fast_wave_sine(x, 0.1)
    U[0] += 0.05 * np.sin(1.3 * y + 0.7 * z)
    U[8] += 0.02 * np.cos(0.9 * x + 1.1 * z)
    U[6] += 0.01 * np.sin(x + y)
    U[7] += 0.01 * np.cos(y - z)
    U += 1e-3 * rng.standard_normal(U.shape)
    return U


def _rel(a, b):
    return abs(a - b) / max(abs(a), abs(b), 1e-300)


def _rhs_case(w, params, u, label, rng):
    torch = _torch()
    odom, ldom, _ = make_pair(w, params)
    E, n3 = odom.E, odom.n ** 3
    act = odom.active
    u = u.copy()
    u[:, ~act] = 0.0
    rep = np.zeros(E, np.int64)
    fd0 = np.zeros((9, E, odom.m, odom.m, odom.m))
    lam = rng.standard_normal(u.shape)
    lam[:, ~act] = 0.0
    delta = rng.standard_normal(u.shape) * np.abs(u).max(axis=(1, 2, 3, 4), keepdims=True)
    delta[:, ~act] = 0.0
    eps = 1e-6
    rep_t = torch.zeros(E, dtype=torch.int32, device="cuda")
    for parts in (1, 2, 3):
        ub = ldom.rhs_adjoint(to_dev(u), rep_t, to_dev(lam), parts=parts).cpu().numpy().reshape(u.shape)
        lhs = float((ub * delta).sum())
        Lp, _ = OR.rhs(odom, u + eps * delta, fd0, rep, parts=parts)
        Lm, _ = OR.rhs(odom, u - eps * delta, fd0, rep, parts=parts)
        rhs_o = float((lam * (Lp - Lm)).sum() / (2 * eps))
        gp, _ = ldom.rhs(to_dev(u + eps * delta), to_dev(fd0), rep_t, parts=parts)
        gm, _ = ldom.rhs(to_dev(u - eps * delta), to_dev(fd0), rep_t, parts=parts)
        rhs_g = float((lam * (gp - gm).cpu().numpy().reshape(u.shape)).sum() / (2 * eps))
        _say(f"rhs adjoint {label} parts={parts}: <ubar,d> {lhs:.12e}  oracle FD {rhs_o:.12e} "
             f"(rel {_rel(lhs, rhs_o):.1e})  library FD {rhs_g:.12e} (rel {_rel(lhs, rhs_g):.1e})")
        assert _rel(lhs, rhs_o) <= TOL, (label, parts)
        assert _rel(lhs, rhs_g) <= TOL, (label, parts)


def test_rhs_adjoint_flat_periodic():
    _torch()
    w = I.workload("wave")
    rng = np.random.default_rng(41)
    odom, _, _ = make_pair(w)
    _rhs_case(w, dict(eta=w["eta"]), _wave_state(odom, w, rng), "wave 2^3 P5", rng)


@pytest.mark.parametrize("N", [3, 6])
def test_rhs_adjoint_ragged_boundaries(N):
    _torch()
    w = dict(n_elem=(3, 2, 1), lower=(-1.0, -0.5, -0.25), upper=(1.0, 0.75, 0.5), degree=N, bc=(1, 1, 0, 0, 1, 1),
             curved=False)
    rng = np.random.default_rng(42 + N)
    odom, _, _ = make_pair(w)
    _rhs_case(w, dict(eta=50.0), _wave_state(odom, w, rng), f"ragged P{N} outflow faces", rng)


def test_rhs_adjoint_kerr_schild_excision():
    _torch()
    w = I.workload("kerr_schild", n_elem=(4, 4, 4), lower=(-16.0,) * 3, upper=(16.0,) * 3)
    rng = np.random.default_rng(44)
    odom, _, _ = make_pair(w)
    dg, _ = curved_state(odom, w, rng)
    _rhs_case(w, dict(eta=w["eta"]), dg, "kerr-schild 4^3 P5", rng)


def _step_case(w, params, u, label, rng, dt=None):
    torch = _torch()
    params = dict(params, hybrid=0)
    odom, ldom, _ = make_pair(w, params)
    E = odom.E
    act = odom.active
    u = u.copy()
    u[:, ~act] = 0.0
    dt = dt or odom.dt()
    fd0 = np.zeros((9, E, odom.m, odom.m, odom.m))
    rep0 = np.zeros(E, np.int64)
    lam = rng.standard_normal(u.shape)
    lam[:, ~act] = 0.0
    delta = rng.standard_normal(u.shape) * np.abs(u).max(axis=(1, 2, 3, 4), keepdims=True)
    delta[:, ~act] = 0.0
    lam_n = ldom.step_adjoint(to_dev(u), to_dev(lam), dt).cpu().numpy().reshape(u.shape)
    lhs = float((lam_n * delta).sum())
    eps = 1e-6
    up = OS.step(odom, OS.State(u + eps * delta, fd0, rep0), dt)
    um = OS.step(odom, OS.State(u - eps * delta, fd0, rep0), dt)
    assert (up.rep == DG).all() and (um.rep == DG).all()
    rhs_o = float((lam * (up.dg - um.dg)).sum() / (2 * eps))
    rep_t = torch.zeros(E, dtype=torch.int32, device="cuda")
    fd_t = to_dev(fd0)
    outs = []
    for sgn in (1.0, -1.0):
        ldom.set_state(to_dev(u + sgn * eps * delta), fd_t, rep_t)
        ldom.step(1, dt)
        outs.append(ldom.get_state()[0].cpu().numpy().reshape(u.shape))
    rhs_g = float((lam * (outs[0] - outs[1])).sum() / (2 * eps))
    _say(f"step adjoint {label}: <lam_n,d> {lhs:.12e}  oracle FD {rhs_o:.12e} (rel {_rel(lhs, rhs_o):.1e})  "
         f"library FD {rhs_g:.12e} (rel {_rel(lhs, rhs_g):.1e})")
    assert _rel(lhs, rhs_o) <= TOL, label
    assert _rel(lhs, rhs_g) <= TOL, label


def test_step_adjoint_wave():
    _torch()
    w = I.workload("wave")
    rng = np.random.default_rng(51)
    odom, _, _ = make_pair(w)
    _step_case(w, dict(eta=w["eta"], cfl=w["cfl"]), _wave_state(odom, w, rng), "wave 2^3 P5", rng)


def test_step_adjoint_no_filter_boundaries_p4():
    _torch()
    w = dict(n_elem=(2, 2, 2), lower=(-1.0, -1.0, -1.0), upper=(1.0, 1.0, 1.0), degree=4, bc=(1, 1, 0, 0, 1, 1),
             curved=False)
    rng = np.random.default_rng(52)
    odom, _, _ = make_pair(w)
    _step_case(w, dict(eta=300.0, cfl=0.25, filter_on=0), _wave_state(odom, w, rng), "P4 outflow, no filter", rng)


def test_step_adjoint_kerr_schild():
    _torch()
    w = I.workload("kerr_schild", n_elem=(4, 4, 4), lower=(-16.0,) * 3, upper=(16.0,) * 3)
    rng = np.random.default_rng(53)
    odom, _, _ = make_pair(w)
    dg, _ = curved_state(odom, w, rng)
    _step_case(w, dict(eta=w["eta"], cfl=w["cfl"]), dg, "kerr-schild 4^3 P5", rng)


def test_autograd_checkpointed_objective():
    torch = _torch()
    from paper_2404_01531_amd import grffe
    from paper_2404_01531_amd.autograd import GRFFEStep
    w = I.workload("wave", n_elem=(2, 2, 2), degree=3)
    rng = np.random.default_rng(54)
    odom, _, _ = make_pair(w)
    u0 = _wave_state(odom, w, rng)
    p = grffe.default_params(eta=1e6, cfl=0.25, hybrid=0)
    dom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], w["degree"], w["bc"], params=p)
    wt = torch.from_numpy(rng.standard_normal(u0.shape).reshape(9, odom.E, -1)).cuda()
    nsteps = 45
    dt = dom.dt()

    def objective(u, every):
        uN = GRFFEStep.apply(u, dom, nsteps, dt, every)
        return (wt * uN).sum()

    u = to_dev(u0).requires_grad_(True)
    J = objective(u, 20)
    J.backward()
    g20 = u.grad.detach().clone()
    u.grad = None
    objective(u, 1).backward()
    g1 = u.grad.detach().clone()
    assert torch.equal(g20, g1), "checkpoint interval changed the gradient"
    delta = torch.from_numpy(rng.standard_normal(u0.shape).reshape(9, odom.E, -1)).cuda()
    eps = 1e-6
    with torch.no_grad():
        jp = float(objective(to_dev(u0) + eps * delta, 20))
        jm = float(objective(to_dev(u0) - eps * delta, 20))
    fd = (jp - jm) / (2 * eps)
    an = float((g20 * delta).sum())
    _say(f"autograd {nsteps} steps (checkpoints every 20): <grad,d> {an:.12e}  FD {fd:.12e}  rel {_rel(an, fd):.1e}")
    assert _rel(an, fd) <= TOL


def test_adjoint_rejects_fd_and_mixed():
    torch = _torch()
    from paper_2404_01531_amd import grffe
    w = I.workload("wave")
    odom, ldom, _ = make_pair(w)
    u = torch.zeros(ldom.dg_shape(), dtype=torch.float64, device="cuda")
    rep = torch.zeros(ldom.E, dtype=torch.int32, device="cuda")
    rep[3] = FD
    with pytest.raises(grffe.GrffeError):
        ldom.rhs_adjoint(u, rep, u)
    _, lmix, _ = make_pair(w, dict(precision=1))
    with pytest.raises(grffe.GrffeError):
        lmix.step_adjoint(u, u)
