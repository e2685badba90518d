"""GPU parity: every C-ABI entry point against the FP64 CPU oracle, element by element.

Tolerance (FP64 path): per evolved component v, max |gpu - oracle| <=
RTOL * max |oracle_v| with RTOL = 1e-12 (the bar the scheme is held to), or
the stated looser bound where a test names one.  Both sides take every
discrete decision (indicator flags, implicit-solve branch) in FP64; the
representation flags must match exactly.
"""
import os
import sys

import numpy as np
import pytest

from oracle import operators as ops
from oracle import rhs as OR
from oracle import step as OS
from oracle import tci as OT
from oracle.domain import DG, FD
from paper_2404_01531_amd import inputs as I

from helpers import curved_state as _curved_state
from helpers import from_dev, group_err, make_pair, node_coords, stiff_tolerance, rel_err, to_dev
from helpers import state_arrays as _state_arrays

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _compare_rhs(odom, ldom, dg, fd, rep, parts, rtol=RTOL, label=""):
    torch = _torch()
    Ldg, Lfd = OR.rhs(odom, dg, fd, rep, parts=parts)
    rep_t = torch.from_numpy(rep.astype(np.int32)).cuda()
    gdg, gfd = ldom.rhs(to_dev(dg), to_dev(fd), rep_t, parts=parts)
    gdg = from_dev(gdg, dg.shape)
    gfd = from_dev(gfd, fd.shape)
    act = odom.active
    dge = np.nonzero(act & (rep == DG))[0]
    fde = np.nonzero(act & (rep == FD))[0]
    worst = 0.0
    for el, G, R in ((dge, gdg, Ldg), (fde, gfd, Lfd)):
        if el.size == 0:
            continue
        e = rel_err(G[:, el], R[:, el])
        worst = max(worst, float(e.max()))
        assert np.all(e <= rtol), (label, e)
    _say(f"rhs parity {label}: worst rel err {worst:.2e}")
    return worst


# ------------------------------------------------------------------ right-hand side


@pytest.mark.parametrize("parts", [1, 2, 3])
def test_rhs_flat_all_dg(parts):
    _torch()
    w = I.workload("wave")
    odom, ldom, _ = make_pair(w)
    rng = np.random.default_rng(11)
    rep = np.zeros(odom.E, np.int64)
    dg, fd = _state_arrays(odom, rng, rep)
    _compare_rhs(odom, ldom, dg, fd, rep, parts, label=f"wave parts={parts}")


@pytest.mark.parametrize("N", [3, 4, 6, 7, 8, 9])
def test_rhs_flat_ragged_degrees(N):
    _torch()
    w = dict(n_elem=(3, 2, 1), lower=(-1.0, -0.5, -0.25), upper=(1.0, 0.75, 0.5), degree=N,
             bc=(0,) * 6, curved=False)
    odom, ldom, _ = make_pair(w)
    rng = np.random.default_rng(20 + N)
    rep = np.zeros(odom.E, np.int64)
    rep[[1, 4]] = FD
    dg, fd = _state_arrays(odom, rng, rep)
    _compare_rhs(odom, ldom, dg, fd, rep, 3, label=f"ragged N={N}")


def test_rhs_flat_mixed_dg_fd():
    _torch()
    w = I.workload("sheet", n_elem=(3, 3, 3))
    odom, ldom, _ = make_pair(w)
    rng = np.random.default_rng(12)
    rep = (rng.random(odom.E) < 0.4).astype(np.int64)
    dg, fd = _state_arrays(odom, rng, rep, smooth_kind="sheet")
    _compare_rhs(odom, ldom, dg, fd, rep, 3, label="sheet mixed")


def test_rhs_fd2_and_no_filter_params():
    _torch()
    w = I.workload("sheet", n_elem=(2, 2, 3))
    odom, ldom, _ = make_pair(w, dict(fd_order=2, eta=10.0))
    rng = np.random.default_rng(13)
    rep = np.array([1, 0, 0, 1, 1, 0, 1, 0, 0, 1, 1, 1], np.int64)
    dg, fd = _state_arrays(odom, rng, rep, smooth_kind="sheet")
    _compare_rhs(odom, ldom, dg, fd, rep, 3, label="fd2")


@pytest.mark.parametrize("N", [5, 3])
def test_rhs_kerr_schild_excision_boundaries(N):
    _torch()
    w = I.workload("kerr_schild", n_elem=(4, 4, 4), lower=(-16.0,) * 3, upper=(16.0,) * 3, degree=N)
    odom, ldom, _ = make_pair(w)
    assert (~odom.active).sum() == 8
    rng = np.random.default_rng(14)
    rep = (rng.random(odom.E) < 0.3).astype(np.int64)
    rep[~odom.active] = DG
    dg, fd = _curved_state(odom, w, rng)
    _compare_rhs(odom, ldom, dg, fd, rep, 3, label=f"kerr-schild N={N}")


# ------------------------------------------------------------- indicator / transfers


def test_tci_project_reconstruct():
    torch = _torch()
    w = I.workload("sheet", n_elem=(4, 3, 2))
    odom, ldom, _ = make_pair(w)
    rng = np.random.default_rng(15)
    rep = (rng.random(odom.E) < 0.5).astype(np.int64)
    dg, fd = _state_arrays(odom, rng, rep, smooth_kind="sheet", noise=3e-3)
    tr, ratio = ldom.tci(to_dev(dg), to_dev(fd), torch.from_numpy(rep.astype(np.int32)).cuda())
    tr, ratio = tr.cpu().numpy(), ratio.cpu().numpy()
    N, M = odom.N, ops.tci_M(odom.N)
    r_dg = OT.tci_ratio(dg, odom.geo_dg, N, M)
    r_fd = OT.tci_ratio(OT.reconstruct_fd_to_dg(fd, N), odom.geo_dg, N, M)
    ref = np.where(rep == FD, r_fd, r_dg)
    thr = np.where(rep == FD, OT.tci_threshold(N, M, 5.0), OT.tci_threshold(N, M, 4.0))
    assert np.abs(ratio - ref).max() <= 1e-12 * max(1e-3, ref.max())
    assert np.array_equal(tr.astype(bool), ref > thr)
    elems = torch.arange(odom.E, dtype=torch.int32, device="cuda")
    pf = from_dev(ldom.project_dg_to_fd(to_dev(dg), elems), fd.shape)
    assert rel_err(pf, OT.project_dg_to_fd(dg, N)).max() <= RTOL
    rd = from_dev(ldom.reconstruct_fd_to_dg(to_dev(fd), elems), dg.shape)
    assert rel_err(rd, OT.reconstruct_fd_to_dg(fd, N)).max() <= RTOL


# ------------------------------------------------------------------------ steps


def _run_steps(w, nsteps, params=None, forced=None, rtol=1e-12, label="", stiff_floor=False, engine=None):
    """Steps of workload w on both sides from the same FD start-up; after every step the
    representation must match and every variable group agree to rtol of the field
    scale.  stiff_floor adds the q~ conditioning floor of a stiff driver current
    (helpers.q_floor: n dt Lambda 8 u eta max|E~| after n steps) to the q~ group."""
    torch = _torch()
    odom, ldom, _ = make_pair(w, params)
    if engine is not None:
        ldom.set_contraction(engine)
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], w["degree"])
    u_fd = I.initial_data(w, xf, yf, zf)
    st = OS.initial_state(odom, u_fd, forced)
    ldom.init_from_fd(to_dev(u_fd), None if forced is None else torch.from_numpy(forced.astype(np.uint8)).cuda())
    dt = ldom.dt()
    assert abs(dt - odom.dt()) <= 1e-14 * dt
    gdg, gfd, grep = ldom.get_state()
    assert np.array_equal(grep.cpu().numpy(), st.rep), "initial representation differs"
    worst = 0.0
    for k in range(nsteps):
        log = []
        st = OS.step(odom, st, dt, log)
        ldom.step(1, dt)
        gdg, gfd, grep = ldom.get_state()
        grep = grep.cpu().numpy()
        assert np.array_equal(grep, st.rep), f"{label}: representation differs after step {k + 1}"
        gdg = from_dev(gdg, st.dg.shape)
        gfd = from_dev(gfd, st.fd.shape)
        act = odom.active
        emax = max(np.abs(st.dg[0:3, act & (st.rep == DG)]).max(initial=0.0),
                   np.abs(st.fd[0:3, act & (st.rep == FD)]).max(initial=0.0))
        for r, G, R in ((DG, gdg, st.dg), (FD, gfd, st.fd)):
            el = np.nonzero(act & (st.rep == r))[0]
            if el.size:
                e = group_err(G[:, el], R[:, el])
                tol = np.full(5, rtol)
                if stiff_floor:
                    tol = stiff_tolerance(odom, dt, k + 1, emax, np.abs(R[:, el]).max(), rtol)
                worst = max(worst, float(e.max()))
                ec = rel_err(G[:, el], R[:, el])
                _say(f"  step {k + 1} rep {r}: group err {np.array2string(e, precision=2)} "
                     f"component err {np.array2string(ec, precision=2)} (q~ bound {tol[4]:.1e})")
                assert np.all(e <= tol), (label, k, r, e.tolist())
    _say(f"step parity {label}: {nsteps} steps, fd elements {int((st.rep == FD).sum())}, worst rel err {worst:.2e}")
    return st, ldom


def test_step_wave_config_10_steps():
    w = I.workload("wave")
    st, _ = _run_steps(w, 10, dict(eta=w["eta"], cfl=w["cfl"]), label="wave 2^3 P5, 10 steps")
    assert (st.rep == DG).all()


def test_step_sheet_adaptive_reduced():
    w = I.workload("sheet", n_elem=(4, 2, 2))
    _run_steps(w, 4, dict(eta=w["eta"], cfl=w["cfl"]), label="sheet 4x2x2 adaptive")


def test_step_forced_partition_and_clamp():
    w = I.workload("sheet", n_elem=(3, 2, 2))
    forced = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 1, 0, 0], bool)
    _run_steps(w, 3, dict(eta=1e6, hybrid=2, ff_clamp=1), forced=forced, label="forced + clamp")


def test_step_dg_only_degree3():
    w = I.workload("wave", n_elem=(3, 2, 2), degree=3)
    _run_steps(w, 3, dict(eta=1e6, hybrid=0), label="dg-only P3")


def test_step_kerr_schild_small():
    w = I.workload("kerr_schild", n_elem=(4, 4, 4), lower=(-16.0,) * 3, upper=(16.0,) * 3)
    _run_steps(w, 2, dict(eta=w["eta"], cfl=w["cfl"]), label="kerr-schild 4^3 P5")


# ------------------------------------------------- Dirichlet faces (the 1D problems)


def test_rhs_dirichlet_faces_dg_and_fd():
    """Dirichlet x faces with DG and FD elements on them: the DG face flux and the FD
    ghost layers take the stored exterior state (a noisy interior, so the face terms
    do not vanish)."""
    w = I.workload("fast_wave_1d", n_elem=(4, 1, 1))
    odom, ldom, _ = make_pair(w, dict(eta=w["eta"], cfl=w["cfl"]))
    rng = np.random.default_rng(1102)
    for rep in ([1, 0, 0, 1], [0, 1, 1, 0], [0, 0, 0, 0], [1, 1, 1, 1]):
        rep = np.array(rep, np.int64)
        dg, fd = _state_arrays(odom, rng, rep)
        _compare_rhs(odom, ldom, dg, fd, rep, 3, label=f"dirichlet faces, rep {rep.tolist()}")


def test_step_fast_wave_dirichlet():
    """The fast-wave problem (kinks on FD) on 8 x 1 x 1 elements between Dirichlet faces."""
    w = I.workload("fast_wave_1d", n_elem=(8, 1, 1))
    st, _ = _run_steps(w, 6, dict(eta=w["eta"], cfl=w["cfl"]), label="fast wave 8x1x1 P5, Dirichlet x faces")
    assert (st.rep == FD).any()


def test_step_pulses_through_dirichlet_faces():
    """Two vacuum pulses reaching the Dirichlet faces (4 x 1 x 1 elements, 40 steps)."""
    w = I.workload("fast_wave_1d", n_elem=(4, 1, 1), lower=(0.0, -0.125, -0.125), upper=(1.0, 0.125, 0.125),
                   kind="pulses_1d")
    _run_steps(w, 40, dict(eta=w["eta"], cfl=w["cfl"]), label="pulses through Dirichlet faces")


def test_dirichlet_state_required_and_checked():
    torch = _torch()
    from paper_2404_01531_amd import grffe
    w = I.workload("fast_wave_1d", n_elem=(4, 1, 1))
    dom = grffe.Domain(w["n_elem"], w["lower"], w["upper"], 5, w["bc"], params=dict(eta=w["eta"], cfl=w["cfl"]))
    with pytest.raises(grffe.GrffeError, match="Dirichlet"):
        dom.step(1)
    bad = I.boundary_states(w)
    bad[0, 2] = np.nan
    with pytest.raises(grffe.GrffeError, match="finite"):
        dom.set_boundary_state(bad)
    dom.set_boundary_state(I.boundary_states(w))
    dom.step(1)
    torch.cuda.synchronize()
    dom.close()
    with pytest.raises(grffe.GrffeError, match="batches"):
        grffe.Batch([dict(n_elem=w["n_elem"], lower=w["lower"], upper=w["upper"], degree=5, bc=w["bc"])])


@pytest.mark.parametrize("N", [3, 4])
def test_step_dirichlet_ragged_degrees_forced_partition(N):
    """Dirichlet x faces on degrees 3 and 4 with a forced partition: FD elements on
    both Dirichlet faces and in the middle.  The fast wave at its own eta = 1e6; the
    stationary Alfven wave at eta = 1e3: its layer carries a parallel current that
    the driver term holds at E.B ~ J.B B^2 / eta, and with eta dt ~ 1e3 the last-bit
    differences of E.B grow to ~1e-9 of the field scale within four steps (the
    problem itself runs at eta = 1e6 in the exact-solution tests)."""
    w = I.workload("fast_wave_1d", n_elem=(8, 1, 1), degree=N)
    _run_steps(w, 4, dict(eta=w["eta"], cfl=w["cfl"], hybrid=2), forced=np.array([1, 0, 0, 1, 0, 0, 0, 1], bool),
               label=f"fast wave P{N}, Dirichlet x faces, forced partition")
    w = I.workload("alfven_1d", n_elem=(10, 1, 1), degree=N)
    _run_steps(w, 4, dict(eta=1e3, cfl=w["cfl"], hybrid=2),
               forced=np.array([1, 0, 0, 0, 1, 0, 0, 0, 0, 1], bool),
               label=f"Alfven wave P{N}, Dirichlet x faces, forced partition")


@pytest.mark.parametrize("N", [3, 5])
def test_step_alfven_paper_eta_forced_partition(N):
    """The stationary Alfven wave at the paper's eta = 1e6 (Sec. IV A 2), DG and FD
    elements (forced partition) with Dirichlet x faces: E, B, psi~, phi~ to 1e-12 of the
    field scale; q~ to that plus the conditioning floor of its stiff flux (the driver
    current eta E.B B / B^2 with E.B relaxed to the rounding level)."""
    w = I.workload("alfven_1d", n_elem=(10, 1, 1), degree=N)
    _run_steps(w, 4, dict(eta=w["eta"], cfl=w["cfl"], hybrid=2),
               forced=np.array([1, 0, 0, 0, 1, 0, 0, 0, 0, 1], bool),
               label=f"Alfven wave P{N}, eta 1e6, forced partition", stiff_floor=True)


def test_step_alfven_paper_eta_adaptive():
    """The same wave at eta = 1e6 with the indicator deciding (levels of Table 1:
    32 P5 elements along x)."""
    w = I.workload("alfven_1d")
    _run_steps(w, 4, dict(eta=w["eta"], cfl=w["cfl"]), label="Alfven wave 32 P5, eta 1e6, adaptive",
               stiff_floor=True)


def _wald_box(N, ne=(2, 2, 2)):
    """The a = 0 Wald field on a box away from the hole, every face a Dirichlet face
    holding the exact field point by point."""
    return dict(n_elem=ne, lower=(4.0, -2.0, -2.0), upper=(8.0, 2.0, 2.0), degree=N, bc=(2,) * 6, curved=True,
                kind="wald_a0", M=1.0, spin=0.0, B0=1.0, boundary_field=True, eta=1e5, cfl=0.25)


@pytest.mark.parametrize("N", [3, 5])
def test_rhs_dirichlet_field_curved(N):
    """Per-point Dirichlet states (the exact Wald field) on a curved background, DG
    and FD elements on the faces, against the oracle."""
    w = _wald_box(N)
    odom, ldom, _ = make_pair(w, dict(eta=w["eta"]))
    x, y, z = node_coords(w)
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], N)
    rng = np.random.default_rng(1103)
    dg = I.wald_a0(x, y, z) + 1e-3 * rng.standard_normal((9,) + x.shape)
    fd = I.wald_a0(xf, yf, zf) + 1e-3 * rng.standard_normal((9,) + xf.shape)
    for rep in ([0] * 8, [1, 0, 0, 1, 0, 1, 1, 0], [1] * 8):
        _compare_rhs(odom, ldom, dg, fd, np.array(rep, np.int64), 3, label=f"Wald field faces P{N}, rep {rep}")


def test_step_dirichlet_field_curved():
    w = _wald_box(5, ne=(3, 2, 2))
    forced = np.array([1, 0, 0, 0, 0, 1, 0, 1, 0, 0, 0, 1], bool)
    _run_steps(w, 3, dict(eta=w["eta"], cfl=w["cfl"], hybrid=2), forced=forced,
               label="Wald field on Dirichlet faces, P5, forced partition")


def test_rhs_kerr_schild_excision_and_dirichlet_field():
    """Both boundary kinds in one domain: Dirichlet outer faces holding the
    Wald-like field point by point, no-incoming-Poynting faces towards the excised
    elements, DG and FD elements mixed."""
    _torch()
    w = dict(I.workload("kerr_schild", n_elem=(4, 4, 4), lower=(-16.0,) * 3, upper=(16.0,) * 3, degree=5),
             bc=(2,) * 6, boundary_field=True)
    odom, ldom, _ = make_pair(w)
    assert (~odom.active).sum() == 8
    rng = np.random.default_rng(15)
    rep = (rng.random(odom.E) < 0.3).astype(np.int64)
    rep[~odom.active] = DG
    dg, fd = _curved_state(odom, w, rng)
    _compare_rhs(odom, ldom, dg, fd, rep, 3, label="kerr-schild, Dirichlet field outside, excision inside")


@pytest.mark.parametrize("N", [8, 9])
def test_step_high_degree_adaptive(N):
    """Degrees 8 and 9 (the paper's exact-Wald table reaches P9): adaptive steps of a
    small current sheet with DG and FD elements."""
    w = I.workload("sheet", n_elem=(3, 2, 2), degree=N)
    _run_steps(w, 2, dict(eta=w["eta"], cfl=w["cfl"]), label=f"sheet 3x2x2 P{N} adaptive")
    # the DG kernels at these degrees: the wave with every element held on DG
    w = I.workload("wave", degree=N)
    st, _ = _run_steps(w, 2, dict(eta=w["eta"], cfl=w["cfl"], hybrid=0), label=f"wave 2^3 P{N}, DG only")
    assert (st.rep == DG).all()


def test_check_finite_reports_blown_up_elements():
    """grffe_check_finite counts the elements holding NaN or infinite values in their
    own representation (a non-finite entry of the other representation is ignored)."""
    torch = _torch()
    from paper_2404_01531_amd import grffe
    w = I.workload("sheet", n_elem=(3, 2, 2))
    _, ldom, _ = make_pair(w, dict(eta=w["eta"], cfl=w["cfl"]))
    xf, yf, zf = I.fd_points(w["n_elem"], w["lower"], w["upper"], w["degree"])
    ldom.init_from_fd(to_dev(I.initial_data(w, xf, yf, zf)))
    assert ldom.check_finite() == 0
    dg, fd, rep = ldom.get_state()
    r = rep.cpu().numpy()
    e_dg, e_fd = int(np.nonzero(r == 0)[0][0]), int(np.nonzero(r == 1)[0][0])
    dg[4, e_dg, 7] = float("nan")
    fd[2, e_fd, 3] = float("inf")
    dg[0, e_fd, 0] = float("nan")  # an FD element's DG entries are not its state
    ldom.set_state(dg, fd, rep)
    assert ldom.check_finite() == 2
    assert "non-finite" in grffe.lib().grffe_last_error().decode()


@pytest.mark.parametrize("curved", [False, True])
def test_mfma_contraction_engine(curved):
    """The DG derivative contraction on the matrix cores (grffe_set_contraction MFMA):
    right-hand sides and adaptive steps against the oracle at the 1e-12 bar, flat (P3,
    P5) and on the Kerr-Schild background with excision (P5)."""
    torch = _torch()
    from paper_2404_01531_amd import grffe
    cases = ([I.workload("kerr_schild", n_elem=(4, 4, 4), lower=(-16.0,) * 3, upper=(16.0,) * 3)] if curved
             else [I.workload("sheet", n_elem=(4, 2, 2), degree=3), I.workload("sheet", n_elem=(4, 2, 2))])
    for w in cases:
        odom, ldom, _ = make_pair(w, dict(eta=w["eta"], cfl=w["cfl"]))
        ldom.set_contraction(grffe.CONTRACTION_MFMA)
        rng = np.random.default_rng(61)
        rep = (rng.random(odom.E) < 0.3).astype(np.int64)
        rep[~odom.active] = DG
        dg, fd = (_curved_state(odom, w, rng) if curved else _state_arrays(odom, rng, rep, smooth_kind="sheet"))
        _compare_rhs(odom, ldom, dg, fd, rep, 3, label=f"MFMA contraction P{w['degree']} curved={curved}")
    st, _ = _run_steps(cases[-1], 2, dict(eta=cases[-1]["eta"], cfl=cases[-1]["cfl"]), label="MFMA contraction steps",
                       engine=grffe.CONTRACTION_MFMA)
