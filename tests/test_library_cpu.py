"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function that include/grffe.h declares,
and its host-built 1D operators must agree with the oracle's independent ones.
"""
import ctypes
import os

import numpy as np
import pytest

from oracle import operators as ops
from paper_2404_01531_amd import grffe

pytestmark = pytest.mark.skipif(not os.path.exists(grffe.LIB_PATH), reason="libgrffe.so not built")


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(grffe.LIB_PATH)
    names = grffe.declared_symbols()
    assert len(names) >= 26
    for name in names:
        assert hasattr(L, name), name


def test_default_params_match_paper_values():
    p = grffe.default_params()
    assert p.eta == 1e6 and p.tci_alpha == 4.0 and p.tci_alpha_fd == 5.0
    assert p.filter_a == 36.0 and p.filter_b == 50.0 and p.fd_order == 4 and p.weno_eps == 1e-40


@pytest.mark.parametrize("N", [3, 4, 5, 6, 7, 8, 9])
def test_host_operators_match_oracle(N):
    n, m = N + 1, 2 * N + 1
    x, w = ops.gll(N)
    M = ops.tci_M(N)
    pairs = [
        (0, x), (1, w), (2, ops.diff_matrix(N).ravel()), (3, ops.filter_matrix(N).ravel()),
        (4, ops.mode_mask_matrix(N, M, True).ravel()), (5, ops.projection_matrix(N).ravel()),
        (6, ops.reconstruction_matrix(N).ravel()), (7, ops.face_eval_matrix(N).ravel()),
    ]
    for which, ref in pairs:
        got = grffe.operator(N, which)
        assert got.shape == ref.shape, which
        assert np.abs(got - ref).max() < 2e-13 * max(1.0, np.abs(ref).max()), (which, np.abs(got - ref).max())


def test_invalid_degree_is_rejected():
    with pytest.raises(grffe.GrffeError):
        grffe.operator(2, 0)


def _grid(**over):
    g = grffe.Grid()
    vals = dict(n_elem=(2, 2, 2), lower=(-1.0,) * 3, upper=(1.0,) * 3, degree=5, bc=(0,) * 6)
    vals.update(over)
    grffe._fill_grid(g, vals["n_elem"], vals["lower"], vals["upper"], vals["degree"], vals["bc"], None)
    return g


@pytest.mark.parametrize("bad, code", [
    (dict(degree=2), -1), (dict(degree=10), -1), (dict(n_elem=(0, 2, 2)), -1),
    (dict(upper=(1.0, -1.0, 1.0)), -1), (dict(bc=(0, 1, 0, 0, 0, 0)), -1), (dict(bc=(0, 0, 7, 7, 0, 0)), -1),
    (dict(bc=(2, 0, 0, 0, 0, 0)), -1), (dict(bc=(3, 3, 0, 0, 0, 0)), -1),
])
def test_init_domain_rejects_bad_grids(bad, code):
    """Validation happens before any device call, so it runs without a GPU."""
    L = grffe.lib()
    g = _grid(**bad)
    p = grffe.default_params()
    h = ctypes.c_void_p()
    rc = L.grffe_init_domain(ctypes.byref(g), ctypes.byref(p), None, None, ctypes.byref(h))
    assert rc == code and not h.value
    assert L.grffe_last_error().decode()


@pytest.mark.parametrize("over, code", [
    (dict(precision=2), -5), (dict(hybrid=3), -1), (dict(fd_order=3), -1), (dict(tci_mode=0), -1),
    (dict(cfl=0.0), -1), (dict(eta=-1.0), -1), (dict(tci_M=6), -1),
])
def test_init_domain_rejects_bad_params(over, code):
    L = grffe.lib()
    g = _grid()
    p = grffe.default_params(**over)
    h = ctypes.c_void_p()
    assert L.grffe_init_domain(ctypes.byref(g), ctypes.byref(p), None, None, ctypes.byref(h)) == code


def test_null_handles_are_rejected():
    L = grffe.lib()
    g = _grid()
    p = grffe.default_params()
    assert L.grffe_init_domain(ctypes.byref(g), ctypes.byref(p), None, None, None) == -1
    assert L.grffe_step(None, 1, 0.0, None) == -1
    assert L.grffe_rhs(None, None, None, None, None, None, 3, None) == -1
    assert L.grffe_destroy(None) == 0
    assert L.grffe_batch_destroy(None) == 0
    h = ctypes.c_void_p()
    arr = (grffe.Grid * 1)(g)
    assert L.grffe_batch_create(arr, 0, ctypes.byref(p), None, None, ctypes.byref(h)) == -1
    bad = (grffe.Grid * 1)(_grid(degree=10))
    assert L.grffe_batch_create(bad, 1, ctypes.byref(p), None, None, ctypes.byref(h)) == -1
    assert L.grffe_batch_step(None, 1, 1, None) == -1
    d = ctypes.c_double()
    assert L.grffe_batch_get_dt(None, 0, ctypes.byref(d)) == -1


def test_dirichlet_entry_points_on_the_host():
    L = grffe.lib()
    state = (ctypes.c_double * 54)()
    assert L.grffe_set_boundary_state(None, state, None) == -1
    assert L.grffe_set_boundary_field(None, None, None, None) == -1
    assert L.grffe_check_finite(None, None, None) == -1
    assert L.grffe_force_flags(None, None, None) == -1
    centre = (ctypes.c_double * 3)()
    assert L.grffe_set_conductor(None, centre, 1.0, 0.2, None) == -1
    p = grffe.default_params()
    h = ctypes.c_void_p()
    arr = (grffe.Grid * 1)(_grid(bc=(2, 2, 0, 0, 0, 0)))
    # batches refuse Dirichlet grids before touching the device
    assert L.grffe_batch_create(arr, 1, ctypes.byref(p), None, None, ctypes.byref(h)) == -5
    assert "Dirichlet" in L.grffe_last_error().decode()


def test_adjoint_entry_points_reject_null_handles():
    L = grffe.lib()
    assert L.grffe_rhs_adjoint(None, None, None, None, None, None, None, None, 3, None) == -1
    assert L.grffe_step_adjoint(None, None, None, None, 0.0, None) == -1
    assert L.grffe_step_adjoint_frozen(None, None, None, None, None, None, None, None, None, 0.0, None) == -1
    assert L.grffe_timing_read(None, 2, None, None) == -1


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


@pytest.mark.parametrize("N, nr, na", [(3, 1, 1), (5, 2, 2), (9, 1, 3)])
def test_shell_points_match_oracle(N, nr, na):
    """The library's host map of the shell (grffe_shell_points) against the oracle's."""
    from oracle import shell as S
    sh = S.Shell(N, nr, na, 1.99, 20.0)
    for fd in (False, True):
        got = grffe.shell_points(N, nr, na, 1.99, 20.0, fd=fd)
        want = sh.points(fd=fd).reshape(3, sh.E, -1)
        assert np.abs(got - want).max() < 1e-13 * 20.0


@pytest.mark.parametrize("shell, over, code", [
    (dict(), dict(hybrid=1, fd_order=4), -5), (dict(), dict(hybrid=2, fd_order=4), -5),
    (dict(), dict(precision=1), -5), (dict(degree=2), dict(), -1),
    (dict(r_in=3.0), dict(), -1), (dict(r_in=0.0), dict(), -1), (dict(n_angular=0), dict(), -1),
    (dict(bc_inner=0), dict(), -1), (dict(bc_outer=7), dict(), -1),
])
def test_init_shell_rejects_unsupported(shell, over, code):
    """Refused before any device call, so it runs without a GPU."""
    L = grffe.lib()
    args = dict(degree=5, n_radial=1, n_angular=1, r_in=2.0, r_out=3.0, bc_inner=3, bc_outer=2)
    args.update(shell)
    s = grffe._fill_shell(**args)
    p = grffe.default_params(**{"hybrid": 0, **over})
    h = ctypes.c_void_p()
    assert L.grffe_init_shell(ctypes.byref(s), ctypes.byref(p), None, None, ctypes.byref(h)) == code
    assert not h.value and L.grffe_last_error().decode()
