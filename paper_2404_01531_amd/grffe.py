"""Python binding of libgrffe (ctypes, argument marshalling only).

Every computation runs in the HIP library; this module only turns torch
tensors into device pointers and the current torch stream into a hipStream_t.
If the library has not been built the import of a domain fails loudly.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libgrffe.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "grffe.h")

BC_PERIODIC = 0
BC_NO_INCOMING_POYNTING = 1
BC_DIRICHLET = 2
BC_OUTFLOW = 3
PART_EXPLICIT, PART_STIFF, PART_ALL = 1, 2, 3
HYBRID_DG_ONLY, HYBRID_ADAPTIVE, HYBRID_FORCED = 0, 1, 2
CONTRACTION_VALU = 0
CONTRACTION_MFMA = 1
KERNEL_FAMILIES = {"dg_substep": 1, "fd_flux": 2, "fd_update": 3, "fd_stage": 4, "fd_trace": 5,
                   "dg_slab": 6, "project": 7, "fd_to_dg": 8, "dg_prestage": 9}


class GrffeError(RuntimeError):
    pass


class Grid(ctypes.Structure):
    _fields_ = [
        ("n_elem", ctypes.c_int32 * 3),
        ("lower", ctypes.c_double * 3),
        ("upper", ctypes.c_double * 3),
        ("degree", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 6),
        ("excised", ctypes.POINTER(ctypes.c_uint8)),
    ]


class ShellGrid(ctypes.Structure):
    _fields_ = [
        ("degree", ctypes.c_int32),
        ("n_radial", ctypes.c_int32),
        ("n_angular", ctypes.c_int32),
        ("r_in", ctypes.c_double),
        ("r_out", ctypes.c_double),
        ("bc_inner", ctypes.c_int32),
        ("bc_outer", ctypes.c_int32),
    ]


def _fill_shell(degree, n_radial, n_angular, r_in, r_out, bc_inner=BC_OUTFLOW, bc_outer=BC_DIRICHLET):
    s = ShellGrid()
    s.degree, s.n_radial, s.n_angular = int(degree), int(n_radial), int(n_angular)
    s.r_in, s.r_out = float(r_in), float(r_out)
    s.bc_inner, s.bc_outer = int(bc_inner), int(bc_outer)
    return s


def shell_points(degree, n_radial, n_angular, r_in, r_out, fd=False):
    """Coordinates (3, E, k^3) of a shell's DG nodes (k = N + 1) or FD cell centres
    (k = 2N + 1), computed by the library on the host."""
    s = _fill_shell(degree, n_radial, n_angular, r_in, r_out)
    E = 6 * int(n_radial) * int(n_angular) ** 2
    k = 2 * int(degree) + 1 if fd else int(degree) + 1
    out = np.empty((3, E, k ** 3), np.float64)
    _check(lib().grffe_shell_points(ctypes.byref(s), 1 if fd else 0,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


class Params(ctypes.Structure):
    _fields_ = [
        ("eta", ctypes.c_double),
        ("kappa_psi", ctypes.c_double),
        ("kappa_phi", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("stab_c", ctypes.c_double),
        ("tci_M", ctypes.c_int32),
        ("tci_mode", ctypes.c_int32),
        ("tci_alpha", ctypes.c_double),
        ("tci_alpha_fd", ctypes.c_double),
        ("filter_a", ctypes.c_double),
        ("filter_b", ctypes.c_double),
        ("filter_on", ctypes.c_int32),
        ("fd_order", ctypes.c_int32),
        ("weno_eps", ctypes.c_double),
        ("ff_clamp", ctypes.c_int32),
        ("ff_margin", ctypes.c_double),
        ("hybrid", ctypes.c_int32),
        ("precision", ctypes.c_int32),
    ]


_lib = None


def lib():
    """Load libgrffe.so (raises GrffeError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GrffeError(f"{LIB_PATH} not found: build it with paper_2404_01531_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.grffe_default_params.argtypes = [ctypes.POINTER(Params)]
    L.grffe_default_params.restype = None
    L.grffe_init_domain.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Params), vp, vp, ctypes.POINTER(vp)]
    L.grffe_shell_points.argtypes = [ctypes.POINTER(ShellGrid), i32, ctypes.POINTER(dbl)]
    L.grffe_init_shell.argtypes = [ctypes.POINTER(ShellGrid), ctypes.POINTER(Params), vp, vp, ctypes.POINTER(vp)]
    L.grffe_set_boundary_state.argtypes = [vp, ctypes.POINTER(dbl), vp]
    L.grffe_set_boundary_field.argtypes = [vp, vp, vp, vp]
    L.grffe_check_finite.argtypes = [vp, ctypes.POINTER(i32), vp]
    L.grffe_check_finite_noalloc.argtypes = [vp, ctypes.POINTER(i32), vp]
    L.grffe_set_conductor.argtypes = [vp, vp, dbl, dbl, vp]
    L.grffe_destroy.argtypes = [vp]
    L.grffe_init_from_fd.argtypes = [vp, vp, vp, vp]
    L.grffe_set_state.argtypes = [vp, vp, vp, vp, vp]
    L.grffe_force_flags.argtypes = [vp, vp, vp]
    L.grffe_set_contraction.argtypes = [vp, ctypes.c_int]
    L.grffe_get_state.argtypes = [vp, vp, vp, vp, vp]
    L.grffe_rhs.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_int, vp]
    L.grffe_step.argtypes = [vp, ctypes.c_int, dbl, vp]
    L.grffe_tci.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.grffe_project_dg_to_fd.argtypes = [vp, vp, vp, vp, i32, vp]
    L.grffe_reconstruct_fd_to_dg.argtypes = [vp, vp, vp, vp, i32, vp]
    L.grffe_get_dt.argtypes = [vp, ctypes.POINTER(dbl)]
    L.grffe_get_counts.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.grffe_operator.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(dbl), ctypes.c_int]
    L.grffe_timing_enable.argtypes = [vp, ctypes.c_int]
    L.grffe_timing_read.argtypes = [vp, ctypes.c_int, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64)]
    L.grffe_timing_period.argtypes = [vp, ctypes.c_int]
    L.grffe_rhs_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp]
    L.grffe_step_adjoint.argtypes = [vp, vp, vp, vp, dbl, vp]
    L.grffe_step_adjoint_frozen.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, dbl, vp]
    L.grffe_get_stages.argtypes = [vp, vp, vp, vp]
    L.grffe_step_adjoint_stages.argtypes = [vp, vp, vp, vp, vp, vp, dbl, vp]
    pvp = ctypes.POINTER(vp)
    L.grffe_batch_create.argtypes = [ctypes.POINTER(Grid), i32, ctypes.POINTER(Params), pvp, vp, pvp]
    L.grffe_batch_destroy.argtypes = [vp]
    L.grffe_batch_size.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.grffe_batch_init_from_fd.argtypes = [vp, pvp, pvp, vp]
    L.grffe_batch_get_state.argtypes = [vp, i32, vp, vp, vp, vp]
    L.grffe_batch_set_state.argtypes = [vp, i32, vp, vp, vp, vp]
    L.grffe_batch_get_dt.argtypes = [vp, i32, ctypes.POINTER(dbl)]
    L.grffe_batch_get_counts.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.grffe_batch_step.argtypes = [vp, i32, i32, vp]
    L.grffe_batch_set_contraction.argtypes = [vp, i32, i32]
    L.grffe_step_logged.argtypes = [vp, dbl, vp, vp]
    L.grffe_batch_get_contraction.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.grffe_last_error.restype = ctypes.c_char_p
    for name in ("grffe_init_domain", "grffe_destroy", "grffe_init_from_fd", "grffe_set_state", "grffe_get_state",
                 "grffe_rhs", "grffe_step", "grffe_tci", "grffe_project_dg_to_fd", "grffe_reconstruct_fd_to_dg",
                 "grffe_get_dt", "grffe_get_counts", "grffe_operator", "grffe_timing_enable",
                 "grffe_timing_read", "grffe_timing_period", "grffe_batch_create", "grffe_batch_destroy", "grffe_batch_size",
                 "grffe_batch_init_from_fd", "grffe_batch_get_state", "grffe_batch_set_state",
                 "grffe_batch_get_dt", "grffe_batch_get_counts", "grffe_batch_step", "grffe_rhs_adjoint",
                 "grffe_step_adjoint", "grffe_step_adjoint_frozen", "grffe_get_stages",
                 "grffe_step_adjoint_stages", "grffe_set_boundary_state", "grffe_set_boundary_field",
                 "grffe_check_finite", "grffe_set_conductor", "grffe_batch_set_contraction",
                 "grffe_batch_get_contraction", "grffe_step_logged", "grffe_shell_points", "grffe_init_shell"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def declared_symbols():
    """Function names declared in include/grffe.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(grffe_[a-z_0-9]+)\s*\(", text)))


def _check(rc):
    if rc < 0:
        raise GrffeError(f"libgrffe error {rc}: {lib().grffe_last_error().decode()}")
    return rc


def default_params(**over):
    p = Params()
    lib().grffe_default_params(ctypes.byref(p))
    for k, v in over.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def operator(degree, which):
    """Host copy of one of the library's 1D operators (see grffe_operator)."""
    n = _check(lib().grffe_operator(degree, which, None, 0))
    buf = (ctypes.c_double * n)()
    _check(lib().grffe_operator(degree, which, buf, n))
    return np.frombuffer(buf, dtype=np.float64).copy()


def _ptr(t):
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise GrffeError("device tensors are required")
    if not t.is_contiguous():
        raise GrffeError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _fill_grid(g, n_elem, lower, upper, degree, bc, excised):
    """Fill a Grid; returns the host excision array that must outlive the call."""
    for k in range(3):
        g.n_elem[k] = int(n_elem[k])
        g.lower[k] = float(lower[k])
        g.upper[k] = float(upper[k])
    g.degree = int(degree)
    for k in range(6):
        g.bc[k] = int(bc[k])
    exc = None
    if excised is not None:
        exc = np.ascontiguousarray(np.asarray(excised, np.uint8))
        g.excised = exc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    return exc


class Domain:
    """A GRFFE domain living on the current HIP device."""

    def __init__(self, n_elem, lower, upper, degree, bc, params=None, bg=None, excised=None):
        import torch
        if not torch.cuda.is_available():
            raise GrffeError("no HIP device available")
        L = lib()
        g = Grid()
        self._exc = _fill_grid(g, n_elem, lower, upper, degree, bc, excised)
        p = params if isinstance(params, Params) else default_params(**(params or {}))
        self.params = p
        self.N = int(degree)
        self.n = self.N + 1
        self.m = 2 * self.N + 1
        self.E = int(np.prod(n_elem))
        if bg is not None:
            bg = bg.contiguous()
            if tuple(bg.shape) != (26, self.E, self.n ** 3) or bg.dtype != torch.float64:
                raise GrffeError("bg must be float64 of shape (26, E, (N+1)^3)")
        h = ctypes.c_void_p()
        _check(L.grffe_init_domain(ctypes.byref(g), ctypes.byref(p), _ptr(bg), _stream(), ctypes.byref(h)))
        self._h = h

    @classmethod
    def shell(cls, degree, n_radial, n_angular, r_in, r_out, bc_inner=BC_OUTFLOW, bc_outer=BC_DIRICHLET,
              params=None, bg=None):
        """A domain on the spherical shell of cubed-sphere wedges (grffe_init_shell);
        bg (26, E, (N+1)^3) float64 at the points of shell_points(..., fd=False)."""
        import torch
        if not torch.cuda.is_available():
            raise GrffeError("no HIP device available")
        L = lib()
        s = _fill_shell(degree, n_radial, n_angular, r_in, r_out, bc_inner, bc_outer)
        self = cls.__new__(cls)
        self._exc = None
        p = params if isinstance(params, Params) else default_params(**(params or {}))
        self.params = p
        self.N = int(degree)
        self.n = self.N + 1
        self.m = 2 * self.N + 1
        self.E = 6 * int(n_radial) * int(n_angular) ** 2
        if bg is not None:
            bg = bg.contiguous()
            if tuple(bg.shape) != (26, self.E, self.n ** 3) or bg.dtype != torch.float64:
                raise GrffeError("bg must be float64 of shape (26, E, (N+1)^3)")
        h = ctypes.c_void_p()
        _check(L.grffe_init_shell(ctypes.byref(s), ctypes.byref(p), _ptr(bg), _stream(), ctypes.byref(h)))
        self._h = h
        return self

    def close(self):
        if getattr(self, "_h", None):
            lib().grffe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- shapes
    def dg_shape(self):
        return (9, self.E, self.n ** 3)

    def fd_shape(self):
        return (9, self.E, self.m ** 3)

    def _check_state(self, dg, fd, rep):
        if dg is not None and tuple(dg.shape) != self.dg_shape():
            raise GrffeError(f"dg must have shape {self.dg_shape()}")
        if fd is not None and tuple(fd.shape) != self.fd_shape():
            raise GrffeError(f"fd must have shape {self.fd_shape()}")
        if rep is not None and tuple(rep.shape) != (self.E,):
            raise GrffeError("rep must have shape (E,)")

    # ------------------------------------------------------------------ calls
    def init_from_fd(self, u_fd, forced=None):
        self._check_state(None, u_fd, None)
        _check(lib().grffe_init_from_fd(self._h, _ptr(u_fd), _ptr(forced), _stream()))

    def set_state(self, dg, fd, rep):
        self._check_state(dg, fd, rep)
        _check(lib().grffe_set_state(self._h, _ptr(dg), _ptr(fd), _ptr(rep), _stream()))

    def set_contraction(self, engine):
        """DG derivative contraction engine: CONTRACTION_VALU (0) or CONTRACTION_MFMA (1)."""
        _check(lib().grffe_set_contraction(self._h, int(engine)))

    def force_flags(self, mask):
        """Host-forced indicator flags (test instrument): mask is a device uint8 tensor
        (3, E), row k - 1 forcing the rollback of its DG elements in substep k of every
        following adaptive step; None switches the forcing off."""
        if mask is not None:
            if tuple(mask.shape) != (3, self.E) or str(mask.dtype) != "torch.uint8":
                raise GrffeError("forced flags must be a uint8 tensor of shape (3, E)")
            mask = mask.contiguous()
        _check(lib().grffe_force_flags(self._h, _ptr(mask), _stream()))
        self._force = mask  # kept alive until the copy on the stream has run

    def set_boundary_state(self, state):
        """Exterior states of the Dirichlet faces: (6, 9) host array, row f = 2 d + s."""
        st = np.ascontiguousarray(np.asarray(state, np.float64))
        if st.shape != (6, 9):
            raise GrffeError("boundary state must have shape (6, 9)")
        _check(lib().grffe_set_boundary_state(self._h, st.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()))

    def set_conductor(self, centre, radius, omega):
        """Rotating perfect conductor of the given centre (3,), radius and angular
        velocity about z; radius <= 0 switches it off."""
        c = np.ascontiguousarray(np.asarray(centre, np.float64).reshape(3))
        _check(lib().grffe_set_conductor(self._h, c.ctypes.data_as(ctypes.c_void_p), float(radius), float(omega),
                                         _stream()))

    def check_finite(self):
        """Number of elements holding NaN or infinite values (0 for a healthy state)."""
        n = ctypes.c_int32(0)
        rc = lib().grffe_check_finite(self._h, ctypes.byref(n), _stream())
        if rc not in (0, -4):
            _check(rc)
        return int(n.value)

    def set_boundary_field(self, ext_dg, ext_fd):
        """Per-point exterior states of the Dirichlet faces: device float64 tensors
        (9, E, 6, n^2) at the DG face nodes and (9, E, 6, 3, m^2) at the FD ghost cells."""
        n2, m2 = self.n ** 2, self.m ** 2
        if tuple(ext_dg.shape) != (9, self.E, 6, n2) or (ext_fd is not None and tuple(ext_fd.shape) != (9, self.E, 6, 3, m2)):
            raise GrffeError(f"boundary field shapes must be (9, E, 6, {n2}) and (9, E, 6, 3, {m2})")
        _check(lib().grffe_set_boundary_field(self._h, _ptr(ext_dg.contiguous()),
                                              _ptr(None if ext_fd is None else ext_fd.contiguous()), _stream()))

    def get_state(self):
        import torch
        dg = torch.empty(self.dg_shape(), dtype=torch.float64, device="cuda")
        fd = torch.empty(self.fd_shape(), dtype=torch.float64, device="cuda")
        rep = torch.empty((self.E,), dtype=torch.int32, device="cuda")
        _check(lib().grffe_get_state(self._h, _ptr(dg), _ptr(fd), _ptr(rep), _stream()))
        return dg, fd, rep

    def get_dg(self):
        """The DG state array alone (grffe_get_state with the FD and flag outputs NULL)."""
        import torch
        dg = torch.empty(self.dg_shape(), dtype=torch.float64, device="cuda")
        _check(lib().grffe_get_state(self._h, _ptr(dg), None, None, _stream()))
        return dg

    def rhs(self, dg, fd, rep, parts=PART_ALL):
        import torch
        self._check_state(dg, fd, rep)
        ddg = torch.zeros_like(dg)
        dfd = torch.zeros_like(fd)
        _check(lib().grffe_rhs(self._h, _ptr(dg), _ptr(fd), _ptr(rep), _ptr(ddg), _ptr(dfd), int(parts), _stream()))
        return ddg, dfd

    def step(self, n_steps=1, dt=0.0):
        _check(lib().grffe_step(self._h, int(n_steps), float(dt), _stream()))

    def step_logged(self, dt=0.0):
        """One step with its decision log (see grffe_step_logged): int32 (5, E) device
        tensor, the representation before the step, after substeps 1-3, after it."""
        import torch
        log = torch.empty((5, self.E), dtype=torch.int32, device="cuda")
        _check(lib().grffe_step_logged(self._h, float(dt), _ptr(log), _stream()))
        return log

    def rhs_adjoint(self, dg, fd, rep, lam_dg, lam_fd, parts=PART_ALL):
        """(ubar_dg, ubar_fd) = (dRHS/du)^T (lam_dg, lam_fd) for a state of DG and FD
        elements chosen by rep (see grffe_rhs_adjoint); the entries of elements in
        the other representation are zero."""
        import torch
        self._check_state(dg, fd, rep)
        self._check_state(lam_dg, lam_fd, None)
        ub_dg = torch.zeros_like(dg)
        ub_fd = torch.zeros_like(fd)
        _check(lib().grffe_rhs_adjoint(self._h, _ptr(dg), _ptr(fd), _ptr(rep), _ptr(lam_dg), _ptr(lam_fd),
                                       _ptr(ub_dg), _ptr(ub_fd), int(parts), _stream()))
        return ub_dg, ub_fd

    def step_adjoint(self, u_dg, lam_next, dt=0.0):
        """(dU^{n+1}/dU^n)^T lam_next for one all-DG step from u_dg (see grffe_step_adjoint)."""
        import torch
        self._check_state(u_dg, None, None)
        self._check_state(lam_next, None, None)
        lam = torch.zeros_like(lam_next)  # excised elements' entries are not written
        _check(lib().grffe_step_adjoint(self._h, _ptr(u_dg), _ptr(lam_next), _ptr(lam), float(dt), _stream()))
        return lam

    def get_stages(self):
        """(U_3, U_4) of the last step, DG (see grffe_get_stages)."""
        import torch
        u3 = torch.empty(self.dg_shape(), dtype=torch.float64, device="cuda")
        u4 = torch.empty_like(u3)
        _check(lib().grffe_get_stages(self._h, _ptr(u3), _ptr(u4), _stream()))
        return u3, u4

    def step_adjoint_stages(self, u_dg, u3, u4, lam_next, dt=0.0):
        """(dU^{n+1}/dU^n)^T lam_next from the step's stored stages (see
        grffe_step_adjoint_stages)."""
        import torch
        for x in (u_dg, u3, u4, lam_next):
            self._check_state(x, None, None)
        lam = torch.zeros_like(lam_next)  # excised elements' entries are not written
        _check(lib().grffe_step_adjoint_stages(self._h, _ptr(u_dg), _ptr(u3), _ptr(u4), _ptr(lam_next), _ptr(lam),
                                               float(dt), _stream()))
        return lam

    def step_adjoint_frozen(self, dg, fd, rep, mu_dg, mu_fd, dt=0.0, with_log=False):
        """(lam_dg, lam_fd) = (dU^{n+1}/dU^n)^T (mu_dg, mu_fd) for one step from (dg, fd, rep)
        with the hybrid decisions of the domain's own forward re-run frozen (see
        grffe_step_adjoint_frozen); entries of elements in the other representation
        are zero.  with_log: also the representation log (5, E) (before the step,
        during substeps 1-3, after the step)."""
        import torch
        self._check_state(dg, fd, rep)
        self._check_state(mu_dg, mu_fd, None)
        lam_dg = torch.zeros_like(mu_dg)
        lam_fd = torch.zeros_like(mu_fd)
        log = torch.empty((5, self.E), dtype=torch.int32, device="cuda") if with_log else None
        _check(lib().grffe_step_adjoint_frozen(self._h, _ptr(dg), _ptr(fd), _ptr(rep), _ptr(mu_dg), _ptr(mu_fd),
                                               _ptr(lam_dg), _ptr(lam_fd), _ptr(log), float(dt), _stream()))
        return (lam_dg, lam_fd, log) if with_log else (lam_dg, lam_fd)

    def tci(self, dg, fd, rep):
        import torch
        self._check_state(dg, fd, rep)
        tr = torch.zeros((self.E,), dtype=torch.uint8, device="cuda")
        ratio = torch.zeros((self.E,), dtype=torch.float64, device="cuda")
        _check(lib().grffe_tci(self._h, _ptr(dg), _ptr(fd), _ptr(rep), _ptr(tr), _ptr(ratio), _stream()))
        return tr, ratio

    def project_dg_to_fd(self, u_dg, elems):
        import torch
        n = int(elems.numel())
        out = torch.zeros((9, n, self.m ** 3), dtype=torch.float64, device="cuda")
        _check(lib().grffe_project_dg_to_fd(self._h, _ptr(u_dg), _ptr(out), _ptr(elems), n, _stream()))
        return out

    def reconstruct_fd_to_dg(self, u_fd, elems):
        import torch
        n = int(elems.numel())
        out = torch.zeros((9, n, self.n ** 3), dtype=torch.float64, device="cuda")
        _check(lib().grffe_reconstruct_fd_to_dg(self._h, _ptr(u_fd), _ptr(out), _ptr(elems), n, _stream()))
        return out

    def dt(self):
        v = ctypes.c_double()
        _check(lib().grffe_get_dt(self._h, ctypes.byref(v)))
        return v.value

    def timing_enable(self, *families, period=1):
        """Time the launches of the given kernel families with HIP events (see
        grffe_timing_enable), in one step of every `period` steps
        (grffe_timing_period); no family switches timing off."""
        mask = 0
        for f in families:
            mask |= 1 << int(f)
        _check(lib().grffe_timing_enable(self._h, mask))
        _check(lib().grffe_timing_period(self._h, int(period)))

    def timing_read(self, family):
        """(summed ms, launches) of one family since timing was enabled or last read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().grffe_timing_read(self._h, int(family), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def counts(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().grffe_get_counts(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


class Batch:
    """Many independent domains stepped together (see grffe_batch_create).

    `grids` is a list of dicts with keys n_elem, lower, upper, degree, bc and
    optionally excised; `bgs` is None (flat) or one (26, E_k, n_k^3) float64
    device tensor per grid."""

    def __init__(self, grids, params=None, bgs=None):
        import torch
        if not torch.cuda.is_available():
            raise GrffeError("no HIP device available")
        L = lib()
        cnt = len(grids)
        if cnt < 1:
            raise GrffeError("a batch needs at least one grid")
        arr = (Grid * cnt)()
        self._keep = []
        self.shapes = []
        for k, gd in enumerate(grids):
            self._keep.append(_fill_grid(arr[k], gd["n_elem"], gd["lower"], gd["upper"], gd["degree"], gd["bc"],
                                         gd.get("excised")))
            N = int(gd["degree"])
            self.shapes.append((int(np.prod(gd["n_elem"])), N))
        p = params if isinstance(params, Params) else default_params(**(params or {}))
        self.params = p
        bg_arr = None
        if bgs is not None:
            if len(bgs) != cnt:
                raise GrffeError("one background per grid")
            for (E, N), b in zip(self.shapes, bgs):
                if tuple(b.shape) != (26, E, (N + 1) ** 3) or b.dtype != torch.float64:
                    raise GrffeError("bg must be float64 of shape (26, E, (N+1)^3)")
            bg_arr = (ctypes.c_void_p * cnt)(*[b.data_ptr() for b in bgs])
        h = ctypes.c_void_p()
        _check(L.grffe_batch_create(arr, cnt, ctypes.byref(p), bg_arr, _stream(), ctypes.byref(h)))
        self._h = h
        self.count = cnt

    def close(self):
        if getattr(self, "_h", None):
            lib().grffe_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def size(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().grffe_batch_size(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def _dims(self, k):
        E, N = self.shapes[k]
        return E, (N + 1) ** 3, (2 * N + 1) ** 3

    def init_from_fd(self, u_fds, forced=None):
        if len(u_fds) != self.count:
            raise GrffeError("one FD array per domain")
        for k, u in enumerate(u_fds):
            E, _, mm = self._dims(k)
            if tuple(u.shape) != (9, E, mm):
                raise GrffeError(f"u_fd[{k}] must have shape {(9, E, mm)}")
            _ptr(u)
        ua = (ctypes.c_void_p * self.count)(*[u.data_ptr() for u in u_fds])
        fa = None
        if forced is not None:
            fa = (ctypes.c_void_p * self.count)(*[(f.data_ptr() if f is not None else None) for f in forced])
        _check(lib().grffe_batch_init_from_fd(self._h, ua, fa, _stream()))

    def get_state(self, k):
        import torch
        E, nn, mm = self._dims(k)
        dg = torch.empty((9, E, nn), dtype=torch.float64, device="cuda")
        fd = torch.empty((9, E, mm), dtype=torch.float64, device="cuda")
        rep = torch.empty((E,), dtype=torch.int32, device="cuda")
        _check(lib().grffe_batch_get_state(self._h, int(k), _ptr(dg), _ptr(fd), _ptr(rep), _stream()))
        return dg, fd, rep

    def set_state(self, k, dg, fd, rep):
        E, nn, mm = self._dims(k)
        if tuple(dg.shape) != (9, E, nn) or tuple(fd.shape) != (9, E, mm) or tuple(rep.shape) != (E,):
            raise GrffeError("state shapes do not match domain")
        _check(lib().grffe_batch_set_state(self._h, int(k), _ptr(dg), _ptr(fd), _ptr(rep), _stream()))

    def dt(self, k):
        v = ctypes.c_double()
        _check(lib().grffe_batch_get_dt(self._h, int(k), ctypes.byref(v)))
        return v.value

    def counts(self, k):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().grffe_batch_get_counts(self._h, int(k), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def step(self, n_steps=1, use_graph=True):
        _check(lib().grffe_batch_step(self._h, int(n_steps), int(bool(use_graph)), _stream()))

    def degrees(self):
        """The degrees of the batch's pools, ascending."""
        return sorted({N for _, N in self.shapes})

    def set_contraction(self, degree, engine):
        """DG contraction engine of the pool of one degree (0: every pool)."""
        _check(lib().grffe_batch_set_contraction(self._h, int(degree), int(engine)))

    def contraction(self, degree):
        v = ctypes.c_int32()
        _check(lib().grffe_batch_get_contraction(self._h, int(degree), ctypes.byref(v)))
        return v.value

    def autotune(self, steps=3, reps=3, margin=0.02):
        """Per-degree choice of the contraction engine by timing the batch's graph step
        with each engine.  Disabled: batches run the VALU contraction (see
        grffe_batch_set_contraction); the tuner's re-captured step graphs with
        matrix-core pools ended in an abort inside the HIP runtime, whose cause is not
        known, so the tuner raises instead of running."""
        raise GrffeError("the batch autotuner is disabled: batches run the VALU contraction")
