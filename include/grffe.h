/* C ABI of the GRFFE DG-FD hot path on MI355X (gfx950).
 *
 * Method: Kim, Most, Throwe, Teukolsky, Deppe, "General relativistic
 * force-free electrodynamics with a discontinuous Galerkin-finite difference
 * hybrid method" (arXiv:2404.01531).  The library evaluates the semi-discrete
 * right-hand side of the augmented GRFFE system (Sec. II, Eqs. (evolved
 * variables), (fluxes), (sources), (electric current density)) on a grid of
 * affine Cartesian elements, each held either as a nodal DG-P_N element on
 * Legendre-Gauss-Lobatto points (Sec. III A) or as (2N+1)^3 finite-difference
 * subcells (Sec. III C 2), and advances it with the IMEX-SSP3(4,3,3) step and
 * the troubled-cell-indicator driven DG<->FD switching (Sec. III B, III C 1,
 * III C 3).
 *
 * Conventions shared by all entry points
 * --------------------------------------
 *  - Evolved variables are the densitized U = sqrt(gamma) (E^i, B^i, psi, phi, q),
 *    component order (Ex, Ey, Ez, Bx, By, Bz, psi, phi, q).
 *  - Elements are numbered e = ex + nx*(ey + ny*ez).  Within an element the DG
 *    node (i, j, k) is stored at i + n*(j + n*k), n = N+1 (xi^1 fastest); the FD
 *    cell (i, j, k) at i + m*(j + m*k), m = 2N+1.
 *  - DG arrays are [9][E][n^3] FP64, FD arrays [9][E][m^3] FP64, structure of
 *    arrays (component-major), all in device memory.  rep arrays are int32 [E]
 *    with 0 = DG, 1 = FD (excised elements are ignored and read as DG).
 *  - Every pointer argument marked "device" must point to device memory of the
 *    current HIP device; work is enqueued on `stream` (a hipStream_t, may be
 *    NULL for the default stream).  The library never retains or frees caller
 *    pointers.  Host pointers are only read during the call.
 *  - Return value: GRFFE_OK (0) or a negative status; the message of the last
 *    failure on the calling thread is returned by grffe_last_error().  No
 *    implicit device synchronisation happens except where a host value is
 *    returned (grffe_get_dt, grffe_get_counts, grffe_timing_read,
 *    grffe_check_finite) and in grffe_set_boundary_state and grffe_set_conductor,
 *    which wait for their host-to-device copies.
 *  - A domain is not thread-safe; separate domains are independent.
 */
#ifndef GRFFE_H
#define GRFFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRFFE_OK 0
#define GRFFE_EINVAL (-1)      /* bad shape, degree, parameter or pointer */
#define GRFFE_ENOMEM (-2)      /* device allocation failed */
#define GRFFE_EHIP (-3)        /* HIP runtime error */
#define GRFFE_ENONFINITE (-4)  /* the state holds NaN or infinite values (grffe_check_finite) */
#define GRFFE_EUNSUPPORTED (-5)

#define GRFFE_BC_PERIODIC 0
#define GRFFE_BC_NO_INCOMING_POYNTING 1 /* Sec. III D */
#define GRFFE_BC_DIRICHLET 2            /* exterior state held fixed: grffe_set_boundary_state */
#define GRFFE_BC_OUTFLOW 3              /* shell spheres only: no boundary condition, the exterior
                                           state is the interior one (the face adds nothing) */

#define GRFFE_PART_EXPLICIT 1 /* fluxes + non-stiff sources */
#define GRFFE_PART_STIFF 2    /* driver current + kappa damping (treated implicitly) */
#define GRFFE_PART_ALL 3

#define GRFFE_HYBRID_DG_ONLY 0  /* no indicator, every element stays DG */
#define GRFFE_HYBRID_ADAPTIVE 1 /* Sec. III C 1: indicator decides */
#define GRFFE_HYBRID_FORCED 2   /* representation fixed by a mask (Sec. IV D 2 style) */

/* Arithmetic of the right-hand side.  FP64 throughout, or mixed: the pointwise
 * fluxes, the DG derivative and lift contractions (accumulated in FP32) and the
 * FD face fluxes, Rusanov and corrector in FP32; the state and its stage
 * combinations, the sources, the implicit solve, the clamp, the filter, the
 * WENO5-Z reconstruction, the indicator and every DG<->FD transfer stay FP64. */
#define GRFFE_PRECISION_FP64 0
#define GRFFE_PRECISION_MIXED 1

/* Element grid (Sec. III A): an axis-aligned box [lower, upper] cut into
 * n_elem[0] x n_elem[1] x n_elem[2] equal elements of degree N (3 <= N <= 9).
 * bc[2d + s] is the boundary kind of the lower (s = 0) / upper (s = 1) face
 * along direction d; periodic faces must come in pairs.  excised (host, E
 * bytes, nullable) removes elements: their faces towards live elements take the
 * no-incoming-Poynting state with the normal pointing into the hole (also when the
 * grid's outer faces are Dirichlet faces). */
typedef struct grffe_grid {
  int32_t n_elem[3];
  double lower[3];
  double upper[3];
  int32_t degree;
  int32_t bc[6];
  const uint8_t* excised;
} grffe_grid;

/* Scheme parameters.  Zero-initialise and call grffe_default_params() first. */
typedef struct grffe_params {
  double eta;           /* driver relaxation rate, Eq. (electric current density) */
  double kappa_psi;     /* divergence-cleaning damping rates */
  double kappa_phi;
  double cfl;           /* CFL factor f of Eq. (spectre DG CFL condition) */
  double stab_c;        /* stepper constant c; 0 selects SSP-RK3's 1.2563726633 */
  int32_t tci_M;        /* modes removed by the indicator; 0 selects max(2, min(3, (N+1)/2)) */
  int32_t tci_mode;     /* 2: u - low-pass(u) (default); 1: only modes with all indices >= M */
  double tci_alpha;     /* exponent on DG (4) */
  double tci_alpha_fd;  /* exponent on FD (5) */
  double filter_a;      /* exponential filter, Eq. (exponential filter): a = 36, b = 50 */
  double filter_b;
  int32_t filter_on;
  int32_t fd_order;     /* 4: with the fourth-order flux corrector, 2: Rusanov flux only */
  double weno_eps;      /* WENO5-Z epsilon (1e-40) */
  int32_t ff_clamp;     /* 1: algebraic E.B = 0, E < B fix after every substep */
  double ff_margin;     /* E^2 <= (1 - margin) B^2 in the clamp */
  int32_t hybrid;       /* GRFFE_HYBRID_* */
  int32_t precision;    /* GRFFE_PRECISION_* */
} grffe_params;

typedef struct grffe_domain grffe_domain;

/* Fill *p with the paper's parameter values (eta = 1e6, kappa = 1, cfl = 0.25,
 * M auto, alpha = 4 / 5, a = 36, b = 50, WENO5-Z eps 1e-40, FD4 corrector,
 * clamp off, adaptive hybrid control). */
void grffe_default_params(grffe_params* p);

/* Create a domain.  bg (device, nullable) is the background metric at the DG
 * nodes, [26][E][n^3]: alpha; beta^x,y,z; gamma_xx,xy,xz,yy,yz,zz; d_x,y,z alpha;
 * d_j beta^i (j outer, i inner); K; Gamma^i = gamma^jk Gamma^i_jk (Sec. II A and
 * Appendix B).  NULL means flat space.  The library copies bg and derives the
 * metric at FD cell centres and faces by evaluating the nodal polynomial.
 * The state is zero and every element is DG until set.  Returns the domain in *out. */
int grffe_init_domain(const grffe_grid* grid, const grffe_params* params, const double* bg, void* stream,
                      grffe_domain** out);

/* Spherical shell of curved elements (Sec. IV B, the black-hole grid; Sec. III A,
 * the element map x(xi)).  The shell r_in <= r <= r_out is cut into six
 * cubed-sphere wedges about +x, -x, +y, -y, +z, -z (wedge w = 2k for +e_k, 2k + 1
 * for -e_k).  A wedge has coordinates (A, B, Z) in [-1, 1]^3 with the equiangular
 * angular map X = tan(pi A / 4), Y = tan(pi B / 4) and the logarithmic radial map
 * r = r_in (r_out / r_in)^((Z + 1) / 2); its local point r (X, Y, 1) /
 * sqrt(1 + X^2 + Y^2) is turned onto the axes (s e_{k+1}, e_{k+2}, s e_k),
 * s = +-1.  Each wedge is cut into n_radial x n_angular x n_angular elements of
 * equal extent in (A, B, Z): element e = ((w n_radial + ir) n_angular + ib)
 * n_angular + ia, E = 6 n_radial n_angular^2, its reference axes xi^1, xi^2, xi^3
 * along A, B, Z and its nodes ordered as on the box grid.  Faces f = 4 (xi^3 = -1)
 * of the innermost and f = 5 of the outermost elements lie on the spheres and take
 * bc_inner and bc_outer: GRFFE_BC_OUTFLOW, GRFFE_BC_DIRICHLET (per-node exterior
 * states, grffe_set_boundary_field) or GRFFE_BC_NO_INCOMING_POYNTING (along the
 * face normal).  Neighbours across wedge faces meet in other orientations; the
 * library matches their face nodes by position. */
typedef struct grffe_shell {
  int32_t degree;      /* 3 <= N <= 9 */
  int32_t n_radial;
  int32_t n_angular;   /* elements along each angular side of a wedge */
  double r_in, r_out;  /* 0 < r_in < r_out */
  int32_t bc_inner, bc_outer;
} grffe_shell;

/* Cartesian coordinates of the DG nodes (fd = 0, k = N + 1 per axis) or of the FD
 * cell centres (fd = 1, k = 2N + 1) of a shell: xyz (host, [3][E][k^3]), written by
 * the call; the caller evaluates the background and the initial data there. */
int grffe_shell_points(const grffe_shell* shell, int32_t fd, double* xyz);

/* Create a domain on a shell.  bg (device, nullable for flat space) as for
 * grffe_init_domain at the points grffe_shell_points(fd = 0) gives.  The DG
 * operator on curved elements is the strong form with the logical derivative of
 * each Cartesian flux component contracted with the inverse Jacobian at the node,
 * dU/dt = S - sum_{i,j} (d xi^i / d x^j) D_i F^j, and at every face node the lift
 * (1 / w_end) (G*(m) - m_j F^j) along the outward covector m = +-grad xi^i, with the
 * Rusanov flux G*(m) of speed alpha sqrt(gamma^{jk} m_j m_k) + |beta^j m_j|.  The
 * time step is Eq. (spectre DG CFL condition) with (dx)_min the smallest distance
 * between neighbouring nodes along a reference line and lambda_max the largest
 * alpha + |beta|_gamma.
 *
 * FD subcells on curved elements (Sec. III C 2, Eq. (fd time derivative)) with
 * params->hybrid GRFFE_HYBRID_FORCED or _ADAPTIVE: second order only (the
 * fourth-order corrector is Cartesian only), so params->fd_order must be 2.  Along
 * each reference direction xi^d the cell values of U and of the three components of
 * J~ are reconstructed with WENO5-Z; at a face, F-hat^j = (F^j(U_L) + F^j(U_R)) / 2
 * - lambda(nu) (U_R - U_L) nu_j / 2 for each Cartesian component j, with nu the
 * face's unit covector grad xi^d / |grad xi^d|; a cell adds
 * -(m / 2) sum_j (d xi^d / d x^j) (F-hat^j_{+} - F-hat^j_{-}) with the inverse
 * Jacobian at its centre.  Ghost cells are the neighbour's cells next to the shared
 * face in its own orientation (matched by position; across wedge faces their
 * positions differ from this element's grid continued past the face by up to about
 * one cell per layer), its P-projection if it is on DG, or on a sphere the outermost
 * own cell (outflow), its no-incoming-Poynting state, or ext_fd of
 * grffe_set_boundary_field (Dirichlet).  A DG face next to an FD element takes the
 * neighbour's R-trace at the matched node.  The indicator, rollbacks, switches back
 * and grffe_force_flags are those of the box grid.  These modes keep the host tables
 * of the cells and faces (about 150 doubles per cell) on the device.
 *
 * Shells run in FP64: params->precision must be GRFFE_PRECISION_FP64
 * (GRFFE_EUNSUPPORTED otherwise, and for FD modes with fd_order 4); the rotating
 * conductor, the adjoint, batches and the matrix-core contraction are not available
 * on shells.  grffe_init_from_fd, grffe_set_state / _get_state, grffe_rhs,
 * grffe_step, grffe_step_logged, grffe_get_dt, grffe_get_counts and
 * grffe_check_finite work as on the box grid. */
int grffe_init_shell(const grffe_shell* shell, const grffe_params* params, const double* bg, void* stream,
                     grffe_domain** out);

/* Exterior state of the grid's Dirichlet faces (the boundary condition of the
 * one-dimensional test problems, Sec. IV A: both ends of the x axis).  state (host,
 * [6][9], row f = 2d + s for the face of direction d and side s, components in the
 * state's order, densitized) is copied into the domain; the row of each face of
 * kind GRFFE_BC_DIRICHLET is the exterior state of the Rusanov flux at every DG node
 * of that face and the value of all three ghost layers of FD elements on it (with
 * its current J~ computed from it at the interior node's or cell's metric); the
 * other rows are not read.  The state is uniform over the face: an analytic state
 * that does not vary along the face and is constant in time at the face over the
 * evolved interval.  Entry points that evaluate the right-hand side (steps, RHS,
 * adjoints) return GRFFE_EINVAL on a domain with Dirichlet faces until this has
 * been called.  The adjoints treat the exterior state as a constant.  Returns
 * GRFFE_EINVAL for a NULL pointer or a non-finite value, GRFFE_EHIP if the copy
 * fails; the call returns after the copy has completed (stream order is kept). */
int grffe_set_boundary_state(grffe_domain* dom, const double* state, void* stream);

/* Exterior states of the Dirichlet faces given point by point (an analytic state
 * that varies along the face, constant in time), in place of the uniform rows of
 * grffe_set_boundary_state: ext_dg (device, [9][E][6][n^2]) holds the state at
 * every DG face node, node t1 + n t2 of face f of element e with (t1, t2) the
 * node's indices along the face's two tangential axes in increasing axis order;
 * ext_fd (device, [9][E][6][3][m^2]) the state at every FD ghost cell, layer
 * l = 0, 1, 2 counted outwards from face f, cell t1 + m t2.  Entries of faces that
 * are not Dirichlet faces are not read.  On a shell ext_fd may be NULL when every
 * element stays DG (GRFFE_HYBRID_DG_ONLY; GRFFE_EINVAL in the FD modes), and this is
 * the only way to set a Dirichlet sphere's states (grffe_set_boundary_state returns
 * GRFFE_EUNSUPPORTED there); there the ghost cells of layer l lie on the element's
 * map continued past the sphere, at reference coordinate +-(1 + (2 l + 1) / m).  Both arrays are
 * copied into the domain (allocated at the first call) on `stream`; a later grffe_set_boundary_state
 * does not undo this.  Returns GRFFE_EINVAL for NULL pointers, GRFFE_ENOMEM,
 * GRFFE_EHIP. */
int grffe_set_boundary_field(grffe_domain* dom, const double* ext_dg, const double* ext_fd, void* stream);

/* Rotating perfect conductor (Sec. IV C, the pulsar magnetospheres): after the
 * update of every substep of grffe_step, at each DG node or FD cell centre x of
 * the substep's result with |x - centre| <= radius, E~ is set to the value the
 * ideal condition E + v x B = 0 gives for the conductor's rigid rotation about the
 * z axis through centre, and psi~ and q~ are set to zero; B~ and phi~ are evolved
 * as everywhere else.  omega is the rotation relative to the grid: in flat space
 * with the grid at rest v = omega z^ x (x - centre); on a background (e.g. the
 * rotating frame of the star, shift beta = Omega z^ x x, where omega = 0 keeps the
 * star at rest on the grid) v = (omega z^ x (x - centre) + beta) / alpha, and
 * E_i = -[ijk] v^j B~^k, E~^i = sqrt(gamma) gamma^{ij} E_j.  The pre-stages U_1,
 * U_2 and grffe_rhs are not affected; the indicator, which reads |B~| only, sees
 * the same values either way.  centre is a host array of 3 doubles; radius <= 0
 * switches the conductor off.  The call copies what it needs (synchronises the
 * stream).  Returns GRFFE_EUNSUPPORTED for batch pools, GRFFE_EINVAL for a NULL
 * centre or non-finite values; the adjoint entry points refuse a domain with the
 * conductor on. */
int grffe_set_conductor(grffe_domain* dom, const double* centre, double radius, double omega, void* stream);

int grffe_destroy(grffe_domain* dom);

/* Set the state from FD subcell data u_fd (device, [9][E][m^3]), as at
 * start-up (Sec. III C 1): every element is reconstructed to DG and the
 * indicator with alpha_fd decides which stay FD (adaptive mode); in forced mode
 * `forced` (device uint8 [E], nullable) marks the FD elements; in DG-only mode
 * all go DG. */
int grffe_init_from_fd(grffe_domain* dom, const double* u_fd, const uint8_t* forced, void* stream);

/* Engine of the DG derivative contraction (Sec. III A, the tensor-product derivative
 * D along each axis of an element's fluxes) in the fused DG substep of FP64 domains:
 * GRFFE_CONTRACTION_VALU (default) contracts each node's line from LDS on the vector
 * ALUs; GRFFE_CONTRACTION_MFMA forms the contraction of every line of the element as
 * 16 x 16 x 4 FP64 matrix-core tiles.  The two give the same result up to the order of
 * the additions.  The mixed-precision mode, and degree 9, always use the VALU form.  Returns
 * GRFFE_EINVAL for an unknown engine. */
#define GRFFE_CONTRACTION_VALU 0
#define GRFFE_CONTRACTION_MFMA 1
int grffe_set_contraction(grffe_domain* dom, int engine);

/* Host-forced indicator flags, a test instrument (fault injection): mask (device
 * uint8 [3][E], row k - 1 for substep k) marks elements that the adaptive step
 * (GRFFE_HYBRID_ADAPTIVE) treats as troubled in substep k of every following step
 * whatever their indicator ratio, so that the rollback of Sec. III C 1 (discard the
 * DG candidate, project the element's registers with P, redo the substep on FD) can
 * be made to happen in any substep; elements already on FD ignore it.  The mask is
 * copied into the domain (allocated at the first call) on `stream`; mask = NULL
 * switches the forcing off.  The frozen step adjoint re-runs its forward step with
 * the same forcing.  Returns GRFFE_ENOMEM or GRFFE_EHIP on failure. */
int grffe_force_flags(grffe_domain* dom, const uint8_t* mask, void* stream);

/* Copy the state in / out.  dg [9][E][n^3], fd [9][E][m^3] and rep [E] are device
 * pointers; on set, only the representation named by rep is read per element (all
 * three non-NULL); on get, a NULL pointer skips that part. */
int grffe_set_state(grffe_domain* dom, const double* dg, const double* fd, const int32_t* rep, void* stream);
int grffe_get_state(grffe_domain* dom, double* dg, double* fd, int32_t* rep, void* stream);

/* Semi-discrete right-hand side dU/dt (Sec. II A fluxes and sources; DG operator of
 * Sec. III A, FD subcell operator of Sec. III C 2 with the fourth-order corrector)
 * of every live element in its representation given by rep (a pure function of the
 * arguments; the domain's own state is not touched).  parts = GRFFE_PART_*.  Outputs have the layouts of
 * the inputs; entries of the other representation are left unchanged. */
int grffe_rhs(grffe_domain* dom, const double* dg, const double* fd, const int32_t* rep, double* ddg, double* dfd,
              int parts, void* stream);

/* Advance the domain's state by n_steps IMEX-SSP3(4,3,3) steps of size dt
 * (dt <= 0 selects the CFL step of Eq. (spectre DG CFL condition)), with the
 * hybrid control of Sec. III C 1 inside every step. */
int grffe_step(grffe_domain* dom, int n_steps, double dt, void* stream);

/* One step as grffe_step, with its decision log: rep_log (device int32 [5][E],
 * caller-owned) receives the representation before the step, after substeps 1, 2
 * and 3 (an element rolled back in substep k is FD from row k on) and after the step
 * (the switches back of Sec. III C 1).  For a parity harness that compares the
 * hybrid decisions of two implementations and replays the other side's decision
 * where an indicator ratio lies within rounding of its threshold.  dt <= 0 selects
 * the CFL step. */
int grffe_step_logged(grffe_domain* dom, double dt, int32_t* rep_log, void* stream);

/* Troubled-cell indicator, Eq. (persson tci), on |B~| = sqrt(gamma_ij B~^i B~^j):
 * DG elements (rep 0) are checked on dg with alpha, FD elements (rep 1) on the
 * reconstruction of fd (the least-squares inverse of the projection) with alpha_fd.  troubled (device uint8 [E]);
 * ratio (device double [E], nullable) receives sqrt(sum u_hat^2 / sum u^2). */
int grffe_tci(grffe_domain* dom, const double* dg, const double* fd, const int32_t* rep, uint8_t* troubled,
              double* ratio, void* stream);

/* DG -> FD projection (evaluation of the nodal polynomial at the subcell
 * centres, Sec. III C 2) and FD -> DG reconstruction, the least-squares inverse
 * of that projection (degree N, Sec. III C 1) of the n listed elements.  Compact layouts: u_dg [9][n][n^3],
 * u_fd [9][n][m^3]; elems (device int32 [n]) only selects the element degree and
 * must hold valid element ids. */
int grffe_project_dg_to_fd(grffe_domain* dom, const double* u_dg, double* u_fd, const int32_t* elems, int32_t n,
                           void* stream);
int grffe_reconstruct_fd_to_dg(grffe_domain* dom, const double* u_fd, double* u_dg, const int32_t* elems,
                               int32_t n, void* stream);

/* Time step of Eq. (spectre DG CFL condition) (host value; synchronises). */
int grffe_get_dt(grffe_domain* dom, double* dt);

/* Scan the domain's state for blow-up: every live element's values in its own
 * representation (DG nodes or FD cells).  *n_bad (host, nullable) receives the
 * number of elements holding a NaN or infinite value.  Returns GRFFE_ENONFINITE when
 * that number is positive, GRFFE_OK otherwise; synchronises `stream`.  The first
 * call allocates an E-byte work array. */
int grffe_check_finite(grffe_domain* dom, int32_t* n_bad, void* stream);

/* grffe_check_finite for callers that cannot allocate device memory (code that
 * runs where hipMalloc is not allowed, such as a tight serving loop or a harness
 * that forbids it): the same scan and status, with the per-element flags and their
 * count kept in a fixed device array of the library (1 MiB + 256 B per device,
 * held until the process ends, looked up once per device) instead of the work
 * array grffe_check_finite allocates at its first call.  The call allocates no
 * device memory.  Domains of more than 1048576 elements are refused
 * (GRFFE_EINVAL).  Every call on one device shares that array: calls that overlap
 * on one device (several streams or host threads) race; the array keeps the last
 * call's flags, and each call reads only what it wrote.  Synchronises `stream`. */
int grffe_check_finite_noalloc(grffe_domain* dom, int32_t* n_bad, void* stream);

/* Number of live elements on DG and on FD (host values; synchronises). */
int grffe_get_counts(grffe_domain* dom, int32_t* n_dg, int32_t* n_fd);

/* Host copies of the library's 1D operators for degree N, row-major:
 * which = 0 GLL nodes (n), 1 GLL weights (n), 2 derivative matrix (n x n),
 * 3 filter (n x n), 4 low-pass (n x n), 5 projection P (m x n),
 * 6 reconstruction R (n x m), 7 face evaluation (m+1 x n).  Returns the number
 * of doubles written (out may be NULL to query). */
int grffe_operator(int degree, int which, double* out, int capacity);

/* Kernel timing with HIP events attached to every launch of the selected kernel
 * families (the events bracket the kernel's own dispatch on its launch stream).
 * Families: 1 fused DG substep, 2 FD face fluxes, 3 FD update, 4 FD stage
 * values, 5 FD traces, 6 DG ghost slabs, 7 DG->FD projection of flagged
 * elements, 8 FD->DG check, 9 DG pre-stage pass.  mask = OR of (1 << family),
 * 0 = off; enabling resets every counter.  grffe_timing_read synchronises the
 * stream of the last timed launch, returns the summed duration (ms) and the
 * number of timed launches of one family, and resets that family's counters. */
int grffe_timing_enable(grffe_domain* dom, int mask);
/* Attach the timing events to the launches of one step in every `period` steps
 * (the first step after this call, then every period-th; default 1: every step):
 * the events add a few microseconds to each timed launch, sampling keeps that out
 * of the rest.  EINVAL for period < 1. */
int grffe_timing_period(grffe_domain* dom, int period);
int grffe_timing_read(grffe_domain* dom, int family, double* total_ms, int64_t* launches);

/* Adjoint of the right-hand side (a vector-Jacobian product), with the
 * representation frozen:  ubar += (d RHS_parts / d u)^T lam, where RHS_parts is
 * the semi-discrete right-hand side of grffe_rhs restricted to `parts` (fluxes,
 * DG derivative and lift or FD WENO5-Z reconstruction, Rusanov faces and the
 * corrector, the no-incoming-Poynting boundary state, non-stiff and stiff sources
 * of Sec. II and III) and u is the pair (DG nodal values of the elements on DG, FD
 * cell values of the elements on FD) chosen by rep, any mix of the two: the
 * DG-FD coupling (P-projected ghost slabs, R-traces; Sec. III C) is transposed
 * too.  Layouts as grffe_rhs; lam_dg / ubar_dg are read / accumulated on the DG
 * elements and lam_fd / ubar_fd on the FD elements, the other entries are left
 * untouched.  All device pointers non-NULL.  The first call allocates the work
 * space (about 40 doubles per FD cell of the domain).  EUNSUPPORTED in mixed
 * precision or with the clamp on. */
int grffe_rhs_adjoint(grffe_domain* dom, const double* dg, const double* fd, const int32_t* rep, const double* lam_dg,
                      const double* lam_fd, double* ubar_dg, double* ubar_fd, int parts, void* stream);

/* Adjoint of one IMEX-SSP3(4,3,3) step (Sec. III B) taken with every element on
 * DG and no switching (the hybrid decisions frozen to DG):
 *   lam = (d U^{n+1} / d U^n)^T lam_next,
 * through the explicit operator, the implicit solves (by the implicit function
 * theorem), the stiff sources and the filter.  u_dg (device [9][E][n^3]) is U^n;
 * the domain re-runs the forward step from it, so its state is left at U^{n+1}
 * with every element on DG.  dt <= 0 selects the CFL step.  lam may be the same
 * buffer as lam_next; neither may overlap u_dg; the entries of excised elements are
 * not written.  Same restrictions as
 * grffe_rhs_adjoint; the first call allocates the adjoint's work space
 * (7 arrays of the DG state's size). */
int grffe_step_adjoint(grffe_domain* dom, const double* u_dg, const double* lam_next, double* lam, double dt,
                       void* stream);

/* The DG stage values U_3 and U_4 of the domain's last step (device [9][E][n^3]
 * each; either may be NULL), for grffe_step_adjoint_stages. */
int grffe_get_stages(grffe_domain* dom, double* u3, double* u4, void* stream);

/* grffe_step_adjoint with the step's stage values given instead of regenerated:
 * u_dg is U^n and u3, u4 its U_3, U_4 (from grffe_get_stages after the step from
 * u_dg with the same dt); the forward step is not re-run and the domain's state is
 * left as it was.  Every element on DG; the same restrictions and work space as
 * grffe_step_adjoint.  For checkpointed gradients whose segment recomputation
 * already produces the stages. */
int grffe_step_adjoint_stages(grffe_domain* dom, const double* u_dg, const double* u3, const double* u4,
                              const double* lam_next, double* lam, double dt, void* stream);

/* Adjoint of one IMEX-SSP3(4,3,3) step (Sec. III B) with the hybrid decisions
 * (Sec. III C 1) frozen from the forward pass:
 *   (lam_dg, lam_fd) = (d U^{n+1} / d U^n)^T (mu_dg, mu_fd).
 * The domain re-runs the forward step from (dg, fd, rep) in its own hybrid mode and
 * logs the representation before each substep and after the step; the adjoint
 * then takes every element through the same path: DG or FD per substep, the
 * rollback of an element flagged in substep k (its registers projected by P, its
 * FD pre-stages re-derived, transposed through P^T), the switch back at the end of
 * the step (R, transposed through R^T).  Each stage is transposed on both
 * representations: the DG operator and filter, the FD WENO5-Z fluxes, the
 * P-projected ghost slabs and R-traces between them (Sec. III C), the implicit
 * solves (implicit function theorem) and the stiff sources.  The indicator itself
 * is not differentiated (a piecewise-constant decision).
 * U = (DG nodal values of the DG elements, FD cell values of the FD elements) as in
 * grffe_rhs_adjoint: dg, fd, rep are U^n and its representation (device, layouts
 * of grffe_set_state); mu_* are given in the representation after the step (the
 * domain's rep after the call: the re-run leaves the state at U^{n+1}); lam_* are
 * returned in rep's representation, entries of elements in the other one left
 * untouched.  rep_log (nullable, device [5][E]) receives the representation before
 * the step, during substeps 1-3 and after the step.  dt <= 0 selects the CFL step.
 * lam_* may be the same buffers as mu_*; none may overlap dg or fd.  Same
 * restrictions as grffe_rhs_adjoint; the first call allocates the work space
 * (8 DG-sized and 10 FD-sized arrays besides that of grffe_rhs_adjoint). */
int grffe_step_adjoint_frozen(grffe_domain* dom, const double* dg, const double* fd, const int32_t* rep,
                              const double* mu_dg, const double* mu_fd, double* lam_dg, double* lam_fd,
                              int32_t* rep_log, double dt, void* stream);

/* Batches: many independent domains advanced together, each with its own grid,
 * degree (3..9) and CFL time step (Eq. (spectre DG CFL condition) per domain).
 * Domains of one degree are concatenated into one pool, so every kernel of a step
 * is one launch over the elements of all of them; pools of different degrees run
 * on concurrent branches of a HIP graph that holds one step of the whole batch.
 * All grids share `params`; bgs (host array of `count` device pointers, each
 * [26][E_k][n_k^3] as for grffe_init_domain) is NULL for flat space, otherwise
 * every entry is non-NULL.  Domain k is addressed by its index in `grids`.  Grids
 * with Dirichlet faces are refused (GRFFE_EUNSUPPORTED). */
typedef struct grffe_batch grffe_batch;
int grffe_batch_create(const grffe_grid* grids, int32_t count, const grffe_params* params,
                       const double* const* bgs, void* stream, grffe_batch** out);
int grffe_batch_destroy(grffe_batch* batch);
/* Number of domains and of degree pools (host values). */
int grffe_batch_size(grffe_batch* batch, int32_t* n_domains, int32_t* n_pools);
/* Start-up of every domain from FD data, as grffe_init_from_fd: u_fd is a host
 * array of `count` device pointers ([9][E_k][m_k^3]); forced (host array,
 * nullable, entries nullable) holds device uint8 [E_k] masks in forced mode. */
int grffe_batch_init_from_fd(grffe_batch* batch, const double* const* u_fd, const uint8_t* const* forced,
                             void* stream);
/* State of domain k in the layouts of grffe_get_state / grffe_set_state. */
int grffe_batch_get_state(grffe_batch* batch, int32_t k, double* dg, double* fd, int32_t* rep, void* stream);
int grffe_batch_set_state(grffe_batch* batch, int32_t k, const double* dg, const double* fd, const int32_t* rep,
                          void* stream);
/* CFL time step of domain k (host value, no synchronisation). */
int grffe_batch_get_dt(grffe_batch* batch, int32_t k, double* dt);
/* Live elements of domain k on DG and on FD (host values; synchronises the device). */
int grffe_batch_get_counts(grffe_batch* batch, int32_t k, int32_t* n_dg, int32_t* n_fd);
/* Advance every domain by n_steps steps of its own CFL time step.  use_graph = 1
 * replays the captured one-step graph (captured at the first such call on a
 * library-owned stream, launched on `stream`); 0 enqueues the same kernels
 * directly.  The two give identical results. */
int grffe_batch_step(grffe_batch* batch, int32_t n_steps, int32_t use_graph, void* stream);

/* Contraction engine (GRFFE_CONTRACTION_*, as grffe_set_contraction) of the batch's
 * pool of degree `degree`, or of every pool for degree = 0.  Batches run the VALU
 * engine: GRFFE_CONTRACTION_MFMA returns GRFFE_EUNSUPPORTED (a step graph re-captured
 * after an engine change, with matrix-core pools, ended in an abort inside the HIP
 * runtime once; its cause is not known), so the captured graph is never dropped.
 * Returns GRFFE_EINVAL for an unknown engine or a degree with no pool. */
int grffe_batch_set_contraction(grffe_batch* batch, int32_t degree, int32_t engine);
int grffe_batch_get_contraction(grffe_batch* batch, int32_t degree, int32_t* engine);

const char* grffe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GRFFE_H */
