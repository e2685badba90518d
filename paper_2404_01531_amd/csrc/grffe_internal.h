// Internal declarations of the GRFFE library: domain layout in HBM, kernel
// argument blocks and launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/grffe.h"

namespace grffe {

constexpr int NV = 9;      // evolved components
constexpr int NW = 12;     // evolved components + densitized current J~
constexpr int NBG = 26;    // background fields at DG nodes / FD cells
constexpr int NBGF = 10;   // background fields at FD faces (alpha, beta, gamma)
constexpr int MAX_DEG = 9; // largest degree with a fused DG kernel
constexpr int NBR_OUTFLOW = -8;  // neighbour code of a face with no boundary condition

// IMEX-SSP3(4,3,3) (Pareschi & Russo 2005): implicit diagonal a, and b, e of the last row.
constexpr double IMEX_A = 0.24169426078821;
constexpr double IMEX_B = 0.06042356519705;
constexpr double IMEX_E = 0.12915286960590;

struct Ops1D {
  int N = 0;
  std::vector<double> x, w, D, F, L, P, Q, R;
};

Ops1D build_ops(int N, double filter_a, double filter_b, int tci_M, int tci_mode);

// Host geometry of a spherical shell (shell.cpp): node coordinates, inverse
// Jacobian, neighbours (with the boundary codes of the spheres) and the matched
// neighbour node of every face node, the smallest node distance.
struct ShellGeom {
  int E = 0;
  std::vector<double> jinv;     // [9][E][n^3]
  std::vector<int32_t> nbr;     // [E][6]
  std::vector<int32_t> fnode;   // [E][6][n^2]
  double dx_min = 0.0;
  // FD subcells (built by shell_fd_geometry when elements may go to FD)
  std::vector<int32_t> nface;   // [E][6] the neighbour's face towards e
  std::vector<int32_t> fcell;   // [E][6][m^2] the neighbour's face cell at face cell t1 + m t2
  std::vector<double> jinv_fd;  // [9][E][m^3] inverse Jacobian at the cell centres
  std::vector<double> nu_face;  // [3][3][E][(m+1) m^2] unit covector grad xi^d / |grad xi^d| at the faces
};
int shell_validate(const grffe_shell* s, std::string& err);
void shell_points(const grffe_shell& s, bool fd, std::vector<double>& xyz);
int shell_geometry(const grffe_shell& s, ShellGeom& g, std::string& err);
int shell_fd_geometry(const grffe_shell& s, ShellGeom& g, std::string& err);
void gll_nodes_weights(int N, std::vector<double>& x, std::vector<double>& w);
int default_tci_M(int N);

// Operators in device memory (row-major), sized for MAX_DEG.
struct DevOps {
  double w[MAX_DEG + 1];
  double D[(MAX_DEG + 1) * (MAX_DEG + 1)];
  double F[(MAX_DEG + 1) * (MAX_DEG + 1)];
  double L[(MAX_DEG + 1) * (MAX_DEG + 1)];
  double P[(2 * MAX_DEG + 1) * (MAX_DEG + 1)];
  double R[(MAX_DEG + 1) * (2 * MAX_DEG + 1)];
};

enum Mode { MODE_RHS = 0, MODE_SUB1 = 1, MODE_SUB2 = 2, MODE_SUB3 = 3 };

// Register set of one representation: U^n, the two stage values, the accumulator.
struct Regs {
  double* Un;
  double* X0;  // U_3 (written in substep 1)
  double* X1;  // U_2 (written by the pre-stage pass), then U_4 (written in substep 2)
  double* A;   // accumulated increments
  double* K;   // [10][E][P] stiff-source terms of substeps 2 and 3 (pre-stage pass), or null
};

// Components of the stiff source that can be non-zero (E~ and psi~, phi~).
constexpr int NK = 5;
__host__ __device__ constexpr int stiff_comp(int k) { return k < 3 ? k : k + 3; }

// Everything a kernel needs; passed by value.
struct KArgs {
  int E;
  const double* eh;        // [E][3] element widths
  const double* edt;       // [E] time step of the element's domain
  const int32_t* nbr;      // [E][6]: neighbour, -1 at a no-incoming-Poynting boundary,
                           // -2 - slot at a Dirichlet face (exterior state bstate[slot]),
                           // NBR_OUTFLOW at an outflow sphere of a shell
  const double* bstate;    // [slots][9] exterior states of Dirichlet faces
  const double* bfield_dg; // [9][E][6][n^2] per-node exterior states of Dirichlet faces, or null
  const double* bfield_fd; // [9][E][6][3][m^2] per-ghost-cell exterior states, or null
  const uint8_t* live;     // [E]
  const double* bg_dg;     // [26][E][n^3] or null
  const float* bg_dg32;    // the same rounded to FP32 (mixed precision on a curved background), or null
  const double* bg_fd;     // [26][E][m^3] or null
  const double* bg_face;   // [3][10][E][(m+1) m^2] or null
  const DevOps* ops;
  // curved element maps (shells), else null: the inverse Jacobian d xi^i / d x^j
  // [9][E][n^3] (row i, column j: component 3 i + j) and, per face node, the node
  // of the neighbour at the same point [E][6][n^2] (flat index in that element)
  const double* jinv;
  const int32_t* fnode;
  const int32_t* nface;     // shells with FD subcells: [E][6]
  const int32_t* fcell;     // [E][6][m^2]
  const double* jinv_fd;    // [9][E][m^3]
  const double* nu_face;    // [3][3][E][(m+1) m^2]
  // state
  Regs dg, fd;
  int32_t* rep0;           // representation at the start of the substep
  int32_t* rep;            // representation being built
  uint8_t* troubled;       // [E] flags of the current substep
  const uint8_t* force;    // [3][E] host-forced indicator flags of substeps 1..3, or null
  double* ratio;           // [E] indicator ratios (diagnostic)
  // scratch
  double* w_fd;            // [12][E][m^3]  FD stage values + J~
  double* trace;           // [12][E][6][n^2]  R-traces of FD elements at their faces
  double* slab;            // [12][E][6][3 m^2]  P-projection of DG stage values next to each face
  double* fhat;            // [3][9][E][m^3] FD flux differences per direction
  // RHS mode outputs
  double* out_dg;
  double* out_fd;
  int parts;
  // scheme parameters; dt > 0 overrides the per-element time steps
  double dt, eta, kpsi, kphi;
  double tci_thr, tci_thr_fd;
  int tci_mode, filter_on, fd_order, ff_clamp, hybrid, precision;
  int contraction;         // GRFFE_CONTRACTION_*: DG derivative on the VALU from LDS, or on the matrix cores
  double weno_eps, ff_margin;
  // work list of the FD kernels: element ids fd_list[0 .. fd_count[sub]), where sub
  // is 0 for the substeps of a step (one list per step) and 3 for a right-hand
  // side evaluation or an adjoint stage
  int32_t* fd_list;
  int32_t* fd_count;
  int sub;
};

// The rotating conductor's kernel arguments.
struct CondArgs {
  const int32_t* list;   // [count] elements that may hold a point of the sphere
  const double* corner;  // [count][3] lower corners of those elements
  const double* ref;     // [N + 1] GLL nodes on [-1, 1]
  int count;
  double cx, cy, cz, r2, omega;  // centre, radius squared, angular velocity about z
};

}  // namespace grffe

// One grid of a pool (a batch concatenates several grids of one degree).
struct grffe_part {
  int off, E, nx, ny, nz;
  double h[3];
  double dt;
  double lambda_max;
};

struct grffe_domain {
  int N, n, m, nn, mm;
  int E, nx, ny, nz;
  std::vector<grffe_part> parts;
  double lower[3], upper[3], h[3];
  int bc[6];
  int bc_missing = 0;         // Dirichlet faces whose exterior state is not set (bit f)
  grffe_params par;
  bool curved;
  bool mapped = false;          // a shell of curved elements (grffe_init_shell)
  double* jinv = nullptr;       // [9][E][n^3] inverse Jacobian (shells)
  int32_t* fnode = nullptr;     // [E][6][n^2] neighbour node of each face node (shells)
  int32_t* nface = nullptr;     // FD subcells on shells: the tables of ShellGeom
  int32_t* fcell = nullptr;
  double* jinv_fd = nullptr;
  double* nu_face = nullptr;
  std::vector<int32_t> nbr_h;
  std::vector<uint8_t> live_h;
  int32_t* nbr = nullptr;
  double* bstate = nullptr;   // [6][9] exterior states of the Dirichlet faces
  double* bfield_dg = nullptr;  // per-point exterior states (grffe_set_boundary_field)
  double* bfield_fd = nullptr;
  uint8_t* bad_flags = nullptr;  // [E] scratch of grffe_check_finite
  uint8_t* force = nullptr;      // [3][E] forced indicator flags (grffe_force_flags)
  int contraction = 0;           // GRFFE_CONTRACTION_* of the DG substep (grffe_set_contraction)
  bool force_on = false;
  // rotating perfect conductor (grffe_set_conductor): the elements meeting its
  // sphere, their lower corners, the GLL nodes; off while cond_count == 0
  int cond_count = 0;
  int32_t* cond_list = nullptr;
  double* cond_corner = nullptr;
  double* cond_ref = nullptr;
  double cond_c[3] = {0.0, 0.0, 0.0};
  double cond_r = 0.0, cond_omega = 0.0;
  uint8_t* live = nullptr;
  double* eh = nullptr;   // [E][3]
  double* edt = nullptr;  // [E]
  std::vector<double> eh_h, edt_h;
  double* bg_dg = nullptr;
  float* bg_dg32 = nullptr;  // FP32 copy of bg_dg read by the mixed-precision DG substep
  double* bg_fd = nullptr;
  double* bg_face = nullptr;
  grffe::DevOps* ops = nullptr;
  grffe::Ops1D ops_h;
  grffe::Regs dg{}, fd{};
  int32_t* rep = nullptr;
  int32_t* rep0 = nullptr;
  uint8_t* troubled = nullptr;
  double* ratio = nullptr;
  double* w_fd = nullptr;
  double* trace = nullptr;
  double* slab = nullptr;
  double* fhat = nullptr;
  int32_t* fd_list = nullptr;   // [E] work list of the FD kernels
  int32_t* fd_count = nullptr;  // [4] list lengths (0: the step's list, 3: right-hand side / adjoint)
  double* adj_ws = nullptr;  // step adjoint: 6 DG-sized arrays, allocated at first use
  double* adj_u0 = nullptr;  // step adjoint: copy of U^n
  double* adj_fd_wbar = nullptr;  // FD adjoint: [3][10][E][m^3]
  double* adj_fd_gbar = nullptr;  // FD adjoint: [10][E][6][3][m^2]
  double* adj_fd_ws = nullptr;    // step adjoint with FD elements: 6 FD-sized arrays
  double* adj_u0_fd = nullptr;    // and the FD copy of U^n
  double* adj_extra = nullptr;    // and the slab transposes of one stage (DG-sized)
  double* adj_hyb = nullptr;      // adaptive steps: U^n adjoints (DG, FD), transfers (DG, FD), mu_fd copy
  int32_t* adj_rep_log = nullptr; // representation before each substep and after the step [5][E]
  double dt_cfl = 0.0;
  double lambda_max = 0.0;
  std::vector<void*> allocs;
  // kernel timing (one family at a time)
  // kernel timing: bit f of timed_mask times family f (1..9)
  static constexpr int NFAM = 10;
  int timed_mask = 0;
  // events on the launches of one step in every timing_period steps
  int timing_period = 1;
  int64_t timing_step = 0;
  bool timing_now = true;
  std::vector<hipEvent_t> ev[NFAM];  // start/stop pairs per family
  size_t ev_used[NFAM] = {};
  hipStream_t ev_stream = nullptr;
};

namespace grffe {

KArgs make_args(grffe_domain* d);

// Event pair armed for the next kernel launch on this host thread (kernel timing).
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
LaunchEvents& armed_launch_events();

// launchers (kernels_mapped.hip)
void launch_dg_mapped(const KArgs& a, int N, bool curved, int mode, bool hybrid, hipStream_t s);
void launch_fd_flux_mapped(const KArgs& a, int N, bool curved, hipStream_t s);
// launchers (kernels_dg.hip)
void launch_dg_substep(const KArgs& a, int N, bool curved, int mode, hipStream_t s);
void launch_dg_slab(const KArgs& a, int N, bool curved, int mode, hipStream_t s);
void launch_dg_prestage(const KArgs& a, int N, bool curved, hipStream_t s);
void launch_to_float(const double* in, float* out, size_t count, hipStream_t s);
// launchers (kernels_fd.hip)
void launch_fd_stage(const KArgs& a, int N, bool curved, int mode, hipStream_t s);
void launch_fd_trace(const KArgs& a, int N, hipStream_t s);
void launch_project_troubled(const KArgs& a, int N, bool curved, int mode, hipStream_t s);
void launch_fd_flux(const KArgs& a, int N, bool curved, hipStream_t s);
void launch_fd_update(const KArgs& a, int N, bool curved, int mode, hipStream_t s);
void launch_fd_to_dg(const KArgs& a, int N, bool curved, int init, hipStream_t s);
void launch_begin_substep(const KArgs& a, bool copy, hipStream_t s);
void launch_tci(const KArgs& a, int N, bool curved, const double* dg, const double* fd, const int32_t* rep,
                uint8_t* troubled, double* ratio, hipStream_t s);
void launch_transfer(const KArgs& a, int N, int to_fd, const double* in, double* out, int count, hipStream_t s);
void launch_bg_derive(const KArgs& a, int N, hipStream_t s);
void launch_lambda_max(const KArgs& a, int N, double* out, hipStream_t s);
// launchers (kernels_adj.hip)
// Stages of the step adjoint (the step's substeps backwards) and of the RHS adjoint.
enum AdjStage { ADJ_A3 = 0, ADJ_B1 = 1, ADJ_B2 = 2, ADJ_B3 = 3, ADJ_RHS = 4 };

// Adjoint registers of one representation ([9][E][P] each, P = n^3 on DG, m^3 on FD).
struct AdjBufs {
  const double* mu;      // adjoint of U^{n+1} (input of the step adjoint), or lambda of the RHS adjoint
  double* un_bar;        // adjoint of U^n (output)
  double* a_bar;         // adjoint of the accumulator
  double* s1_bar;        // adjoint of S_stiff(U_1)
  double* s2_bar;        // adjoint of S_stiff(U_2)
  double* v_in;          // vector the transposed explicit operator is applied to (read by neighbours)
  double* v_out;         // the next stage's vector
  double* w;             // vector the transposed stiff source is applied to (pointwise)
  const double* extra;   // DG only, nullable: adjoint contributions of the ghost slabs at this stage
  // Step adjoint with the decisions of an adaptive step frozen (nullable: the
  // representation does not change within the substep).  a.rep0 is the
  // representation at the start of the substep whose operator a stage transposes
  // (what neighbours read, and the one of the combination the stage transposes);
  // rep_upd the one that updated each element in that substep.  An element on DG in
  // rep0 and on FD in rep_upd was rolled back there: its DG neighbours read its DG
  // values and its FD neighbours its ghost slab, while it was updated on FD from
  // its projected registers.  The FD stage kernel writes the adjoint of its
  // substep input to `transfer` (FD) and stops; the DG stage kernel takes
  // `transfer` (DG, after P^T) and the neighbours' terms in place of its own
  // operator adjoint.
  const int32_t* rep_upd;
  double* transfer;
  int parts;             // RHS adjoint: GRFFE_PART_* of lambda
};

void launch_rhs_adjoint(const KArgs& a, int N, bool curved, const double* lam, double* ubar, int parts,
                        hipStream_t s);
void launch_dg_adjoint_stage(const KArgs& a, int N, bool curved, int stage, const AdjBufs& b, hipStream_t s);
void launch_step_adjoint(const KArgs& a, int N, bool curved, const double* mu, double* lam, double* ws,
                         hipStream_t s);
// launchers (kernels_fd_adj.hip)
void launch_fd_rhs_adjoint(const KArgs& a, int N, bool curved, const double* lam, double* ubar,
                           const double* lam_dg, double* ubar_dg, int parts, double* wbar, double* gbar,
                           hipStream_t s);
// step adjoint with FD elements: the couplings and the flux adjoint of one stage
// (V vectors v_fd, v_dg; slab transposes added to extra_dg), then the FD cells' stage
void launch_fd_step_coupling(const KArgs& a, int N, bool curved, const double* v_fd, const double* v_dg,
                             const double* x_dg, double* extra_dg, double* wbar, double* gbar,
                             const int32_t* rep_upd, hipStream_t s);
void launch_fd_step_stage(const KArgs& a, int N, bool curved, int stage, const AdjBufs& r, double* wbar,
                          double* gbar, hipStream_t s);
// launchers (kernels_adj_hybrid.hip): the frozen decisions of an adaptive step
void launch_adj_rollback(const KArgs& a, int N, bool curved, const AdjBufs& rd, const AdjBufs& rf,
                         const int32_t* rep_upd, const double* t_fd, double* t_dg, int k, hipStream_t s);
void launch_adj_flags(const KArgs& a, const int32_t* rep_upd, hipStream_t s);
void launch_adj_switch_back(const KArgs& a, int N, const int32_t* rep3, const int32_t* repF, const double* mu_dg,
                            double* mu_fd, hipStream_t s);
void launch_adj_project_un(const KArgs& a, int N, const int32_t* rep0, const int32_t* rep3, const double* un_dg,
                           double* un_fd, hipStream_t s);
void launch_copy_rep(const KArgs& a, const int32_t* rep, int want, int P, const double* src, double* dst,
                     hipStream_t s);

}  // namespace grffe
