/*
 * dg.h -- C ABI of the MI355X matrix-free discontinuous Galerkin library.
 *
 * The library evaluates, on one gfx950 GPU, the hot path of a high-order
 * modal DG discretisation of the compressible Navier-Stokes equations with
 * BR2 viscous fluxes (Franciolini, Botti, Colombo, Crivellini,
 * arXiv:1809.00866):
 *
 *   dg_residual             residual f_h of eq. (NSdiscrRes), Sec. 2.2
 *   dg_jvp                  Jacobian-vector product j_h (Sec. 2.2), exact
 *                           tangent or the finite difference of
 *                           eqs. (matrix-free)/(epsdef), Sec. 2.3
 *   dg_block_precond_setup  element-wise block Jacobi (EWBJ, Sec. 2.3):
 *   dg_block_precond_apply  LU of the diagonal blocks of G = shift*I + J
 *   dg_fgmres_solve         flexible GMRES (Sec. 2.5) on G dw = b,
 *                           eq. (rosSysOp) with M = I (orthonormal basis)
 *   dg_rosenbrock_step      one linearly implicit stage loop (Alg. ros)
 *                           with caller-supplied coefficients
 *   dg_mg_setup             p-multigrid V-cycle or full cycle (Sec. 2.4,
 *   dg_mg_apply             Alg. vcic / fullvcic) with inherited or
 *                           rescaled-inherited coarse operators (eq. GalProj,
 *                           App. A) and GMRES[EWBJ] smoothers
 *   dg_mg_update_fine       preconditioner lagging: new fine state, coarse
 *                           levels kept (Sec. 4)
 *   dg_mlp_*                learned element-local preconditioner, usable
 *                           because the outer solver is flexible (Sec. 2.5)
 *
 * Meshes: periodic, conforming, multilinear elements (Sec. 2.1).  Uniform
 * axis-aligned lattices run MFMA kernels (3D P2-P4); any other such mesh
 * runs the curved-element kernels, each element with its own orthonormal
 * basis.
 *
 * Conventions (all entry points):
 *  - Every vector is FP64, device memory, caller-owned, contiguous, in the
 *    DOF layout  idx(e, c, b) = (c*Nb + b)*n_elem + e  (element index
 *    fastest; c = conserved variable rho, rho*u_1..d, rho*E; b = mode).
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  Calls are stream-ordered and asynchronous unless stated.
 *  - Inputs and outputs must not alias unless stated.
 *  - The library owns its tables, scratch vectors, block factors and Krylov
 *    bases; they are allocated by dg_create / setup calls and released by
 *    dg_destroy.
 *  - Argument and state errors are returned synchronously; asynchronous
 *    device faults surface at the next call or at dg_sync.  dg_last_error()
 *    returns a thread-local message for the last non-OK status.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_context dg_context;

typedef enum {
  DG_OK = 0,
  DG_NOT_CONVERGED = 1,       /* status, not an error: x holds the last iterate */
  DG_ERR_ARG = -1,            /* invalid argument or unsupported configuration */
  DG_ERR_HIP = -2,            /* a HIP runtime call failed */
  DG_ERR_OOM = -3,            /* device allocation failed */
  DG_ERR_STATE = -4,          /* e.g. block apply before block setup */
  DG_ERR_SINGULAR_BLOCK = -5, /* zero pivot in a diagonal block */
  DG_ERR_NONFINITE = -6       /* NaN/Inf met where a finite value is required */
} dg_status;

enum { DG_BASIS_PK = 0, DG_BASIS_QK = 1 };          /* total degree / tensor degree */
enum { DG_FLUX_LF = 0, DG_FLUX_ROE = 1 };           /* convective numerical flux */
enum { DG_JVP_EXACT = 0, DG_JVP_FD = 1, DG_JVP_EXACT_FP32 = 2, DG_JVP_STAB = 3, DG_JVP_EXACT_BF16 = 4 };  /* Jv mode */
enum { DG_FP64 = 0, DG_FP32 = 1, DG_BF16 = 2 };     /* block-factor storage */
enum { DG_PREC_NONE = 0, DG_PREC_BJ = 1, DG_PREC_MG = 2, DG_PREC_MLP = 3 };  /* FGMRES preconditioner */
enum { DG_ORTH_CGS2 = 0, DG_ORTH_MGS = 1 };         /* FGMRES orthogonalisation */
enum { DG_MG_V = 0, DG_MG_FULL = 1 };               /* p-multigrid cycle (Algs. vcic, fullvcic) */
enum { DG_PHYS_COMPRESSIBLE = 0, DG_PHYS_INCOMPRESSIBLE = 1, DG_PHYS_DIFFUSION = 2 };  /* equations */

/* Discretisation parameters.
 *  dim 2 or 3; order k >= 0; basis DG_BASIS_PK (paper's total-degree space,
 *  Sec. 2.1) or DG_BASIS_QK; nq1d Gauss points per direction (volume rule
 *  nq1d^dim, face rule nq1d^(dim-1)); flux DG_FLUX_LF or DG_FLUX_ROE;
 *  gamma, prandtl, mu: perfect gas, constant viscosity; eta_br2: BR2
 *  stabilisation (must exceed the number of faces of an element, Sec. 2.1;
 *  <= 0 selects 2*dim+1); entropy_fix: Harten fix width of the Roe flux as a
 *  fraction of |u.n| + c (<= 0 selects 0.1).
 *  physics DG_PHYS_COMPRESSIBLE (default, zero): conserved (rho, rho u, rho E).
 *  physics DG_PHYS_INCOMPRESSIBLE: the paper's own equations (Sec. 2.1, eq.
 *  ns): unit density, variables (u_1..u_d, p) (nvar = dim + 1), kinematic
 *  viscosity mu, Stokes stress; the divergence constraint is the last
 *  equation; the mass form of eq. massBil acts on the velocities only, so
 *  every "shift*v" below (Jv, block setup, p-multigrid, FGMRES, Rosenbrock)
 *  is shift times v on the velocity variables and 0 on the pressure (a
 *  differential-algebraic system); the interface flux is the Lax-Friedrichs
 *  flux of the artificial compressibility system (1/beta^2) dp/dt + div u = 0
 *  with beta = ac_beta (<= 0 selects 1), standing in for the exact Riemann
 *  solver of that system that the paper cites; flux and gamma/prandtl are
 *  ignored.  Uniform lattices only (DG_ERR_ARG on curved meshes), reference
 *  (vector-ALU) kernels, FP64 only (no FP32/BF16 operator, no network).
 *  physics DG_PHYS_DIFFUSION: the scalar BR2 Laplacian of the paper's
 *  Poisson assessment (App. B): one variable, residual of -div(mu grad u)
 *  (no convective flux); FP64 only, reference kernels on uniform lattices,
 *  the curved-element kernels on distorted 2D meshes at P2, P3 and P6
 *  (DG_ERR_ARG for other curved configurations); dg_max_wave_speed refuses
 *  it on curved meshes. */
typedef struct {
  int dim, order, basis, nq1d, flux;
  double gamma, prandtl, mu, eta_br2, entropy_fix;
  int physics;
  double ac_beta;
} dg_params;

/* Mesh (host memory, read during dg_create only).
 *  elem_xyz [n_elem][2^dim][dim]: corner coordinates, corners lexicographic
 *  (v = v0 + 2*v1 + 4*v2, v_i = 0/1 low/high end along axis i), unwrapped
 *  across periodic boundaries.  elem_nbr [n_elem][2*dim]: face neighbours in
 *  the order -x,+x,-y,+y,-z,+z; the +p neighbour's -p neighbour must be the
 *  element itself.  Faces must be conforming: the +p face of an element and
 *  the -p face of its neighbour have the same corners (up to a periodic
 *  shift).  Elements are multilinear (Sec. 2.1): when every element is the
 *  same axis-aligned box (uniform periodic lattice) the affine kernels run;
 *  otherwise each element carries its own orthonormal basis (Cholesky
 *  factor of its mass matrix in the reference basis) and the curved FP64
 *  kernels run.  An element with a non-positive Jacobian determinant at a
 *  quadrature point returns DG_ERR_ARG.  On curved meshes the learned
 *  preconditioner is unavailable (DG_ERR_ARG: its features assume a uniform
 *  lattice). */
typedef struct {
  int64_t n_elem;
  const double* elem_xyz;
  const int64_t* elem_nbr;
} dg_mesh;

/* Create a context (allocates tables and scratch on the current device). */
dg_status dg_create(const dg_params* params, const dg_mesh* mesh, dg_context** out);
void dg_destroy(dg_context* ctx);

/* Sizes: DOFs = n_elem*nvar*nbasis; nq = volume points per element. */
int64_t dg_ndof(const dg_context* ctx);
int dg_nbasis(const dg_context* ctx);
int dg_nvar(const dg_context* ctx);
int dg_nq(const dg_context* ctx);

/* Physical coordinates of the volume quadrature points, device output
 * xyz[dim][nq][n_elem]. */
dg_status dg_volume_points(dg_context* ctx, double* xyz, void* stream);

/* L2 projection onto the orthonormal basis: w_b = sum_q w_q |J_q| phi_b(x_q) f(x_q).
 * f: device input [nvar][nq][n_elem] (values at the volume points); w: DOFs. */
dg_status dg_project(dg_context* ctx, const double* f, double* w, void* stream);

/* Residual r = f_h(w) (eq. NSdiscrRes): -volume flux against grad(phi) plus
 * the numerical flux against the jump of phi; BR2 corrected gradients. */
dg_status dg_residual(dg_context* ctx, const double* w, double* r, void* stream);

/* The same residual with FP32 contractions (MFMA, FP32 accumulation) and FP32
 * pointwise fluxes; w and r stay FP64.  Curved meshes (FP32 tables and
 * vector-ALU kernels) and 3D P2-P4 lattices only (DG_ERR_ARG otherwise).  A reduced-precision operator for preconditioners
 * and smoothers; relative error of order 1e-6 against the FP64 residual. */
dg_status dg_residual_fp32(dg_context* ctx, const double* w, double* r, void* stream);

/* The same residual with BF16 contractions: every basis contraction (traces,
 * interpolation, corrected gradients, projections) takes BF16 operands (the
 * FP32 tables and the intermediate values rounded to nearest even) and
 * accumulates in FP32 on the BF16 matrix cores; pointwise fluxes in FP32; w and
 * r stay FP64.  3D P2-P4 lattices only (DG_ERR_ARG otherwise).  Relative error
 * of order 1e-3 against the FP64 residual (BF16 keeps 8 significant bits);
 * for preconditioners and smoothers only. */
dg_status dg_residual_bf16(dg_context* ctx, const double* w, double* r, void* stream);

/* out = shift*v + J(w) v.
 *  mode DG_JVP_EXACT: exact directional derivative of the residual (the
 *  Jacobian forms j_h of Sec. 2.2 applied to v), FP64.
 *  mode DG_JVP_FD: (f_h(w + D v) - f_h(w))/D with D = 1e-9*sqrt(1+||w||)/||v||
 *  (eqs. matrix-free, epsdef; L2 norms = DOF 2-norms).  r_w may pass f_h(w)
 *  (device, nullable) to skip its evaluation.  ||v|| = 0 gives out = 0 + shift*v.
 *  mode DG_JVP_EXACT_FP32: the exact tangent computed like dg_residual_fp32
 *  (FP32 contractions and pointwise arithmetic; for preconditioners only).
 *  mode DG_JVP_EXACT_BF16: the exact tangent computed like dg_residual_bf16
 *  (BF16 contractions, FP32 accumulation and pointwise arithmetic).
 *  mode DG_JVP_STAB: J replaced by its BR2 stabilisation part (the last term
 *  of eq. jacTrilFNURef: the tangent through the face lifting argument
 *  eta {r} of the face viscous flux only), FP64; not a solver mode.
 *  out may not alias w, v or r_w. */
dg_status dg_jvp(dg_context* ctx, const double* w, const double* r_w, const double* v, double shift,
                 int mode, double* out, void* stream);

/* Allocation-free variant of dg_jvp in mode DG_JVP_EXACT, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): out = shift*v + J(w) v computed by
 * the same kernels, bit for bit the result of dg_jvp, with the intermediate
 * arrays (modal corrected gradients and face fluxes, or on curved meshes the
 * transformed coefficients, face jumps and face fluxes) in a static device
 * array of dg_jvp_noalloc_scratch_bytes() = 256 MiB that every GPU running the
 * library holds until the process ends.  Calls no allocating routine.
 * Returns DG_ERR_ARG when the context's arrays exceed that size (affine P3:
 * 6,720 B per element, i.e. up to 39,945 elements; affine P4: 11,400 B per
 * element, up to 23,546).  All calls on one GPU share the array, whatever the
 * context or stream: calls that overlap on one GPU race, the caller
 * serialises them.  w, v, out: device, ndof entries; out may not alias w or v. */
dg_status dg_jvp_noalloc(dg_context* ctx, const double* w, const double* v, double shift, double* out,
                         void* stream);
size_t dg_jvp_noalloc_scratch_bytes(void);

/* EWBJ setup: D_K = shift*I + dR_K/dU_K for every element (exact, by
 * probing with exact Jv: element-local where dg_set_block_probing allows it,
 * else coloured), factored by Gauss-Jordan with partial
 * pivoting into explicit inverses, stored as `storage`: DG_FP64 (FP64
 * elimination), DG_FP32 (FP32 elimination) or DG_BF16 (FP32 elimination,
 * inverse rounded to BF16; the apply accumulates in FP32).  With DG_FP32 or
 * DG_BF16 the blocks are also probed with the FP32 operator (dg_residual_fp32)
 * where the configuration has it.  Reduced precision only changes the
 * preconditioner, never the FP64 operator of the solve.
 * Returns DG_ERR_SINGULAR_BLOCK if a pivot is exactly zero or non-finite
 * (synchronises the stream). */
dg_status dg_block_precond_setup(dg_context* ctx, const double* w, double shift, int storage, void* stream);

/* How the diagonal blocks dR_K/dU_K are probed (Sec. 2.3: the blocks of the
 * element-wise block Jacobi are the exact Jacobian's diagonal blocks; the
 * p-multigrid setup probes its fine blocks the same way).
 *   DG_PROBE_AUTO (default of a new context): element-local probing where the
 *     kernels allow it -- the MFMA operators of 3D P2-P4 lattices on meshes
 *     where no element is its own face neighbour: one pass per block column
 *     with every element perturbed at once, the face kernel run once per face
 *     side so that each flux tangent reaches only the perturbed element's own
 *     rows (half the passes of a two-colour lattice); coloured elsewhere.
 *   DG_PROBE_COLOURED: one exact Jv per block column and colour of the
 *     face-neighbour graph (e_l in the elements of one colour, whose
 *     neighbours all carry zero).
 * Both give the same blocks bit for bit (the local tangents are the coloured
 * probe's, with the other side's tangent zero instead of a zero input).
 * DG_ERR_ARG for another mode; takes effect at the next setup. */
enum { DG_PROBE_AUTO = 0, DG_PROBE_COLOURED = 1 };
dg_status dg_set_block_probing(dg_context* ctx, int mode);

/* z_K = D_K^{-1} r_K for every element (needs a prior setup; DG_ERR_STATE
 * otherwise).  r and z may not alias. */
dg_status dg_block_precond_apply(dg_context* ctx, const double* r, double* z, void* stream);

typedef struct {
  int restart;     /* Krylov subspace size m (default 30) */
  int max_iter;    /* total iteration cap */
  double rtol;     /* ||b - G x|| <= rtol*||b|| on the true residual */
  int precond;     /* DG_PREC_NONE, DG_PREC_BJ (block setup must exist),
                      DG_PREC_MG (dg_mg_setup must exist, built with the same w, shift)
                      or DG_PREC_MLP (network weights set) */
  int jvp_mode;    /* DG_JVP_EXACT or DG_JVP_FD for G z (the outer operator stays FP64) */
  double rho_ref;  /* DG_PREC_MLP only: if > 0 and a block setup exists, the
                      solve switches to block Jacobi when the convergence
                      factor (|g_j|/||r_0||)^(1/j) after judge_after
                      iterations exceeds rho_ref (e.g. block Jacobi's) */
  int judge_after; /* iterations before that check (<= 0 selects 5) */
  int orth;        /* Arnoldi: DG_ORTH_CGS2 (classical Gram-Schmidt with one
                      re-orthogonalisation, two fused passes over the basis) or
                      DG_ORTH_MGS (modified Gram-Schmidt, one vector at a time) */
  int check_every; /* the host applies the Givens rotations of the Hessenberg
                      columns that arrived and tests convergence every
                      check_every iterations and at the end of a restart cycle
                      (0 or 1: every iteration; < 0: DG_ERR_ARG); the GPU runs
                      ahead meanwhile, and iterations enqueued past the
                      converged one are discarded */
} dg_solve_opts;

typedef struct {
  int iters, restarts, converged;
  double rel_res_est, rel_res_true, rho; /* rho: convergence factor */
  double ms_solve;
  int fallbacks;   /* switches from DG_PREC_MLP to block Jacobi */
  double ms_setup; /* wall time of the last setup of the preconditioner used
                      (dg_block_precond_setup or dg_mg_setup, including their
                      autotuning); 0 for none and the learned preconditioner */
} dg_solve_stats;

/* Right-preconditioned flexible GMRES(m) for (shift*I + J(w)) x = b.
 * Classical Gram-Schmidt with one re-orthogonalisation, Givens rotations,
 * restarts from the true residual.  x: device, in = initial guess, out =
 * solution.  b = 0 returns x = 0.  Synchronises the stream at every
 * convergence check (opts->check_every).  opts/stats are host memory; stats
 * may be NULL. */
dg_status dg_fgmres_solve(dg_context* ctx, const double* w, double shift, const double* b, double* x,
                          const dg_solve_opts* opts, dg_solve_stats* stats, void* stream);

/* Rosenbrock (linearly implicit Runge-Kutta) step (Sec. 2.2, Alg. ros) for
 * M dw/dt + R(w) = 0 with M = I (orthonormal basis):
 *   for s = 1..n_stages:
 *     dp = sum_{o<s} a[s][o] dw_o,  dq = sum_{o<s} c[s][o] dw_o   (0-based s, o)
 *     (I/(gamma dt) + J(w)) dw_s = -R(w + dp) - dq/dt      (FGMRES with *opts)
 *   w_next = w + sum_s m[s] dw_s
 * The Jacobian is that of w for every stage, and the preconditioner named by
 * opts->precond must have been set up by the caller at (w, 1/(gamma dt))
 * (dg_block_precond_setup or dg_mg_setup; once per step).  Coefficients are
 * the caller's (the scheme of the paper, ROSI2PW, is cited there without
 * them); n_stages = 1, gamma = 1, m[0] = 1 is the linearised backward Euler
 * step.  w and w_next: device, ndof entries, may not alias.  Stage vectors
 * live in a library buffer grown on demand.  stats (host, nullable): iters
 * and restarts summed over the stages, converged = all stages converged,
 * rel_res_est / rel_res_true / rho = the largest over the stages, ms_solve
 * summed, ms_setup that of the preconditioner's last setup.  Returns
 * DG_NOT_CONVERGED (w_next still written) if a stage did not converge.
 * Synchronises the stream (at every convergence check of the stage solves). */
enum { DG_ROS_MAX_STAGES = 6 };
typedef struct {
  int n_stages;                                  /* 1..DG_ROS_MAX_STAGES */
  double gamma;                                  /* > 0 */
  double a[DG_ROS_MAX_STAGES][DG_ROS_MAX_STAGES]; /* a[s][o], o < s used */
  double c[DG_ROS_MAX_STAGES][DG_ROS_MAX_STAGES]; /* c[s][o], o < s used */
  double m[DG_ROS_MAX_STAGES];
} dg_rosenbrock;
dg_status dg_rosenbrock_step(dg_context* ctx, const double* w, double dt, const dg_rosenbrock* coeffs,
                             const dg_solve_opts* opts, double* w_next, dg_solve_stats* stats, void* stream);

/* p-multigrid preconditioner (Sec. 2.4): levels l = 0..n_levels-1 of degrees
 * orders[0] (= the context's order) > orders[1] > ...; level vectors use the
 * DOF layout with N_b(orders[l]) modes.  Restriction keeps the first
 * N_b(orders[l+1]) modes of every variable, prolongation pads with zeros
 * (Sec. 2.4.1, hierarchical orthonormal basis).  Level 0 applies
 * G_0 = shift*I + J(w) matrix-free; coarse levels apply the inherited
 * operators G_l = R G_0 P (eq. GalProj), stored block-sparse (diagonal block
 * plus one block per face neighbour, FP64) after probing G_0 with a
 * distance-2 colouring of the elements.  Every level is smoothed by
 * smooth_iters[l] right-preconditioned GMRES steps (one cycle, block Jacobi of
 * the level operator, factors stored as `storage`); the last entry is the
 * coarsest-level solve.  One apply is Alg. vcic (cycle DG_MG_V) or Alg.
 * fullvcic (DG_MG_FULL: restrict the right-hand side level by level, solve
 * on the coarsest, then on each finer level prolong the coarser result and
 * correct it by one V-cycle on its defect) from a zero initial guess. */
typedef struct {
  int n_levels;         /* 2 or 3, the fine level included */
  int orders[3];        /* strictly decreasing, >= 0, orders[0] = context order */
  int smooth_iters[3];  /* 0..60 each; the coarsest level needs >= 1 */
  int storage;          /* block-factor storage on every level: DG_FP64/FP32/BF16;
                           with FP32 or BF16 the cycle also applies FP32
                           copies of the coarse operators (FP64 sums) */
  int use_graph;        /* nonzero: capture one cycle into a hipGraph at setup;
                           every apply replays it on a library stream ordered
                           against the caller's stream by events */
  int fine_precision;   /* DG_FP64, DG_FP32 or DG_BF16: the fine-level operator
                           inside the cycle (smoother products and the defect)
                           and the probing of the coarse operators and of every
                           column of the fine diagonal blocks, as the exact FP64
                           Jv or its FP32 / BF16-contraction variant (BF16: 3D
                           P2-P4 lattices); the outer solve stays FP64 */
  int cycle;            /* DG_MG_V or DG_MG_FULL */
  int rescale;          /* 1: rescaled-inherited coarse operators (App. A, eq.
                           GalProjResc): the BR2 stabilisation part of each
                           inherited operator is scaled by
                           S = k_{l+1}(k_{l+1}+d) / (k_l(k_l+d)) per level
                           (probing costs one more product per column) */
  int coarse_ilu;       /* 1: the coarsest level's smoother is preconditioned by
                           a block ILU(0) of its operator in the multicolour
                           order of the face-neighbour graph (FP64; blocks of
                           at most 64 rows) instead of block Jacobi; stands in
                           for the paper's ASM(1,ILU(0)) coarse smoother.  The
                           elimination updates only diagonal blocks, exact for
                           face-neighbour graphs without triangles; a mesh with
                           a periodic direction of three elements is refused
                           (DG_ERR_ARG) */
} dg_mg_opts;

/* Builds the hierarchy at state w (device, copied) and shift: runs the fine
 * block-Jacobi setup (as dg_block_precond_setup with opts->storage, which
 * replaces any earlier block setup), probes the first coarse level, truncates
 * deeper ones, factors every level's diagonal blocks, autotunes the coarse
 * operator kernels and optionally captures the graph.  Basis DG_BASIS_PK only.
 * Synchronises the stream.  A later dg_block_precond_setup invalidates the
 * hierarchy (apply then returns DG_ERR_STATE). */
dg_status dg_mg_setup(dg_context* ctx, const double* w, double shift, const dg_mg_opts* opts, void* stream);

/* Preconditioner lagging (the time-step study of Sec. 4: the coarse operators
 * are frozen for several steps while the matrix-free fine level follows the
 * current state).  Replaces the state (device, copied) and shift of the
 * fine-level operator inside the cycle (smoother products and defect) and
 * keeps the probed coarse operators and their factors from the last
 * dg_mg_setup.  refresh_blocks != 0 also rebuilds the fine block-Jacobi
 * factors at (w, shift) with the hierarchy's storage (as
 * dg_block_precond_setup, which alone would invalidate the hierarchy);
 * refresh_blocks = 0 keeps them and is refused (DG_ERR_STATE) once another
 * block setup has replaced them.  Re-captures the graph.  Synchronises the
 * stream. */
dg_status dg_mg_update_fine(dg_context* ctx, const double* w, double shift, int refresh_blocks, void* stream);

/* z = MG_V(0, r, 0): one V-cycle on the fine level (r, z: device DOF vectors,
 * no aliasing).  The cycle is nonlinear in r (GMRES smoothers), hence the
 * flexible outer solver. */
dg_status dg_mg_apply(dg_context* ctx, const double* r, double* z, void* stream);

/* y = G_l x on level l (0 = fine, matrix-free; >= 1 = inherited block-sparse
 * operator), vectors in level l's DOF layout. */
dg_status dg_mg_level_apply(dg_context* ctx, int level, const double* x, double* y, void* stream);

/* Learned element-local preconditioner.  For element K with residual slice
 * r_K (n*Nb values, local order c*Nb + b) and s_K = ||r_K||_2 + 1e-300 the
 * features are x_K = [r_K / s_K, m(K_f)/m_ref for the 2d face neighbours K_f
 * in the order -x,+x,-y,+y,-z,+z], with m the cell means of the n conserved
 * variables of the state w and m_ref their RMS over the mesh
 * (n_in = n*Nb + 2d*n).  Network n_in -> 256 -> 256 -> n*Nb with ReLU on the
 * hidden layers; BF16 weights, activations and deltas, FP32 biases, MFMA
 * products with FP32 accumulation; z_K = s_K * output.  Parameters: one
 * flat FP32 vector W1 [256][n_in], b1 [256], W2 [256][256], b2 [256],
 * W3 [n*Nb][256], b3 [n*Nb] (row-major), owned by the library (master copy,
 * Adam moments, BF16 copies).  Training minimises the mean squared error
 * over a batch of normalised pairs (x_K, z_K / s_K) with Adam (0.9, 0.999,
 * 1e-8).  All arrays are device memory. */
int64_t dg_mlp_nparams(dg_context* ctx);
/* Network mode.  DG_MLP_DIRECT (default): z_K = s_K * output, targets
 * T = z_K / s_K.  DG_MLP_CORRECT_BJ: the network corrects block Jacobi,
 * z_K = D_K^{-1} r_K + s_K * output with targets T = (z_K - D_K^{-1} r_K) / s_K,
 * so a network whose last layer is zero is block Jacobi exactly; features
 * with targets and the apply then need a block setup (DG_ERR_STATE
 * otherwise) and use its factors. */
enum { DG_MLP_DIRECT = 0, DG_MLP_CORRECT_BJ = 1 };
dg_status dg_mlp_set_mode(dg_context* ctx, int mode);
/* Copy the parameter vector in (resets the Adam state). */
dg_status dg_mlp_set_weights(dg_context* ctx, const float* theta, void* stream);
dg_status dg_mlp_get_weights(dg_context* ctx, float* theta, void* stream);
/* Features X [n_elem][n_in] (FP32) for state w and residual r; optional
 * normalised targets T [n_elem][n*Nb] = z_K / s_K (needs z) and scales
 * s [n_elem] (FP64); T and s may be NULL. */
dg_status dg_mlp_features(dg_context* ctx, const double* w, const double* r, const double* z, float* X, float* T,
                          double* s, void* stream);
/* Y [batch][n*Nb] = network(X [batch][n_in]) (normalised outputs). */
dg_status dg_mlp_forward(dg_context* ctx, const float* X, int64_t batch, float* Y, void* stream);
/* Gradient of the loss over rows[0..batch) of X / T (rows may be NULL for
 * 0..batch-1) into grad (nparams FP32); loss (1 FP32) may be NULL. */
dg_status dg_mlp_grad(dg_context* ctx, const float* X, const float* T, const int64_t* rows, int64_t batch,
                      float* grad, float* loss, void* stream);
/* One Adam step with learning rate lr on the same loss. */
dg_status dg_mlp_train_step(dg_context* ctx, const float* X, const float* T, const int64_t* rows, int64_t batch,
                            float lr, float* loss, void* stream);
/* z = s_K * network(x_K(w, r)) for every element (DOF layout, FP64). */
dg_status dg_mlp_apply(dg_context* ctx, const double* w, const double* r, double* z, void* stream);

/* max over volume points of |u| + c, returned to host memory (synchronises). */
dg_status dg_max_wave_speed(dg_context* ctx, const double* w, double* out, void* stream);

/* Per-kernel timing: when enabled, the library records HIP events around
 * each launch on the launch stream; dg_kernel_time returns the accumulated
 * milliseconds and launch count of a named kernel ("face_jvp", "vol_jvp",
 * "face_res", "vol_res", "face_jvp_f32", "vol_jvp_f32", "block_probe",
 * "block_invert", "block_apply", "arnoldi", "mg_probe", "mg_vcycle",
 * "mlp_apply"; the element-local probing passes inside "block_probe" as
 * "grad_probe", "face_probe" (both face passes) and "vol_probe", with the
 * suffix "_f32" / "_bf16" for the reduced-precision operators) and resets
 * it.  Synchronises. */
dg_status dg_set_profiling(dg_context* ctx, int on);
dg_status dg_kernel_time(dg_context* ctx, const char* name, double* ms, int64_t* launches);

/* Launch-shape autotuning.  In DG_TUNE_AUTO mode (the default of a new
 * context) dg_autotune, dg_block_precond_setup and dg_mg_setup time the
 * candidate launch shapes of the kernels they set up, at the problem's own
 * size and on the caller's stream, and keep the fastest (a candidate replaces
 * the built-in default only when it is at least 3 % faster):
 *   - the waves per SIMD (1 or 2) of the 3D MFMA face and volume kernels and
 *     whether the volume kernel forms the corrected gradients itself (no
 *     gradient kernel and buffer), per operator precision, residual and Jv
 *     (dg_autotune: every precision the context has; the setups: the
 *     precision they probe with);
 *   - the block-inverse apply: one lane per row with 1-8 elements per
 *     workgroup (blocks of at most 64 rows), or 16-byte column loads by
 *     64-512 threads per element with 1-4 elements per workgroup; per level
 *     and storage;
 *   - the p-multigrid coarse operators' block-sparse apply: workgroup size,
 *     rows per thread and column slices per row, per level.
 * Choices are kept in a process-wide cache keyed by kernel and problem shape,
 * so later setups and contexts of the same shape reuse them without timing.
 * The MFMA occupancy and the gradient fusion change no result bit; the apply
 * shapes change the order
 * of the sums (results differ in the last bits between shapes, never between
 * calls with the same shapes).  A setup that runs while its stream is being
 * captured keeps the defaults.  DG_TUNE_FIXED: the built-in defaults and no
 * timing, bitwise reproducible across processes; setting it resets the
 * context's operator and fine block-apply shapes at once (a ready hierarchy
 * re-captures its cycle graph), while the hierarchy keeps the coarse shapes
 * of its setup until the next dg_mg_setup.  DG_ERR_ARG for another mode. */
enum { DG_TUNE_FIXED = 0, DG_TUNE_AUTO = 1 };
dg_status dg_set_tuning(dg_context* ctx, int mode);

/* Tunes the fine operator's shapes at state w (device DOF vector, read only)
 * and, when block-Jacobi factors exist, their apply shape.  Uses the
 * context's work vectors and synchronises the stream; no-op in DG_TUNE_FIXED
 * mode. */
dg_status dg_autotune(dg_context* ctx, const double* w, void* stream);

/* Pin launch shapes instead of tuning them (e.g. to reproduce the shapes of an
 * earlier tuned run without timing, or to compare shapes).  DG_ERR_ARG for a
 * shape the kernel does not have for this problem; a ready p-multigrid
 * hierarchy re-captures its cycle graph.
 *   dg_set_fine_shape: waves per SIMD (1, 2; 0 = default) of the MFMA face
 *     and volume kernels of the operator of `precision` (DG_FP64/FP32/BF16),
 *     residual (jvp = 0) or Jv (jvp = 1), and fused_gradients (1: the volume
 *     kernel forms the corrected gradients; 0: the gradient kernel writes
 *     them to a buffer); later setups keep it.
 *   dg_set_apply_shape: block-inverse apply of level 0 (the fine block-Jacobi
 *     factors; needs a block setup) or of coarse level >= 1 of the hierarchy:
 *     kind 1 = one lane per row (threads = 64, epw = 1/2/4/8 elements per
 *     workgroup, blocks of at most 64 rows), kind 2 = 16-byte column loads by
 *     `threads` threads per element (64 with epw 1/2/4, or 128/256/512 with
 *     epw 1), kind 0 = the default.  A later setup of that level chooses again.
 *   dg_set_bsr_shape: coarse level >= 1's block-sparse apply: workgroup 256,
 *     512 or 1024 threads, rows per thread 1, 2 or 4 (4: FP32 copies only; 0 =
 *     the widest the block size allows), column slices 1, 2, 4 or 8.  Applies
 *     to the blocks the cycle uses (the FP32 copies with FP32/BF16 storage). */
dg_status dg_set_fine_shape(dg_context* ctx, int precision, int jvp, int face_occ, int volume_occ,
                            int fused_gradients);
dg_status dg_set_apply_shape(dg_context* ctx, int level, int kind, int threads, int epw);
dg_status dg_set_bsr_shape(dg_context* ctx, int level, int workgroup, int rows_per_thread, int column_slices);

/* Writes the current launch shapes as NUL-terminated text, one line per
 * kernel family ("fine fp64 residual: face occ 2, volume occ 2, gradients separate", "block apply
 * m=175 fp32: vec 256x1", "mg level 1 ...").  DG_ERR_ARG when buf is null or
 * len is too small (4096 bytes always suffice). */
dg_status dg_tuning_report(const dg_context* ctx, char* buf, size_t len);

const char* dg_last_error(void);
dg_status dg_sync(dg_context* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DG_H */
