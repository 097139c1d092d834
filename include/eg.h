/*
 * eg.h -- C ABI of the MI355X exponential p-multigrid (eMG) library.
 *
 * The library solves the steady compressible Euler equations discretised by
 * a modal discontinuous Galerkin method (arXiv:1807.01151, Section 3) with
 * the eMG V-cycle (Section 2.4): an s-stage element-block-preconditioned
 * Runge-Kutta smoother (Section 2.3) on orders p >= 1 and the EXP1
 * exponential step (Sections 2.1-2.2) on p = 0.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - d = 2 (quads) or 3 (hexes); V = d + 2 conserved variables
 *    (rho, rho v_1..rho v_d, rho E); gamma from eg_params.
 *  - A level-p coefficient vector holds N_p = (p+1)^d modes per variable,
 *    contiguous FP64, layout [elem][var][mode], modes in hierarchical order
 *    (sort key: largest 1D degree, then the degrees along axes 0, 1, 2), so
 *    level p-1 is the leading N_{p-1} slice of each [elem][var] row.
 *    Coefficients refer to the per-element orthonormal basis psi_i of
 *    Section 3.2 (mass matrix = identity), built from tensor Legendre
 *    polynomials on the reference element.
 *  - Pointers named *_dev are HIP device pointers owned by the caller; *_host
 *    are host pointers.  Every entry point enqueues its work on the stream
 *    passed to eg_init_mesh; entry points returning host values synchronise
 *    that stream.
 *  - Errors: a non-EG_OK status leaves caller buffers untouched when it is
 *    EG_ERR_ARG or EG_ERR_MESH (all checks precede any launch); the message is
 *    available from eg_last_error().  No C++ exception crosses this ABI.
 *  - One handle per stream; a handle is not safe for concurrent use.
 */
#ifndef EG_H
#define EG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eg_handle eg_handle;

typedef enum {
  EG_OK = 0,
  EG_ERR_ARG = 1,            /* invalid argument (null pointer, size, order) */
  EG_ERR_MESH = 2,           /* unmatched / non-conforming face, inverted element */
  EG_ERR_ALLOC = 3,          /* device allocation failed */
  EG_ERR_HIP = 4,            /* a HIP call failed; message has hipGetErrorString */
  EG_ERR_NOT_CONVERGED = 5,  /* eg_solve_steady hit max_cycles (history filled) */
  EG_ERR_DIVERGED = 6,       /* non-finite residual norm (history filled) */
  EG_ERR_UNSUPPORTED = 7     /* valid request this build does not implement */
} eg_status;

/* Boundary tags of eg_mesh.bface_tag.  A symmetry plane (Section 5.2) takes
   the slip-wall ghost state (the mirror image of the inside state) but is not
   part of the body surface the drag integrates.  Other values: EG_ERR_MESH. */
enum { EG_FACE_INTERIOR = 0, EG_FACE_WALL = 1, EG_FACE_FARFIELD = 2, EG_FACE_SYMMETRY = 4 };

typedef struct {
  int dim;                  /* 2 or 3 */
  int n_vert;
  const double* xyz;        /* host, [n_vert][dim]; copied */
  int n_elem;
  const int32_t* elem_vert; /* host, [n_elem][2^dim]; local vertex a+2b(+4c) sits at
                               reference corner (2a-1, 2b-1[, 2c-1]); copied */
  const int8_t* bface_tag;  /* host, [n_elem][2 dim]; local face 2r+s is xi_r = -1 (s=0)
                               or +1 (s=1).  0 interior (matched to the neighbour
                               that shares its vertices), 1 slip wall, 2 far-field,
                               4 symmetry plane */
  const double* elem_geo;   /* host, optional (null = straight-sided elements): nodes of
                               a quadratic curved element map (Sections 5.1, 5.2 meshes).
                               2D: [n_elem][9][2], biquadratic, node a+3b at reference
                               point (a-1, b-1); 3D: [n_elem][27][3], triquadratic, node
                               a+3b+9c at (a-1, b-1, c-1).  The nodes at the corners
                               (every digit 0 or 2) must equal the vertices, and both
                               sides of an interior face must place its nodes (3 per
                               edge, 9 per quadrilateral) at the same points (within
                               1e-12 relative), else EG_ERR_MESH.  Copied */
} eg_mesh;

typedef struct {
  int p_max;          /* highest order, 0..4 (2D) or 0..3 (3D) */
  int rk_stages;      /* s of the PRK smoother (Section 2.3); paper: 4 */
  double cfl_max;     /* upper bound of the CFL ramp (Section 4, eq. (cfl)); paper: 100 */
  int krylov_m;       /* Krylov dimension of EXP1 (Section 5: m = 30), 1..48 */
  int relative_ramp;  /* 1: the ramp uses ||R(rho_n)|| / ||R(rho_1)||; 0: the printed absolute norm */
  double gamma;       /* ratio of specific heats (paper: 7/5) */
  double mach;        /* free-stream Mach number; rho_inf = 1, p_inf = 1/gamma */
  double alpha_deg;   /* free-stream angle in the x-y plane */
  double beta_deg;    /* 3D only: angle out of the x-y plane */
  int precision;      /* EG_FP64 or EG_MIXED (see below) */
  int flux;           /* numerical flux of the face integrals: EG_FLUX_RUSANOV or EG_FLUX_ROE */
} eg_params;

/* Numerical flux (eg_params.flux), Section 3.1 after eq. (euler3) and
 * Section 3.3 (the same flux with a ghost state on boundary faces):
 *  EG_FLUX_RUSANOV  local Lax-Friedrichs, dissipation max over both sides of
 *                   |v . n| + c;
 *  EG_FLUX_ROE      the paper's Roe solver: Roe-averaged (sqrt(rho)-weighted)
 *                   velocity and total enthalpy, wave decomposition of the
 *                   jump, Harten's entropy fix on the two acoustic waves for
 *                   |lambda| < c / 10 (the paper names no fix).
 * Every kernel (residual, element blocks, p = 0 operator, J v, J^T w, drag)
 * uses the handle's flux; its Jacobians come from the same dual-number
 * evaluation. */
enum { EG_FLUX_RUSANOV = 0, EG_FLUX_ROE = 1 };

/* Arithmetic of the smoother (eg_params.precision).
 *  EG_FP64:  every kernel in FP64.
 *  EG_MIXED: state, forcings, transfers, the p = 0 level (EXP1, Arnoldi,
 *            phi_1) and every residual norm stay FP64; the element blocks of
 *            the levels p >= 1, their LU factors (stored FP32) and the PRK
 *            stage solves are FP32.  A steady solve runs in two phases:
 *            phase A also evaluates the residuals of the levels p >= 1 in
 *            FP32, with an FP64 defect at p_max (d = R64(u^n) - R32(u^n) is
 *            that level's forcing for the cycle); it ends for good once the
 *            FP64 norm r_n <= 1e-4 r_1, has not reached a new minimum for
 *            100 cycles, or r_n > 0.9 r_{n-50} (less than 10% progress in
 *            50 cycles).  Phase B evaluates every residual in FP64, so the
 *            FP32 blocks only precondition an FP64 defect correction
 *            (Section 2.3, eq. (prk_scalar) with P in FP32) and the
 *            converged state is the FP64 steady state.  eg_vcycle runs
 *            phase B when r_n <= 1e-4 rref, else phase A. */
enum { EG_FP64 = 0, EG_MIXED = 1 };

/* Builds faces, orientation codes, geometry and per-element basis data, and
 * allocates every device workspace.  hip_stream may be NULL (default stream).
 * On failure *out may still receive a handle (so that eg_last_error can be
 * read); release it with eg_free. */
eg_status eg_init_mesh(const eg_mesh* mesh, const eg_params* params, void* hip_stream, eg_handle** out);

void eg_free(eg_handle* h);

const char* eg_last_error(const eg_handle* h);

/* Sizes: number of elements, modes per variable at level p, variables. */
eg_status eg_sizes(const eg_handle* h, int p, int* n_elem, int* n_modes, int* n_vars);

/* u_dev <- uniform free stream at level p (all higher modes zero). */
eg_status eg_set_freestream(eg_handle* h, int p, double* u_dev);

/* DG residual R_p(u) of Section 3.1, eq. (euler3) (no source term):
 *   R_{E,i} = -sum_faces int psi_i F~.n dsigma + int_E F . grad psi_i dx,
 * the handle's numerical flux (eg_params.flux), (p+2)^d Gauss points per
 * element and (p+2)^(d-1) per face.
 * u_dev, r_dev: level-p vectors.  Evaluated in the smoother's arithmetic:
 * FP32 for p >= 1 on an EG_MIXED handle (FP64 inputs and outputs), else FP64.
 * Asynchronous. */
eg_status eg_residual(eg_handle* h, int p, const double* u_dev, double* r_dev);

/* Local pseudo-time step of Section 4, eq. (x3d):
 *   dtau_E = cfl h_E / ((2 p + 1)(|v| + c)),  h_E = 2 d |E| / |dE|,
 * v and c from the element-mean state of the level-p_level vector u_dev.
 * dtau_dev: [n_elem].  Asynchronous. */
eg_status eg_timestep(eg_handle* h, int p, int p_level, double cfl, const double* u_dev, double* dtau_dev);

/* Element-diagonal Jacobian blocks D_E = dR_E/du_E at level p
 * (Section 3.3, eq. (jac1)), layout [elem][(var,mode)][(var,mode)], row
 * (v, i) = v N_p + i.  Asynchronous. */
eg_status eg_element_jacobian(eg_handle* h, int p, const double* u_dev, double* D_dev);

/* One s-stage PRK step at level p >= 1 (Section 2.3, eq. (prk_scalar)):
 *   u^(k) = u^n + beta_k P^{-1} [R_p(u^(k-1)) + f],  beta_k = 1/(s-k+1),
 * P_E = I/dtau_E - D_E(u^n) (dtau at order p and the given cfl).
 * u_dev is updated in place; f_dev (level p) may be NULL.  Asynchronous. */
eg_status eg_prk_step(eg_handle* h, int p, double cfl, double* u_dev, const double* f_dev);

/* p = 0 Jacobian (Section 3.3 at p = 0): diagonal blocks [elem][V][V] and
 * neighbour blocks [elem][2d][V][V] (zero on boundary faces); nbr_dev
 * (may be NULL) receives [elem][2d] neighbour indices, -1 on boundaries. */
eg_status eg_jacobian_p0(eg_handle* h, const double* u0_dev, double* diag_dev, double* off_dev, int32_t* nbr_dev);

/* One EXP1 step on the p = 0 level (Sections 2.1-2.2, eqs. (EXP1), (final)):
 *   u0 <- u0 + phi_1(A) b,  A = T J_0(u0),  b = T [R_0(u0) + f0],
 * T = diag(dt_E), dt_E = (p_max + 1) dtau_E (dtau at order p_max, Section 4),
 * phi_1(A) b ~ beta V_m phi_1(H_m) e_1 with krylov_m Arnoldi steps.
 * f0_dev may be NULL.  m_used_host (may be NULL) gets the Krylov dimension
 * actually used (smaller after a happy breakdown); synchronises if non-NULL. */
eg_status eg_exp1_step(eg_handle* h, double cfl, double* u0_dev, const double* f0_dev, int* m_used_host);

/* Density-residual norm of Section 4: ||R(rho)|| = (1/|Omega|) (int R_rho^2)^(1/2)
 * of a level-p_max residual vector.  Synchronises. */
eg_status eg_rnorm(eg_handle* h, const double* r_dev, double* rn_host);

/* The norm of eg_rnorm without allocation or synchronisation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  r_dev: level-p_max
 * residual (psi coordinates, as eg_rnorm); rn_dev: device pointer to one
 * double that receives the norm.  Enqueued on the handle's stream; calls
 * no allocating routine.  Its only workspace is a static per-device array
 * of 4096 partial sums (32 KiB, held by each GPU the library runs on until
 * the process ends), so the handle may have at most 1,048,576 elements
 * (else EG_ERR_ARG with a message).  Every call on one GPU shares that
 * array: calls that overlap on one GPU (other streams or threads) race.
 * Batch handles: EG_ERR_ARG. */
eg_status eg_rnorm_noalloc(eg_handle* h, const double* r_dev, double* rn_dev);

/* One eMG V-cycle (Section 2.4) on the level-p_max state u_dev, cycle index
 * n >= 1 (enters the CFL ramp).  rref is the reference norm of the ramp
 * (r_1 for the relative ramp, 1 for the absolute one; 0 = use the state's
 * own norm, i.e. a first cycle).  rn_host receives r_n of the entry state,
 * cfl_host (may be NULL) the CFL used.  Synchronises once. */
eg_status eg_vcycle(eg_handle* h, double* u_dev, int n, double rref, double* rn_host, double* cfl_host);

/* Steady solve: repeat V-cycles until r_n <= drop_tol r_1 or max_cycles.
 * hist_host[0..*n_cycles_host] receives r_1, r_2, ... (caller provides
 * max_cycles + 1 entries).  Returns EG_OK, EG_ERR_NOT_CONVERGED or
 * EG_ERR_DIVERGED (history filled in every case). */
eg_status eg_solve_steady(eg_handle* h, double* u_dev, double drop_tol, int max_cycles, double* hist_host,
                          int* n_cycles_host);

/* Continues the last eg_solve_steady / eg_solve_resume of this handle on
 * u_dev: same r_1 and cycle numbering (the CFL ramp carries on), starting by
 * re-evaluating the norm of the cycle at which the previous call stopped;
 * hist_host[0..*n_cycles_host] as for eg_solve_steady.  Lets a caller run a
 * long solve in chunks. */
eg_status eg_solve_resume(eg_handle* h, double* u_dev, double drop_tol, int max_cycles, double* hist_host,
                          int* n_cycles_host);

/* Graph replay (enable != 0): the steady-solve entries (eg_solve_steady,
 * eg_solve_resume, eg_solve_batch) capture the V-cycle below the entry norm
 * once (one graph per mixed-precision phase) into a HIP graph on an
 * internal stream of the handle, ordered after and before the handle's
 * stream by events, and replay it every cycle; the CFL of each cycle is
 * read from device memory.  Results are identical to the eager launches.
 * Off by default; profiling (eg_profile) runs eagerly. */
eg_status eg_set_graphs(eg_handle* h, int enable);

/* Tile autotuner (no passage of the paper: a tuning of this implementation).
 * For every order p <= p_max and both arithmetic precisions, times the
 * residual kernel (eq. (euler3)) with three element tiles per workgroup
 * (half, the default and 1.5 x the default) on a free-stream state, reps
 * launches each with HIP events on the handle's stream, and keeps the
 * fastest for every later residual of the handle (results do not depend on
 * the tile: every output is formed by one thread with the same sums).
 * tiles_host (nullable, host memory, 2 (p_max + 1) ints): the chosen
 * elements per workgroup, [p][FP64, FP32].  Uses the handle's scratch
 * buffers and rt; call it before a solve, not between eg_solve_steady and
 * eg_solve_resume.  Drops captured V-cycle graphs (they are recaptured). */
eg_status eg_autotune(eg_handle* h, int reps, int* tiles_host);

/* ---- Batched independent solves ----
 * n_solves steady problems (Section 2.4 eMG each) in one handle: meshes of
 * any size with the same dim, p_max, rk_stages, krylov_m, cfl_max,
 * relative_ramp, gamma and precision; mach, alpha_deg and beta_deg may
 * differ.  The meshes are concatenated into one disconnected mesh, so every
 * kernel launch covers all solves; the residual norms, the CFL ramp and the
 * EXP1 Krylov process (Arnoldi, phi_1, breakdown) are per solve.  Level-p
 * vectors are the solves' vectors one after another (eg_layout gives the
 * offsets).  On a batch handle eg_vcycle, eg_solve_steady, eg_solve_resume,
 * eg_rnorm, eg_drag and eg_adjoint_solve return EG_ERR_ARG; the per-element
 * entries (eg_residual, eg_prk_step, ...) act on all solves with one CFL. */
eg_status eg_init_batch(const eg_mesh* meshes, const eg_params* params, int n_solves, void* hip_stream,
                        eg_handle** out);

/* Offset (in doubles) of solve `solve` in a level-p vector, its modes per
 * variable and its element count (a single-solve handle is solve 0). */
eg_status eg_layout(const eg_handle* h, int solve, int p, int64_t* offset, int* n_modes, int* n_elem);

/* Batched steady solve: V-cycles of all solves together until every solve
 * has r_n <= drop_tol r_1 (its own r_1) or max_cycles.  hist_host is
 * [n_solves][max_cycles + 1]: solve s's norms r_1, r_2, ... up to the cycle
 * it reached the drop, which n_cycles_host[s] receives.  The kernels keep
 * covering converged solves until all are done, but each converged solve's
 * state is saved at the cycle whose norm reached the drop and is what u_dev
 * returns for it.  A solve whose norm becomes non-finite is marked diverged
 * (its history ends there) and the others continue; its values never reach
 * the other solves.  Returns EG_OK when all converged, else EG_ERR_DIVERGED
 * if any diverged, else EG_ERR_NOT_CONVERGED. */
eg_status eg_solve_batch(eg_handle* h, double* u_dev, double drop_tol, int max_cycles, double* hist_host,
                         int* n_cycles_host);

/* Several batch handles (typically one per polynomial order of a
 * heterogeneous set of solves) advanced together, V-cycle by V-cycle, each
 * with the arithmetic and bookkeeping of eg_solve_batch (Section 2.4; the
 * CFL ramp of eq. (cfl) per solve).  Per cycle: the entry residual norms
 * of every running handle, one synchronisation, then one launch of the
 * cycle: when every handle has graph replay enabled (eg_set_graphs) a
 * single graph whose children are the handles' captured V-cycles (no
 * ordering between them, so the groups may overlap on the GPU), else the
 * handles' V-cycles one after another, eagerly.  A handle whose solves
 * have all converged or diverged stops running.  hs[nh]: distinct batch
 * handles on one device (all their work runs on hs[0]'s stream; the others'
 * streams must have no work the call depends on after it starts, and the
 * call synchronises before it returns); u_devs[k], hist_hosts[k] and
 * n_cycles_hosts[k] as the arguments of eg_solve_batch for handle k;
 * status_host[nh] (host): each handle's eg_solve_batch status.  Returns
 * the first error, else EG_ERR_DIVERGED if a solve diverged, else
 * EG_ERR_NOT_CONVERGED if a handle reached max_cycles, else EG_OK. */
eg_status eg_solve_multi(eg_handle* const* hs, int nh, double* const* u_devs, double drop_tol, int max_cycles,
                         double* const* hist_hosts, int* const* n_cycles_hosts, int* status_host);

/* ---- Adjoint drag sensitivity (discrete adjoint of the steady problem) ----
 * The paper solves R(u) = 0 (Section 2.1, eq. (starteq) at steady state);
 * these entries give d(functional)/d(parameter) for a converged u by the
 * discrete adjoint: (dR/du)^T lambda + dJ/du = 0, then
 * dJ/dtheta = dJ/dtheta|_u + lambda . dR/dtheta|_u. */

/* Pressure drag coefficient of the level-p_max state u_dev on the slip walls:
 *   C_D = -(1 / (q_inf S_ref)) sum_{wall faces} int p(U) n . dir dsigma,
 * n the element's outward unit normal (into the body), q_inf = |v_inf|^2 / 2
 * (rho_inf = 1), U the element's trace, the residual's face quadrature.
 * dir_host: host [d] direction (normally the free stream's); sref > 0.
 * cd_host receives C_D; grad_dev (may be NULL) dC_D/du (level p_max, psi
 * coordinates).  Synchronises. */
eg_status eg_drag(eg_handle* h, const double* u_dev, const double* dir_host, double sref, double* cd_host,
                  double* grad_dev);

/* Jacobian of the residual applied to a vector (Section 3.3, eqs. (jac1)
 * and (jac2): element-diagonal and neighbour blocks together), matrix free:
 * out_dev = (dR_p/du)(u_dev) v_dev at any level 0 <= p <= p_max, by
 * forward-mode differentiation of the residual (dual numbers with one
 * tangent at every quadrature point; the flux, ghost-state and Rusanov
 * derivatives are exact, with the tie rules of the block Jacobians).  All
 * level-p vectors in the ABI's psi coordinates.  Uses the handle's residual
 * workspace of level p (not while a solve runs on the handle).
 * Asynchronous. */
eg_status eg_jacobian_apply(eg_handle* h, int p, const double* u_dev, const double* v_dev, double* out_dev);

/* Transposed Jacobian of the residual (Section 3.3, eqs. (jac1), (jac2),
 * transposed): out_dev = (dR_p/du)(u_dev)^T w_dev at level p >= 1, matrix
 * free from the pointwise flux Jacobians at u_dev.  All level-p vectors.
 * Asynchronous. */
eg_status eg_adjoint_apply(eg_handle* h, int p, const double* u_dev, const double* w_dev, double* out_dev);

/* Adjoint solve (dR/du)(u_dev)^T lambda + g_dev = 0 at level p_max by the
 * transposed linear V-cycle: transposed PRK smoother (Section 2.3 with
 * P^T, blocks frozen at u_dev with dtau at cfl_max), truncation / padding
 * transfers, and on p = 0 one EXP1 step (Sections 2.1-2.2) of the linear
 * adjoint problem with the transposed p = 0 operator.  lam_dev: initial
 * guess in, solution out.  Stops when the 2-norm of the adjoint residual
 * has dropped by drop_tol; hist_host[0..*n_cycles_host] as for
 * eg_solve_steady.  Orders with a transposed block solve: 2D p <= 4 and 3D
 * p <= 3 (else EG_ERR_UNSUPPORTED).
 * Runs in FP64 on every handle.  Synchronises. */
eg_status eg_adjoint_solve(eg_handle* h, const double* u_dev, const double* g_dev, double* lam_dev, double drop_tol,
                           int max_cycles, double* hist_host, int* n_cycles_host);

/* One component of the adjoint gradient of the drag coefficient with
 * respect to a parameter theta of the problem (free-stream Mach number, a
 * wall-bump amplitude, ...): with lambda the adjoint solution at the
 * converged state u (eg_adjoint_solve with g = dC_D/du),
 *   dC_D/dtheta = dC_D/dtheta|_u + lambda . dR/dtheta|_u,
 * both partial derivatives at fixed coefficients u taken as central
 * differences over the handles hp and hm, built at theta + step and
 * theta - step (same mesh topology, element count, order and device; their
 * own geometry and free stream).  u_dev, lam_dev: level-p_max vectors
 * (psi coordinates); dir_host, sref: as eg_drag.  The residuals, their
 * difference and the dot product with lambda run in the library's kernels
 * (FP64, deterministic sums); uses both handles' residual workspaces.
 * dj_host receives dC_D/dtheta.  Synchronises both streams. */
eg_status eg_param_sensitivity(eg_handle* hp, eg_handle* hm, double step, const double* u_dev, const double* lam_dev,
                               const double* dir_host, double sref, double* dj_host);

/* Profiling aid: HIP-event timing of the solver's own kernel launches, by
 * kernel class and level, recorded on the handle's stream while enabled.
 * eg_profile(h, 1) clears the records and starts recording, eg_profile(h, 0)
 * stops; eg_profile_read sums the durations of class kernel_class at level p
 * (p < 0: all levels).  Both synchronise the stream. */
enum {
  EG_K_RESIDUAL = 0,     /* DG residual */
  EG_K_JACOBIAN_LU = 1,  /* element Jacobian block assembly + LU of the PRK block */
  EG_K_PRK_STAGE = 2,    /* PRK stage block solve and update */
  EG_K_TRANSFER = 3,     /* restriction, FAS forcing, prolongation, state copies */
  EG_K_TIMESTEP = 4,     /* pseudo-time step */
  EG_K_P0_SETUP = 5,     /* p = 0 residual, Jacobian blocks and right-hand side */
  EG_K_ARNOLDI = 6,      /* Arnoldi process (two grid-wide kernels per step) */
  EG_K_PHI1 = 7,         /* phi_1 of the Hessenberg matrix */
  EG_K_EXP1_UPDATE = 8,  /* Krylov combination of the EXP1 update */
  EG_K_NORM = 9,         /* residual norm */
  EG_K_COUNT = 10
};
eg_status eg_profile(eg_handle* h, int enable);
eg_status eg_profile_read(eg_handle* h, int kernel_class, int p, double* total_ms, int* launches);

/* Achievable peaks of the current device, for roofline fractions (a
 * measurement aid, no passage of the paper): kind 0 = HBM bandwidth in GB/s
 * (1 GiB streaming copy, bytes read + written), 1 = FP64 matrix-core
 * TFLOP/s (16 x 16 x 4 FP64 products, eight independent chains per
 * wavefront), 2 = FP64 vector FMA TFLOP/s (sixteen independent chains per
 * lane).  Allocates and frees its own device buffers; runs on hip_stream
 * (NULL: default stream) and synchronises it.  EG_ERR_ARG for another kind,
 * EG_ERR_HIP if a HIP call fails. */
eg_status eg_measure_peak(int kind, void* hip_stream, double* value_host);

/* ------------------------------------------------------------------------
 * Tetrahedra and prisms with the Cartesian basis (Section 3.2).
 *
 * The paper's basis: on every element the normalised monomials
 * chi_j(x) = prod_k ((x_k - xc_k) / L_k)^{a_k} of total degree <= p
 * (eq. (basis2); xc the element centroid, L_k half the element's extent
 * along axis k), orthonormalised by modified Gram-Schmidt in the element's
 * L2 inner product (eq. (basis)): psi_i = sum_{j<=i} S_ij chi_j, S lower
 * triangular.  N_p = (p+1)(p+2)(p+3)/6 modes, ordered by total degree, then
 * a_x descending, then a_y descending, so level p-1 is the leading slice.
 * Coefficient vectors are [elem][var][mode] FP64, V = 5 variables.
 *
 * Mesh (eg_poly_mesh, host arrays, copied): elem_type 0 = tetrahedron
 * (first four vertices, det(v1-v0, v2-v0, v3-v0) > 0), 1 = prism (bottom
 * v0 v1 v2, top v3 v4 v5, v_{a+3} above v_a, det(v1-v0, v2-v0, v3-v0) > 0);
 * elem_vert [n_elem][6] (tetrahedra pad with -1); bface_tag [n_elem][5]
 * with the tags of eg_mesh.  Local faces: tetrahedron face k omits v_k;
 * prism faces (v0 v1 v2), (v3 v4 v5), (v0 v1 v4 v3), (v1 v2 v5 v4),
 * (v2 v0 v3 v5).  Interior faces are matched through their vertex sets.
 * Straight-sided elements only.
 *
 * Quadrature with Q = p+2 Gauss-Legendre points per direction on [0, 1],
 * collapsed on simplices: tetrahedron barycentrics l1 = t1(1-t2)(1-t3),
 * l2 = t2(1-t3), l3 = t3 (weight factor (1-t2)(1-t3)^2); prism triangle
 * l1 = t1(1-t2), l2 = t2 (factor 1-t2) times zeta = t3 with the pointwise
 * Jacobian of the map; triangular faces l1 = t1(1-t2), l2 = t2 over the
 * face's vertices in ascending global id; quadrilateral faces the tensor
 * rule on the bilinear patch of the corners, cyclic from the lowest id
 * towards its lower-id neighbour.  The basis of every level comes from the
 * volume rule of p_max.
 * ------------------------------------------------------------------------ */
typedef struct eg_poly_handle eg_poly_handle;

typedef struct {
  int n_vert;
  const double* xyz;         /* host, [n_vert][3] */
  int n_elem;
  const int8_t* elem_type;   /* host, [n_elem]: 0 tetrahedron, 1 prism */
  const int32_t* elem_vert;  /* host, [n_elem][6] */
  const int8_t* bface_tag;   /* host, [n_elem][5]: 0 interior, 1 wall, 2 far-field, 4 symmetry */
} eg_poly_mesh;

/* Set-up on the current device: face matching, centroids, extents and the
 * per-element MGS basis (on the host), device copies.  Uses p_max (0..3),
 * rk_stages (>= 1), krylov_m (1..48), cfl_max (> 0), gamma, mach,
 * alpha_deg, beta_deg and flux of prm; the other fields are ignored.  EG_ERR_ARG for bad sizes or parameters, EG_ERR_MESH for an
 * unmatched face, a bad tag or vertex id, a non-positive element or a
 * degenerate basis; EG_ERR_ALLOC / EG_ERR_HIP for device failures.  *out is
 * set (and must be freed) whenever the status is not EG_ERR_ARG from a null
 * out pointer. */
eg_status eg_poly_init(const eg_poly_mesh* mesh, const eg_params* prm, void* hip_stream, eg_poly_handle** out);
void eg_poly_free(eg_poly_handle* h);
const char* eg_poly_last_error(const eg_poly_handle* h);

/* Uniform free stream at level p: u_{E,v,0} = U_inf,v / S_00, other modes 0
 * (u_dev: n_elem * 5 * N_p doubles, device). */
eg_status eg_poly_freestream(eg_poly_handle* h, int p, double* u_dev);

/* DG residual R_p(u) of eq. (euler3) on the tetrahedra and prisms:
 * R_{E,i} = -sum_faces int psi_i F~ . n dsigma + int_E F . grad psi_i dx,
 * with the handle's numerical flux and the ghost states of eg_mesh tags
 * (Section 3.3).  u_dev, r_dev: n_elem * 5 * N_p doubles, device, distinct.
 * Enqueued on the handle's stream, no synchronisation. */
eg_status eg_poly_residual(eg_poly_handle* h, int p, const double* u_dev, double* r_dev);

/* Element block D_E = dR_E / du_E of the level-p residual (Section 3.3,
 * eq. (jac1): volume term and the own-side derivative of every face flux,
 * ghost states included; neighbours held fixed), exact (forward-mode dual
 * numbers at the quadrature points).  D_dev: n_elem * n * n doubles,
 * n = 5 N_p, element after element, each block row-major with rows and
 * columns ordered (v, i) (variable-major, the layout of a coefficient
 * vector).  u_dev: level-p state (device).  No synchronisation. */
eg_status eg_poly_element_block(eg_poly_handle* h, int p, const double* u_dev, double* D_dev);

/* One s-stage PRK step on the tetrahedra and prisms (Section 2.3,
 * eq. (prk_scalar)), in place on the level-p state u_dev (device, p >= 1):
 * u^(k) = u^n + beta_k P^{-1} [R(u^(k-1)) + f], beta_k = 1/(s-k+1), with
 * P = I/dtau_E - D_E (dtau of eg_poly_timestep at this cfl, D_E of
 * eg_poly_element_block, both at u^n) factorised by LU with partial
 * pivoting.  f_dev: forcing (level p, device) or NULL; must not alias u_dev.
 * The first call allocates the handle's work buffers for p_max
 * (n_elem (5 N)^2 doubles for the blocks).  Synchronises the stream.
 * EG_ERR_DIVERGED (message set) if a block has a zero or non-finite pivot. */
eg_status eg_poly_prk_step(eg_poly_handle* h, int p, int s, double cfl, double* u_dev, const double* f_dev);

/* EXP1 on the p = 0 level (Section 2.1, eq. (EXP1); Section 2.2), the step
 * of the hexahedra: u0 += phi_1(A) b approximated by beta V_m phi_1(H_m) e_1
 * (krylov_m of eg_poly_init), A = T J_0 with the exact p = 0 Jacobian J_0
 * (element and neighbour blocks), b = T (R_0(u0) + f0),
 * T = diag((p_max+1) dtau_E), dtau at p_max and this cfl from the cell means.
 * u0_dev: level-0 state (device), updated in place; f0_dev: forcing or NULL
 * (not aliasing u0_dev).  Synchronises the stream.  EG_ERR_DIVERGED if phi_1
 * fails (non-finite Hessenberg matrix). */
eg_status eg_poly_exp1_step(eg_poly_handle* h, double cfl, double* u0_dev, const double* f0_dev);

/* One eMG V-cycle (Section 2.4) on the level-p_max state u_dev (p_max >= 1),
 * the cycle of the hexahedra with the parameters of eg_poly_init
 * (rk_stages, krylov_m, cfl_max): PRK on p >= 1, FAS forcing
 * f_{p-1} = Trunc(R_p(u) + f_p) - R_{p-1}(Trunc u), EXP1 on p = 0, the coarse
 * correction added to the leading modes.  Cycle n >= 1 and the reference
 * norm rref (0: the entry norm) enter the CFL ramp of eq. (cfl); rn_host and
 * cfl_host (may be NULL) receive the entry norm and the CFL.  The first call
 * allocates the level and Krylov buffers.  Synchronises.  EG_ERR_DIVERGED on
 * a non-finite norm, a zero pivot or a failed phi_1. */
eg_status eg_poly_vcycle(eg_poly_handle* h, double* u_dev, int n, double rref, double* rn_host, double* cfl_host);

/* Steady solve: V-cycles until r_n <= drop_tol r_1 (EG_OK) or max_cycles
 * (EG_ERR_NOT_CONVERGED); hist_host[0..*n_cycles_host] receives r_1, r_2, ...
 * (max_cycles + 1 entries); the ramp uses r_1 as its reference. */
eg_status eg_poly_solve_steady(eg_poly_handle* h, double* u_dev, double drop_tol, int max_cycles, double* hist_host,
                               int* n_cycles_host);

/* Pseudo-time step (Section 4, eq. (x3d)), the definition of the
 * hexahedra: dtau_E = cfl h_E / ((2p+1)(|v| + c)), h_E = 2 d |E| / |dE|,
 * v and c from the cell-mean state u_{E,.,0} psi_0.  u_dev: n_elem * 5 * N_p
 * doubles, dtau_dev: n_elem doubles (device).  No synchronisation. */
eg_status eg_poly_timestep(eg_poly_handle* h, int p, double cfl, const double* u_dev, double* dtau_dev);

/* Density-residual norm (Section 4, the norm under eq. (cfl)):
 * (1/|Omega|) (sum over elements and modes of r_{E,0,i}^2)^(1/2), the L2
 * norm of the density residual in the orthonormal basis.  r_dev: level-p
 * vector (device); *rn_host receives the value.  Synchronises the stream;
 * uses a small buffer of the handle, so calls on one handle must not
 * overlap. */
eg_status eg_poly_rnorm(eg_poly_handle* h, int p, const double* r_dev, double* rn_host);

/* Transfers between levels pc <= pf (Section 2.4, modal truncation): with
 * the hierarchical basis, restriction copies the leading N_pc modes of each
 * [elem][var] row (yc_dev: level pc, xf_dev: level pf), prolongation adds
 * the coarse vector to those leading modes (zero padding).  Device buffers,
 * distinct; no synchronisation. */
eg_status eg_poly_restrict(eg_poly_handle* h, int pf, int pc, const double* xf_dev, double* yc_dev);
eg_status eg_poly_prolong_add(eg_poly_handle* h, int pc, int pf, const double* yc_dev, double* xf_dev);

/* Copies of the set-up (host buffers): S [n_elem][N_pmax][N_pmax] (row i
 * holds S_ij, j <= i), xc [n_elem][3], L [n_elem][3], vol [n_elem]; any
 * pointer may be NULL. */
eg_status eg_poly_basis(const eg_poly_handle* h, double* S_host, double* xc_host, double* L_host, double* vol_host);

#ifdef __cplusplus
}
#endif

#endif /* EG_H */
