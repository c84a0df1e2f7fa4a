/*
 * tcf.h - C ABI of the MI355X (gfx950) thermocapillary two-phase flow step.
 *
 * The library advances incompressible two-phase volume-of-fluid flow with
 * temperature-dependent surface tension (Zimbrod, Schreter, Schilp 2022,
 * arXiv 2209.09671) by one projection step on a uniform Cartesian MAC grid:
 *
 *   S1  WENO5 upwind transport of the volume fraction alpha (eq. 1) and the
 *       temperature T (energy equation, named in Section "Theory"), SSP-RK3,
 *       face velocity frozen at u^n;
 *   S2  material laws from clamp(alpha, 0, 1); surface tension computed as a
 *       field sigma(T) (Section "Implementation");
 *   S3  interface geometry: delta_s = |grad alpha| (eq. 6), n = grad alpha /
 *       delta_s (eq. 7), curvature kappa = -div n, Marangoni vector
 *       M = delta_s (I - n n^T) grad sigma (eqs. 4, 5);
 *   S4  face CSF force (eq. 4): normal part sigma kappa grad alpha plus the
 *       tangential Marangoni part;
 *   S5  momentum predictor u* (WENO5 convection, variable-viscosity stress,
 *       CSF force divided by the face density);
 *   S6  b = D u* / dt made mean-free;
 *   S7  A p = b with A = D (1/rho_f) G, matrix free, solved by conjugate
 *       gradients preconditioned by a geometric multigrid V-cycle, warm
 *       started from p^n, gauge mean(p) = 0;
 *   S8  projection u^{n+1} = u* - dt (1/rho_f) G p.
 *
 * Layout (every field): structure of arrays, C order, x fastest.
 *   cell fields alpha, T, p : nx*ny*nz values, index i + nx*(j + ny*k)
 *   x-face velocity u       : (nx+1)*ny*nz,   index i + (nx+1)*(j + ny*k)
 *   y-face velocity v       : nx*(ny+1)*nz,   index i + nx*(j + (ny+1)*k)
 *   z-face velocity w       : nx*ny*(nz+1),   index i + nx*(j + ny*k)   (3D only)
 * Cell (i,j,k) has centre ((i+1/2)h, (j+1/2)h, (k+1/2)h).  Wall faces
 * (index 0 and n along their own axis) carry zero velocity.  In 2D nz == 1
 * and there is no w.  Phase 1 is alpha = 0, phase 2 alpha = 1.
 *
 * Pointers passed to tcf_set_fields / tcf_get_fields / tcf_solve_pressure /
 * tcf_predictor / tcf_apply_A are DEVICE pointers to FP64 arrays in both
 * precision modes (the FP32 mode converts internally).  The caller owns them
 * and the workspace; the library never allocates device memory.
 *
 * Streams: all device work is enqueued on the hip_stream given at init.
 * Calls synchronise that stream only where they must read a device value on
 * the host (pressure-solver convergence tests, and info when requested).
 *
 * Errors: every call returns a tcf_status, never throws and never aborts;
 * tcf_last_error() returns a message for the calling thread.  TCF_E_INVALID
 * leaves the state unchanged.  TCF_E_NOT_CONVERGED completes the step with
 * the best pressure iterate.  TCF_E_NONFINITE stops at the first step whose
 * residual or fields are not finite and leaves that step's output in place.
 */
#ifndef TCF_H_
#define TCF_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TCF_OK = 0,
  TCF_E_INVALID = 1,       /* bad argument; nothing changed */
  TCF_E_DEVICE = 2,        /* a HIP runtime call failed */
  TCF_E_NOT_CONVERGED = 3, /* pressure solve reached its iteration limit */
  TCF_E_NONFINITE = 4,     /* NaN/Inf in the residual or the fields */
  TCF_E_STATE = 5,         /* fields not set yet */
  TCF_E_WORKSPACE = 6      /* workspace too small or misaligned */
} tcf_status;

typedef enum {
  TCF_FP64 = 0,        /* everything in FP64 */
  TCF_FP32_REFINE = 1  /* FP32 stencils and inner Poisson solve; FP64 refinement
                          residual, CG scalars, sums, and u, v, w, p storage */
} tcf_precision;

enum {
  TCF_TRANSPORT_ONLY = 1, /* tcf_step runs S1 only (velocity frozen, p kept) */
  TCF_WITH_ADJOINT = 2    /* reserve adjoint workspace (needs precision TCF_FP64) */
};

typedef struct tcf_grid tcf_grid; /* opaque, host side */

/* Plain parameter block, copied at init. */
typedef struct tcf_config {
  int dim, nx, ny, nz;     /* dim 2 => nz must be 1 */
  double h;                /* uniform cell size */
  int precision;           /* tcf_precision */
  int flags;               /* TCF_TRANSPORT_ONLY or 0 */
  double rho1, rho2, mu1, mu2, rhocp1, rhocp2, lambda1, lambda2; /* phase 1 (alpha=0), phase 2 */
  double sigma0, dsigma_dT, T0;  /* sigma(T) = sigma0 + dsigma_dT (T - T0) */
  int T_bc[6];             /* walls -x,+x,-y,+y,-z,+z : 0 Neumann, 1 Dirichlet */
  double T_wall[6];        /* Dirichlet wall temperatures */
  double q_power, q_radius, q_x0, q_y0, q_vx, q_vy; /* Gaussian surface heat flux, 0 power = off */
  double weno_eps;         /* WENO smoothness epsilon (1e-6) */
  double normal_eps;       /* regularisation of |grad alpha| (1e-6 / h) */
  double p_rtol;           /* FP64 relative residual target of the pressure solve */
  int p_maxit;             /* CG iteration limit (FP64 mode; per inner solve in FP32 mode) */
  double inner_rtol;       /* FP32 inner solve relative tolerance */
  int refine_maxit;        /* FP64 refinement sweeps limit (FP32 mode) */
  int mg_levels;           /* 0 = automatic */
  int mg_nu;               /* Jacobi sweeps before and after the coarse correction */
  /* Initial guess of each step's pressure solve: the polynomial
   * extrapolation in time of order p_extrapolate (0, 1 or 2) through the
   * last pressures, 0: p^n; 1: 2 p^n - p^(n-1); 2: 3 p^n - 3 p^(n-1) +
   * p^(n-2).  The order is limited by the previous pressures the grid holds
   * (none after tcf_set_fields; one more after each step, or as given to
   * tcf_set_pressure_history).  With integrator 1 each of the three stage
   * solves extrapolates that stage's pressures of the last steps (kept
   * inside the grid, cleared by tcf_set_fields, not exposed).  Only the
   * iteration count changes: every solve still runs to p_rtol.
   * (tcf_step_backward sets the state without history: its recomputed
   * forward step starts from the pressure of the state it was given for
   * the step after.) */
  int p_extrapolate;
  /* Solutal Marangoni (eq. 5: the surface-tension gradient is the chain rule
   * over temperature and concentration; in-situ alloying).  species = 1
   * carries a concentration field c (cell centres, set with tcf_set_species)
   * with the same WENO5 / SSP-RK3 transport as alpha (no diffusion, no flux
   * through walls) and adds dsigma_dc (c - c0) to sigma.  0 = no species
   * (dsigma_dc, c0 ignored).  Not combined with TCF_WITH_ADJOINT. */
  int species;
  double dsigma_dc, c0;
  /* Time integrator.  0: SSP-RK3 transport of alpha, T (and c) with the
   * velocity frozen at u^n, then one forward-Euler momentum predictor and
   * one projection (first order in time overall).  1: time-accurate
   * variant, SSP-RK3 (Shu-Osher) over the whole state (alpha, T, c, u) with
   * a projection in every stage: each stage takes all right-hand sides
   * (transport with the stage velocity, heat source at the stage time t,
   * t + dt, t + dt/2, geometry, CSF force, predictor) at the stage state and
   * projects the combined velocity with that state's density (three
   * pressure solves per step, third order in time).  The paper does not
   * state its integrator.  1 is not combined with TCF_WITH_ADJOINT. */
  int integrator;
  /* N-phase VOF (eq. 1 for every phase of several in one domain).  0 or 2:
   * the two-phase model (alpha = phase 2, phase 1 the rest).  3 or 4: the
   * fractions of phases 3 and 4 (set with tcf_set_phases) are carried by
   * the same WENO5 / SSP-RK3 transport as alpha; phase 1 is the background
   * with alpha_1 = 1 - the others.  Material laws are linear in each clamped
   * fraction relative to phase 1 (P = P_1 + sum_j clamp(alpha_j)(P_j - P_1),
   * phases 1 and 2 from rho1, rho2, ... above, phases 3 and 4 from the
   * arrays below).  Every pair of phases i < j has its own surface tension
   * sigma_ij = pair_sigma0 + pair_dsigma_dT (T - T0), acting through the
   * pair gradient alpha_i grad alpha_j - alpha_j grad alpha_i with the
   * curvature and Marangoni terms of eqs. 4-7; pairs are ordered (1,2),
   * (1,3), (1,4), (2,3), (2,4), (3,4) (sigma0, dsigma_dT are not used).  The
   * heat source acts at the boundary of the condensed fraction 1 - alpha_1.
   * Not combined with species, integrator 1 or TCF_WITH_ADJOINT. */
  int nphases;
  double rho34[2], mu34[2], rhocp34[2], lambda34[2];
  double pair_sigma0[6], pair_dsigma_dT[6];
} tcf_config;

typedef struct tcf_step_info {
  int cg_iters;      /* CG iterations of the last step (summed over refinements) */
  int refine_iters;  /* FP64 refinement sweeps of the last step (FP32 mode) */
  double p_relres;   /* ||b - A p|| / ||b|| in FP64 after the last step */
  double div_rel;    /* ||D u^{n+1}|| / ||D u*|| of the last step */
  double sum_alpha;  /* sum of alpha over cells (FP64) after the last step */
  double alpha_min, alpha_max;
  double cfl_max;    /* dt max|u_f| / h after the last step */
  int nonfinite;     /* 1 if a non-finite value was seen */
} tcf_step_info;

/* Bytes of device workspace needed for this configuration (0 if invalid). */
size_t tcf_workspace_bytes(const tcf_config* cfg);

/* Validate cfg and carve the caller's workspace (device memory, 256-byte
 * aligned, at least tcf_workspace_bytes bytes).  hip_stream is a hipStream_t
 * (NULL = default stream).  *out receives a host-side handle.  Besides the
 * workspace the grid holds a 320-byte block of pinned host memory, mapped
 * and coherent, into which the device writes the solver scalars the host
 * reads (the host polls it, querying the stream now and then, so that a
 * failed stream ends the wait with TCF_E_DEVICE), a second stream of the
 * current device for work that overlaps within a step, and three events;
 * tcf_destroy releases them.  TCF_E_DEVICE if any of them cannot be made. */
tcf_status tcf_init_grid(const tcf_config* cfg, void* workspace, size_t bytes, void* hip_stream,
                         tcf_grid** out);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): tcf_init_grid with
 * the workspace taken from a fixed device array inside the library instead
 * of a caller allocation.  Each GPU holds one such array of
 * TCF_STATIC_WORKSPACE_BYTES (128 MiB) from its first use until the process
 * ends; the grid lives on the device current at the call.  The call
 * allocates nothing: no device or pinned host memory (the handle and its
 * host mirror of the solver scalars are slots inside the library, one per
 * GPU) and, after the first call on a device, no event either.  Every other
 * entry point works on the handle as on any grid, and tcf_destroy releases
 * the slot.
 *   TCF_E_WORKSPACE : tcf_workspace_bytes(cfg) exceeds the fixed array
 *                     (e.g. 2D up to 512^2, 3D up to 128 x 64 x 64 fit);
 *   TCF_E_STATE     : a grid on this GPU's fixed workspace is still open
 *                     (one at a time per GPU; destroy it first);
 *   TCF_E_INVALID   : as tcf_init_grid.
 * Successive grids on one GPU share the array and find the last grid's
 * contents in it: the call clears what must start at zero, and everything
 * else is written before it is read.  The handle's calls are ordered on its
 * stream; calls on it from several host threads at once race, as on any
 * grid.  Its solver scalars are read back through pageable host memory, with
 * a stream synchronisation per read (no overlap of that read with queued
 * work). */
#define TCF_STATIC_WORKSPACE_BYTES ((size_t)128 << 20)
tcf_status tcf_init_grid_static(const tcf_config* cfg, void* hip_stream, tcf_grid** out);

/* Copy the state in (device FP64 pointers, layout above).  w must be NULL in
 * 2D; p may be NULL (zero pressure).  Wall-face velocities are forced to 0. */
tcf_status tcf_set_fields(tcf_grid* g, double t, const double* alpha, const double* T, const double* u,
                          const double* v, const double* w, const double* p);

/* Copy the state out (device FP64 pointers; any may be NULL to skip). */
tcf_status tcf_get_fields(const tcf_grid* g, double* t, double* alpha, double* T, double* u, double* v,
                          double* w, double* p);

/* Previous pressures of the extrapolated initial guess (p_extrapolate > 0):
 * held = how many are held (0 .. p_extrapolate), p1 = p^(n-1), p2 =
 * p^(n-2) (device FP64, cell layout like p; p1 is read / written when held
 * >= 1, p2 when held = 2, otherwise they may be NULL).  A run restarted
 * from tcf_get_fields plus this history repeats the uninterrupted run
 * bitwise.  tcf_set_fields clears the history.  TCF_E_STATE on a grid that
 * keeps no such history (p_extrapolate = 0, or integrator 1, whose
 * per-stage histories stay internal); TCF_E_INVALID on a NULL grid or held pointer, held
 * out of range, or a NULL pointer that held requires. */
tcf_status tcf_get_pressure_history(const tcf_grid* g, double* p1, double* p2, int* held);
tcf_status tcf_set_pressure_history(tcf_grid* g, const double* p1, const double* p2, int held);

/* Species field of a grid made with species = 1: copy in / out (device FP64,
 * nx*ny*nz cells in the layout above).  TCF_E_STATE on a grid without a
 * species; TCF_E_INVALID on a NULL pointer.  tcf_step needs it set once. */
tcf_status tcf_set_species(tcf_grid* g, const double* c);

/* Fractions of phases 3 and 4 of a grid made with nphases = 3 or 4: copy in
 * / out (device FP64, cell layout like alpha; a4 is ignored and may be NULL
 * when nphases = 3).  TCF_E_STATE on a two-phase grid or (get) before they
 * are set; TCF_E_INVALID on a missing pointer.  tcf_step needs them set. */
tcf_status tcf_set_phases(tcf_grid* g, const double* a3, const double* a4);
tcf_status tcf_get_phases(const tcf_grid* g, double* a3, double* a4);
tcf_status tcf_get_species(const tcf_grid* g, double* c);

/* Advance nsteps steps of size dt (S1..S8 each).  info may be NULL; when set
 * it receives the diagnostics of the last step (forces a stream sync). */
tcf_status tcf_step(tcf_grid* g, double dt, int nsteps, tcf_step_info* info);

/* Solve A p = rhs (S7) with the operator built from the grid's current alpha.
 * rhs is made mean-free first; p holds the initial guess on entry and the
 * mean-free solution on exit.  Device FP64 pointers of nx*ny*nz values. */
tcf_status tcf_solve_pressure(tcf_grid* g, const double* rhs, double* p, tcf_step_info* info);

/* Diagnostics of single sub-steps (parity checks of the path's parts).
 * tcf_predictor: S2..S5 with the grid's current alpha, T, u taken as
 * (alpha^{n+1}, T^{n+1}, u^n); writes u* (device FP64, face layouts).
 * tcf_apply_A: y = A x with the grid's current alpha. */
tcf_status tcf_predictor(tcf_grid* g, double dt, double* us, double* vs, double* ws);
tcf_status tcf_apply_A(tcf_grid* g, const double* x, double* y);

/* Adjoint of one step (the transposed linearisation of S1..S8 at state n),
 * row "adjoint" of the path; needs a grid created with TCF_WITH_ADJOINT.
 *   state_n  : alpha, T, u, v, w, p at step n (device FP64; w NULL in 2D; p
 *              may be NULL - it is only the warm start of the recomputed solve)
 *   adj_np1  : dL/d(alpha, T, u, v, w) at step n+1 (wall-face entries ignored)
 *   adj_n    : written with dL/d(alpha, T, u, v, w) at step n (wall faces 0)
 *   dL_dsigmaT: device FP64 scalar, incremented by dL/d(dsigma_dT) of this step
 * The forward step is recomputed from state_n inside the call (WENO weights
 * and interface geometry are recomputed, not stored).  The pressure adjoint
 * reuses the symmetric operator of S7 (one extra solve at p_rtol).  The
 * derivative of clamp(alpha,0,1) is taken as 1 inside (0,1) and 0 outside,
 * and the upwind side follows the sign of the advecting velocity.  Adjoint
 * sums use FP64 atomics: results agree to rounding, not bitwise, run to run.
 * Afterwards the grid's fields are unspecified: call tcf_set_fields again
 * before tcf_step.  Entries of adj_n must not alias adj_np1 or state_n.
 * TCF_E_INVALID on a grid created with TCF_TRANSPORT_ONLY (whose step is S1
 * alone; tcf_adjoint_transport is its adjoint). */
tcf_status tcf_step_backward(tcf_grid* g, double t_n, double dt, const double* const state_n[6],
                             const double* const adj_np1[5], double* const adj_n[5], double* dL_dsigmaT);

/* The same adjoint step with the forward step's intermediates supplied
 * instead of recomputed (a checkpointed rollout replays each segment anyway):
 *   tcf_step_keep: one forward step exactly as tcf_step(g, dt, 1, NULL) on a
 *     TCF_WITH_ADJOINT grid, which also writes the transport's stage values
 *     alpha^(1), T^(1), alpha^(2), T^(2) (SSP-RK3 stages 1 and 2, device FP64,
 *     nx*ny*nz each, caller-owned, distinct and not the grid's own arrays)
 *     into stages[0..3]; the transport writes them there directly.  With
 *     p_np1 non-NULL (device FP64, nx*ny*nz) the pressure solve S6-S7 is
 *     skipped and p_np1 is taken as p^{n+1}: given the pressure an earlier
 *     run of the same step returned (tcf_get_fields after it), the new state
 *     is bitwise that run's (a rollout that kept every step's pressure
 *     replays its segments without solving).  The grid's pressure becomes
 *     p_np1 and its pressure history is emptied.
 *   tcf_step_backward_kept: tcf_step_backward(g, t_n, dt, state_n, adj_np1,
 *     adj_n, dL_dsigmaT) given stages (from tcf_step_keep of this step) and
 *     state_np1 = alpha, T, p of step n+1 (the state that step produced).
 *     Only the interface geometry and the pressure operator of step n+1 are
 *     recomputed; the transport, predictor and forward solve are not run.
 *     The result equals tcf_step_backward's to rounding when the inputs are
 *     those of one forward step (other inputs give the adjoint of a step that
 *     did not happen).  Same errors as tcf_step_backward, and TCF_E_INVALID
 *     for a NULL stage or state_np1 pointer; the grid's fields are left
 *     unspecified in the same way. */
tcf_status tcf_step_keep(tcf_grid* g, double dt, double* const stages[4], const double* p_np1);
tcf_status tcf_step_backward_kept(tcf_grid* g, double t_n, double dt, const double* const state_n[6],
                                  const double* const stages[4], const double* const state_np1[3],
                                  const double* const adj_np1[5], double* const adj_n[5], double* dL_dsigmaT);

/* Adjoints of single sub-steps at the grid's current fields (checks of the
 * adjoint against finite differences of tcf_step(TCF_TRANSPORT_ONLY) and
 * tcf_predictor).  tcf_adjoint_transport: (ab_in, Tb_in) is dL/d(alpha, T)
 * after S1; writes dL/d(alpha, T) before it and dL/d(u, v, w) (all device
 * FP64, no aliasing of in and out).  tcf_adjoint_predictor: (usb, vsb, wsb)
 * is dL/du*; writes dL/d(alpha, T, u, v, w) and sbar = dL/d(dsigma_dT)
 * (device scalar, overwritten). */
tcf_status tcf_adjoint_transport(tcf_grid* g, double dt, const double* ab_in, const double* Tb_in, double* ab_out,
                                 double* Tb_out, double* ub, double* vb, double* wb);
tcf_status tcf_adjoint_predictor(tcf_grid* g, double dt, const double* usb, const double* vsb, const double* wsb,
                                 double* ab, double* Tb, double* ub, double* vb, double* wb, double* sbar);

/* Measurement: time every launch of one kernel family with HIP events on
 * the grid's stream ("transport", "geometry", "predictor", "smooth" = the
 * finest-level Jacobi sweeps, "spmv", "update" = the fused CG update and
 * first sweep, "resid64", "project", "species" = the species transport
 * stages; NULL or "" turns
 * timing off and clears the totals).  tcf_profile_read synchronises on the
 * last recorded event and returns the summed milliseconds and the number of
 * timed launches since tcf_profile was called. */
tcf_status tcf_profile(tcf_grid* g, const char* family);
tcf_status tcf_profile_read(tcf_grid* g, double* total_ms, long* launches);

/* Release the handle (the workspace stays the caller's). */
void tcf_destroy(tcf_grid* g);

/* Message of the last failed call on this thread ("" if none). */
const char* tcf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TCF_H_ */
