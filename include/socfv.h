/*
 * socfv — steady state-of-charge (SOC) solve on voxelised porous electrodes, MI355X.
 *
 * C ABI of the GPU library libsocfv.so.  Plain pointers and sizes only.
 *
 * The method (Emanuel & Rycroft, "Digital Twin for Porous Electrodes in Redox Flow
 * Batteries"): at a fixed flow field, the state of charge s obeys the transport equation
 * of Eq. (nernst-planck-soc), whose Butler-Volmer source is affine in s at a controlled
 * voltage (Eq. (rate-from-soc-gen)): a k0 K (s_eq - s).  The steady state is reached by the
 * explicit pseudo-time iteration of the Algorithm "SOC at Mass Transport Limit"
 * (s <- F s, electrode cells reset), stopped by the rule of Eq. (convergence-bv-change).
 * Its figure of merit is the utilisation U (Eq. (utilization-def)); in the fast-kinetics
 * limit (Eqs. (np-fast-interior), (np-fast-boundary)) with s_in = 0 and s = 1 on the
 * electrode it is U_mt (Eq. (umt-def)).
 *
 * Units.  Everything is nondimensional: voxel size h = 1, diffusivity D = 1, time in
 * h^2 / D.  Face velocities are given in units of D / h (a face Peclet number).  The
 * reaction enters as Da = k0 K h / D per fibre face of a surface cell, with
 * K = e^{alpha V} + e^{(alpha-1) V} the slope of the affine rate.
 *
 * Layout.  Grids are (nz, ny, nx), x fastest, cell index x + nx*(y + ny*z); flow enters
 * through the x = 0 plane and leaves through x = nx.  Staggered face velocities, positive
 * along +axis: ux (nz, ny, nx+1), uy (nz, ny+1, nx), uz (nz+1, ny, nx), FP64.
 *
 * Discretisation (finite volumes, one definition shared by every entry point):
 *   R_P(s) = sum_f [ -max(w_f,0) s_P - min(w_f,0) s_up(f) + G_f (s_nb(f) - s_P) ]
 *            + lam_P (s_eq - s_P),          lam_P = Da * kappa_P * n_f(P)
 * w_f = outward normal velocity of face f; interior faces (pore on both sides): upwind
 * value of the neighbour, G = 1; inlet faces: upwind value s_in, G = 2 (Dirichlet value
 * on the face); outlet faces: upwind value s_P, G = 0 (no concentration gradient); faces
 * shared with a fibre voxel and the y / z walls carry no flux and must have w = 0.
 * n_f(P) = number of faces P shares with fibre voxels (its specific area a = n_f / h).
 * Iteration: s <- s + dt R(s), dt = cfl / max_P (sum_f max(w_f,0) + sum_f G_f + lam_P)
 * (the maximum is scanned once per operator: again after socfv_set_velocity,
 * socfv_set_activity, or a solve with another Da or mode).
 * Residual: res = tau * sqrt(mean over pore cells of R_P^2) = (tau/dt)||s^{n+1}-s^n||_rms
 * with tau = nx*ny*nz / Q (nominal volume over inlet flow).
 *
 * Ownership.  Every pointer argument is owned by the caller.  Device pointers
 * (marked "device") must stay valid for the duration of the call only: the library
 * copies what it keeps into buffers it owns, freed by socfv_destroy.  All device work is
 * enqueued on the caller's HIP stream (NULL = default stream); calls return when their
 * outputs are complete.
 *
 * Errors.  Every int-returning call returns a socfv_status.  No exception crosses the
 * ABI; socfv_last_error() gives a message for the calling thread's last failure.
 * A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef SOCFV_H
#define SOCFV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SOCFV_OK = 0,
  SOCFV_NOT_CONVERGED = 1,   /* max_iter reached; outputs are still written */
  SOCFV_INVALID_ARG = -1,
  SOCFV_BAD_GEOMETRY = -2,   /* pore cell not face-connected to the inlet, no inlet/outlet pore */
  SOCFV_BAD_VELOCITY = -3,   /* non-finite, flux through a closed face, Q <= 0,
                                or divergence above the tolerance */
  SOCFV_DIVERGED = -4,       /* non-finite residual or s outside [min(s_in,s_eq), max(..)] */
  SOCFV_HIP_ERROR = -5,
  SOCFV_OOM = -6
} socfv_status;

enum { SOCFV_FINITE_RATE = 0, SOCFV_PINNED = 1 };
enum {
  SOCFV_FP64 = 0,            /* every sweep in FP64 */
  SOCFV_FP32 = 1,            /* FP32 sweeps on a correction against an FP64 residual,
                                FP64 reductions, FP64 refresh and polish */
  SOCFV_FP32_PLAIN = 2       /* FP32 sweeps on s itself until FP32 stagnates (diagnostic) */
};

typedef struct socfv_ctx socfv_ctx;

typedef struct {
  double s_in;        /* inlet Dirichlet value */
  double s_eq;        /* equilibrium SOC of the electrode (sigma(V)) */
  double Da;          /* reaction number per fibre face, k0 K h / D (FINITE_RATE) */
  int mode;           /* SOCFV_FINITE_RATE or SOCFV_PINNED (electrode cells held at s_eq) */
  int precision;      /* SOCFV_FP64, SOCFV_FP32 or SOCFV_FP32_PLAIN */
  double cfl;         /* dt = cfl / max diag; 0 < cfl <= 1 keeps the iteration monotone */
  double tol;         /* stop when res < tol */
  long max_iter;      /* cap on explicit sweeps (all precisions, FP64 polish included;
                         socfv_batch_solve counts in whole chunks of check_every sweeps) */
  int check_every;    /* sweeps between residual checks (>= 2, even; rounded up to even) */
  int polish_iters;   /* FP32 mode: FP64 sweeps after the last refresh once the residual
                         is below tol (0 = check_every), clipped to what max_iter leaves */
} socfv_params;

typedef struct {
  long iterations;    /* explicit sweeps done in total */
  long it_fp32;       /* FP32 sweeps */
  long it_fp64;       /* FP64 sweeps (FP64 mode, refreshes and polish) */
  int cycles;         /* FP32 mode: FP64 residual refreshes */
  int status;         /* socfv_status of the solve */
  double residual;    /* final residual tau * rms(R) (FP64 in FP64 / FP32 modes) */
  double dt, tau;     /* pseudo-time step and flow-through time */
  double U;           /* (sbar_out - s_in) / (s_eq - s_in) */
  double s_out;       /* outlet flux-weighted mean SOC, sum_out w s / sum_out w */
  double flux_in;     /* advective + diffusive inlet flux of s */
  double flux_in_adv; /* advective inlet flux only, sum_in u s_in */
  double flux_out;    /* sum_out w s */
  double reaction;    /* sum lam (s - s_eq) (finite rate) or what held cells absorb (pinned) */
  double sum_R;       /* sum of R over updated cells: flux_in - flux_out - reaction */
  double q_out;       /* outlet flow, sum_out w */
  double seconds;     /* wall time of the call */
  double ms_fp32;     /* GPU time of the FP32 sweeps (HIP events around each chunk) */
  double ms_fp64;     /* GPU time of the FP64 sweeps (excluding refreshes) */
  double ms_refresh;  /* GPU time of the FP64 residual refreshes */
  long sweeps_fp64;   /* FP64 sweeps excluding refreshes */
  int tile_y, z_chunk; /* launch shape of the sweeps used */
} socfv_stats;

/* Fill p with defaults: s_in 1, s_eq 0, Da 0.45, FINITE_RATE, FP32, cfl 0.4, tol 1e-8,
 * max_iter 10^8, check_every 200, polish_iters 0. */
void socfv_default_params(socfv_params *p);

/*
 * Geometry (pore / fibre voxels, the electrode's implicit-function description reduced to
 * voxels).  solid: device, uint8 (nz, ny, nx), nonzero = fibre voxel.  Builds the per-cell
 * flags (which faces touch fibre, pore bit) on the GPU and checks on the host that every
 * pore cell is face-connected to a pore cell of the inlet plane and that the outlet plane
 * has a pore cell (BAD_GEOMETRY otherwise).  *out receives a new context.
 */
int socfv_setup_geometry(socfv_ctx **out, int nx, int ny, int nz, const uint8_t *solid,
                         void *hip_stream);

/*
 * Face velocities (device, FP64, staggered layout above), multiplied by q (the flow is
 * linear in the driving pressure in the Stokes regime, so one field serves every flow
 * rate).  Stored in FP32 and FP64.  Rejects (BAD_VELOCITY) non-finite values, non-zero
 * velocity on a face shared with a fibre voxel or on a y/z wall, no net inflow (Q <= 0),
 * and a cell divergence above 1e-6 times the largest face velocity.  Flow may leave through
 * part of the inlet (a pressure-driven flow does so next to an obstacle near the inlet):
 * such a face carries the cell's value out (upwind), its Dirichlet diffusion unchanged.
 */
int socfv_set_velocity(socfv_ctx *c, const double *ux, const double *uy, const double *uz,
                       double q, void *hip_stream);

/* Per-voxel reaction activity kappa (device, FP32 (nz, ny, nx); NULL = 1 everywhere).
 * lam_P = Da * kappa_P * n_f(P). */
int socfv_set_activity(socfv_ctx *c, const float *kappa, void *hip_stream);

/*
 * Steady state by the explicit iteration.  In FP32 mode the loop's stop rule and refresh
 * decisions are taken on the device after every check_every sweeps; the host enqueues chunks
 * ahead and reads the state between groups of them.  s_init (device FP64 (nz,ny,nx), nullable):
 * start state (default s_in on pore cells); held cells always start at s_eq.
 * s_out (device FP64 (nz,ny,nx), nullable): steady state (fibre cells 0).  The state is
 * also kept in the context for socfv_solve_soc_adjoint.  st (host, nullable): stats,
 * including U and the flux balance of the final state.
 * Returns OK, NOT_CONVERGED (max_iter reached), DIVERGED or an error.
 */
int socfv_solve_soc_steady(socfv_ctx *c, const socfv_params *p, const double *s_init,
                           double *s_out, socfv_stats *st, void *hip_stream);

/*
 * Mass-transport-limited utilisation U_mt: the PINNED solve with s_in = 0, s_eq = 1
 * (p's mode, s_in, s_eq and Da are ignored; its precision, cfl, tol, max_iter,
 * check_every are used; p may be NULL for defaults).  *U_mt (host) receives the result;
 * s_out / st as in socfv_solve_soc_steady.
 */
int socfv_compute_umt(socfv_ctx *c, const socfv_params *p, double *U_mt, double *s_out,
                      socfv_stats *st, void *hip_stream);

/*
 * U and the flux balance of a given state s (device FP64 (nz,ny,nx); NULL = the state
 * of the last solve) under p's s_in / s_eq / Da / mode.  Writes the output fields of st
 * (U ... q_out) and st->residual (FP64 residual of that state).
 */
int socfv_evaluate(socfv_ctx *c, const socfv_params *p, const double *s, socfv_stats *st,
                   void *hip_stream);

/*
 * socfv_evaluate without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and kernels as socfv_evaluate; its per-block partials and reduced
 * values live in a static device array of 4 MiB per GPU (held until the process ends)
 * instead of the context's buffers, and it calls no hipMalloc / hipFree.  The context must
 * live on the current device (INVALID_ARG otherwise).  Limit: the grid's FP64 reduction
 * blocks, ceil(nx / 128) ceil(ny / 4) ceil(nz / zc) (64 for 128 when nx is odd; zc a power
 * of two from 2 to 128 picked by the march's chunk rule), times 8 partials plus 8 results must fit 2^19
 * doubles: at most 65,535 blocks (a 1024 x 512 x 256 grid has 2,048; a grid 2 cells wide and
 * 262,144 deep has 65,536) (INVALID_ARG beyond).  The array is shared by every
 * call on that GPU and keeps the last call's contents (every value is written before it is
 * read, so nothing needs clearing); calls that overlap on one GPU, from any thread or
 * context, race and must be serialised by the caller.
 */
int socfv_evaluate_noalloc(socfv_ctx *c, const socfv_params *p, const double *s,
                           socfv_stats *st, void *hip_stream);

/*
 * Discrete adjoint of U at the last steady state of this context (which must come from
 * socfv_solve_soc_steady with the same s_in, s_eq, Da, mode and cfl): solves
 * A^T psi = g, g = dU/ds (g_P = w_out,P / (Q_out (s_eq - s_in)) on outlet cells), by the
 * same explicit iteration with reversed advection, psi <- psi + dt (g - A^T psi), until
 * ||g - A^T psi||_2 / ||g||_2 < p->tol (FP64 sweeps, or FP32 sweeps on a correction
 * against FP64 refreshes, by p->precision).  Then
 *   dU_dkappa[P] = Da n_f(P) psi_P (s_eq - s_P)   (device FP64 (nz,ny,nx), nullable;
 *                                                 FINITE_RATE only, 0 elsewhere)
 *   *dU_dlnq     = sum_P psi_P Radv_P(s)          (host; derivative in ln q for u = q u0:
 *                                                 divide by q for dU/dq)
 * with Radv the advective part of R.  psi_out (device FP64, nullable) receives psi; held
 * cells (PINNED) get psi = 0 (no design variable enters their rows).
 */
int socfv_solve_soc_adjoint(socfv_ctx *c, const socfv_params *p, double *dU_dkappa,
                            double *dU_dlnq, double *psi_out, socfv_stats *st,
                            void *hip_stream);

/*
 * Many problems (contexts with geometry and velocity set; uneven sizes allowed) solved
 * together.  With every p[i].precision == SOCFV_FP32, each FP32 sweep is one launch over
 * a tile work list spanning all unfinished problems (persistent blocks taking tiles from a
 * device counter), and each problem keeps its own dt, tau, FP64 refreshes and stopping rule
 * (its own p[i]), all decided on the device: one chunk of check_every sweeps (rounded up to
 * a multiple of 4) with the work lists, the per-problem residuals and decisions and the
 * refreshes is captured once as a hipGraph and replayed, the host reading the problems'
 * states every few chunks to re-tile the remaining ones; the single-sweep block shape is
 * chosen by timing candidates on the batch.  The FP64 polish of the converged problems runs
 * as one launch per sweep over all of them (st[i].ms_fp64 is that shared time).  Other
 * precisions solve the problems one after another.  p, st: host arrays of n entries;
 * s_out: host array of n device pointers (nullable, entries nullable).  Returns the worst
 * status (OK < NOT_CONVERGED) or the first error.
 */
int socfv_batch_solve(int n, socfv_ctx *const *ctxs, const socfv_params *p,
                      double *const *s_out, socfv_stats *st, void *hip_stream);

/*
 * Explicit Nernst model (Sec. "Steady State Reaction Model (Nernst)", Algorithm "Explicit
 * Nernst Model", with the electrode value of Eq. (nernst-model-s-update)); FP64.  Electrode
 * cells (pore cells with a fibre face) are held at sigma(V - eta), V = logit(s_eq); every
 * iteration takes the transport step (advection and diffusion) on all pore cells, then on
 * electrode cells eta <- (1 - omega) eta + omega eta_I with eta_I = 2 asinh(-R_t /
 * (2 a k0 sqrt(s (1 - s)))) (Eq. (nernst-eta-inst-def), R_t the transport rate of the step,
 * a k0 = Da kappa n_f sqrt(s_eq (1 - s_eq)) per cell) and s = sigma(V - eta).  Its fixed
 * point is the finite-rate steady state of socfv_solve_soc_steady (alpha = 1/2).
 * Needs FINITE_RATE, 0 < s_eq < 1, Da > 0, 0 < omega <= 1 (INVALID_ARG otherwise).  The
 * relaxation is stable for omega below about 2 / (1 + M), M = D_P sqrt(s (1 - s)) / (a k0
 * cosh(eta / 2)) with D_P the transport diagonal (~6 + advection): small omega for slow
 * kinetics; DIVERGED reports an unstable omega.  Uses p's s_in, s_eq, Da, cfl (on the
 * transport-only diagonal), tol (on tau rms((s' - s) / dt)), max_iter, check_every.
 * Outputs: s_out, eta_out (device, FP64 (nz, ny, nx), nullable), st (iterations, residual,
 * U and the balance).  The state becomes the context's forward state (as after a solve with
 * p).
 */
int socfv_solve_nernst(socfv_ctx *c, const socfv_params *p, double omega, double *s_out,
                       double *eta_out, socfv_stats *st, void *hip_stream);

/*
 * Iterative upsampling: converge on the unrefined grid, then start the refined problem from
 * the interpolated steady state (the paper's technique for the flow, Sec. "Incompressible
 * Fluid Flow"), here for this solve with the grid coarsened by two in every direction.
 *
 * socfv_coarsen writes the coarse problem of the context's current geometry and velocity
 * (q included); nx, ny, nz must be even (INVALID_ARG otherwise; velocity must be set).
 *   solid_c: device, uint8 (nz/2, ny/2, nx/2): 1 where all eight children are fibre.
 *   ux_c, uy_c, uz_c: device, FP64, the staggered layout above for the coarse grid: each
 *   coarse face velocity in coarse grid units (h doubled, same physical flux) is
 *   ((v00 + v01) + (v10 + v11)) / 2 over its four fine faces, v_ab with a the offset along
 *   the slower transverse axis (z for x and y faces, y for z faces) and b along the faster.
 * Buffers are the caller's; the call returns when they are written.
 *
 * socfv_solve_soc_upsampled solves the coarse problem (reaction 2 Da per coarse fibre face,
 * uniform activity, the other parameters of p) to steady state, prolongates it (each fine
 * pore cell takes its parent's value) and solves the fine problem from that state, which
 * has the plain solve's fixed point.  st: the fine solve's statistics with seconds covering
 * the whole call; coarse_st (nullable): the coarse solve's.  s_out as in
 * socfv_solve_soc_steady.  Temporary device memory is allocated and freed inside the call.
 * Returns the fine solve's status (or the first error).
 */
int socfv_coarsen(socfv_ctx *c, uint8_t *solid_c, double *ux_c, double *uy_c, double *uz_c,
                  void *hip_stream);
int socfv_solve_soc_upsampled(socfv_ctx *c, const socfv_params *p, double *s_out,
                              socfv_stats *st, socfv_stats *coarse_st, void *hip_stream);

/*
 * Upstream flow step: the steady velocity field this solve takes as input, from the
 * incompressible flow equations (Eqs. (navier-stokes), (incompressibility)) in the Stokes
 * regime of Eq. (stokes-flow), by the projection method of Eqs. (cp1)-(cp4) (Algorithm "Flow
 * Simulation", explicit momentum diffusion; momentum advection omitted), to the stop rule of
 * Eq. (flow-cnvg).  Nondimensional: h = rho = mu = 1; the field is linear in p_in, so one
 * solve serves every applied pressure (scale it with q in socfv_set_velocity).
 *
 * Discretisation: normal velocity on open faces (both cells pore, or the inlet / outlet face
 * of a pore cell); pressure in pore cells; pressure p_in at the inlet face x = 0 and 0 at the
 * outlet face x = nx; no-slip on fibre voxel faces and on the y / z walls (zero normal
 * velocity; tangential wall on the voxel face); zero normal gradient of the velocity across
 * the inlet and outlet planes.  Each step: u* = u + dt L u; (-D G) p = D gbc - D u* / dt by
 * Jacobi-preconditioned CG from the previous pressure, stopped when dt ||r|| < cg_theta x the
 * previous step's ||u' - u|| or after cg_max iterations; u' = u* - dt (G p + gbc).  The fixed
 * point is the discrete Stokes solution (L u = G p on open faces, D u = 0 on pore cells)
 * whatever cg_theta.  dt = cfl / 24 (Eq. (time-step-flow) with C_V = 6, C_A = C_F = 0).
 *
 *   p_in        applied inlet pressure (outlet at 0)
 *   cfl         C_CFL, in (0, 4) (explicit diffusion is stable below 4); paper value 0.5
 *   tol         eps_flow of Eq. (flow-cnvg): stop when ||u' - u||_2 < tol ||u'||_2 (1e-9)
 *   cg_theta    pressure CG stop factor (0.1)
 *   max_steps, check_every   step cap; steps between host checks of the stop rule
 *   cg_max      cap on CG iterations per step
 *   resume      0: start from rest (u = 0, p = 0); 1: start from the velocity in ux, uy, uz
 *               and, if p_out is given, the pressure in p_out (continuing an earlier call)
 *
 * ux, uy, uz: device, FP64, the staggered layout of socfv_set_velocity, written with the
 * flow (closed faces 0); they also serve as the iteration's velocity, so they hold the last
 * iterate on NOT_CONVERGED or DIVERGED (and the start with resume).  p_out (nullable): device,
 * FP64 (nz, ny, nx), the pressure (0 in fibre cells; the start pressure with resume).  Needs a context from socfv_setup_geometry (velocity not
 * needed).  Temporary device memory (~72 B per cell) is allocated and freed inside the call.
 * Returns OK, NOT_CONVERGED (outputs written), DIVERGED, INVALID_ARG, HIP_ERROR or OOM.
 */
typedef struct {
  double p_in, cfl, tol, cg_theta;
  long max_steps;
  int check_every, cg_max;
  int resume;
} socfv_flow_params;
typedef struct {
  long steps, cg_iterations;
  double change;       /* final ||u' - u|| / ||u'|| */
  double divergence;   /* max over pore cells of |D u| */
  double Q, Q_out;     /* flow rate through the inlet / outlet plane */
  double u_max, dt, seconds;
  int status;
} socfv_flow_stats;
void socfv_default_flow_params(socfv_flow_params *p);
int socfv_solve_stokes(socfv_ctx *c, const socfv_flow_params *p, double *ux, double *uy,
                       double *uz, double *p_out, socfv_flow_stats *st, void *hip_stream);

/*
 * Launch shapes.  Single sweeps work on (64 x tile_y) lanes marching z_chunk cells along z;
 * with two_sweeps set (the default), FP32 sweeps run two sweeps per launch on blocks of 1024
 * lanes marching z_chunk2 cells: rows of 64 lanes (16 rows) or, where that wastes fewer lanes
 * on the box, rows of 32 lanes (32 rows), two cells per lane for even nx and one for odd.
 * socfv_set_tiles overrides them for a context (0 = keep; two_sweeps: -1 keep, 0 off, 1 on
 * with the row width chosen for the box, 2 on with 64-lane rows, 3 on with 32-lane rows; a
 * new row width re-picks z_chunk2 unless given); socfv_autotune times candidate shapes on
 * this context's problem (`sweeps` sweeps each) and keeps the fastest; best[3] (host,
 * nullable) receives tile_y, z_chunk, z_chunk2.
 */
int socfv_set_tiles(socfv_ctx *c, int tile_y, int z_chunk, int z_chunk2, int two_sweeps);
int socfv_autotune(socfv_ctx *c, int sweeps, int best[3], void *hip_stream);

/* Problem facts: dims[3] = nx, ny, nz; counts[3] = pore cells, reactive cells,
 * cells not connected (always 0 after a successful setup). */
int socfv_info(const socfv_ctx *c, int dims[3], long counts[3]);

void socfv_destroy(socfv_ctx *c);
const char *socfv_last_error(void);
int socfv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SOCFV_H */
