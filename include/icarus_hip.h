/*
 * icarus_hip.h -- C-ABI of the MI355X heliospheric ideal-MHD library.
 *
 * The library advances the solar wind in the frame co-rotating with the Sun
 * on a radially stretched spherical grid starting at the 0.1 AU inner
 * boundary (Icarus 3.0, arXiv 2501.15923):
 *   - ideal MHD, Sect. 2 Eqs. (1)-(6), mu0 = 1 in code units, gravity and the
 *     centrifugal + Coriolis force F with energy source v.F, rotation rate
 *     Omega taken from the parameters (Sect. 2);
 *   - inner boundary from primitive-variable boundary maps (Sect. 2.1), the
 *     same value in every ghost layer (Sect. 2.1), linear interpolation in
 *     time between successive maps (Sect. 3), cone CMEs written only into
 *     the boundary points inside the cone (Sect. 3.2, bc_icarus);
 *   - initial state by radial expansion of the first map (Sect. 2.1);
 *   - sampling along spacecraft trajectories interpolated from tables
 *     (Sect. 2, particle sampling on stretched grids).
 * The finite-volume scheme (not printed in the paper): primitive MUSCL
 * reconstruction with a minmod or MC limiter, TVD-Lax-Friedrichs or HLL face
 * fluxes, exact spherical finite-volume divergence with area-difference
 * pressure sources, SSP-RK2 in time, dt = CFL / max over cells of
 * sum_d (|v_d| + c_f,d) / dx_d.
 *
 * Conventions
 *   - Every call returns ICR_OK (0) or a negative ICR_ERR_* code; the message
 *     of the last failure on the calling thread is icr_last_error().
 *   - Arguments are validated on the host before any GPU work.
 *   - Host inputs are copied; the caller keeps ownership of every buffer it
 *     passes.  Device memory for the solver comes from the caller: query
 *     icr_workspace_bytes(), allocate that many bytes of device memory
 *     (256-byte aligned) and keep it alive until icr_destroy().  No call
 *     allocates device memory: host <-> device copies of states, tracers
 *     and divergences go through a staging region of that workspace in
 *     chunks of 65536 cells.
 *   - API quantities are SI: metres, seconds, kg/m^3, m/s, Pa, tesla,
 *     radians.  theta is colatitude, phi longitude in the co-rotating frame.
 *   - Primitive channel order (maps and states):
 *       rho, v_r, v_theta, v_phi (co-rotating frame), p, B_r, B_theta, B_phi.
 *   - Layouts: maps [n_maps][8][n_theta][n_phi]; states [8][n_phi][n_theta][n_r]
 *     (active cells only, r fastest); all row-major, float64 at the ABI.
 *   - Work is enqueued on the HIP stream given at creation; calls that return
 *     host data synchronise that stream.
 *   - A solver is not thread-safe: one host thread at a time per solver.
 */
#ifndef ICARUS_HIP_H
#define ICARUS_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ICR_OK = 0,
  ICR_ERR_ARG = -1,          /* invalid argument (size, range, ordering)   */
  ICR_ERR_STATE = -2,        /* call out of order (e.g. step before maps)  */
  ICR_ERR_NONPHYSICAL = -3,  /* rho <= 0, p <= 0 or non-finite value found */
  ICR_ERR_HIP = -4,          /* HIP runtime failure                         */
  ICR_ERR_UNSUPPORTED = -5   /* option not implemented                      */
};

/* Face fluxes: TVDLF (Rusanov), HLL, and HLLD (Miyoshi & Kusano 2005: the
 * fast, rotational and contact waves; both face states use the mean normal
 * field, whose own flux is the HLL value; single solvers only). */
enum { ICR_FLUX_TVDLF = 0, ICR_FLUX_HLL = 1, ICR_FLUX_HLLD = 2 };
/* Reconstruction on primitives: minmod or MC limited slopes (two ghost
 * layers), or WENO5 (Jiang & Shu 1996; three ghost layers, the
 * thread-per-cell stage kernel only, single solvers only; a face state with
 * rho or p <= 0 falls back to its cell value). */
enum { ICR_LIM_MINMOD = 0, ICR_LIM_MC = 1, ICR_LIM_WENO5 = 2 };
enum { ICR_PREC_F64 = 64, ICR_PREC_F32 = 32 };
/* Transverse quantities (v_theta, v_phi, B_theta, B_phi) at the inner
 * boundary (Sect. 2.1).  MAP: every ghost layer takes the map's values
 * (after time interpolation and the cone-CME overwrite), like rho, v_r, p
 * and B_r.  ASYMM: the paper's default for the quantities a coronal model
 * does not provide; ghost layer g takes minus the primitive of active cell
 * g-1 (the mirror image about r_in), so they vanish on the boundary
 * surface, while rho, v_r, p and B_r still come from the map.  ASYMM needs
 * n_r >= the ghost width (2; 3 for WENO5). */
enum { ICR_BCT_MAP = 0, ICR_BCT_ASYMM = 1 };

/* State kinds for icr_set_state / icr_get_state. */
enum {
  ICR_STATE_PRIM_SI = 0,   /* primitive, SI units, float64                */
  ICR_STATE_CONS_CODE = 1  /* conservative, code units, float64           */
};

/* Grid and capacities.  The radial edges are r_in * q^i, q = (r_out /
 * r_in)^(1/n_r) (radially stretched grid, Sect. 2); colatitude uniform on
 * [th_min, th_max] with reflecting edges (mirror rows, v_theta and B_theta
 * negated; the paper does not state this boundary); longitude uniform and
 * periodic on [0, 2 pi); zero-gradient outflow at r_out.  The
 * capacities size the workspace: boundary maps, cone CMEs, probes, points
 * per trajectory table and rows of the device probe log. */
typedef struct {
  int n_r, n_theta, n_phi;   /* >= 1 each, product < 2^29 (one variable's
                                array below 4 GiB)                      */
  double r_in, r_out;        /* m, 0 < r_in < r_out                     */
  double th_min, th_max;     /* rad, 0 < th_min < th_max < pi           */
  int max_maps;              /* >= 1                                     */
  int max_cmes;              /* >= 0                                     */
  int max_probes;            /* >= 0                                     */
  int max_traj_pts;          /* >= 2 when max_probes > 0                 */
  int probe_log_rows;        /* >= 0: rows of [max_probes][12] in the log */
} icr_grid;

/* Physics and numerics (Sect. 2: gamma = 1.5, co-rotating frame with the
 * equatorial rotation rate, gravity of the Sun). */
typedef struct {
  double gamma;              /* adiabatic index, > 1                     */
  double omega;              /* rotation rate, rad/s (0 = inertial)      */
  double cfl;                /* Courant number, (0, 1]                   */
  int flux;                  /* ICR_FLUX_*                               */
  int limiter;               /* ICR_LIM_*                                */
  int precision;             /* ICR_PREC_F64 or ICR_PREC_F32             */
  int gravity;               /* 1: include -GM/r^2 e_r                   */
  int corotation;            /* 1: centrifugal + Coriolis sources        */
  int tracer;                /* 1: carry the passive CME tracer          */
  int bc_transverse;         /* ICR_BCT_MAP or ICR_BCT_ASYMM             */
} icr_phys;

/* Clock: time [s] since the map time origin, completed RK2 steps, the dt of
 * the last step [s], the CFL dt the next step will use (before clipping)
 * [s], the last relaxation residual ||rho^{n+1}-rho^n||_2/||rho^n||_2, and
 * the time in code units for exact restarts (icr_set_clock_code). */
typedef struct {
  double t;
  long long step;
  double last_dt;
  double next_dt;
  double residual;
  double t_code;
} icr_clock;

/* Result of icr_step.  bad_cell = -1, or the linear index k*n_theta*n_r +
 * j*n_r + i of the first active cell found with rho <= 0, p <= 0 or a
 * non-finite value after the step that produced it. */
typedef struct {
  int steps_taken;
  int status;
  long long bad_cell;
  double t;
  double last_dt;
  double residual;
} icr_step_info;

typedef struct icr_solver icr_solver;

/* Message of the last failed call on this thread ("" if none). */
const char *icr_last_error(void);

/* Code units: time, length, density, pressure, field, velocity (SI per code
 * unit).  out: 6 doubles. */
int icr_units(double *out);

/* Device bytes the solver needs for this grid and physics. */
int icr_workspace_bytes(const icr_grid *grid, const icr_phys *phys,
                        size_t *bytes);

/* Create a solver on the current HIP device.  dev_workspace: caller-owned
 * device memory of at least icr_workspace_bytes(); hip_stream: a
 * hipStream_t (NULL = default stream).  Computes the grid metric on the
 * device.  The state is undefined until icr_init_radial or icr_set_state. */
int icr_create(const icr_grid *grid, const icr_phys *phys, void *dev_workspace,
               size_t workspace_bytes, void *hip_stream, icr_solver **out);

/* Release the solver (not the caller's workspace).  NULL is allowed. */
void icr_destroy(icr_solver *s);

/* Grid edges: r [n_r+1] m, theta [n_theta+1] rad, phi [n_phi+1] rad.  Any
 * pointer may be NULL. */
int icr_grid_edges(const icr_solver *s, double *r_edges, double *th_edges,
                   double *ph_edges);

/* Boundary maps at 0.1 AU (Sect. 2.1 lookup table, Sect. 3 time series):
 * n_maps <= max_maps primitive maps in SI, [n_maps][8][n_theta][n_phi],
 * at strictly ascending times t_s [n_maps] (s).  Between two map times the
 * boundary is the linear interpolation of the bracketing maps; before the
 * first / after the last map time it is that map.  Requires rho > 0 and
 * p > 0 everywhere (ICR_ERR_ARG otherwise).  maps_on_device: 1 if maps_si
 * is a device pointer (t_s is always host). */
int icr_set_boundary_maps(icr_solver *s, int n_maps, const double *t_s,
                          const double *maps_si, int maps_on_device);

/* Stream later maps into a run (long dynamic runs with more maps than fit,
 * e.g. an extended domain with an hourly map cadence; Sect. 3 and 4).
 * Appends n maps in the layout of icr_set_boundary_maps, with times strictly
 * after the last map held.  First the maps that can no longer bracket any
 * time from the clock on are dropped: those before the last map time <= t.
 * The boundary values at times >= t are unchanged by the drop.  If the maps
 * still needed plus the new ones exceed max_maps, nothing changes and
 * ICR_ERR_STATE asks to step further first.  *n_held (may be NULL) receives
 * the number of maps held afterwards.  Setting the clock back before the
 * first map held later clamps to that map, as for any time before the first
 * map. */
int icr_append_boundary_maps(icr_solver *s, int n_maps, const double *t_s,
                             const double *maps_si, int maps_on_device, int *n_held);

/* Cone CMEs (Sect. 3.2 bc_icarus; Table 2 parameters): n <= max_cmes rows
 * of 8 SI values: insertion start [s], duration [s], latitude [rad],
 * co-rotating longitude [rad], half-width [rad], speed [m/s], density
 * [kg/m^3], temperature [K].  While t_start <= t < t_start + duration the
 * boundary points whose great-circle distance to the cone axis is <= the
 * half-width get rho, v_r = speed, v_theta = 0, v_phi = -Omega r_in
 * sin(theta), p = 2 (rho/m_p) k_B T; B is unchanged (the cone CME is not
 * magnetised).  n = 0 removes all CMEs. */
int icr_set_cmes(icr_solver *s, int n, const double *rows);

/* Initial state by radial expansion of the first map (Sect. 2.1):
 * rho ~ r^-2, v_r constant, v_theta = 0, v_phi = -Omega r sin(theta),
 * p ~ r^(-2 gamma), B_r ~ r^-2, B_theta = 0, B_phi ~ r^-1, from r_in.
 * Sets the clock to t = 0, step 0 and computes the first dt. */
int icr_init_radial(icr_solver *s);

/* Replace the state.  kind: ICR_STATE_*; data: [8][n_phi][n_theta][n_r]
 * float64, host (on_device = 0) or device (on_device = 1) pointer.
 * Recomputes the CFL dt; the clock time is kept. */
int icr_set_state(icr_solver *s, const double *data, int kind, int on_device);

/* Copy the state out (same layout and kinds as icr_set_state). */
int icr_get_state(icr_solver *s, double *out, int kind, int on_device);

int icr_get_clock(icr_solver *s, icr_clock *out);
/* Set time [s] and step count; recomputes the CFL dt. */
int icr_set_clock(icr_solver *s, double t, long long step);
/* Set the time in code units (bit-exact restart from icr_clock.t_code). */
int icr_set_clock_code(icr_solver *s, double t_code, long long step);

/* Advance up to n_steps SSP-RK2 steps (n_steps >= 0).  If t_end_s > 0 the
 * last step is shortened to land on t_end_s and no step starts at or after
 * it.  The clock, dt and map bracket stay on the device; steps are replayed
 * from captured HIP graphs; one host synchronisation per call.  Returns
 * ICR_ERR_NONPHYSICAL (and stops advancing) when a step produced an
 * invalid cell; info may be NULL. */
int icr_step(icr_solver *s, int n_steps, double t_end_s, icr_step_info *info);

/* For callers that cannot allocate device memory or instantiate graphs
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): icr_step with direct kernel launches instead of graph
 * replays, and the stage-2 kernel's per-block CFL / residual / validity
 * partials in a fixed device array of the library instead of the
 * workspace.  Same arguments, results and errors as icr_step (bit-identical
 * states).  The array holds 32768 blocks (1 MiB, one copy per device, kept
 * until the process ends): a solver whose stage launch has more blocks
 * gets ICR_ERR_ARG (choose more phi planes per block with icr_set_launch).
 * Call it with the solver's device current (ICR_ERR_ARG otherwise).  Every
 * call on one device shares that device's array: calls for different
 * solvers that overlap in time on one device (other host threads, other
 * streams) race and must be serialised by the caller.  Nothing in the
 * array needs to start at zero: each step writes every slot it reads. */
int icr_step_noalloc(icr_solver *s, int n_steps, double t_end_s, icr_step_info *info);

/* Probes (Sect. 2 particle sampling): n <= max_probes trajectory tables
 * traj [n][n_pts][4] of rows (t [s], r [m], theta, phi_inertial [rad]),
 * ascending t, unwrapped phi, 2 <= n_pts <= max_traj_pts.  Positions are
 * linear in t between rows (clamped outside), phi' = phi - Omega t.
 * cadence_s: > 0 logs a record each time t crosses a multiple of cadence_s,
 * = 0 logs after every step, < 0 disables the device log.  Clears the log. */
int icr_set_probes(icr_solver *s, int n, int n_pts, const double *traj,
                   double cadence_s);

/* Sample every probe at the current time: out [n][12] host doubles: t, r,
 * theta, phi', rho, v_r, v_theta, v_phi (inertial frame), p, B_r, B_theta,
 * B_phi (SI), trilinear in (r, theta, phi) between the 8 surrounding cell
 * centres.  Outside the range of cell centres the 8 plasma values are NaN. */
int icr_sample_probes(icr_solver *s, double *out);

/* Copy the device probe log to host: up to cap records, each [n][12] as in
 * icr_sample_probes; *n_rec receives the number of records logged (may
 * exceed cap; the log keeps the first probe_log_rows records). */
int icr_read_probe_log(icr_solver *s, double *out, int cap, int *n_rec);

/* Relaxation diagnostic: rho [kg/m^3] and v_r [m/s] on the sphere r_m for
 * every (theta, phi) column, linear in r between the bracketing cell centres
 * (clamped to the first / last centre): out [2][n_theta][n_phi] host. */
int icr_sample_shell(icr_solver *s, double r_m, double *out);

/* Passive CME tracer (the CME density tracer the paper plots and refines on,
 * Fig. 7 and Sect. 4; solvers created with icr_phys.tracer = 1).  tau is the
 * mass fraction of CME material, [n_phi][n_theta][n_r] like the state.  The
 * solver carries rho tau and advects it with each RK stage's own mass
 * fluxes and the upwind tau.  Material enters through the inner boundary:
 * tau = 1 where a cone CME is being inserted, 0 elsewhere.  Beyond r_out
 * and the colatitude edges the edge cell's own tau is used.
 * icr_init_radial and icr_set_state reset tau to 0.
 * icr_set_tracer converts tau to rho tau with the current density.
 * on_device selects device or host memory, as for the state.
 * ICR_ERR_STATE without the tracer or before a state exists. */
int icr_set_tracer(icr_solver *s, const double *tau, int on_device);
int icr_get_tracer(icr_solver *s, double *tau, int on_device);

/* Velocity divergence of the current state [1/s] (the div V diagnostic of the
 * paper's shock refinement criterion, Fig. 7), [n_phi][n_theta][n_r].
 * Finite-volume divergence in the co-rotating frame.  The face velocity is
 * the mean of the two neighbouring cell centres.  The inner ghost is the
 * boundary primitive at the current time; beyond r_out zero-gradient;
 * mirror rows (v_theta negated) beyond the colatitude edges; phi periodic. */
int icr_divv(icr_solver *s, double *out, int on_device);

/* Inner-boundary primitive (SI) the solver would impose at time t_s, after
 * time interpolation and the CME overwrite: out [8][n_theta][n_phi] host. */
int icr_boundary_at(icr_solver *s, double t_s, double *out);

/* Launch configuration of the fused stage kernels.  variant: 0 = default
 * (2), 1 = one thread per cell with on-the-fly neighbour primitives, 2 =
 * face-once kernel (LDS tile with halo in r/theta, registers along phi).
 * tile_r: lanes along r per block (variant 1: 64, 128, 256; variant 2: 32,
 * 64, of which the first two and the last two hold the r halo, so a block
 * updates tile_r - 4 cells along r; 0 = 64; a solver with the passive
 * tracer keeps 64 for variant 2; a WENO5 solver's variant 2 is its own
 * 64-lane tile of 58 cells along r, and with the tracer it runs variant 1);
 * 256 threads per block.  planes: phi planes per block of
 * variant 2 (1..n_phi, 0 = 8).  use_graphs: 1 replays steps from captured
 * HIP graphs.  All tiles and plane counts of one variant give bit-identical
 * results; the two variants agree to rounding. */
int icr_set_launch(icr_solver *s, int variant, int tile_r, int planes,
                   int use_graphs);

/* Advance n_steps (> 0) steps with direct launches, timing each kernel with
 * HIP events on the solver's stream.  avg_ms[4] receives the mean duration
 * of the boundary driver, stage 1, stage 2 and the finalize kernel (clock,
 * dt and probe record).  Same results as icr_step. */
int icr_profile_steps(icr_solver *s, int n_steps, double *avg_ms);

/* Accuracy diagnostic of the FP64 reciprocal and square root the face-once
 * stage kernels use instead of division and sqrt (hardware estimate refined
 * by two Newton-Raphson steps, and by two Goldschmidt iterations plus a
 * residual correction): rcp[q] = 1/x[q], sq[q] = sqrt(x[q]) for n device
 * doubles (positive normal x).  All pointers device memory; synchronises
 * the stream. */
int icr_fast_math(const double *x, long long n, double *rcp, double *sq, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched ensemble (not in the paper; many independent runs on one GPU).
 * n_runs solvers with their own grids, boundary maps, cone CMEs, clocks and
 * CFL dt, stepped together: each ensemble step walks all runs' boundary
 * columns, stage-1 tiles, stage-2 tiles and per-run finalize (with the
 * passive tracer, a tracer list of all runs' cells follows each stage).  In the
 * persistent mode one kernel launch performs the steps with a device-wide
 * barrier between those phases (its grid never exceeds the resident block
 * capacity; a barrier that cannot complete turns into ICR_ERR_HIP instead of
 * a hang); in the batched mode each phase is one launch.  Steps are replayed
 * from captured HIP graphs.  Every run's state is bit-identical to stepping
 * that run alone with icr_step.
 * ------------------------------------------------------------------------ */
typedef struct icr_ensemble icr_ensemble;

/* Device bytes for n_runs grids (grids[n_runs]) sharing one icr_phys.
 * Every flux, limiter and the tracer are supported, except WENO5 together
 * with the tracer (ICR_ERR_UNSUPPORTED): the WENO5 tile keeps no face mass
 * fluxes. */
int icr_ens_workspace_bytes(int n_runs, const icr_grid *grids,
                            const icr_phys *phys, size_t *bytes);

/* Create the ensemble in caller-owned device memory (256-byte aligned). */
int icr_ens_create(int n_runs, const icr_grid *grids, const icr_phys *phys,
                   void *dev_workspace, size_t workspace_bytes,
                   void *hip_stream, icr_ensemble **out);

/* Release the ensemble and its run solvers (not the workspace). */
void icr_ens_destroy(icr_ensemble *e);

/* The solver of run r (owned by the ensemble): use it with
 * icr_set_boundary_maps, icr_set_cmes, icr_init_radial, icr_set_state,
 * icr_get_state and icr_get_clock.  Do not destroy it. */
int icr_ens_run(icr_ensemble *e, int r, icr_solver **out);

/* Phi planes per tile for run r (1..n_phi); the autotuner's knob.  The
 * result does not depend on it. */
int icr_ens_set_planes(icr_ensemble *e, int r, int planes);

/* persistent: 1 (default) one launch for many steps, 0 one launch per phase;
 * grid_blocks: 0 = all resident blocks, else a multiple of 8 not above that;
 * use_graphs: 1 replays chunks of 8 steps from a captured HIP graph. */
int icr_ens_set_mode(icr_ensemble *e, int persistent, int grid_blocks,
                     int use_graphs);

/* Advance every run up to n_steps RK2 steps (each with its own dt); if
 * t_end_s > 0 each run's last step lands on t_end_s and runs at t_end_s stay
 * put.  info: NULL or an array of n_runs results.  ICR_ERR_NONPHYSICAL if
 * any run produced an invalid cell (that run stops advancing, the others
 * continue). */
int icr_ens_step(icr_ensemble *e, int n_steps, double t_end_s, icr_step_info *info);

/* ------------------------------------------------------------------------
 * Block-structured adaptive mesh refinement (Sect. 3.2 and Sect. 4: the
 * 2015 runs refine the radially stretched grid up to five levels where the
 * CME tracer ('tracing'), a compression or shock ('shock') or either
 * ('combined') is present in a block).
 *
 * The grid of icr_grid is level 1, cut into blocks of block_r x block_theta
 * x block_phi cells; a level-(l+1) block is one octant of a level-l block
 * at twice the resolution in r (edges split at the geometric mean), theta
 * and phi.  One dt for all levels (CFL over every leaf cell), SSP-RK2 on the
 * leaves, two ghost layers per block: copies, volume-weighted restriction
 * of finer leaves, conservative minmod-limited prolongation of the coarser
 * leaf; the physical edges of the uniform solver (inner boundary: the map
 * value of the base column containing a cell, the cone CME tested at the
 * cell's own centre).  A coarse cell next to finer leaves takes their
 * area-weighted face fluxes (mass and B_r conserved to round-off).  The
 * passive CME tracer is always carried.  Every regrid_every steps a leaf
 * below max_level is split when its criterion holds (max tau >=
 * tau_threshold; max over its cells of -div(V) r / (2 |v_r|) >=
 * shock_threshold), and 8 leaf children none of which holds it are merged;
 * face neighbours stay within one level.  FP64; minmod or MC with TVDLF,
 * HLL or HLLD; the map transverse rule.
 * ------------------------------------------------------------------------ */
enum { ICR_AMR_TRACING = 0, ICR_AMR_SHOCK = 1, ICR_AMR_COMBINED = 2 };

typedef struct {
  int block_r, block_theta, block_phi;  /* >= 4 each, dividing the grid   */
  int max_level;                        /* 1 (no refinement) .. 6          */
  int criterion;                        /* ICR_AMR_*                       */
  double tau_threshold;                 /* tracing: CME mass fraction      */
  double shock_threshold;               /* shock: dimensionless compression */
  int regrid_every;                     /* steps between regrids, >= 1     */
  int max_blocks;                       /* block pool over all levels      */
} icr_amr_params;

typedef struct icr_amr icr_amr;

/* Device bytes of a refined run (caller-owned, as for icr_create). */
int icr_amr_workspace_bytes(const icr_grid *grid, const icr_phys *phys,
                            const icr_amr_params *params, size_t *bytes);
int icr_amr_create(const icr_grid *grid, const icr_phys *phys,
                   const icr_amr_params *params, void *dev_workspace,
                   size_t workspace_bytes, void *hip_stream, icr_amr **out);
void icr_amr_destroy(icr_amr *a);
/* Boundary maps and cone CMEs: as icr_set_boundary_maps (host maps) and
 * icr_set_cmes. */
int icr_amr_set_boundary_maps(icr_amr *a, int n_maps, const double *t_s,
                              const double *maps_si);
int icr_amr_set_cmes(icr_amr *a, int n, const double *rows);
/* Level-1 leaves from the radial expansion of the first map (Sect. 2.1),
 * tracer 0, clock at 0, first dt. */
int icr_amr_init_radial(icr_amr *a);
/* n_steps RK2 steps with a regrid after every regrid_every-th step of the
 * run; t_end_s as in icr_step.  ICR_ERR_STATE when the block pool is full,
 * ICR_ERR_NONPHYSICAL on an invalid cell (bad_cell = slot * cells per block
 * + cell). */
int icr_amr_step(icr_amr *a, int n_steps, double t_end_s, icr_step_info *info);
/* Split the given leaves (keys [n][4]: level, block index along r, theta,
 * phi at that level) and the coarser leaves the one-level rule needs. */
int icr_amr_force_refine(icr_amr *a, int n, const int *keys);
/* Leaves in (level, i, j, k) order: *n receives the count, keys [cap][4]
 * receives the first cap of them (cap = 0: the count only, keys may be NULL). */
int icr_amr_leaves(icr_amr *a, int cap, int *keys, int *n);
/* One leaf's cells, conservative in code units (the 8 variables of
 * ICR_STATE_CONS_CODE, then rho tau): [9][block_phi][block_theta][block_r]
 * host doubles. */
int icr_amr_get_block(icr_amr *a, const int *key, double *out);
int icr_amr_get_clock(icr_amr *a, icr_clock *out);

#ifdef __cplusplus
}
#endif
#endif /* ICARUS_HIP_H */
