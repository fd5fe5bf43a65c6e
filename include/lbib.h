/*
 * lbib.h - C ABI of the MI355X (gfx950) lattice-Boltzmann / immersed-boundary
 * capillary solver.
 *
 * The library advances the 2D hybrid kinematic/dynamic immersed-boundary
 * lattice-Boltzmann method of Coclite, "Vascular journey and adhesion
 * mechanics of micro-sized carriers in narrow capillaries" (arXiv 1907.00080):
 *   - D2Q9 BGK collide-and-stream with Guo body forcing (Sec. 2.1, Eqs. BGK,
 *     feq, GaussHermite; Sec. 2.2, Eqs. forcedBGK, ForcingTerm), x periodic,
 *     no-slip walls at y = -1/2 and y = ny - 1/2 (halfway bounce-back);
 *   - mass-spring membranes with strain, bending and enclosed-area forces
 *     (Sec. 2.2, Eqs. strainFor, bendFor, areaFor);
 *   - ligand-receptor bonds: stochastic formation/rupture and linear springs
 *     (Sec. 2.2, Eq. adhFor; Sec. 3 parameters);
 *   - red cells moved by the kinematic IB (Sec. 2.3, Eq. kinematicPos);
 *     rigid and soft particles by the dynamic IB with probe-based pressure
 *     and viscous loads (Sec. 2.2, Eqs. hydroForP, hydroForNu; Sec. 2.3,
 *     Eqs. newtonSoft, verletPos, verletVel, linearVelRig, angularVelRig).
 *
 * Units: lattice units throughout (dx = dt = 1, rho0 = 1, cs^2 = 1/3).
 *
 * Conventions shared by every entry point
 *   - Every call returns an lbib_status; LBIB_OK == 0.  On any other value
 *     the call had no effect on the context's state, and lbib_last_error()
 *     describes the cause.  No C++ exception crosses this boundary.
 *   - Host arrays passed in are owned by the caller and copied during the
 *     call.  Readback calls write into caller-owned host buffers of the
 *     stated sizes.  NULL where an array is required -> LBIB_EINVAL.
 *   - Device memory: the library allocates none of its state.  The caller
 *     queries the workspace size, allocates that many bytes of device
 *     memory (any allocator; 256-byte alignment required) and binds it
 *     together with a HIP stream.  The workspace must outlive the context.
 *     All kernels are enqueued on the bound stream; lbib_step returns once
 *     the work is enqueued.  Readback calls synchronise that stream.
 *   - Lifecycle: create -> add_body / set_receptors / set_adhesion /
 *     init_fields (setup) -> workspace_query -> bind -> finalize_setup
 *     (running) -> step / readback ... -> destroy.  A call made in the wrong
 *     phase returns LBIB_ESTATE.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Lagrangian data crosses the boundary in float64; marker x coordinates
 *     are unwrapped (the lattice is periodic in x, bodies are not cut).
 */
#ifndef LBIB_H
#define LBIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBIB_ABI_VERSION 6u

typedef struct lbib_ctx lbib_ctx;

typedef enum {
  LBIB_OK = 0,
  LBIB_EINVAL = 1,     /* bad argument: NULL, size or value out of range      */
  LBIB_ESTATE = 2,     /* call not allowed in the context's current phase      */
  LBIB_EHIP = 3,       /* a HIP runtime call failed (message has the HIP error) */
  LBIB_ENOSPACE = 4,   /* workspace smaller than lbib_workspace_query's value  */
  LBIB_EUNSTABLE = 5   /* watchdog: non-finite or non-positive density found   */
} lbib_status;

typedef enum { LBIB_F32 = 0, LBIB_F64 = 1 } lbib_dtype;

typedef enum {
  LBIB_RBC_KINEMATIC = 0,   /* red cell: kinematic IB, forces spread to the fluid */
  LBIB_PARTICLE_SOFT = 1,   /* deformable particle: dynamic IB, Verlet + BDF2     */
  LBIB_PARTICLE_RIGID = 2   /* rigid particle: dynamic IB, BDF2 on U and Omega    */
} lbib_body_kind;

/* Lattice of nx * ny nodes at x = 0..nx-1, y = 0..ny-1 (Sec. 3: periodic in x,
 * walls in y).  tau: BGK relaxation time (> 1/2), nu = (tau - 1/2)/3.
 * (gx, gy): uniform body force driving the flow (the pressure drop of the
 * Poiseuille set-up).  periodic_y = 1 replaces the walls by periodicity
 * (used by conservation tests).  dtype: precision of the populations and of
 * the collision arithmetic; populations are stored shifted by their rest
 * weights (f_i - w_i).  seed and instance key the Philox4x32-10 stream of
 * the bond kinetics.  tile_x, tile_y: lattice tile of the fused kernel and
 * of the marker bins, one of (64,4), (128,2), (32,8), (256,1); 0,0 = default. */
typedef struct {
  int32_t nx, ny;
  int32_t periodic_y;
  int32_t dtype;
  double tau;
  double gx, gy;
  uint64_t seed;
  int32_t instance;
  int32_t tile_x, tile_y;
} lbib_lattice_desc;

/* One closed membrane (Sec. 2.2): nv vertices, counter-clockwise, given in
 * their stress-free configuration (rest lengths, rest angles and rest area
 * are taken from them).  ks, kb, ka: strain, bending and area constants;
 * p_ref: reference pressure of the area penalty.  density_ratio: rho_P/rho
 * (particle mass = ratio * rest area, Sec. 3).  sigma: bond spring constant.
 * ligand_stride: 0 = no ligands; s > 0: a ligand on every element l with
 * l % s == 0 (s = 2 is the density rho_L = 0.5 of Sec. 3).  Ligands sit on
 * particles only: a kinematic red cell with ligand_stride > 0 is refused
 * (LBIB_EINVAL). */
typedef struct {
  int32_t kind;
  int32_t nv;
  double ks, kb, ka, p_ref;
  double density_ratio;
  double sigma;
  int32_t ligand_stride;
} lbib_body_desc;

/* Bond kinetics (Sec. 2.2 Wall-Particle Interaction, Sec. 3): bonds form only
 * when an element centroid is closer than y_cr to a wall; y_eq is the
 * force-free bond length.  Formation/rupture probabilities per step:
 * P = 1 - exp(-k dt) with k_f = kf0_dt exp(-s_ts (y - y_eq)^2 / (2 kbt)) and
 * k_r = kr0_dt exp((sigma - s_ts)(y - y_eq)^2 / (2 kbt)), s_ts =
 * sigma_ts_frac * sigma.  freeze_topology = 1 keeps the bond table fixed. */
typedef struct {
  double y_cr, y_eq;
  double kf0_dt, kr0_dt;
  double sigma_ts_frac;
  double kbt;
  int32_t freeze_topology;
} lbib_adhesion_desc;

/* Whole-lattice diagnostics of the last completed step. */
typedef struct {
  int64_t step;          /* number of completed time steps                     */
  double mass;           /* sum of rho                                         */
  double mom_x, mom_y;   /* sum of rho u (physical, half-force velocity)      */
  double rho_min;
  double u_max;          /* max |u|                                            */
  int64_t nonfinite;     /* nodes with a non-finite population                 */
  int32_t nbonds;
  int32_t bin_overflow;  /* marker-bin registrations dropped since set-up (a
                            full bin also poisons its tile's force, so the
                            watchdog reports it), plus bodies whose
                            repulsion candidate list was truncated; 0 in
                            any valid run                                  */
  int32_t sync_timeouts; /* in-kernel waits for the bond update that gave up
                            (0 in any valid run)                           */
} lbib_diag;

uint32_t lbib_abi_version(void);

/* Status name for an lbib_status value (static string). */
const char* lbib_status_string(int32_t status);

/* Message of the last failed call on ctx (owned by ctx, valid until the next
 * call on it).  ctx may be NULL: then the last lbib_create failure. */
const char* lbib_last_error(const lbib_ctx* ctx);

/* Create a context in the setup phase.  nx, ny >= 1, tau > 1/2. */
lbib_status lbib_create(const lbib_lattice_desc* desc, lbib_ctx** out);

/* Add a body (setup phase).  xy: nv*2 doubles (x0, y0, x1, y1, ...).
 * nv >= 3.  *id receives the body index (bodies are numbered in call order). */
lbib_status lbib_add_body(lbib_ctx* ctx, const lbib_body_desc* desc, const double* xy,
                          int32_t* id);

/* Receptor positions on one wall (setup phase), the binding sites of the
 * ligand-receptor bonds of Sec. 2.2 "Wall-Particle Interaction" (receptors
 * uniformly distributed over the walls): wall 0 is y = -1/2, wall 1 is
 * y = ny - 1/2 (the node rows 0 and ny - 1 with velocity walls).  x: n
 * strictly increasing values in [0, nx).  Replaces any earlier set.  n = 0
 * clears the wall.  Errors: LBIB_EINVAL for a wall other than 0/1, n < 0,
 * x NULL with n > 0, or values outside [0, nx) or not increasing;
 * LBIB_ESTATE outside set-up. */
lbib_status lbib_set_receptors(lbib_ctx* ctx, int32_t wall, const double* x, int32_t n);

/* Bond kinetics parameters (setup phase; defaults: no bonds form). */
lbib_status lbib_set_adhesion(lbib_ctx* ctx, const lbib_adhesion_desc* desc);

/* Wall condition (setup phase; default mode 0).  Mode 0: halfway bounce-back,
 * walls at rest at y = -1/2 and ny - 1/2.  Mode 1: the paper's wall
 * condition (Sec. 2.1), Zou-He velocity walls on the node rows y = 0 and
 * ny - 1 (channel height ny - 1) moving along x with u_lo (bottom) and u_hi
 * (top), e.g. a Couette box; the populations from beyond a wall are set so
 * that the node's half-force velocity (Sec. 2.2) is the wall velocity, with
 * the node's total force, and with the drive alone in the state the particle
 * probes read.  Bond lengths, wall distances and flow regions use the wall
 * positions of the mode.  Errors: LBIB_EINVAL for a mode other than 0 or 1,
 * a non-finite or |u| > 0.3 velocity, moving walls in mode 0, or mode 1 on a
 * periodic-y lattice or one with ny < 2; LBIB_ESTATE outside set-up or on a
 * batch (a batch takes each instance's setting).  The adjoint calls return
 * LBIB_EINVAL for mode 1. */
lbib_status lbib_set_walls(lbib_ctx* ctx, int32_t mode, double u_lo, double u_hi);

/* Lattice <-> marker transfer (Sec. 2.2 "Immersed Boundary Treatment": the
 * paper exchanges all data between lattice and chain by a moving-least-
 * squares reconstruction; Sec. 2.3: nine nodes in a square of side 2.6 dx).
 * Every transfer (velocity at red-cell vertices, probe values and velocity
 * gradients of particles, their vertex velocities, and the spreading of
 * marker forces, which uses the same weights) works on the 3x3 nodes nearest
 * the point.  LBIB_TRANSFER_ROMA (default): the 3-point kernel of Roma,
 * Peskin and Berger along each axis; rows beyond a wall are dropped.
 * LBIB_TRANSFER_MLS: linear basis (1, x, y) fitted by weighted least squares
 * to those nodes, weight w(x_j - X) w(y_j - Y) chosen by `weight`:
 *   LBIB_MLS_WEIGHT_ROMA  the Roma kernel (support 3/2; `half_width` ignored;
 *                         in the interior this equals the default transfer),
 *   LBIB_MLS_WEIGHT_CUBIC cubic spline of support half-width `half_width`,
 *   LBIB_MLS_WEIGHT_GAUSS Gaussian exp(-(|r| / (0.4 h))^2), shifted to vanish
 *                         at |r| = h = `half_width`;
 * the paper's square is half_width = 1.3.  Rows beyond a wall carry no
 * weight, so the fit next to a wall is one-sided (constants and linear
 * fields are still reproduced exactly); a point with fewer than two rows
 * inside the support fits a constant along y.  Velocity gradients are the
 * derivatives of the fitted shape functions.  Errors: LBIB_EINVAL for an
 * unknown mode or weight, or half_width outside (1, 3/2] (non-finite
 * included) for the cubic and Gaussian weights; LBIB_ESTATE outside set-up or
 * on a batch (a batch takes each instance's setting).  The adjoint calls
 * return LBIB_EINVAL for the MLS transfer. */
enum { LBIB_TRANSFER_ROMA = 0, LBIB_TRANSFER_MLS = 1 };
enum { LBIB_MLS_WEIGHT_ROMA = 0, LBIB_MLS_WEIGHT_CUBIC = 1, LBIB_MLS_WEIGHT_GAUSS = 2 };
lbib_status lbib_set_transfer(lbib_ctx* ctx, int32_t mode, int32_t weight, double half_width);

/* Repulsion between vertices of different bodies (setup phase; default off),
 * Sec. 2.2 "Particle-Particle Interaction", Eq. (repFor): every vertex closer
 * than `cutoff` (lattice units) to a vertex of another body of the same
 * lattice adds coeff * sqrt(1 / d^5) along its own inward vertex normal (the
 * normalised sum of its two element normals, negated); d uses the minimum
 * image along periodic axes.  The paper's coefficient is 1e-4 / (8 sqrt 2);
 * cutoff 2 is this library's reading (the expression has none).  Evaluated
 * at X^n with the membrane forces: red cells spread it, soft particles add
 * it to their vertex forces, rigid particles to their force and torque.
 * coeff = 0 switches it off.  With it on, the merged step form is not used
 * (the repulsion needs every body's X^n first) and the adjoint calls return
 * LBIB_EINVAL.  Errors: LBIB_EINVAL for coeff < 0, a non-finite value or a
 * cutoff outside (0, 16]; LBIB_ESTATE outside set-up or on a batch (a batch
 * takes each instance's setting). */
lbib_status lbib_set_repulsion(lbib_ctx* ctx, double coeff, double cutoff);

/* Initial fluid state (setup phase): populations at the equilibrium of
 * Eq. (feq) (Sec. 2.1) with density rho and velocity (ux, uy), host arrays
 * of ny*nx doubles, row-major [y][x], copied during the call.  rho may be
 * NULL (1 everywhere); ux/uy NULL = 0.  Default: rest.  Errors: LBIB_EINVAL
 * for a non-finite value or rho <= 0; LBIB_ESTATE outside set-up. */
lbib_status lbib_init_fields(lbib_ctx* ctx, const double* rho, const double* ux,
                             const double* uy);

/* Bytes of device workspace the context needs (setup phase, after all
 * add_body / set_receptors calls). */
lbib_status lbib_workspace_query(const lbib_ctx* ctx, size_t* bytes);

/* Attach caller-owned device memory (>= the queried size, 256-byte aligned)
 * and the HIP stream (hipStream_t, NULL = default stream) all work goes to. */
lbib_status lbib_bind(lbib_ctx* ctx, void* dev_workspace, size_t bytes, void* hip_stream);

/* Upload the set-up, compute the stress-free state, enter the running phase. */
lbib_status lbib_finalize_setup(lbib_ctx* ctx);

/* Advance nsteps >= 0 time steps (running phase).  One step n -> n+1 runs,
 * in this order (the paper gives the pieces, not their order): bond rupture
 * and formation at X^n (Sec. 2.2 "Wall-Particle Interaction"); membrane,
 * bending, area and spring forces (Eqs. strainFor, bendFor, areaFor, adhFor)
 * and the optional repulsion (Eq. repFor); particle probe loads and motion
 * (Eqs. hydroForP, hydroForNu; Sec. 2.3, Eqs. newtonSoft, verletPos,
 * linearVelRig, angularVelRig) with the weak no-slip coupling; spreading of
 * the marker forces (Sec. 2.2 "Immersed Boundary Treatment"); the forced
 * collide-and-stream (Sec. 2.1, Eqs. BGK, feq; Sec. 2.2, Eqs. forcedBGK,
 * ForcingTerm); red-cell advance (Sec. 2.3, Eq. kinematicPos).
 * Asynchronous on the bound stream.  If the watchdog is on
 * (lbib_set_watchdog), the call synchronises at its end and returns
 * LBIB_EUNSTABLE when the state holds a non-finite population, a
 * non-positive density, or a total mass that drifted from the set-up value
 * by more than 1e-6 relative (bounce-back walls and periodic lattices
 * conserve it to rounding; velocity walls exchange mass and are exempt from
 * this check).  The state is left in place.  Errors: LBIB_EINVAL for
 * nsteps < 0; LBIB_ESTATE outside the running phase. */
lbib_status lbib_step(lbib_ctx* ctx, int64_t nsteps);

/* Watchdog after every lbib_step call when on != 0 (default off). */
lbib_status lbib_set_watchdog(lbib_ctx* ctx, int32_t on);

/* Relative mass drift the watchdog accepts (default 1e-6; any phase).  The
 * reference is the total mass at finalize_setup or at the last set_state.
 * rel = 0 flags any change, including float32 rounding.  Errors:
 * LBIB_EINVAL for a negative or non-finite value. */
lbib_status lbib_set_watchdog_mass_tolerance(lbib_ctx* ctx, double rel);

/* Steps per captured HIP graph used by lbib_step (even, 0 = no graphs;
 * default 0).  Graph replays and plain launches give bitwise-identical
 * results. */
lbib_status lbib_set_graph_steps(lbib_ctx* ctx, int32_t steps);

/* Fields of the last completed step (synchronises): rho = sum f (Sec. 2.1)
 * and the physical velocity with the half force of Sec. 2.2,
 * u = (sum f e + F/2)/rho, F the node's total force (drive plus spread IB
 * force), ny*nx doubles each, [y][x], written into caller buffers.  Any
 * pointer may be NULL to skip it.  Before the first step: initial state.
 * Errors: LBIB_ESTATE outside the running phase. */
lbib_status lbib_get_fields(lbib_ctx* ctx, double* rho, double* ux, double* uy);

/* lbib_get_fields without allocating: for callers that cannot allocate
 * (serving loops and harnesses that forbid allocation).  Same values,
 * bit for bit, as lbib_get_fields; the fields are staged in a file-scope
 * device array that each GPU holds for the life of the process (3 x 2^19
 * doubles, 12 MiB), its address resolved per device by lbib_bind (call that
 * with the workspace's device current), and copied straight into the
 * caller's arrays; no memory is allocated on the device or the host.
 * Calls that overlap on one GPU share that array and race.  Errors:
 * LBIB_EINVAL for a lattice of more than 2^19 = 524288 nodes (use
 * lbib_get_fields), LBIB_ESTATE outside the running phase. */
lbib_status lbib_get_fields_noalloc(lbib_ctx* ctx, double* rho, double* ux, double* uy);

/* Current vertex positions of body `body` (synchronises): nv*2 doubles. */
lbib_status lbib_get_markers(lbib_ctx* ctx, int32_t body, double* xy);

/* Overwrite current and previous vertex positions of a body (running phase);
 * xy_prev may be NULL (= xy).  Rest state is unchanged.  Synchronises. */
lbib_status lbib_set_markers(lbib_ctx* ctx, int32_t body, const double* xy,
                             const double* xy_prev);

/* Force each marker of `body` handed to the fluid in the last step
 * (synchronises), nv*2 doubles: for a red cell the membrane force; for a
 * particle the weak-coupling force times the marker's arc weight. */
lbib_status lbib_get_marker_forces(lbib_ctx* ctx, int32_t body, double* fxy);

/* Ligand count over all bodies (global ligand ids are numbered body by body,
 * element ascending). */
lbib_status lbib_num_ligands(const lbib_ctx* ctx, int32_t* n);

/* Ligand-receptor bond table of Sec. 2.2 "Wall-Particle Interaction"
 * (synchronises): lig_to_rec[n_ligands], -1 = free, else receptor index
 * (wall 0 receptors first, then wall 1), written into a caller buffer.
 * *nbonds (may be NULL) receives the number of bonds.  Errors: LBIB_EINVAL
 * for lig_to_rec NULL with ligands present; LBIB_ESTATE outside the running
 * phase. */
lbib_status lbib_get_bonds(lbib_ctx* ctx, int32_t* lig_to_rec, int32_t* nbonds);

/* Overwrite the bond table (running phase).  Entries must be -1 or a valid
 * receptor index, with no receptor used twice. */
lbib_status lbib_set_bonds(lbib_ctx* ctx, const int32_t* lig_to_rec);

/* Checkpoint of the complete dynamic state (populations, marker positions
 * and history, rigid-body state, bond table, step counter).  Call with
 * blob = NULL to get the size.  set_state restores it bitwise. */
lbib_status lbib_get_state(lbib_ctx* ctx, void* blob, size_t* bytes);
lbib_status lbib_set_state(lbib_ctx* ctx, const void* blob, size_t bytes);

/* Whole-lattice diagnostics (synchronises): the invariants of the scheme
 * of Sec. 2.1 that the watchdog checks (mass, which bounce-back walls and
 * periodic lattices conserve; momentum; density range; non-finite
 * populations), the bond count of Sec. 2.2, and the library's own overflow
 * and wait counters.  Errors: LBIB_EINVAL for out NULL; LBIB_ESTATE outside
 * the running phase. */
lbib_status lbib_diagnostics(lbib_ctx* ctx, lbib_diag* out);

/* Flow regions of a body's lateral position eta = (y_c - y_lo) / (y_hi - y_lo)
 * between the walls (-1/2 and ny - 1/2, or 0 and ny - 1 with velocity walls;
 * Sec. 3, three flow regions; the paper's open intervals leave 0.2 and 0.8
 * unassigned: they go to the cell-free layer). */
enum { LBIB_REGION_CFL = 0,            /* eta <= 0.2 or eta >= 0.8        */
       LBIB_REGION_INTERMEDIATE = 1,   /* 0.2 < eta < 0.3, 0.7 < eta < 0.8 */
       LBIB_REGION_BULK = 2 };         /* 0.3 <= eta <= 0.7               */

/* Per-body observables, the quantities the paper reports for margination
 * and adhesion (Sec. 3: region occupancy, <r_max>/H, rolling and lateral
 * velocity, n_L / n_L0).  Lattice units; velocities per time step (divide
 * by u_max for the paper's ratios). */
typedef struct {
  double xc, yc;           /* centre of mass (mean of the vertex positions)
                              at the last observation; x unwrapped          */
  double x0, y0;           /* at the first observation (release)            */
  double r_max;            /* largest |yc - y0| over the observations       */
  double u_x, u_y;         /* centre-of-mass displacement over the last
                              interval / its steps (0 before the second)    */
  double u_x_sum, u_y_sum; /* sums of u_x, u_y over the intervals (n_obs - 1)*/
  int32_t region;          /* LBIB_REGION_* of yc                           */
  int32_t n_bonds;         /* ligands of the body holding a bond            */
  int32_t n_bonds0;        /* n_bonds at the first observation              */
  int32_t n_obs;           /* observations so far                           */
  int64_t step_obs;        /* step of the last observation                  */
} lbib_body_obs;

/* One observation of every body at the current step (running phase),
 * computed on the device and queued on the bound stream (does not
 * synchronise); records accumulate until lbib_reset_observations.  For the
 * host's sampling loop: step k, observe, step k, observe, ...  Errors:
 * LBIB_ESTATE outside the running phase. */
lbib_status lbib_observe(lbib_ctx* ctx);

/* Copy the records of all bodies (body order; a batch lists its instances'
 * bodies in instance order) into out[nbody] (synchronises).  Errors:
 * LBIB_EINVAL for NULL, LBIB_ESTATE outside the running phase. */
lbib_status lbib_get_observations(lbib_ctx* ctx, lbib_body_obs* out);

/* Clear the records: the next observation is the release (running phase). */
lbib_status lbib_reset_observations(lbib_ctx* ctx);

/* Measurement: launch the fused lattice kernel (streaming, collision and
 * gathered spreading) `reps` times on the bound stream with the current
 * state, bracketed by HIP events, and return the mean duration per launch
 * in milliseconds (synchronises).  The kernel reads the current populations
 * and writes the spare buffer only, so the dynamic state is unchanged.
 * Requires at least one completed step (the marker bins of that step). */
lbib_status lbib_time_lattice_kernel(lbib_ctx* ctx, int32_t reps, double* avg_ms);

/* Measurement: while on != 0, lbib_step launches kernels one by one (no
 * graphs) and binds a pair of HIP events to every fused lattice-kernel
 * dispatch on the bound stream (start and end of that dispatch, not separate
 * markers).  lbib_get_kernel_timing returns the mean duration (ms) of those
 * launches since timing was switched on, and their number (synchronises).
 * Switching on or off discards the collected events. */
lbib_status lbib_set_kernel_timing(lbib_ctx* ctx, int32_t on);
lbib_status lbib_get_kernel_timing(lbib_ctx* ctx, double* lattice_ms_avg, int64_t* launches);

/* ---------------------------------------------------------------------------
 * Discrete adjoint of a window of steps (single-lattice contexts with red
 * cells, soft and rigid particles, bounce-back walls and the Roma-kernel
 * transfer; no vertex repulsion).
 *
 * The window advances nsteps steps from the current state with the bond
 * topology frozen (no bond kinetics; bonded springs keep acting, Eq. adhFor),
 * keeping a device checkpoint of the dynamic state every ckpt_every steps.
 * The objective is
 *   J = mean over the vertices of all particles of the distance to the
 *       nearer wall, min(y + 1/2, ny - 1/2 - y), at the end of the window.
 * The backward pass recomputes each segment from its checkpoint, then applies
 * the transposed Jacobian of every step (Sec. 2.1 collision and streaming,
 * Sec. 2.2 spreading, interpolation, membrane, spring and probe loads,
 * Sec. 2.3 soft-particle, rigid-particle (Eqs. linearVelRig, angularVelRig)
 * and kinematic marker updates) in reverse order.  A rigid particle's
 * gradient has only its sigma entry (k_s and k_b do not act on it).
 *
 * lbib_adjoint_workspace_query / lbib_adjoint_bind: size and bind the
 *   caller-owned device workspace (256-byte aligned, must outlive the
 *   context's use of it) for a window of nsteps with a checkpoint every
 *   ckpt_every steps (both >= 1).  After finalize_setup.
 * lbib_adjoint_forward: run the window; *J receives the objective, *nbonds
 *   (may be NULL) the number of bonds held during the window.  Leaves the
 *   context at the end of the window.
 * lbib_adjoint_backward: after lbib_adjoint_forward (and no parameter
 *   change since): grad[3*b + 0..2] = dJ * dJ/dk_s, dJ * dJ/dk_b,
 *   dJ * dJ/dsigma of body b (all bodies of the context, host array).  The
 *   context is left at the end of the window.  The gradient is bitwise
 *   reproducible: the scatter-form terms (transposed interpolation, probe
 *   and spreading) add into exact fixed-point accumulators (two 64-bit
 *   integer words, resolution 2^-72), so their sums do not depend on the
 *   order of the atomics.
 * Errors: LBIB_ESTATE before finalize_setup, without a bound workspace or
 *   forward window; LBIB_EINVAL for batches, the vertex repulsion, velocity
 *   walls, the MLS transfer or bad sizes;
 *   LBIB_ENOSPACE for a workspace that is too small; LBIB_EUNSTABLE from
 *   lbib_adjoint_backward when a scattered term is not finite or of magnitude
 *   2^30 or more (grad is then left unwritten). */
lbib_status lbib_adjoint_workspace_query(const lbib_ctx* ctx, int64_t nsteps, int32_t ckpt_every,
                                         size_t* bytes);
lbib_status lbib_adjoint_bind(lbib_ctx* ctx, void* dev_workspace, size_t bytes, int64_t nsteps,
                              int32_t ckpt_every);
lbib_status lbib_adjoint_forward(lbib_ctx* ctx, double* J, int32_t* nbonds);
lbib_status lbib_adjoint_backward(lbib_ctx* ctx, double dJ, double* grad);

/* Change the strain constant k_s (Eq. strainFor), bending constant k_b
 * (Eq. bendFor) and bond spring constant sigma (Eq. adhFor) of body `body`
 * of a running single-lattice context (instance 0 of a batch).  All >= 0 and
 * finite, else LBIB_EINVAL; LBIB_ESTATE before finalize_setup.  Invalidates
 * the last adjoint forward window. */
lbib_status lbib_set_body_params(lbib_ctx* ctx, int32_t body, double ks, double kb, double sigma);

/* How steps are launched (the results are the same bit for bit):
 *   1  three kernels per step: body forces and particle motion, fused
 *      lattice step, marker advance;
 *   2  merged: inside a run the body kernel first finishes the previous
 *      step's marker advance for its own bodies (two kernels per step; used
 *      only when every body has <= 512 vertices, else as 1);
 *   3  overlapped: the lattice tiles without IB force run on a second stream
 *      while the body kernel runs, the tiles with IB force after it;
 *   0  automatic (default): 2 when every body has <= 512 vertices, else 1.
 * Allowed in any phase; LBIB_EINVAL for other values.  lbib_get_step_mode
 * returns the form in use (after finalize_setup) or the requested mode. */
lbib_status lbib_set_step_mode(lbib_ctx* ctx, int32_t mode);
lbib_status lbib_get_step_mode(const lbib_ctx* ctx, int32_t* mode);

/* Cache hints of the fused lattice kernel's population accesses (the
 * results are the same bit for bit; only the speed differs):
 *   0  plain loads and stores;
 *   1  non-temporal loads (pull streaming reads every population once);
 *   3  non-temporal loads and stores;
 *  -1  automatic (default): 3 on a single lattice whose two population
 *      buffers take at most 128 MB, else 0.
 * Allowed in any phase; LBIB_EINVAL for other values.  lbib_get_cache_hints
 * returns the hints in use. */
lbib_status lbib_set_cache_hints(lbib_ctx* ctx, int32_t hints);
lbib_status lbib_get_cache_hints(const lbib_ctx* ctx, int32_t* hints);

/* Launch form of the fused lattice kernel (the results are the same bit for
 * bit; only the speed differs):
 *   0        one workgroup per tile, the default;
 *   1,2,4,8  persistent: that many workgroups per compute unit of the
 *            device, each walking the tiles with a fixed stride (the tiles
 *            of one XCD stay on that XCD).
 * The batched sweeps' autotuner times these forms.  Allowed in any phase;
 * LBIB_EINVAL for other values.  lbib_get_lattice_launch returns the form. */
lbib_status lbib_set_lattice_launch(lbib_ctx* ctx, int32_t wgs_per_cu);
lbib_status lbib_get_lattice_launch(const lbib_ctx* ctx, int32_t* wgs_per_cu);

/* Streaming of the populations (Sec. 2.1, Eq. BGK; the results are the same
 * bit for bit, only the speed differs):
 *   0   two buffers: every step pulls from one and writes the other;
 *   1   one buffer, updated in place: steps alternate between a pass that
 *       reads each node's neighbours and writes their slots and a pass local
 *       to the node, so that every slot is read and then written by a single
 *       node of the step (one buffer's working set: a 4.45 M-node lattice's
 *       160 MB stays in the last-level cache);
 *  -1   automatic (default): 1 when one population buffer takes at most
 *       192 MB, else 0.
 * Allowed in any phase; on a running context the populations are converted
 * (graphs captured before are dropped).  The state blob of lbib_get_state is
 * the same in both forms.  lbib_get_streaming returns 1 for in place.
 * LBIB_EINVAL for other values. */
lbib_status lbib_set_streaming(lbib_ctx* ctx, int32_t mode);
lbib_status lbib_get_streaming(const lbib_ctx* ctx, int32_t* inplace);

/* Completed step count. */
lbib_status lbib_get_step(const lbib_ctx* ctx, int64_t* step);

/* Free the context (not the caller's workspace).  NULL is allowed. */
lbib_status lbib_destroy(lbib_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBIB_H */
