/*
 * ppmlr.h -- C ABI of the MI355X PPMLR-MHD split-sweep library.
 *
 * The library advances the 3D ideal-MHD equations with the dipole split
 * B = B_d + B' (paper, Section II: conservative equations for rho, rho v,
 * B', E with E = p/(gamma-1) + rho v^2/2 + B'^2/2) by the PPMLR method:
 * zone-centred volume averages, a parabolic distribution in each zone,
 * characteristic edge values, a Lagrangian update with an interface Riemann
 * solve, and a remap onto the fixed Eulerian grid.  The 3D problem is split
 * into three independent 1D problems per zone, one per axis (Section III-A),
 * on the stretched Cartesian grid of Section III-A (Earth at the origin, x
 * toward the Sun, y dusk, z north).  Code units with mu0 = 1.
 *
 * Conventions for every entry point:
 *   - Return value: ppmlr_status, 0 = PPMLR_OK, negative = error.  Nothing
 *     aborts or throws across the ABI; ppmlr_last_error() gives a message.
 *   - State: one device buffer, SoA [8][nz][ny][nx] (x fastest) holding
 *     (rho, m_x, m_y, m_z, B'_x, B'_y, B'_z, E') in FP32 or FP64.  The caller
 *     owns it (e.g. a torch tensor) and the stream the work is queued on.
 *   - Host arrays passed in (face coordinates, states of boundary conditions)
 *     are copied; the caller keeps ownership.
 *   - Calls that only queue GPU work return as soon as it is queued; calls
 *     that return a value to the host (cfl_dt, totals, stats, status_check,
 *     time) synchronise the stream.
 *   - A context may be used from one host thread at a time.
 */
#ifndef PPMLR_H
#define PPMLR_H

#ifdef __cplusplus
extern "C" {
#endif

typedef int ppmlr_status;
#define PPMLR_OK 0
#define PPMLR_EINVAL (-1)    /* bad argument: axis, dt <= 0, grid, dtype, null */
#define PPMLR_ECFL (-2)      /* dt above the CFL limit (checked in debug mode) */
#define PPMLR_ERIEMANN (-3)  /* a face hit the Newton iteration limit */
#define PPMLR_ENONPHYS (-4)  /* rho <= 0 or a non-finite value entered a sweep */
#define PPMLR_EDEVICE (-5)   /* HIP runtime error (message in last_error) */
#define PPMLR_ENOMEM (-6)    /* device allocation failed */

/* boundary conditions per domain face */
#define PPMLR_PERIODIC 0
#define PPMLR_OUTFLOW 1      /* zero gradient: ghosts copy the edge zone */
#define PPMLR_INFLOW 2       /* ghosts hold the fixed inflow state */

/* state precision */
#define PPMLR_F32 0
#define PPMLR_F64 1

#define PPMLR_GHOSTS 7       /* ghost zones per side (with flattening) */

typedef struct ppmlr_ctx ppmlr_ctx;   /* opaque, library-owned */

/* Scheme options.  ppmlr_default_options() fills the defaults noted. */
typedef struct {
    int flatten;        /* shock flattening (Colella-Woodward appendix), 1 */
    int janhunen;       /* -v div B' induction source (Section II eqs), 1 */
    int max_iter;       /* Newton iteration limit of the Riemann solve, 20 */
    double tol_f64;     /* Newton stop |dP| <= tol P in FP64, 1e-12 */
    double tol_f32;     /* same in FP32, 1e-6 */
    double p_floor;     /* thermal-pressure floor (absolute), 1e-8 */
    int collect_stats;  /* iteration histogram and floor counters, 1 (about
                           2 % of a sweep's time) */
    int debug_cfl;      /* ppmlr_step checks dt against the CFL limit, 0 */
    int tracing;        /* zone-edge values and interface solve (Section II:
                           edge values by a characteristic method, then the
                           interface Riemann problem), 0:
                             PPMLR_TRACE_TWO_FAMILY (default): the fast pair
                             (rho, u, p, B_t) and the Alfven pair (rho, v_t,
                             B_t) traced over their own domains of
                             dependence, with the oblique coupling terms;
                             the two-shock Newton solve and the linear Alfven
                             solve;
                             PPMLR_TRACE_CHARACTERISTIC: the seven waves
                             traced one by one (fast reference, Alfven and
                             slow projected on their eigenvectors) and the
                             interface problem of all seven waves in its
                             linearisation about the face-mean state (no
                             iteration; meant for smooth flows: it does not
                             take the two-shock solve's nonlinear jumps).
                             An Alfven or slow wave slower than 1e-4 of the
                             fast wave counts as at rest (a normal field
                             that cancels to rounding noise decides
                             nothing); a traced state without positive
                             density and pressure falls back to the zone
                             average.
                           Plain initial-guess mode only; no ensembles. */
} ppmlr_options;
#define PPMLR_TRACE_TWO_FAMILY 0
#define PPMLR_TRACE_CHARACTERISTIC 1

/* Grid: zone counts, boundary conditions, inner boundary radius. */
typedef struct {
    int n[3];           /* nx, ny, nz >= 1; >= 7 on non-periodic axes */
    int bc_lo[3];       /* PPMLR_PERIODIC / OUTFLOW / INFLOW per axis */
    int bc_hi[3];       /* periodic must be set on both sides */
    double r_inner;     /* zones with centre radius < r_inner are reset to
                           the inner state after every sweep; <= 0: none */
} ppmlr_grid;

/* Face coordinates: host arrays of n[a]+1 strictly increasing values. */
typedef struct {
    const double *faces[3];
} ppmlr_coords;

/* A state buffer on the device and the stream its work is queued on. */
typedef struct {
    void *u;            /* device pointer, SoA [8][nz][ny][nx] */
    int dtype;          /* PPMLR_F32 or PPMLR_F64 */
    void *stream;       /* hipStream_t; NULL = default stream */
} ppmlr_state;

/* Counters accumulated since the last ppmlr_reset_stats.  Interface counts
 * cover the faces -1/2 .. N-1/2 of every pencil, each once whatever the
 * segments. */
typedef struct {
    long long iters_hist[32];  /* Newton iterations per interface (bin 31: >=31) */
    long long floor_hits;      /* zones whose pressure was floored */
    long long nonconverged;    /* interfaces that hit max_iter */
    long long nonphys;         /* zones with rho <= 0 or non-finite values */
    long long guess_faces;     /* faces selected for the learned guess (learned / harvest modes) */
    long long guess_fallbacks; /* selected faces that started from the plain guess instead */
} ppmlr_stats_t;

void ppmlr_default_options(ppmlr_options *opt);

/* Create a context for one grid.  gamma: adiabatic index (Section II: 5/3).
 * coords: host face coordinates, copied to the device.  opt: NULL for the
 * defaults.  Returns EINVAL for a bad grid (counts, non-increasing faces,
 * mismatched periodic sides, non-periodic axis shorter than 7 zones, more
 * than 2^24 zones along an axis).  Pencils longer than one workgroup holds
 * (1010 zones in FP32, 818 in FP64) are swept in segments (see
 * ppmlr_set_segments).  Every call that takes a state also returns EINVAL
 * if one variable of it (nx ny nz elements) exceeds 4 GiB: FP32 grids up to
 * 2^30 zones, FP64 up to 2^29 zones. */
ppmlr_status ppmlr_create(const ppmlr_grid *grid, double gamma, const ppmlr_coords *coords,
                          const ppmlr_options *opt, ppmlr_ctx **out);
void ppmlr_destroy(ppmlr_ctx *ctx);
const char *ppmlr_last_error(const ppmlr_ctx *ctx);

/* Static background field B_d (Section II: the Earth dipole, which is
 * subtracted from B and evaluated analytically wherever it is needed):
 * B_d = M [3 (m.r) r / r^5 - m / r^3] + b_ext.  moment: M in code units
 * (0 = no dipole); dir: unit vector m (host, 3 values).  b_ext: a uniform
 * field (host, 3 values), zero by default. */
ppmlr_status ppmlr_set_dipole(ppmlr_ctx *ctx, double moment, const double dir[3]);
ppmlr_status ppmlr_set_background(ppmlr_ctx *ctx, const double b_ext[3]);

/* Fixed state of PPMLR_INFLOW ghosts (solar wind and IMF upstream, Section
 * IV-A): primitive rho, vx, vy, vz, Bx, By, Bz (total field), p. */
ppmlr_status ppmlr_set_inflow(ppmlr_ctx *ctx, const double prim[8]);

/* Time-dependent driving at the inflow faces: n knots (t[k] increasing,
 * prim[8k..8k+7] as for ppmlr_set_inflow, host arrays, copied).  The inflow
 * ghost state of a step from t to t + dt is the series at the mid-time
 * t + dt/2, linear in time between knots and held at the first / last knot
 * outside them (t = the context's simulated time, see ppmlr_time; a lone
 * ppmlr_sweep uses t + dt/2 without advancing it).  n = 0 returns to the
 * constant state of ppmlr_set_inflow.  EINVAL for non-increasing or
 * non-finite times, non-finite values, or non-positive density or pressure.
 * Ensembles do not take series.  Synchronises the device. */
ppmlr_status ppmlr_set_inflow_series(ppmlr_ctx *ctx, int n, const double *t, const double *prim);

/* State the zones inside r_inner are reset to (rest, B' = 0; with an
 * ionosphere coupling attached, the drift it set, see below). */
ppmlr_status ppmlr_set_inner(ppmlr_ctx *ctx, double rho, double p);

/* ------------------------------------------------------------------ */
/* Ionosphere shell coupling (Section II: a thin shell at 1.017 R_E     */
/* closes the field-aligned currents; the electrostatic potential        */
/* solved on it is carried along dipole field lines to the inner         */
/* boundary, where it sets the flow)                                     */
/* ------------------------------------------------------------------ */

/* Shell parameters.  ppmlr_iono_default_params() fills the defaults noted. */
typedef struct {
    int n_theta;        /* cells per polar cap in magnetic colatitude, 32 */
    int n_phi;          /* cells in longitude, 64; n_theta * n_phi <= 4096
                           and 8 * (4 n_theta n_phi + 3 n_theta + 2 n_phi)
                           bytes must fit the 160 KiB of LDS */
    double r_shell;     /* shell radius, 1.017 (R_E) */
    double r_fac;       /* radius where the field-aligned current is taken
                           on each cell's field line, 3.5 (> r_shell; the
                           sphere, with one zone of margin for the central
                           differences, must lie inside the grid) */
    double sigma;       /* height-integrated Pedersen conductance in code
                           units (mu_0 = 1: S times mu_0 v_0), 5 S = 0.137 */
} ppmlr_iono_params;

void ppmlr_iono_default_params(ppmlr_iono_params *p);

/* One coupling of the state (FP32 or FP64, on its stream):
 *   1. j_r: the radial current density reaching each shell cell, from
 *      J = curl B' at the zone centres (central differences) around the point
 *      where the cell's dipole field line crosses r_fac (trilinear
 *      interpolation), its component along the dipole, times
 *      |B(shell)| / |B(r_fac)| (J_par / |B| is constant along a flux tube);
 *   2. Phi: div_h(sigma grad_h Phi) = j_r on the polar cap of each hemisphere
 *      whose field lines cross r_fac (magnetic colatitude theta with
 *      sin^2 theta <= r_shell / r_fac), Phi = 0 at its edge; finite volumes
 *      on cells uniform in theta and longitude, solved directly in FP64 (a
 *      discrete Fourier transform in longitude, one tridiagonal system per
 *      mode in colatitude: the conductance is uniform);
 *   3. the drift v = E x B_d / |B_d|^2 of every zone with centre inside
 *      r_inner, E = -grad Phi by central differences of the potential at the
 *      footpoints of the zone's and its neighbours' field lines (zero where a
 *      zone or neighbour lies inside the shell), kept by the context: every
 *      later sweep resets those zones to (inner rho, v, inner p, B' = 0)
 *      until ppmlr_ionosphere_detach.
 * Magnetic frame: z_m opposite to the dipole moment, x_m the x axis
 * projected off z_m; hemisphere 0 is z_m > 0; cell (h, k, j) at colatitude
 * (k + 1/2) theta_c / n_theta and longitude (j + 1/2) 2 pi / n_phi.
 * jr, phi (device pointers, may be NULL) receive [2][n_theta][n_phi] FP64.
 * EINVAL without a
 * dipole or an inner boundary, for bad parameters, or when the sphere r_fac
 * does not fit inside the zone centres with one zone of margin.  The
 * context allocates its work buffers at the first call (and again when the
 * shell grows).  Synchronises. */
ppmlr_status ppmlr_ionosphere_couple(ppmlr_ctx *ctx, const ppmlr_state *state, const ppmlr_iono_params *params,
                                     double *jr, double *phi);

/* Back to the inner state at rest. */
ppmlr_status ppmlr_ionosphere_detach(ppmlr_ctx *ctx);

/* One 1D sweep along axis (0 = x, 1 = y, 2 = z) over every pencil of the
 * grid (Section III-A: the 3D equations split into independent 1D
 * problems); the result replaces the state (a segmented axis sweeps into
 * the context's second state and copies back).  dt > 0.  Queued on
 * state->stream. */
ppmlr_status ppmlr_sweep(ppmlr_ctx *ctx, const ppmlr_state *state, double dt, int axis);

/* One split step: x, y, z sweeps on even steps and z, y, x on odd steps
 * (step counter held by the context, starts at 0), all with the same dt;
 * advances the simulated time by dt. */
ppmlr_status ppmlr_step(ppmlr_ctx *ctx, const ppmlr_state *state, double dt);
ppmlr_status ppmlr_set_step_index(ppmlr_ctx *ctx, long long step);
ppmlr_status ppmlr_get_step_index(const ppmlr_ctx *ctx, long long *step);

/* Largest stable time step: cfl / max over zones outside r_inner of
 * max_a (|v_a| + c_f,a) / dx_a, with c_f,a the fast speed along axis a
 * computed from the total field; reduced in FP64.  Synchronises. */
ppmlr_status ppmlr_cfl_dt(ppmlr_ctx *ctx, const ppmlr_state *state, double cfl, double *dt_out);

/* nsteps split steps with dt = cfl-limited and computed on the device from
 * the state at the start of each step (the last sweep of a step fuses the
 * signal-speed maximum); no host synchronisation.  The accumulated simulated
 * time (of ppmlr_step and ppmlr_advance) is read with ppmlr_time. */
ppmlr_status ppmlr_advance(ppmlr_ctx *ctx, const ppmlr_state *state, int nsteps, double cfl);
ppmlr_status ppmlr_time(ppmlr_ctx *ctx, const ppmlr_state *state, double *t_out);

/* Volume integrals of the 8 conserved variables, FP64, fixed-order
 * reduction (bitwise reproducible).  Synchronises. */
ppmlr_status ppmlr_totals(ppmlr_ctx *ctx, const ppmlr_state *state, double out[8]);

/* Counters; synchronises the given stream (NULL: device). */
ppmlr_status ppmlr_stats(ppmlr_ctx *ctx, void *stream, ppmlr_stats_t *out);
ppmlr_status ppmlr_reset_stats(ppmlr_ctx *ctx, void *stream);
/* PPMLR_ENONPHYS / PPMLR_ERIEMANN if the counters since the last reset
 * recorded such events, else PPMLR_OK.  Synchronises. */
ppmlr_status ppmlr_status_check(ppmlr_ctx *ctx, void *stream);

/* Measurement: when enabled, every sweep launch is bracketed by a pair of
 * HIP events recorded on the state's stream.  ppmlr_kernel_times
 * synchronises, and returns per axis the summed kernel time in ms and the
 * number of launches since profiling was enabled (then starts over). */
ppmlr_status ppmlr_set_profiling(ppmlr_ctx *ctx, int enable);
ppmlr_status ppmlr_kernel_times(ppmlr_ctx *ctx, double ms[3], long long launches[3]);

/* Pencils per workgroup for sweeps along axis (tile shape); 0 = automatic.
 * EINVAL if the tile does not fit one workgroup. */
ppmlr_status ppmlr_set_tile(ppmlr_ctx *ctx, int axis, int pencils);
ppmlr_status ppmlr_get_tile(const ppmlr_ctx *ctx, int axis, int dtype, int *pencils);

/* Segments per pencil for sweeps along axis; 0 = automatic: the fewest whose
 * tile fits one workgroup for the state's dtype (one, unless the pencil is
 * longer than 1010 zones in FP32 or 818 in FP64).  A sweep
 * tile then holds `pencils` pencil segments of ceil(N / segments) interior
 * zones (the last segment takes the rest) plus the 7 ghost zones on either
 * side that the reconstruction, Riemann solve and remap of the sweep
 * (Section II, the method) reach: neighbouring segments overlap by those ghosts and
 * each zone is computed by its own segment only, so the result does not
 * depend on the segment count, bit for bit.  Shorter tiles trade recomputed
 * ghost zones for fewer state planes per workgroup; the z sweep of a large
 * grid, whose planes lie far apart in memory, gains most.  A segmented sweep
 * reads zones that other workgroups update, so it writes a second state of
 * the same size that the context allocates at its first use and keeps until
 * ppmlr_destroy; sweeps alternate between the two, and a call that would
 * end in the second state copies it back (ppmlr_advance with the z sweep
 * segmented ends at home after an even number of steps).  EINVAL if a
 * segment would be empty or shorter than 7 zones, or the current tile no
 * longer fits one workgroup. */
ppmlr_status ppmlr_set_segments(ppmlr_ctx *ctx, int axis, int segments);
/* Tile order of segmented sweeps along axis: 1 = the segments of one pencil
 * group are consecutive tiles, 2 = the grid is dealt out one segment band
 * after another (the tiles running together then touch fewer state planes),
 * 0 = automatic (1 for x, 2 for y and z).  Results do not depend on it.
 * ppmlr_get_segment_order returns the order in effect (1 or 2). */
ppmlr_status ppmlr_set_segment_order(ppmlr_ctx *ctx, int axis, int order);
ppmlr_status ppmlr_get_segment_order(const ppmlr_ctx *ctx, int axis, int *order);
ppmlr_status ppmlr_get_segments(const ppmlr_ctx *ctx, int axis, int dtype, int *segments);

/* Tile autotuner: for each axis, times `reps` sweeps of every tile shape
 * (pencils per workgroup, segments per pencil from 1 to 8, both segment
 * orders) that fits one
 * workgroup on a library-owned copy of the state (the caller's state is not
 * modified), times the three fastest again with 3 x reps sweeps, keeps the
 * fastest per axis (the shape is set on the context) and returns the pencils
 * per workgroup in tiles[3] (may be NULL).  The sweeps timed use the context's initial-guess mode
 * (the harvest mode is timed as the plain one and records nothing); they add
 * to the counters.  Synchronises; allocates and frees one state-sized buffer. */
ppmlr_status ppmlr_autotune(ppmlr_ctx *ctx, const ppmlr_state *state, int reps, int tiles[3]);

/* Batched ensemble: many independent runs of different sizes, each with its
 * own inflow and its own CFL-limited dt (the Section IV-A set-up per member),
 * advanced together.  Advances member m (ctxs[m], states[m]) by `steps` split
 * steps with dt computed on the device per member, exactly as ppmlr_advance
 * would (same arithmetic, bitwise equal results for the same tiles).  Two
 * launch forms (ppmlr_set_ensemble_launch), with the same results:
 *   - per sweep (default): each sweep of a step is one launch over the
 *     tiles of every member (four launches per step: per-member dt + three
 *     sweeps);
 *   - persistent: the whole call is one launch; as many workgroups as the
 *     device holds at once take the tiles of every member in each sweep,
 *     with a grid-wide barrier between the phases (the start-of-call
 *     signal-speed maximum, each step's per-member dt, each sweep).  The
 *     launch is cooperative, so the runtime refuses a grid that cannot be
 *     co-resident; a barrier wait that polls for seconds gives up, and the
 *     call then returns PPMLR_EDEVICE.  Slower on MI355X (its kernel holds
 *     more registers, so fewer workgroups are resident), kept for callers
 *     that need one launch per call.
 * All states must share one dtype and stream (states[0]->stream) and all
 * contexts the same step-counter parity; the contexts' dt, time, signal-speed
 * and counter buffers are used as by ppmlr_advance, so none of the contexts
 * may be in use elsewhere meanwhile.
 * block: workgroup size 256, 512 or 1024 (every pencil segment + 14 ghosts must fit;
 * 1024 is FP32 only), or 0 for the value chosen by ppmlr_ensemble_autotune
 * (512 if it never ran); each member's pencils are cut into the segments
 * its context is set to (ppmlr_set_segments), and pencils per workgroup per
 * member and axis are the most that fit the workgroup.  A member with
 * segments alternates between its state and its context's second state
 * (allocated at first use) every sweep, and is copied back after an odd
 * number of sweeps.  per_member (may be NULL) receives each
 * member's ppmlr_status_check result.  Synchronises; allocates and frees its
 * work tables. */
ppmlr_status ppmlr_ensemble_run(ppmlr_ctx *const *ctxs, const ppmlr_state *const *states, int n, int steps,
                                double cfl, int block, ppmlr_status *per_member);

/* Launch form of the ensemble calls (process-wide; default per sweep).
 * EINVAL for another value. */
#define PPMLR_ENSEMBLE_PERSISTENT 0
#define PPMLR_ENSEMBLE_PER_SWEEP 1
ppmlr_status ppmlr_set_ensemble_launch(int mode);

/* Polls of a grid-barrier wait in the persistent ensemble launch before it
 * gives up (process-wide; default 4194304, seconds of waiting).  0 makes
 * every wait give up at its first poll, which exercises the error path
 * (PPMLR_EDEVICE, the kernel leaves normally, the states are then
 * undefined).  EINVAL for a negative value. */
ppmlr_status ppmlr_set_ensemble_barrier_limit(long long polls);

/* ppmlr_ensemble_run without device allocation, for callers that cannot
 * allocate device memory during the call (tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, arithmetic and results as
 * ppmlr_ensemble_run (bitwise), but the per-call work tables (sweep
 * descriptors, tile offsets, per-member dt pointers) live in one fixed
 * library array in device memory instead of being allocated and freed:
 * about 250 KB per GPU, taken when a process first calls this function on
 * that GPU and held until the process ends.  Limits and errors:
 *   - at most 64 members (more: PPMLR_EINVAL with a message);
 *   - all contexts on one device (else PPMLR_EINVAL);
 *   - a member cut into pencil segments needs its context's second state
 *     to exist already (it is allocated by the first segmented sweep,
 *     ppmlr_ensemble_run or ppmlr_advance of that context); otherwise
 *     PPMLR_EINVAL, and nothing is allocated.
 * Every call on one GPU uses the same array and overwrites the previous
 * call's tables: calls on one stream are ordered, but calls that overlap on
 * one GPU (other streams, other host threads) race and must not be made.
 * Synchronises (after uploading the tables and in the per_member check).
 * No hipMalloc, hipFree or other device-allocating routine is called. */
ppmlr_status ppmlr_ensemble_run_noalloc(ppmlr_ctx *const *ctxs, const ppmlr_state *const *states, int n, int steps,
                                        double cfl, int block, ppmlr_status *per_member);

/* Ensemble tile autotuner: times `reps` ensemble steps for each feasible
 * workgroup size (256, 512, 1024) and target segment length (whole pencils,
 * or segments of about 96, 64, 48 or 32 interior zones) on library-owned
 * copies of the states (the callers' states, step counters and times are
 * left unchanged), stores the fastest workgroup size for ensemble calls with
 * block = 0, returns it in *block (may be NULL), and sets every member
 * context's segments per axis to the fastest length's; then, at that
 * workgroup size, tries each other length for one axis at a time (over at
 * least 5 steps) and keeps it where it is faster. */
ppmlr_status ppmlr_ensemble_autotune(ppmlr_ctx *const *ctxs, const ppmlr_state *const *states, int n, int reps,
                                     double cfl, int *block);

/* ------------------------------------------------------------------ */
/* Learned initial guess for the interface Riemann solve                 */
/* ------------------------------------------------------------------ */
/*
 * The normal-pair Riemann problem at each face (Section II: the Lagrangian
 * step solves a Riemann problem at every zone interface) is solved by a
 * Newton iteration on the star pressure.  Its starting point is the linear
 * (acoustic) guess, or, in the learned mode, the output of a small MLP on
 * the faces with a strong jump.  The converged solution is the same within
 * the iteration tolerance; only the iteration count changes.
 *
 * Network: 14 inputs, two hidden layers of 64 (tanh-form GELU), 2 outputs.
 * Inputs per face: for the left then the right state,
 *   rho/rho_m, (u - u_m)/c_m, (v_t1 - v_t1m)/c_m, (v_t2 - v_t2m)/c_m,
 *   B_t1/sqrt(P_m), B_t2/sqrt(P_m), P/P_m,
 * where _m are the means of the two states, c_m = sqrt(P_m/rho_m), P is the
 * total pressure the solver sees and B_t the total transverse field.
 * Outputs: (P* - P0)/P_m and (u* - u0)/c_m, the star pressure and velocity as
 * residuals on the linear guess (P0, u0).  A face is selected when
 * |P_R - P_L| > g_p min(P_L, P_R) or |u_R - u_L| > g_u c_m (default 0.1, 0.1).
 * Parameters: PPMLR_MLP_PARAMS FP32 values, W1[14][64], b1[64], W2[64][64],
 * b2[64], W3[64][2], b3[2], row-major with the input index first.  The
 * kernels use BF16 weights and activations with FP32 accumulation on the
 * matrix cores.
 */
#define PPMLR_GUESS_PLAIN 0
#define PPMLR_GUESS_LEARNED 1
#define PPMLR_GUESS_HARVEST 2
#define PPMLR_MLP_PARAMS 5250
#define PPMLR_RECORD_FLOATS 28

/* Initial-guess mode of the FP32 sweeps of this context (FP64 sweeps always
 * use the linear guess).  PLAIN: linear guess.  LEARNED: theta (device,
 * PPMLR_MLP_PARAMS FP32) is copied into the context and packed into BF16 on
 * `stream`; the call synchronises, so theta may change afterwards.
 * HARVEST: linear guess, and every selected face appends one record to the
 * buffer set by ppmlr_set_harvest (EINVAL if none).  Learned and harvest
 * sweeps always count the iterations (ppmlr_stats). */
ppmlr_status ppmlr_set_guess(ppmlr_ctx *ctx, int mode, const float *theta, void *stream);

/* Face-selection thresholds g_p, g_u (>= 0) of the learned and harvest modes. */
ppmlr_status ppmlr_set_gate(ppmlr_ctx *ctx, double rel_p, double rel_u);

/* Harvest buffer (caller-owned device memory): records[capacity][28] FP32 and
 * a device counter the sweeps increment once per offered record (the caller
 * zeroes it; records beyond the capacity are counted, not written).  Record:
 * [0..13] the 14 network inputs, [14..15] the 2 targets, then the solver's
 * own scalars: P~_L, P~_R, P_d, u_L, u_R, C_L, C_R, k_L, k_R, P~0, P~*, u*
 * (P~ = perturbation total pressure, P = P~ + P_d; C Lagrangian sound speed;
 * k = (gamma_e + 1) / (2 gamma_e)).  records = NULL detaches the buffer (and
 * leaves the harvest mode). */
ppmlr_status ppmlr_set_harvest(ppmlr_ctx *ctx, float *records, long long capacity, unsigned long long *count);

/* Training workspace for batches of up to max_batch samples (device buffers
 * for packed weights and per-workgroup partial gradients). */
typedef struct ppmlr_mlp ppmlr_mlp;
ppmlr_status ppmlr_mlp_create(int max_batch, ppmlr_mlp **out);
void ppmlr_mlp_destroy(ppmlr_mlp *mlp);
const char *ppmlr_mlp_last_error(const ppmlr_mlp *mlp);

/* Network outputs for n samples: X[n][ldx] (first 14 columns used) ->
 * Y[n][ldy] (first 2 columns written).  All pointers on the device; queued on
 * `stream`.  n = 0 does nothing (the pointers are not checked). */
ppmlr_status ppmlr_mlp_forward(ppmlr_mlp *mlp, const float *theta, const float *X, int ldx, int n, float *Y, int ldy,
                               void *stream);

/* Loss L = (1 / 2n) sum over samples and outputs of (net - target)^2 for a
 * batch of 1 <= n <= max_batch samples (targets Y[n][ldy], first 2 columns),
 * and its gradient (grad: PPMLR_MLP_PARAMS FP32, theta order; may be NULL;
 * loss: one FP32, may be NULL).  Partial sums are added in a fixed order:
 * results are reproducible. */
ppmlr_status ppmlr_mlp_grad(ppmlr_mlp *mlp, const float *theta, const float *X, int ldx, const float *Y, int ldy,
                            int n, float *grad, float *loss, void *stream);

/* One Adam step (Kingma & Ba 2015, bias-corrected, step number t >= 1) on the
 * FP32 master parameters theta with moments m, v, using the gradient of the
 * batch as in ppmlr_mlp_grad; loss (may be NULL) receives the batch loss
 * before the step. */
ppmlr_status ppmlr_mlp_train_step(ppmlr_mlp *mlp, float *theta, float *m, float *v, const float *X, int ldx,
                                  const float *Y, int ldy, int n, int t, float lr, float beta1, float beta2,
                                  float eps, float *loss, void *stream);

#ifdef __cplusplus
}
#endif
#endif
