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
    int collect_stats;  /* iteration histogram and floor counters, 1 */
    int debug_cfl;      /* ppmlr_step checks dt against the CFL limit, 0 */
} ppmlr_options;

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

/* Counters accumulated since the last ppmlr_reset_stats. */
typedef struct {
    long long iters_hist[32];  /* Newton iterations per interface (bin 31: >=31) */
    long long floor_hits;      /* zones whose pressure was floored */
    long long nonconverged;    /* interfaces that hit max_iter */
    long long nonphys;         /* zones with rho <= 0 or non-finite values */
} ppmlr_stats_t;

void ppmlr_default_options(ppmlr_options *opt);

/* Create a context for one grid.  gamma: adiabatic index (Section II: 5/3).
 * coords: host face coordinates, copied to the device.  opt: NULL for the
 * defaults.  Returns EINVAL for a bad grid (counts, non-increasing faces,
 * mismatched periodic sides, non-periodic axis shorter than 7 zones). */
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

/* State the zones inside r_inner are reset to (rest, B' = 0). */
ppmlr_status ppmlr_set_inner(ppmlr_ctx *ctx, double rho, double p);

/* One 1D sweep along axis (0 = x, 1 = y, 2 = z) over every pencil of the
 * grid, in place (Section III-A: the 3D equations split into independent 1D
 * problems).  dt > 0.  Queued on state->stream. */
ppmlr_status ppmlr_sweep(ppmlr_ctx *ctx, const ppmlr_state *state, double dt, int axis);

/* One split step: x, y, z sweeps on even steps and z, y, x on odd steps
 * (step counter held by the context, starts at 0), all with the same dt. */
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
 * time is read with ppmlr_time. */
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

/* Tile autotuner: for each axis, times `reps` sweeps of every tile shape that
 * fits one workgroup on a library-owned copy of the state (the caller's state
 * is not modified), keeps the fastest per axis and returns them in tiles[3]
 * (may be NULL).  Synchronises; allocates and frees one state-sized buffer. */
ppmlr_status ppmlr_autotune(ppmlr_ctx *ctx, const ppmlr_state *state, int reps, int tiles[3]);

/* Batched ensemble: many independent runs of different sizes, each with its
 * own inflow and its own CFL-limited dt (the Section IV-A set-up per member),
 * advanced together.  Advances member m (ctxs[m], states[m]) by `steps` split
 * steps with dt computed on the device per member, exactly as ppmlr_advance
 * would (same arithmetic, bitwise equal results for the same tiles).  Each
 * sweep of a step is one launch that covers the tiles of every member, so
 * the device sees one large grid instead of many small ones; per step there
 * are four launches (per-member dt + three sweeps) whatever the member count.
 * All states must share one dtype and stream (states[0]->stream) and all
 * contexts the same step-counter parity; the contexts' dt, time, signal-speed
 * and counter buffers are used as by ppmlr_advance, so none of the contexts
 * may be in use elsewhere meanwhile.
 * block: workgroup size 256, 512 or 1024 (every pencil + 14 ghosts must fit;
 * 1024 is FP32 only), or 0 for the value chosen by ppmlr_ensemble_autotune
 * (512 if it never ran); pencils per workgroup per member and axis are the
 * most that fit the workgroup.  per_member (may be NULL) receives each
 * member's ppmlr_status_check result.  Synchronises; allocates and frees its
 * work tables. */
ppmlr_status ppmlr_ensemble_run(ppmlr_ctx *const *ctxs, const ppmlr_state *const *states, int n, int steps,
                                double cfl, int block, ppmlr_status *per_member);

/* Ensemble tile autotuner: times `reps` ensemble steps for each feasible
 * workgroup size on library-owned copies of the states (the callers' states,
 * step counters and times are left unchanged), stores the fastest for
 * ensemble calls with block = 0 and returns it in *block (may be NULL). */
ppmlr_status ppmlr_ensemble_autotune(ppmlr_ctx *const *ctxs, const ppmlr_state *const *states, int n, int reps,
                                     double cfl, int *block);

#ifdef __cplusplus
}
#endif
#endif
