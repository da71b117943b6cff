/*
 * swe.h -- C ABI of the MI355X (gfx950) implementation of the eta-based,
 * well-balanced central-upwind finite-volume scheme for the rotational
 * shallow-water equations of Brodtkorb & Holm, "Real-World Oceanographic
 * Simulations on the GPU using a Two-Dimensional Finite-Volume Scheme"
 * (arXiv 1912.02457).
 *
 * Conventions used by every entry point:
 *   - Cell fields are row-major [ny][nx] float32, x fastest; corner depths
 *     are [ny+1][nx+1] float32 (equilibrium depth H, metres, positive
 *     downwards, at the cell intersections: the piecewise bilinear bathymetry
 *     of the section "Mathematical formulation", Figure 1b).
 *   - The land mask is an optional uint8 [ny][nx] array (nonzero = land).
 *   - Units are SI.  Times are float64 seconds.
 *   - Host arrays passed in are read during the call and copied; the library
 *     never keeps a host pointer.  Device memory comes from ONE caller-owned
 *     workspace (size from swe_workspace_bytes) that stays borrowed for the
 *     lifetime of the domain handle; the library allocates no device memory
 *     of its own for a domain.
 *   - All GPU work of a domain is issued on the HIP stream given at init
 *     (NULL = the null stream).  Calls marked "asynchronous" only enqueue.
 *   - Every function returns SWE_OK (0) or a negative error code; the message
 *     of the last error on the calling thread is in swe_last_error().  No C++
 *     exception crosses this interface.
 */
#ifndef SWE_H
#define SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define SWE_OK 0
#define SWE_E_ARG (-1)      /* invalid size, parameter, pointer or non-finite input */
#define SWE_E_NOMEM (-2)    /* caller workspace too small */
#define SWE_E_HIP (-3)      /* HIP runtime error; message in swe_last_error() */
#define SWE_E_UNSTABLE (-4) /* a non-finite state, or a water depth eta + Hbar below -kappa in a
                               non-land cell, was seen by the CFL reduction (a flag raised on the
                               device after a step, swe_set_state or init; cleared by swe_set_state) */
#define SWE_E_STATE (-5)    /* call out of order (e.g. nested sides without boundary data) */

/* boundary kinds, per side in the order West, East, South, North */
#define SWE_BC_WALL 0     /* reflective wall, section "Global wall boundary conditions" */
#define SWE_BC_PERIODIC 1 /* periodic; must be set on both sides of an axis */
#define SWE_BC_NESTED 2   /* external state + flow relaxation, section "Nesting the model" */

/* bed shear stress laws, section "Wind forcing and bed friction source terms";
 * the source is -S(Q) (hu, hv) with h* the desingularised depth of eq. desing_ours */
#define SWE_FRICTION_NONE 0
#define SWE_FRICTION_LINEAR 1    /* S = r / h*           (r in m/s)            */
#define SWE_FRICTION_QUADRATIC 2 /* S = r |u| / h*^2     (eq. swe as printed)  */
#define SWE_FRICTION_MANNING 3   /* S = g n^2 |u| / h*^(4/3)                   */

/* forcing kinds for swe_set_forcing */
#define SWE_FORCING_WIND_STRESS 0 /* uniform wind stress (N/m^2), snapshots in time */
#define SWE_FORCING_BOUNDARY 1    /* external (eta, hu, hv) along the perimeter      */

typedef struct swe_params {
    int32_t nx, ny;          /* cells, each >= 2 */
    double dx, dy;           /* cell size (m) */
    double g;                /* gravity (m/s^2), e.g. 9.81 */
    double courant;          /* C in dt = C * 1/4 * min(dx/(|u|+c), dy/(|v|+c)), eq. cfl; 0 < C <= 1 */
    double theta;            /* generalized-minmod parameter in [1, 2] */
    double kappa;            /* desingularisation / dry tolerance (m), eq. desing_ours; > 0 */
    int32_t bc[4];           /* SWE_BC_* for W, E, S, N */
    int32_t friction;        /* SWE_FRICTION_* */
    double friction_coeff;   /* r (m/s), r (-), or Manning n (s m^-1/3) */
    double rho_w;            /* sea-water density (kg/m^3) dividing the wind stress, e.g. 1025 */
    int32_t frs_width;       /* relaxation zone width W in cells (1..32), eq. frs */
    double frs_d0;           /* relaxation length d0 in cells, eq. frs; > 0 */
    int32_t north_projection;/* 0: Coriolis as f (hv, -hu); 1: evaluate the north-vector
                                projection of the section "Coriolis force" literally
                                (reads the north angle every stage) */
    int32_t compensated_state;/* 0: the state is stored in float32, as in the paper;
                                1: each stored value of Q^n and Q* also keeps its
                                rounding error (a second plane per field holding
                                the error's upper 16 bits, a bfloat16), updated
                                by an error-free sum, so that storing the state
                                rounds away about 2^-10 of a float32 ulp per
                                step instead of up to half of one; the arithmetic
                                of a stage stays float32.  Six more half-size
                                planes of workspace. */
} swe_params;

typedef struct swe_domain swe_domain;

/* Bytes of device workspace that swe_init_domain needs for these parameters
 * (state double buffer, bathymetry, Coriolis field -- every plane with a
 * frame of two ghost cells on each side --, forcing tables, control block).  max_bnd_times / max_wind_times bound the forcing snapshots that
 * swe_set_forcing may later hold.  Returns SWE_E_ARG for invalid parameters. */
int swe_workspace_bytes(const swe_params *p, int32_t max_wind_times, int32_t max_bnd_times,
                        size_t *bytes);

/* Create a domain: validate p, upload the problem statement of the sections
 * "Mathematical formulation" and "Efficient simulation of real-world ocean
 * currents" -- corner depths Hc [ny+1][nx+1], optional land mask [ny][nx],
 * Coriolis parameter f [ny][nx] (section "Coriolis force"), north angle theta
 * [ny][nx] (radians between the grid y-axis and north, may be NULL = 0) and
 * the initial state eta, hu, hv [ny][nx] -- into the caller's device
 * workspace (device pointer, 256-byte aligned, `bytes` long, borrowed until
 * swe_destroy), and compute the first CFL time step on the device.  Host
 * arrays are copied.  Launches go on `hip_stream` (a hipStream_t, may be
 * NULL); the call synchronises that stream before returning.
 * Errors: SWE_E_ARG (sizes < 2, non-finite inputs, bad parameters, periodic
 * on one side only, periodic seam depths that differ), SWE_E_NOMEM, SWE_E_HIP. */
int swe_init_domain(const swe_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
                    int32_t max_wind_times, int32_t max_bnd_times, const float *Hc,
                    const uint8_t *land, const float *f, const float *theta, const float *eta,
                    const float *hu, const float *hv, swe_domain **out);

/* Forcing snapshots, linearly interpolated in time in float64 on the device
 * (eq. windstress_interpol; nesting data as in the section "Nesting the
 * model"), clamped outside [times[0], times[n-1]].
 *   SWE_FORCING_WIND_STRESS: data = n_times x 2 (tau_x, tau_y) in N/m^2; the
 *     momentum source is tau / rho_w (uniform in space).
 *   SWE_FORCING_BOUNDARY: data = n_times x 3 x (2 ny + 2 nx) for (eta, hu, hv)
 *     along the West strip (by row), East strip, South strip (by column) and
 *     North strip.  Ghost cells of nested sides take these values and the
 *     relaxation zone is nudged toward them.
 * times must increase strictly.  Host arrays, copied; synchronises the stream.
 * Errors: SWE_E_ARG (n_times < 1 or above the workspace bound, non-finite
 * data, unknown kind), SWE_E_HIP. */
int swe_set_forcing(swe_domain *d, int32_t kind, int32_t n_times, const double *times,
                    const float *data);

/* Boundary snapshots given at their own spacing (section "Nesting the
 * model": boundary data interpolated linearly in time and space like the
 * wind, so that it need not match the grid, e.g. after a refinement):
 * data = n_times x 3 x (2 n_y + 2 n_x) for (eta, hu, hv) along the West side
 * (n_y samples, south to north), East side, South side (n_x samples, west to
 * east) and North side.  A side's samples sit at the centres of n equal
 * parts of it; each boundary cell takes the linear interpolation at its
 * centre (held at the end samples), once per snapshot, and the result is
 * used as by swe_set_forcing(SWE_FORCING_BOUNDARY) (interpolation in space
 * and in time are both linear, so the order does not matter).  n_x = nx and
 * n_y = ny give the data unchanged.  Host arrays, copied; synchronises.
 * Errors: SWE_E_ARG (counts, times, non-finite data, more snapshots than
 * the workspace holds), SWE_E_STATE inside an ensemble, SWE_E_HIP. */
int swe_set_boundary_field(swe_domain *d, int32_t n_times, int32_t n_x, int32_t n_y, const double *times,
                           const float *data);

/* Wind at 10 m on its own grid (section "Wind"): n_times snapshots at
 * increasing times of ny_w x nx_w samples of (u, v) in m/s, laid out
 * [n_times][ny_w][nx_w][2].  The samples sit at the centres of an nx_w x ny_w
 * partition of the domain; each stage interpolates them bilinearly in space
 * (held at the edge samples outside their hull) and linearly in time (eq.
 * windstress_interpol; clamped outside the snapshot times), then adds the
 * stress of Large and Pond, (rho_air / rho_w) C_D |W| W with C_D = 1.2e-3
 * below 11 m/s and (0.49 + 0.065 |W|) 1e-3 above, to the momentum equations
 * (on top of any stress from swe_set_forcing).  The data is copied into
 * dev_buffer: caller-owned device memory of swe_wind_field_bytes bytes,
 * 256-byte aligned, borrowed until the field is replaced or removed
 * (n_times = 0) or the domain destroyed.  Synchronises.  Errors: SWE_E_ARG,
 * SWE_E_NOMEM (buffer too small), SWE_E_STATE inside an ensemble. */
int swe_wind_field_bytes(int32_t n_times, int32_t nx_w, int32_t ny_w, size_t *bytes);
int swe_set_wind_field(swe_domain *d, int32_t n_times, int32_t nx_w, int32_t ny_w, const double *times,
                       const float *w10, double rho_air, void *dev_buffer, size_t bytes);

/* The same grid, interpolation and buffer rules for a field of wind STRESS:
 * tau (N/m^2) at the samples, [n_times][ny_w][nx_w][2], interpolated
 * bilinearly in space and linearly in time as it is and divided by rho_w.
 * The section calls the interpolated quantity both the wind and the wind
 * stress; swe_set_wind_field interpolates the wind and takes the stress per
 * cell, this call takes the stress at the samples.  One gridded field at a
 * time: this replaces a wind field and the other way round; n_times = 0
 * removes it.  Errors as swe_set_wind_field. */
int swe_set_stress_field(swe_domain *d, int32_t n_times, int32_t nx_w, int32_t ny_w, const double *times,
                         const float *tau, void *dev_buffer, size_t bytes);

/* Advance n_steps SSP-RK2 steps (eq. rk2_semiimp with the spatial operator of
 * eq. sw_semidiscrete), each with the dt of eq. cfl computed on the device
 * from the state at the start of the step.  Asynchronous: no host
 * synchronisation.  Steps run as replays of captured HIP graphs of the two
 * stage kernels: chunks of 16 steps, then the remaining n_steps mod 16 as
 * one graph of that length; each graph is captured (and instantiated) on
 * its first use at a given step parity and kept until the domain is
 * destroyed or its tiling or forcing changes, so a caller that times
 * repeated calls should make one untimed call of the same length at the
 * same parity first.  Errors: SWE_E_ARG (n_steps < 0), SWE_E_STATE
 * (nested side without boundary data), SWE_E_HIP. */
int swe_step(swe_domain *d, int32_t n_steps);

/* Like swe_step but with the time step of step k given by dts[k] (host
 * array of n_steps float64 values > 0): replays a known dt sequence.
 * Asynchronous. */
int swe_step_dt(swe_domain *d, int32_t n_steps, const double *dts);

/* Advance until t == t_end: the last step is shortened on the device so that
 * t lands on t_end exactly.  Synchronises; *steps_taken (may be NULL) gets
 * the number of steps.  Returns SWE_E_UNSTABLE if the state became
 * non-finite. */
int swe_run_until(swe_domain *d, double t_end, int64_t *steps_taken);

/* Time-step update policy.  interval = 0 (the default): dt from eq. cfl at
 * the start of every step.  interval > 0: the policy of the paper's
 * real-world runs (section "Real-world simulations": dt updated every 20
 * simulated minutes, Courant number 0.8) -- a step takes the dt
 * of the last update until the time of the next update is reached; the step
 * that starts at or after it takes the CFL dt of its state, and the next
 * update moves one interval on (to one interval past that step's start if
 * that is not later).  The first step after this call (or after
 * swe_set_state) updates.  swe_run_until still clamps the last step to its
 * end time; swe_step_dt ignores the policy.  The CFL maximum is still
 * reduced every step (the state's wave speed stays observable).
 * Errors: SWE_E_ARG (negative or non-finite interval), SWE_E_STATE (member
 * of an ensemble), SWE_E_HIP.  Synchronises the stream. */
int swe_set_dt_policy(swe_domain *d, double interval);

/* Copy the state into caller buffers (each [ny][nx] float32; host or device
 * pointers, any may be NULL) and report time t and the dt of the next step.
 * Synchronises.  Returns SWE_E_UNSTABLE if the device flag is set. */
int swe_read_state(swe_domain *d, float *eta, float *hu, float *hv, double *t, double *dt_next);

/* Replace the state (host arrays [ny][nx]) and the time; recomputes the
 * next dt.  For checkpoint/resume.  Synchronises. */
int swe_set_state(swe_domain *d, const float *eta, const float *hu, const float *hv, double t);

/* Float64 reductions over non-land cells: mass = sum (eta + Hbar) dx dy and
 * energy = sum (|hu|^2 / (2 h*) + g eta^2 / 2) dx dy, Hbar the mean of the
 * four corner depths.  Deterministic order.  Synchronises. */
int swe_diagnostics(swe_domain *d, double *mass, double *energy);

/* SWE_OK, or SWE_E_UNSTABLE once a step (or the state given at init or to
 * swe_set_state) had a non-finite value or a water depth below -kappa in a
 * non-land cell; swe_last_error() says which.  Synchronises. */
int swe_status(swe_domain *d);

/* Measures both stage kernels of this domain for rows per tile in {2..64}
 * and, around the fastest, for tails of 1-4-row bands (swe_set_stage_tiling),
 * then the winner under the other tile orders (a few launches each), times
 * the three fastest candidates again, and keeps the fastest tiling per
 * stage.  Before anything is timed, stage-1 launches run for about 25 ms of
 * device time so that the clocks have come up.  The state and the
 * control block are saved to host memory first and restored afterwards, so
 * the simulation does not advance.  *rows_per_wave gets stage 1's choice
 * (may be NULL; swe_get_tiling reports each stage).  Synchronises.  Errors:
 * SWE_E_STATE inside an ensemble or without boundary data for nested sides,
 * SWE_E_HIP. */
int swe_autotune_tiling(swe_domain *d, int32_t *rows_per_wave);

/* Work decomposition of the stage kernels: each wavefront updates a strip of
 * 60 columns over rows_per_wave rows (0 = the built-in choice per stage
 * kernel, which fills the wave slots its register use allows in whole
 * rounds); order picks the tile numbering
 * (bit 0: row-block-major instead of strip-major, bit 1: no grouping of
 * neighbouring tiles per XCD; -1 = default).  Used by the autotuner; results
 * do not depend on it (bitwise).  swe_get_tiling reports the values and the
 * wavefronts per launch of stage kernel `stage` (1 or 2). */
int swe_set_tiling(swe_domain *d, int32_t rows_per_wave, int32_t order);
int swe_get_tiling(swe_domain *d, int32_t stage, int32_t *rows_per_wave, int32_t *order, int32_t *waves);

/* Tiling of one stage kernel (1 or 2) with two band heights: bands of
 * rows_per_wave rows (>= 1) from the top, and when 0 < tail_rows_per_wave <
 * rows_per_wave, the last rows -- at least tail_rows of them, 0 < tail_rows <
 * ny, with at least one band of rows_per_wave rows before them -- in bands of
 * tail_rows_per_wave rows whose waves are launched after all the others, so
 * that a launch ends on short waves.  Other tail values give one band height.
 * order as in swe_set_tiling (-1 keeps the current one).  Results do not
 * depend on it (bitwise).  swe_get_stage_tiling reports the values (tail
 * rows per wave and the number of tail rows 0 for one band height) and the
 * wavefronts per launch; any output pointer may be NULL.  Errors: SWE_E_ARG,
 * SWE_E_STATE inside an ensemble. */
int swe_set_stage_tiling(swe_domain *d, int32_t stage, int32_t rows_per_wave, int32_t tail_rows_per_wave,
                         int32_t tail_rows, int32_t order);

/* Every tiling swe_autotune_tiling may time for stage kernel `stage` on this
 * domain (the one-height tilings, then the tails tried around each height;
 * the tuner also times the winner under the four tile orders, which are not
 * listed), as triples (rows_per_wave, tail_rows_per_wave, tail_rows) in the form of
 * swe_get_stage_tiling, into out[3 * max_tilings] (caller-owned host array;
 * NULL when max_tilings is 0).  *n_tilings gets the total count, which may
 * exceed max_tilings (then only the first max_tilings are written).  Lets a
 * profiler run cover every tiling the tuner can settle on.  Errors: SWE_E_ARG. */
int swe_list_tilings(swe_domain *d, int32_t stage, int32_t *out, int32_t max_tilings, int32_t *n_tilings);
int swe_get_stage_tiling(swe_domain *d, int32_t stage, int32_t *rows_per_wave, int32_t *tail_rows_per_wave,
                         int32_t *tail_rows, int32_t *order, int32_t *waves);

/* Average device time per launch of each stage kernel (milliseconds) over
 * the launches issued since the last call with reset != 0, measured with HIP
 * events recorded around every stage launch on the domain's stream while
 * timing is enabled (swe_enable_timing).  Synchronises. */
int swe_enable_timing(swe_domain *d, int32_t on);
int swe_stage_times(swe_domain *d, double *ms_stage1, double *ms_stage2, int64_t *launches,
                    int32_t reset);

void swe_destroy(swe_domain *d);
const char *swe_last_error(void);

/* ---- batched ensemble ---------------------------------------------------
 * Many domains of uneven sizes advanced together: each RK stage of all
 * members is ONE persistent kernel launch that drains a device queue of
 * (member, tile) work items (largest members first, split into 8
 * partitions taken in chunks with one atomic each).  Every member keeps its
 * own parameters, forcing, time and CFL time step (eq. cfl per member), so
 * a member's result is bitwise the one it gets stepped alone.  Steps are
 * replayed as captured HIP graphs.  Used for ensembles of perturbed runs and
 * by the serving loop.  Members are borrowed; while they belong to the
 * ensemble their own stepping calls return SWE_E_STATE and all their work
 * (including swe_read_state) is ordered on the ensemble's stream. */
typedef struct swe_ensemble swe_ensemble;

/* Device workspace for an ensemble of these members with rows_per_wave rows
 * per tile (0 = default) -- the member table, the work queue and its
 * counters.  Errors: SWE_E_ARG. */
int swe_ensemble_workspace_bytes(swe_domain *const *members, int32_t n, int32_t rows_per_wave, size_t *bytes);

/* Group n >= 1 ready domains (boundary data set where nested; all with the
 * same north_projection) into an ensemble using the caller's device workspace
 * (256-byte aligned, borrowed until swe_ensemble_destroy) and stream.
 * chunk = work items taken per atomic (0 = default 1).  Synchronises. */
int swe_ensemble_create(swe_domain *const *members, int32_t n, void *dev_workspace, size_t bytes,
                        void *hip_stream, int32_t rows_per_wave, int32_t chunk, swe_ensemble **out);

/* Advance every member n_steps SSP-RK2 steps, each with its own dt.
 * Asynchronous. */
int swe_ensemble_step(swe_ensemble *e, int32_t n_steps);

/* Reports the work decomposition (rows per tile, chunk, work items per
 * stage, blocks of the persistent launch). */
int swe_ensemble_info(swe_ensemble *e, int32_t *rows_per_wave, int32_t *chunk, int64_t *items, int32_t *blocks);

/* HIP-event timing of the two ensemble stage kernels, as swe_stage_times. */
int swe_ensemble_enable_timing(swe_ensemble *e, int32_t on);
int swe_ensemble_stage_times(swe_ensemble *e, double *ms_stage1, double *ms_stage2, int64_t *launches,
                             int32_t reset);

/* on = 1 (default): swe_ensemble_step replays captured HIP graphs of 16
 * steps and one of the remaining n_steps mod 16 steps (each captured on its
 * first use at a given step parity, as in swe_step); on = 0: every stage is
 * launched directly (no capture cost, for ensembles that live only a few
 * steps, as in the serving loop). */
int swe_ensemble_use_graphs(swe_ensemble *e, int32_t on);

/* Releases the ensemble; the members return to their own streams. */
void swe_ensemble_destroy(swe_ensemble *e);

/* ---- serving loop (continuous batching) ----------------------------------
 * Forecast requests (a domain, its initial state and forcing, and a
 * simulated-time horizon) arrive at any time; the server keeps the active
 * ones resident in a caller-provided device arena and advances them together
 * as one batched ensemble in ticks of a fixed number of SSP-RK2 steps.  At
 * every tick boundary finished requests leave (their final state is copied
 * to the caller's host buffers and their arena block is freed) and waiting
 * requests join in arrival order while their HBM footprint (the
 * swe_workspace_bytes of their domain) fits in the arena and an active slot
 * is free.  Each request's last step is clamped so that it ends exactly at
 * its horizon (the run-to-time rule of the scheme); a request's result is
 * bitwise the one it gets when run alone.  The active set is of one kind
 * (params.north_projection and params.compensated_state): a waiting request
 * of another kind stays at the head of the queue, and the ones behind it
 * wait too, until the active set has drained.  swe_server_submit may be called
 * from another thread while a tick runs; no other calls on one server may
 * overlap. */
typedef struct swe_server swe_server;

typedef struct swe_request {
    int64_t id;           /* caller's tag, reported on completion */
    swe_params params;    /* as for swe_init_domain */
    double horizon;       /* simulated seconds to advance, >= 0 */
    const float *Hc;      /* host inputs as for swe_init_domain; copied by swe_server_submit */
    const uint8_t *land;  /* may be NULL */
    const float *f;
    const float *theta;   /* may be NULL */
    const float *eta, *hu, *hv;
    int32_t n_wind;       /* 0 = no wind, else n_wind times and (n_wind x 2) stresses, N/m^2 */
    int32_t n_bnd;        /* boundary snapshots for nested sides (as swe_set_forcing), 0 if none */
    const double *wind_t;
    const float *wind_tau;
    const double *bnd_t;
    const float *bnd;
    float *out_eta, *out_hu, *out_hv; /* host [ny][nx]; caller-owned, must stay valid until the
                                         request is reported by swe_server_poll; may be NULL */
} swe_request;

typedef struct swe_completion {
    int64_t id;
    double t;        /* simulated time reached (= horizon unless status != SWE_OK) */
    int64_t steps;   /* time steps taken */
    int64_t tick;    /* tick after which it completed */
    int32_t status;  /* SWE_OK; SWE_E_UNSTABLE (non-finite state, stopped early); SWE_E_NOMEM
                        (its workspace and work queue do not fit even in the empty arena);
                        SWE_E_ARG (its inputs were refused when it was started) */
    int32_t pad;
} swe_completion;

typedef struct swe_server_stats {
    int64_t submitted, admitted, completed, ticks;
    int64_t cell_steps;             /* sum over requests of cells x steps taken so far */
    size_t arena_bytes, arena_used, arena_peak;
    int32_t active, pending;
    /* host wall time spent in the parts of swe_server_tick, seconds:
     * rebuilding the work queue, launching the steps, admitting (uploads),
     * waiting for the device, retiring (result copies, frees) */
    double host_rebuild_s, host_launch_s, host_admit_s, host_wait_s, host_retire_s;
} swe_server_stats;

/* dev_arena: caller-owned device memory (256-byte aligned) from which every
 * admitted request's workspace and the ensemble's queue are carved.  Work
 * runs on hip_stream; uploads of joining requests on upload_stream (may be
 * the same), overlapping the running tick.  max_active >= 1;
 * steps_per_tick >= 1; rows_per_wave / chunk as for the ensemble (0 =
 * default).  Errors: SWE_E_ARG. */
int swe_server_create(void *dev_arena, size_t arena_bytes, void *hip_stream, void *upload_stream, int32_t max_active,
                      int32_t steps_per_tick, int32_t rows_per_wave, int32_t chunk, swe_server **out);

/* Queue a request (inputs are validated and copied).  SWE_E_ARG for invalid
 * inputs, SWE_E_NOMEM if its footprint exceeds the whole arena. */
int swe_server_submit(swe_server *s, const swe_request *r);

/* One tick: launch steps_per_tick steps of the active set, admit waiting
 * requests (uploading them while the steps run), then retire the finished
 * ones.  Synchronises.  Reports the active and waiting counts after the tick. */
int swe_server_tick(swe_server *s, int32_t *n_active, int32_t *n_pending);

/* Pops up to max completions (oldest first) into out; *n = number written. */
int swe_server_poll(swe_server *s, swe_completion *out, int32_t max, int32_t *n);

/* Counters of the server (requests, ticks, cell-steps, arena use). */
int swe_server_get_stats(swe_server *s, swe_server_stats *st);

/* Drops every active and waiting request and frees the server. */
void swe_server_destroy(swe_server *s);

/* ---- preprocessing of the input fields ----------------------------------
 * Init-time steps that turn model data into the inputs of swe_init_domain,
 * run on the device.  Every array pointer is a DEVICE pointer to a dense
 * row-major array (row pitch = width, x fastest); outputs must not overlap
 * inputs; planes of refined outputs must be 8-byte aligned.  The calls only
 * enqueue kernels on hip_stream (a hipStream_t, may be NULL) and return;
 * launch failures give SWE_E_HIP.  Non-finite input values propagate to the
 * output; they are not detected.  No device memory is allocated. */

/* Corner depths from cell-centre depths (section "Bathymetry"): the initial
 * guess of eqs. recon_1-3 -- a minmod-limited plane per cell (a difference
 * toward land or outside the domain counts as 0), evaluated at the cell's
 * corners and averaged over the water cells meeting at each corner -- then
 * `iters` rounds of: misfit Hm - (mean of the cell's four corners) on water
 * cells, its corner estimate by the same equations ADDED to the corners,
 * and smoothing H <- (1 - smooth) H + (smooth/4) (sum of the 4 neighbours),
 * a neighbour outside the domain replaced by the corner itself (smooth =
 * 0.5 gives H/2 + sum/8).  Corners touching no water cell hold the mean of
 * the four cell values around them (edge cells repeated).
 *   Hm [ny][nx] metres, positive down; land [ny][nx] (nonzero = land) or NULL;
 *   Hc [ny+1][nx+1] output; scratch [ny+1][nx+1] floats, required when
 *   iters > 0 (contents overwritten).  nx, ny >= 1; iters in [0, 100000];
 *   smooth in [0, 1].
 * Errors: SWE_E_ARG (sizes, NULL pointers, a corner plane of 4 GiB or more,
 * parameters out of range), SWE_E_HIP. */
int swe_reconstruct_bathymetry(int32_t nx, int32_t ny, const float *Hm, const uint8_t *land, int32_t iters,
                               float smooth, float *Hc, float *scratch, void *hip_stream);

/* swe_reconstruct_bathymetry for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and the same result (bitwise), but the
 * corner plane the rounds alternate with Hc is a device array of the
 * library's own -- 16 MiB per GPU, reserved on every GPU the library is
 * loaded on and held until the process ends -- so no scratch argument.
 * The caller still passes Hm, land, Hc and the stream as above.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine);
 * on its first use on a device it looks up that device's copy of the array.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (on different streams or threads) race and give undefined corners; run
 * them on one stream or one after the other.
 * Limit: (nx + 1) * (ny + 1) <= 4194304 corners.
 * Errors: SWE_E_ARG (the limit, and as swe_reconstruct_bathymetry), SWE_E_HIP. */
int swe_reconstruct_bathymetry_noalloc(int32_t nx, int32_t ny, const float *Hm, const uint8_t *land,
                                       int32_t iters, float smooth, float *Hc, void *hip_stream);

/* One erosion of the land mask (section "Bathymetry", Figure erode_land):
 * a land cell with a water 4-neighbour (cells outside the domain count as
 * land) becomes water of depth land_depth, its eta the largest eta among
 * those water neighbours (gray dilation), its momenta 0; every other cell is
 * copied.  land_out holds 0/1.  eta, hu, hv may each be NULL (with their
 * outputs NULL).  Repeat the call to erode further.
 * Errors: SWE_E_ARG (sizes, missing land/Hm/outputs, mismatched optional
 * pairs, non-finite land_depth), SWE_E_HIP. */
int swe_erode_land(int32_t nx, int32_t ny, const uint8_t *land, const float *Hm, const float *eta,
                   const float *hu, const float *hv, float land_depth, uint8_t *land_out, float *Hm_out,
                   float *eta_out, float *hu_out, float *hv_out, void *hip_stream);

/* Factor-two refinement (section "Refinement and coarsening of grid"):
 *   fields: n_fields planes [n_fields][ny][nx] -> fields_out
 *     [n_fields][2ny][2nx]; each cell's linear reconstruction with slopes
 *     minmod(theta D-, (D- + D+)/2, theta D+) (a difference toward land or
 *     outside the domain is 0; land cells stay constant) evaluated at the
 *     four sub-cell centres, which preserves the cell average;
 *   land -> land_out [2ny][2nx] (children inherit; needs n_fields >= 1;
 *     land may be NULL = all water, land_out may be NULL);
 *   Hc [ny+1][nx+1] -> Hc_out [2ny+1][2nx+1]: the bilinear surface at the
 *     refined intersections (both NULL to skip).
 * theta in [1, 2] (1 = plain minmod).
 * Errors: SWE_E_ARG (sizes, pointers, theta, a refined corner plane of
 * 4 GiB or more), SWE_E_HIP. */
int swe_refine2(int32_t nx, int32_t ny, int32_t n_fields, const float *fields, const uint8_t *land, float theta,
                float *fields_out, uint8_t *land_out, const float *Hc, float *Hc_out, void *hip_stream);

/* Factor-two coarsening (same section) of a grid with even nx, ny >= 2:
 * a coarse cell is the average of its water children (of all four when all
 * are land) and is land when all four children are; corner depths are
 * sampled at the coarse intersections.  Shapes: fields [n_fields][ny][nx]
 * -> [n_fields][ny/2][nx/2]; land -> [ny/2][nx/2] (land_out needs land and
 * n_fields >= 1); Hc [ny+1][nx+1] -> [ny/2+1][nx/2+1].
 * Errors: SWE_E_ARG (odd or small sizes, pointers), SWE_E_HIP. */
int swe_coarsen2(int32_t nx, int32_t ny, int32_t n_fields, const float *fields, const uint8_t *land,
                 float *fields_out, uint8_t *land_out, const float *Hc, float *Hc_out, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
