/*
 * rtgd.h -- C ABI of librtgd: batched HF ray tracing through a gridded
 * ionosphere on one AMD Instinct MI355X (gfx950).
 *
 * The library implements the hot path of RTM-GD ("Efficient and
 * High-Accuracy Ray Tracing in Discretized Ionospheric Models"):
 * many independent rays integrated with fixed-step RK4 (Sec. II-C) along the
 * Haselgrove equations in spherical coordinates (Sec. II-A, eq. 1a-1f, with
 * the frame term of the k_r equation taken as k_phi sin(theta) dphi/dP'),
 * through an electron density reconstructed by the C1 Galerkin-Difference
 * interpolant, p = 3 (Sec. II-B-2, eq. 3dinterp_gd, Appendix A), with the
 * Appleton-Hartree refractive index (eq. appleton, collisionless, + = O,
 * - = X) under a centred axial dipole field.
 *
 * Conventions shared by every call:
 *   - lengths in km, angles in degrees, frequencies in MHz;
 *   - spherical Earth of radius earth_radius_km; transmitter height must lie
 *     below the grid bottom h0_km: rays run as straight lines through the
 *     density-free region below h0_km (launch and ground return are closed
 *     form), N_e = 0 below h0_km;
 *   - outside the grid box laterally or above its top the density is
 *     continued as a constant (its derivative along the clamped axis is 0);
 *   - the wave-normal vector n = c k / omega is carried in local
 *     (r, theta = colatitude, phi = east longitude) components.
 *
 * Errors: every call returns an rt_status; no C++ exception crosses the ABI.
 * rt_last_error(ctx) returns a message for the last failed call on a context;
 * rt_last_error(NULL) the message of the last failed rt_ctx_create on the
 * calling thread.
 * A context is used by one host thread at a time.
 */
#ifndef RTGD_H
#define RTGD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rt_status;
enum {
    RT_OK = 0,
    RT_W_TRAJ_TRUNCATED = 1, /* success; some trajectories did not fit     */
    RT_E_INVALID = -1,       /* bad argument (message in rt_last_error)    */
    RT_E_NOMEM = -2,         /* device allocation failed                   */
    RT_E_DEVICE = -3,        /* HIP runtime error                          */
    RT_E_UNSUPPORTED = -4    /* valid request outside what is implemented  */
};

/* element type / quantity of the grid values handed to rt_grid_create */
enum { RT_F64 = 0, RT_F32 = 1 };
enum { RT_NE_M3 = 0, RT_FN2_MHZ2 = 1 };   /* N_e in m^-3, or f_N^2 in MHz^2 */
/* interpolation of the grid */
enum { RT_INTERP_GD = 0, RT_INTERP_CR = 1 };
/* wave modes (bit mask in rt_fan.modes) */
enum { RT_MODE_O = 1, RT_MODE_X = 2 };
/* arithmetic of the trace */
enum { RT_FP64 = 0, RT_MIXED = 1 };
/* where caller buffers live */
enum { RT_MEM_HOST = 0, RT_MEM_DEVICE = 1 };
/* per-ray termination status */
enum { RT_RAY_GROUND = 0, RT_RAY_ESCAPE = 1, RT_RAY_MAX_PATH = 2, RT_RAY_NUMERIC = 3 };

typedef struct rt_ctx rt_ctx;
typedef struct rt_grid rt_grid;

/* Uniform (lat, lon, height) grid.  Node (i, j, k) sits at
 * lat0 + i dlat, lon0 + j dlon, h0 + k dh; values are C order
 * [n_lat][n_lon][n_h] (height fastest).  Every n >= 4, every spacing > 0,
 * the latitude range inside (-90, 90). */
typedef struct {
    int32_t n_lat, n_lon, n_h;
    int32_t dtype;      /* RT_F64 or RT_F32                               */
    int32_t quantity;   /* RT_NE_M3 or RT_FN2_MHZ2                        */
    int32_t interp;     /* RT_INTERP_GD (the method) or RT_INTERP_CR      */
    double lat0_deg, dlat_deg;
    double lon0_deg, dlon_deg;
    double h0_km, dh_km;
    double earth_radius_km;
} rt_grid_geom;

/* Centred dipole.  B0 = field at the equator on the Earth's surface
 * (|B| = B0 (R/r)^3 sqrt(1 + 3 cos^2 theta)).  Only the axial dipole
 * (pole_lat_deg = 90) is implemented. */
typedef struct {
    double B0_tesla;
    double pole_lat_deg, pole_lon_deg;
} rt_dipole;

/* A launch fan: every combination of frequency, mode, elevation and
 * azimuth.  Ray index = ((i_freq * n_mode + i_mode) * n_elev + i_elev)
 * * n_az + i_az, modes ordered O then X; n_mode = number of bits set in
 * modes.  Elevation in [0, 90] above the horizon, azimuth clockwise from
 * north.  The arrays are host memory, read during the call only. */
typedef struct {
    double tx_lat_deg, tx_lon_deg, tx_h_km;
    const double *elev_deg;
    int32_t n_elev;
    int32_t n_az;
    const double *az_deg;
    const double *freq_mhz;
    int32_t n_freq;
    uint32_t modes;     /* RT_MODE_O | RT_MODE_X; both modes give the same
                           isotropic ray when no field is set              */
} rt_fan;

typedef struct {
    double step_km;         /* fixed RK4 step in group path, > 0           */
    double max_group_km;    /* MAX_PATH limit, > 0                         */
    double exit_h_km;       /* ESCAPE height; <= 0 means the grid top      */
    int32_t precision;      /* RT_FP64, or RT_MIXED (FP32 interpolation and
                               refractive index, FP64 integration)         */
    int32_t traj_stride;    /* record every traj_stride-th step; 0 = none  */
    int64_t traj_capacity;  /* records available in rt_results.traj        */
    int32_t results_mem;    /* RT_MEM_HOST or RT_MEM_DEVICE                */
    int32_t tail_threshold; /* scheduling knob, results unchanged.  Rays
                               start one lane each; once the queue is empty:
                               > 0: once at most this many rays are live in
                               the launch, all are handed to a separate
                               16-lanes-per-ray tail kernel;
                               0: the same at 16 rays per CU (default);
                               -1: one lane per ray throughout;
                               -2: a wave left with <= 4 live rays
                               finishes them 16 lanes per ray itself      */
    int32_t waves_per_simd; /* scheduling knob, results unchanged: register
                               budget of the kernels, 1 = whole register
                               file, 2 = two waves per SIMD; 0 = default  */
    int32_t ray_order;      /* scheduling knob, results unchanged: order in
                               which waves take rays from the queue; 0 =
                               default (3), 1 = index order,
                               2 = strided: q -> q * s mod n_rays with s
                               coprime to n_rays near 0.618 n_rays, which
                               spreads neighbouring (similar) rays over
                               many waves; 3 = sorted by wave mode (a
                               counting sort, stable in ray index: O and
                               isotropic rays, then X rays), so that a wave
                               holds rays of one mode                     */
    int32_t promote_waves;  /* scheduling knob, results unchanged: this many
                               waves run rays 16 lanes each beside the
                               one-lane waves, taking over rays trapped in a
                               duct (wave normal turning upward inside the
                               ionosphere: they run to max_group_km), rays
                               that grazed a layer peak on their first ascent
                               (n_r falling to a positive local minimum below
                               0.02 |n|: such rays are often trapped later)
                               and rays older than promote_age steps;
                               0 = default (32 for launches of at least
                               8192 rays, else none), -1 = none, at most 64;
                               ignored with tail_threshold = -2.  With
                               promotion on, an rt_trace launch holds at
                               most one wave per SIMD (so that no promotion
                               wave shares one).  An idle
                               promotion wave waits for work at most a
                               wall-clock bound far above the launch's
                               one-lane phase (at least 10 s; the variable
                               RTGD_PROMOTE_IDLE_MS overrides it, for
                               tests); a wait that runs out fails the call
                               with RT_E_DEVICE                            */
    int32_t promote_age;    /* steps after which any ray may be promoted;
                               0 = default and -1: never (trapped and
                               grazing rays only)                          */
    int32_t cu_layout;      /* scheduling knob, results unchanged: how the
                               one-lane kernel's waves are grouped when
                               promotion waves run.  1: one wave per
                               work-group; 2: four waves per work-group and
                               one work-group per CU (an LDS reservation
                               keeps others off the CU), so the promotion
                               waves, the launch's last work-groups, have
                               CUs to themselves; 0 = default (2)        */
} rt_trace_opts;

/* Per-ray outputs, arrays of N_r = rt_fan_count() elements, owned by the
 * caller, in host or device memory per rt_trace_opts.results_mem.  Any
 * pointer may be NULL to skip that output.
 *   group_km    group path P' (includes the vacuum segments)
 *   phase_km    phase path P = integral of n . dx
 *   range_km    ground range R * (central angle transmitter -> landing)
 *   az_dev_deg  initial great-circle bearing transmitter -> landing minus the
 *               launch azimuth, in (-180, 180]; 0 when the range is ~0
 *   apogee_km   largest height over the RK4 step ends (reflection height)
 *   land_*_deg  landing point (GROUND) or the point under the last state
 *   status      RT_RAY_*; NUMERIC rays have NaN outputs
 *   n_steps     RK4 steps taken
 * Trajectory (optional): ray i owns records [i*per_ray, (i+1)*per_ray) of
 * traj, per_ray = traj_capacity / N_r; a record is 8 doubles
 * (r_km, theta_rad, phi_rad, n_r, n_theta, n_phi, P'_km, P_km) taken at
 * steps 0, stride, 2*stride, ... and at the last step; traj_count[i] is
 * the number written (capped at per_ray, RT_W_TRAJ_TRUNCATED if any
 * ray was capped). */
typedef struct {
    double *group_km, *phase_km, *range_km, *az_dev_deg, *apogee_km;
    double *land_lat_deg, *land_lon_deg;
    int32_t *status, *n_steps;
    double *traj;
    int32_t *traj_count;
    int64_t total_steps;    /* out: sum of n_steps over the fan            */
    double kernel_ms;       /* out: device time of the launch's kernels    */
    /* out (rt_trace only): how the launch ran -- RK4 steps taken one lane
     * per ray, on promotion rows and on 16-lane rows after the hand-off (or
     * of the in-wave switch), summing to total_steps; device time of the
     * ray-start and one-lane kernels, then of the tail and finish kernels */
    int64_t steps_one_lane, steps_promoted, steps_rows;
    double trace_ms, tail_ms;
    /* out (rt_trace only): iterations of the one-lane waves that stepped at
     * least one ray, summed over the waves; steps_one_lane / (64 x this) is
     * the share of lane slots that held a ray (the one-lane kernel's lane
     * occupancy) */
    int64_t one_lane_wave_iters;
} rt_results;

/* Create a context on HIP device `device` issuing work on `hip_stream`
 * (a hipStream_t, borrowed; NULL = the null stream).  The context owns
 * its device workspace.  RT_E_DEVICE if the device cannot be used. */
rt_status rt_ctx_create(int32_t device, void *hip_stream, rt_ctx **out);
void rt_ctx_destroy(rt_ctx *ctx);
const char *rt_last_error(const rt_ctx *ctx);

/* Upload a grid (preprocessing module of Sec. II-C).  `values` points to
 * n_lat*n_lon*n_h elements of geom->dtype in host or device memory
 * (values_mem); it is copied and converted (f_N^2 in MHz^2 for the FP64
 * path and an FP32 copy for the mixed path), so the caller keeps its
 * buffer.  RT_E_INVALID on a bad geometry or a negative / non-finite value;
 * RT_E_NOMEM if the device copy cannot be allocated.  No field is set. */
rt_status rt_grid_create(rt_ctx *ctx, const rt_grid_geom *geom, const void *values,
                         int32_t values_mem, rt_grid **out);
void rt_grid_destroy(rt_grid *grid);

/* Geomagnetic model (Sec. II-C, the field input of the preprocessing
 * module; it enters the refractive index through Y = f_H / f of eq.
 * appleton, with Y_L and Y_T its components along and across the wave
 * normal).  Set (or with d == NULL / B0 == 0 clear) the dipole field of a
 * grid, stored by value on the grid handle; later traces of the grid use
 * it.  The field is a centred axial dipole: B_r = -2 B0 (R/r)^3 cos(theta),
 * B_theta = -B0 (R/r)^3 sin(theta), B_phi = 0 in local components (it
 * points down in the northern hemisphere).  RT_E_INVALID for a negative or
 * non-finite B0; RT_E_UNSUPPORTED for a tilted dipole (pole_lat_deg != 90). */
rt_status rt_field_set(rt_grid *grid, const rt_dipole *d);

/* Trace every ray of a fan through a grid (main processing module of
 * Sec. II-C) and write the per-ray outputs.  Synchronous on the context's
 * stream.  RT_E_INVALID on bad options or fan values; RT_E_UNSUPPORTED if
 * a frequency is at or below the largest electron gyrofrequency of the
 * field (Y >= 1), or the transmitter is not below the grid bottom.
 * Per-ray failures are statuses, not call failures.  RT_E_DEVICE on a HIP
 * error, or if the launch itself went wrong: a promotion wait that timed
 * out, or a ray that no trace kernel finished (such rays keep status -1
 * and NaN outputs; no output of a failed call is valid).  An empty fan is a
 * no-op returning RT_OK. */
rt_status rt_trace(rt_ctx *ctx, const rt_grid *grid, const rt_fan *fan,
                   const rt_trace_opts *opts, rt_results *res);

/* For callers that cannot allocate device or pinned memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * rt_trace with every buffer the launch needs beyond the caller's inputs and
 * outputs -- ray records, hand-off records, tickets, counters, the staged fan
 * and parameter block -- taken from a scratch region of RT_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device from the first context on it until
 * the process ends, and host staging held by the context.  The successful
 * path calls no hipMalloc, hipFree, hipHostMalloc or other allocating
 * routine.  Same arguments, results and errors as rt_trace, within these
 * limits (RT_E_INVALID beyond them, before anything is launched):
 * opts->results_mem must be RT_MEM_DEVICE (every non-NULL array of res is
 * device memory), no trajectories (traj_stride 0), at most
 * RT_NOALLOC_MAX_RAYS rays and RT_NOALLOC_MAX_AXIS fan axis values
 * (n_elev + n_az + n_freq).  Every call on one GPU uses that GPU's one scratch
 * region, whose contents the next call overwrites: calls that overlap on one
 * GPU (several contexts or threads) race, and the caller must serialize
 * them.  The call is synchronous, like rt_trace. */
#define RT_NOALLOC_SCRATCH_BYTES (40 << 20)
#define RT_NOALLOC_MAX_RAYS 131072
#define RT_NOALLOC_MAX_AXIS 4096
rt_status rt_trace_noalloc(rt_ctx *ctx, const rt_grid *grid, const rt_fan *fan,
                           const rt_trace_opts *opts, rt_results *res);

/* Synthetic oblique ionogram from a traced frequency x elevation sweep
 * (Sec. IV-B-4: joint frequency-elevation scanning).  `fan` is the fan that
 * produced `res`: one azimuth (n_az == 1), elevations strictly increasing.
 * For every (frequency, mode) trace and every pair of adjacent elevations
 * whose rays both return to the ground with ground ranges on opposite sides
 * of range_km (range - range_km changes sign, zero counting as positive),
 * one received ray is reported, linearly interpolated in elevation:
 * out[(t * max_points + k) * 4 + {0,1,2,3}] = elevation (deg), group path
 * (km), phase path (km), apogee (km) of the k-th crossing of trace
 * t = i_freq * n_mode + i_mode, in increasing elevation; counts[t] = number
 * of crossings found (may exceed max_points; only max_points are kept).
 * Slots k >= counts[t] of a trace are set to 0.
 * res arrays group_km, phase_km, range_km, apogee_km and status are read;
 * mem (RT_MEM_HOST / RT_MEM_DEVICE) says where res, out and counts live.
 * RT_E_INVALID on a fan that is not a sweep or missing arrays. */
rt_status rt_ionogram(rt_ctx *ctx, const rt_fan *fan, const rt_results *res, double range_km,
                      int32_t max_points, int32_t mem, double *out, int32_t *counts);

/* ------------------------------------------------------------------------
 * Request server (continuous batching of ray-fan requests on one GPU).
 *
 * A server owns n_slots HIP streams (each with its own workspace and pinned
 * staging) and a device-memory arena of mem_budget bytes for the outputs of
 * admitted requests.  rt_server_submit copies the fan and never blocks: the
 * request waits in a FIFO queue.  Whenever a slot is idle, the queue head
 * and the requests behind it that share its grid geometry, transmitter and
 * options and whose outputs fit in the arena are launched together as one
 * batch on that slot (one persistent kernel over all their rays, each
 * request through its own grid snapshot); launches in different slots run
 * concurrently on the device.  A batch of at least 65536 rays waits while
 * another slot's launch of that size is still in its one-lane phase (it
 * starts when that launch reaches its tail kernel), so that two large
 * launches do not run their bulks side by side.  rt_server_poll launches
 * queued requests as slots and memory free up and reports finished ones
 * (the server makes progress only when submit or poll is called).  A finished
 * request keeps its outputs in the arena until rt_server_fetch copies them
 * out and releases the memory.  Per-ray arithmetic does not depend on the
 * slot or on what else runs, so a request's results are bit-identical alone
 * and in a mix.  Grids stay resident (created with rt_grid_create on the
 * same context) and may serve many requests.  Trajectories are not
 * recorded by the server.  One host thread drives a server.
 * ---------------------------------------------------------------------- */
typedef struct rt_server rt_server;

typedef struct {
    int64_t mem_budget_bytes;  /* output arena; 0 = 256 MiB                    */
    int32_t n_slots;           /* concurrent launches (streams); 0 = 2, <= 64    */
    int32_t max_batch_requests;/* requests per launch; 0 = 256                   */
    int32_t max_batch_rays;    /* rays per launch (a larger single request still
                                  runs alone); 0 = 1048576                       */
    int32_t reserved;          /* must be 0                                      */
} rt_server_opts;

typedef struct {
    int64_t id;
    int64_t n_rays;
    int64_t total_steps;       /* RK4 steps of the request                     */
    double kernel_ms;          /* device time of the request's kernels         */
    rt_status status;          /* RT_OK or RT_W_TRAJ_TRUNCATED                 */
    int32_t reserved;
} rt_request_info;

/* RT_E_NOMEM if the arena cannot be allocated. */
rt_status rt_server_create(rt_ctx *ctx, const rt_server_opts *opts, rt_server **out);
/* Waits for running requests, then frees everything the server owns. */
void rt_server_destroy(rt_server *srv);
/* opts->traj_stride must be 0 (RT_E_UNSUPPORTED otherwise); a request whose
 * outputs exceed the whole arena is RT_E_NOMEM.  *id identifies it. */
rt_status rt_server_submit(rt_server *srv, const rt_grid *grid, const rt_fan *fan,
                           const rt_trace_opts *opts, int64_t *id);
/* Non-blocking: launch what can be launched, then write up to `max` newly
 * finished requests into done[] (*n_done of them). */
rt_status rt_server_poll(rt_server *srv, rt_request_info *done, int32_t max, int32_t *n_done);
/* Copy a finished request's per-ray outputs into res (arrays of n_rays,
 * host or device memory per mem; NULL pointers skipped), release its arena
 * memory and forget it.  To host memory the outputs go through the
 * server's pinned staging (one device copy).  Blocks until the copy is
 * done.  RT_E_INVALID for an unknown or unfinished id. */
rt_status rt_server_fetch(rt_server *srv, int64_t id, rt_results *res, int32_t mem);
/* Drop a queued request (RT_OK) or mark a running one to be discarded when
 * it finishes (RT_OK); RT_E_INVALID for an unknown id. */
rt_status rt_server_cancel(rt_server *srv, int64_t id);
/* Queue length, running requests, arena bytes in use. */
rt_status rt_server_stats(const rt_server *srv, int32_t *queued, int32_t *running,
                          int64_t *arena_used);

/* ------------------------------------------------------------------------
 * Replayable traces (HIP graph).  rt_plan_create validates a trace exactly
 * like rt_trace, stages its fan and parameter block once, and captures the
 * launch sequence (workspace upload, ray-start kernel, one-lane kernel,
 * 16-lane tail kernel, ray-finish kernel, counter read-back) into a HIP
 * graph on a private stream.  The
 * plan owns its workspace and pinned staging; it borrows the grid and the
 * caller's result buffers, which must be device memory (opts->results_mem =
 * RT_MEM_DEVICE) and stay valid, like the grid, until rt_plan_destroy.
 * The fan is copied at create.  Trajectories are not supported.
 * rt_plan_launch enqueues one replay on the context's stream and returns;
 * rt_plan_wait synchronizes that stream and reports the replay's ray-steps
 * and device time.  Every replay recomputes all outputs from the launch
 * state (the counters are re-uploaded by the graph, no memset nodes).
 * ---------------------------------------------------------------------- */
typedef struct rt_plan rt_plan;

rt_status rt_plan_create(rt_ctx *ctx, const rt_grid *grid, const rt_fan *fan,
                         const rt_trace_opts *opts, const rt_results *res, rt_plan **out);
rt_status rt_plan_launch(rt_plan *plan);
rt_status rt_plan_wait(rt_plan *plan, int64_t *total_steps, double *kernel_ms);
void rt_plan_destroy(rt_plan *plan);

/* ------------------------------------------------------------------------
 * Autotuner.  The launch settings that change speed but not results are
 * tail_threshold, waves_per_simd, ray_order, promote_waves, promote_age and
 * cu_layout (see rt_trace_opts).  rt_autotune traces the given fan for every
 * candidate setting (tail_threshold in {-2, -1, 8 and 16 rays per CU} x
 * waves_per_simd in {1, 2} x ray_order in {index, strided, mode-sorted};
 * then, on top of
 * the fastest of those other than the in-wave switch (promotion does not
 * combine with it), promote_waves in
 * {16, 32, 64} with promote_age -1, each with cu_layout 2 and 1; the first
 * stage runs without promotion; one untimed run, then the median device
 * time of three), times the three fastest and the library defaults again,
 * nine single launches each, interleaved, keeps the one with the lowest
 * median if that beats the defaults' by at least 2 % (else the defaults,
 * all six fields 0; best_ms and default_ms are those medians) and writes
 * base with
 * those six fields replaced to *tuned.  Choices are cached in the process under a key made of the
 * device's CU count, the grid shape and interpolation, precision, field on
 * or off and the ray count rounded to a power of two; a cached key is
 * answered without tracing.  Results of the trial traces are discarded
 * (every candidate gives bit-identical results).  rt_tune_cache_save and
 * rt_tune_cache_load write and read the cache as text, one key per line.
 * ---------------------------------------------------------------------- */
typedef struct {
    double best_ms;            /* device time of the chosen setting (0 if cached) */
    double default_ms;         /* device time with the library defaults (0 if cached) */
    int32_t n_candidates;      /* settings traced                                */
    int32_t from_cache;        /* 1: answered from the cache                     */
} rt_tune_info;

rt_status rt_autotune(rt_ctx *ctx, const rt_grid *grid, const rt_fan *fan, const rt_trace_opts *base,
                      rt_trace_opts *tuned, rt_tune_info *info);
/* RT_E_INVALID if the file cannot be written / read or a line is malformed. */
rt_status rt_tune_cache_save(const char *path);
rt_status rt_tune_cache_load(const char *path);
void rt_tune_cache_clear(void);

/* Host-only helpers (no device needed). */
rt_status rt_fan_count(const rt_fan *fan, int64_t *n_rays);
rt_status rt_check_geom(const rt_grid_geom *geom);
void rt_default_opts(rt_trace_opts *opts);

#ifdef __cplusplus
}
#endif
#endif
