/*
 * gcloak.h -- C ABI of the MI355X (gfx950) Newtonian ray tracer for grating
 * cloaks (Halimeh, Schmied, Wegener, "Newtonian photorealistic ray tracing
 * of grating cloaks and correlation-function-based cloaking-quality
 * assessment", Opt. Express 2010).
 *
 * The library renders what a pinhole camera sees in a metal grating mirror
 * covered by the grating cloak and scores the image against a flat-mirror
 * reference:
 *   - index profile n = 1 / |1 + W0(i c k e^{ik(x+iy)})|, c = iA,
 *     k = 2 pi / Lambda (Sec. 2, eq. (1); W0 is the principal Lambert
 *     function, eq. (13)), truncated to n = 1 outside a finite box;
 *   - rays obey the Newton-type law of Sec. 3 (eq. (11)); the library
 *     integrates the equivalent form dr/dtau = p, dp/dtau = grad(n^2)/2 with
 *     |p| = n (dt = n^2 dtau), refracts with Snell's law at the box faces
 *     (Sec. 3) and reflects off the trochoid metal grating of eq. (2);
 *   - escaped rays sample a procedural sky (an 8 x 8 latitude-longitude
 *     checkerboard smoothed by tanh of sharpness K);
 *   - images are compared with the zero-shift cross-correlation of
 *     eqs. (14)-(15).
 *
 * Conventions for every call:
 *   - All pointers named d_* are DEVICE pointers on the context's device;
 *     the caller owns them.  Scene, camera and option structs are host
 *     memory, read during the call only.  The library never returns memory.
 *   - Work is enqueued on the given stream (0 = the null stream) and runs
 *     asynchronously, except that calls returning host scalars (C0, ncc,
 *     gc_stats) synchronise that stream before returning.
 *   - Every call returns GC_OK (0) or a negative gc_status.  On error a
 *     message is available from gc_last_error() (per host thread) and no
 *     output is guaranteed.  No C++ exception crosses this interface.
 *   - Per-ray failures are not call errors: they appear in the per-ray
 *     status array or in gc_stats.failed, and a failed sample shades black.
 *   - One gc_ctx per host thread; calls on one context must not overlap.
 */
#ifndef GCLOAK_H
#define GCLOAK_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GC_OK = 0,
    GC_EINVAL = -1,        /* bad argument (null pointer, size, NaN, ...) */
    GC_EDOMAIN = -2,       /* A k >= 1 or A < 0: W0 is not single-valued on the cloak */
    GC_ENOMEM = -3,        /* device scratch allocation failed */
    GC_EDEVICE = -4,       /* a HIP call failed */
    GC_EUNSUPPORTED = -5   /* option combination not provided */
} gc_status;

typedef enum { GC_F64 = 0, GC_F32 = 1 } gc_precision;
typedef enum { GC_RK4 = 0, GC_DOPRI5 = 1 } gc_integrator;

typedef enum {
    GC_RAY_OK = 0,
    GC_RAY_MAX_STEPS = 1,       /* more than max_steps accepted steps in the cloak */
    GC_RAY_MAX_EVENTS = 2,      /* more than max_events interface events */
    GC_RAY_NONFINITE = 3,       /* a non-finite value appeared in the ray state */
    GC_RAY_STEP_UNDERFLOW = 4   /* DOPRI5 step fell below h_min */
} gc_ray_status;

/* What fills the box |x| <= half_width, grating < y <= y_top (n = 1 outside):
 *   GC_CLOAK_NONE        nothing (the box does not exist);
 *   GC_CLOAK_EQ1         the index of eq. (1) (Sec. 2);
 *   GC_CLOAK_REFERENCED  eq. (1) divided by its minimum n_min = 1 / (1 + A k),
 *                        so that no index is below the air's (Sec. 4,
 *                        Figs. 5-7 (c));
 *   GC_CLOAK_PLATE       a homogeneous dielectric plate of index
 *                        1 / n_min = 1 + A k (Sec. 4: with the flat mirror,
 *                        the ideal image of the referenced cloak, Figs. 5-7
 *                        (a); with the grating, Figs. 5-7 (b)). */
typedef enum { GC_CLOAK_NONE = 0, GC_CLOAK_EQ1 = 1, GC_CLOAK_REFERENCED = 2, GC_CLOAK_PLATE = 3 } gc_cloak;

/* What a ray that leaves the scene shows:
 *   GC_BACKDROP_SKY    a sky at infinity, an 8 x 8 latitude-longitude
 *                      checkerboard smoothed by tanh of sharpness sky_K;
 *   GC_BACKDROP_PLANE  the plane y = backdrop_y (the photograph in front of
 *                      which the camera sits, Sec. 4), patterned with
 *                      m = 1/2 + 1/2 tanh(sky_K cos(2 pi x / P))
 *                      tanh(sky_K cos(2 pi z / P)), P = backdrop_period, at
 *                      the point the ray meets it; a ray that does not rise
 *                      to the plane sees m = 0.
 * Both colour a ray Cb + m (Ca - Cb), Ca = (0.95, 0.85, 0.30),
 * Cb = (0.10, 0.20, 0.55). */
typedef enum { GC_BACKDROP_SKY = 0, GC_BACKDROP_PLANE = 1 } gc_backdrop;

/* Scene (Sec. 2).  Grating x = xi - A sin(k xi), y = A cos(k xi) (eq. (2)),
 * infinite in x and z; the box holds `cloak` (gc_cloak); half_width and
 * y_top may be +inf.  mirror = 1 replaces the grating by the flat mirror
 * y = 0 (with cloak = GC_CLOAK_NONE: the reference image; with the plate:
 * the plate reference).  sky_K is the backdrop's tanh sharpness (+inf:
 * hard squares).  fresnel = 0: the box faces refract by Snell's law (total
 * internal reflection where it allows no transmission), weight 1;
 * fresnel = 1: Fresnel-weighted faces (Sec. 3): the primary ray goes on with
 * the transmitted fraction T of unpolarised light at each face crossing, and
 * the reflected fraction R starts a branch that is traced to its end without
 * further splitting (rays reflected more than once are neglected); the
 * sample's colour sums the weighted backdrop of all its paths (gc_render in
 * FP64 only). */
typedef struct {
    double Lambda;
    double A;
    double half_width;
    double y_top;
    int32_t cloak;          /* gc_cloak */
    int32_t mirror;
    double sky_K;
    int32_t fresnel;
    int32_t backdrop;       /* gc_backdrop */
    double backdrop_y;
    double backdrop_period;
} gc_scene;

/* Pinhole camera (Sec. 4: a virtual point camera).  right = forward x up,
 * image up = right x forward, with `up` the up hint (all zero: +y); row 0
 * at the top.  fov_y_deg is the full vertical opening angle; fov_x_deg the
 * horizontal one, or 0 for square pixels (the paper's camera opens 50 deg
 * horizontally and 42 vertically).  Sample s of pixel (i, j) passes through
 * (i + u, j + v), with u, v the SplitMix64 outputs number 2c and 2c + 1
 * (c = ((scene_index H + j) W + i) spp + s) of the generator seeded with
 * `seed`, each mapped to [0,1) by its top 53 bits; u = v = 1/2 when
 * jitter = 0. */
typedef struct {
    double eye[3];
    double target[3];
    double fov_y_deg;
    int32_t width;
    int32_t height;
    int32_t spp;
    int32_t jitter;
    uint64_t seed;
    int64_t scene_index;
    double up[3];
    double fov_x_deg;
} gc_camera;

/* Integration options.  RK4: classical 4-stage, fixed step h.  DOPRI5:
 * Dormand-Prince 5(4) with an RMS error norm over (x, y, p_x, p_y) scaled
 * by atol + rtol max(|y_n|, |y_n+1|), step factor clamp [0.2, 5], safety
 * 0.9, no growth right after a rejection, first step h0, caps h_max and
 * h_min.  Step sizes are in tau (|dr/dtau| = n).  w_fallback is the
 * |1 + W| threshold below which the FP32 path hands a step to FP64; the
 * FP64 kernel keeps the ray while |1 + W| < 2 w_fallback.  fp64_stay > 0:
 * from the fp64_stay-th hand-over of a ray on, the FP64 kernel keeps it
 * for the rest of its visit of the box (at most 16384 steps per round), so
 * that a ray that keeps returning near the branch point does not cost a
 * round per return; 0 (default): never.  An event (box face or grating) ends a step at the
 * partial step of the same integrator that lands on the surface. */
typedef struct {
    int32_t prec;          /* gc_precision */
    int32_t integ;         /* gc_integrator */
    double h;              /* RK4 step */
    double rtol, atol;     /* DOPRI5 tolerances */
    double h_max, h0, h_min;
    double w_fallback;     /* default 1e-2 */
    int32_t max_events;    /* default 32 */
    int32_t fp64_stay;     /* default 0 (FP32 path only) */
    int64_t max_steps;     /* default 10^5 */
} gc_opts;

typedef struct {
    int64_t rays;            /* samples traced */
    int64_t accepted_steps;  /* integrator steps kept inside the cloak (all precisions) */
    int64_t rejected_steps;  /* DOPRI5 attempts rejected */
    int64_t events;          /* box entries/exits, internal reflections, grating contacts */
    int64_t fallbacks;       /* FP32 path: steps handed to FP64 because a stage needed it */
    int64_t failed;          /* samples with status != GC_RAY_OK */
    int64_t fp64_steps;      /* FP32 path: accepted in-box steps taken in FP64 (hand-overs) */
    int64_t rounds;          /* FP32 path: in-cloak / event rounds */
    int64_t tail_rays;       /* batch plan: rays put at the front of the first round's queue */
    int64_t hot_steps;       /* FP32 path: accepted steps taken by the FP32 in-cloak kernel */
    double hot_ms;           /* FP32 path: device time of the FP32 in-cloak kernel (HIP events) */
    double event_ms;         /* FP32 path: device time of the FP64 event and air kernels */
    double tail_ms;          /* FP32 path: device time of the tail kernel */
    double total_ms;         /* FP32 path: device time of the whole call */
    int64_t first_pass_steps; /* gc_render_grad: forward steps the first pass took (stopped traces included) */
} gc_stats;

typedef struct gc_ctx gc_ctx;

/* Scheduling of the FP32 pipeline, per context.  It changes only which
 * lane integrates which ray and when: every ray's result is the same for
 * any setting.  The in-cloak kernel is persistent: each
 * wave takes rays from queues of box entries, one visit of the box at a
 * time, and a visit cannot be split, so the longest visits bound the
 * length of a launch unless they start early and run fast.
 *   slow_pxy        a box entry whose unit direction has an in-plane part
 *                   |(d_x, d_y)| below this goes to the slow queue (it
 *                   crosses the box slowly in tau); 0: a single queue
 *   slow_wave_div   every slow_wave_div-th wave takes the slow queue first;
 *                   a wave holding slow rays raises its issue priority on
 *                   its SIMD; 0: no wave prefers the slow queue
 *   refill          a wave claims new rays once at least this many of its
 *                   64 lanes are idle (1 .. 64)
 *   waves_per_simd  resident waves per SIMD of the in-cloak kernel
 *                   (1 .. 8; 0: as many as fit)
 *   plan_lanes      a batch plan made while this is G >= 2 splits its
 *                   scenes into G groups (balanced by sample count), each
 *                   with its own queues, rounds and graphs on a stream of
 *                   its own, so that the long serial tail of one group
 *                   (its last visits and FP64 hand-overs) overlaps the work
 *                   of the others (0 or 1: one pipeline; at most 3) */
typedef struct {
    double slow_pxy;
    int32_t slow_wave_div;
    int32_t refill;
    int32_t waves_per_simd;
    int32_t plan_lanes;
} gc_tune;

/* Create a context on HIP device `hip_device` (made current for the call).
 * Returns GC_EINVAL for a null `out` or a bad device, GC_EDEVICE on HIP
 * failure. */
gc_status gc_create(gc_ctx** out, int hip_device);

/* Release the context and its device scratch.  Null is ignored. */
void gc_destroy(gc_ctx* ctx);

/* Message of the last failed call on this host thread ("" if none). */
const char* gc_last_error(void);

/* Fill `opts` with the defaults: FP64, RK4, h = 1e-3, rtol = atol = 1e-8,
 * h_max = 0.02, h0 = 1e-3, h_min = 1e-12, w_fallback = 1e-2,
 * max_events = 32, max_steps = 10^5. */
void gc_default_opts(gc_opts* opts);

/* Fill `tune` with the defaults (the setting a new context starts with). */
void gc_default_tune(gc_tune* tune);

/* Set / read the context's scheduling.  GC_EINVAL for a null pointer or a
 * value out of range (slow_pxy outside [0, 1], slow_wave_div < 0, refill
 * outside 1 .. 64, waves_per_simd outside 0 .. 8, plan_lanes outside
 * 0 .. 3). */
gc_status gc_set_tune(gc_ctx* ctx, const gc_tune* tune);
gc_status gc_get_tune(const gc_ctx* ctx, gc_tune* tune);

/* Batched FP32 render as HIP graphs (S7: one launch sequence for many
 * scenes and their correlations).  gc_batch_plan_create renders the
 * workload once eagerly (which fixes the number of pipeline rounds it
 * needs: every ray's path is deterministic), then captures, on a stream of
 * its own: the counters' reset (a kernel, no memset node), the flight of
 * every camera ray to the box, that many rounds of the in-box / FP64 / air
 * kernels, the pixel averages into d_rgb[i], and, when d_ref is non-null,
 * for each scene the flat-mirror reference into d_ref[i] (if render_refs)
 * and the zero-shift correlation C0 (eq. (15)) of d_rgb[i] against
 * d_ref[i]; 1 + 2 x rounds graphs, each round's in-box kernel in a graph of
 * its own.  The plan owns its pipeline buffers (the context's are not
 * touched) and keeps the image pointers and the context's gc_tune of the
 * moment: the images must stay allocated while the plan lives.  The eager
 * run also records the longest first visits of the box (at least 1000
 * steps; the 4096 longest): the replays put those rays at the front of the
 * first round's queue, so that they start when the launch does (scheduling
 * only: every result is the same).  Launch enqueues the graphs back to back
 * on a stream (asynchronous); results synchronises that stream and returns
 * C0[n_scenes] and the counters of the last replay (total_ms from HIP
 * events around it, hot_ms from events between the graph launches around
 * each in-box kernel, event_ms 0; tail_rays = the number of those front
 * rays).  GC_EUNSUPPORTED for prec != GC_F32 or a flat-mirror scene;
 * GC_EDEVICE if the replay left rays unfinished (the workload changed under
 * the plan). */
typedef struct gc_batch_plan gc_batch_plan;
gc_status gc_batch_plan_create(gc_ctx* ctx, int32_t n_scenes, const gc_scene* scenes, const gc_camera* cameras,
                               const gc_opts* opts, float* const* d_rgb, float* const* d_ref, int32_t render_refs,
                               gc_batch_plan** out);
gc_status gc_batch_plan_launch(gc_batch_plan* plan, hipStream_t stream);
gc_status gc_batch_plan_results(gc_batch_plan* plan, double* C0, gc_stats* stats, hipStream_t stream);
void gc_batch_plan_destroy(gc_batch_plan* plan);

/* Autotuner of the FP32 pipeline: the DOPRI5 tolerance rtol (= atol), the
 * step cap h_max and the scheduling (gc_tune), picked for a workload (one
 * or more scenes with their cameras) subject to accuracy bounds against
 * the FP64 path.
 *
 * Reference: the FP64 path with the same options except prec = GC_F64 and
 * rtol = atol = ref_rtol (the FP64 path follows the CPU oracle to
 * rounding).  Checks, per scene:
 *   - exit directions of the camera's rays at width / dir_scale x
 *     height / dir_scale (same spp, jitter and seed): rays whose FP64 exit
 *     moves by more than dir_tol when the initial direction moves by 1e-6
 *     (two fixed perpendicular perturbations), or whose status or event
 *     count then changes, are ill-conditioned and not compared; of the
 *     others, the fraction whose status or event count differs from the
 *     reference must be at most max_changed, and the rest must have their
 *     99th percentile angle error at most dir_tol and their maximum at most
 *     30 dir_tol;
 *   - the zero-shift correlation C0 (eq. (15)) of the image at
 *     width / cc_scale x height / cc_scale against the flat-mirror
 *     reference must be within cc_tol of the FP64 image's (with
 *     cc_scale = 1 the timed full-size renders are the ones checked).
 * Candidates (DOPRI5): rtol x {3, 1, 1/3} times h_max x {1, 2.5, 5,
 * 10, 25} (RK4 keeps its step: one candidate), at FP64 hand-over
 * thresholds w_fallback in {the given one, 0.1, 0.3}: after the given
 * one, the levels of 0.1 and 0.3 that exceed it are tried, in increasing
 * order, only while no candidate has passed (at most 45 candidates).  Of the candidates that pass, the one with the shortest FP32 render of the whole workload is
 * chosen (best of `reps`); if none passes, the fastest that is nowhere less
 * accurate than the options as given (see `chosen`); then, if tune_sched, a fixed set of gc_tune
 * settings is timed the same way and the fastest is installed in the
 * context.  Results never depend on gc_tune.  C0 differences near 1e-4 are
 * at the level by which two correct integrations (FP64 at rtol 1e-7 and
 * 1e-8) differ on images of ~10^4 pixels, so the correlation check wants
 * the full-size images. */
typedef struct {
    int32_t dir_scale;     /* default 4 */
    int32_t cc_scale;      /* default 1 */
    double dir_tol;        /* default 1e-4 rad */
    double cc_tol;         /* default 1e-4 */
    double max_changed;    /* default 0.01 */
    double ref_rtol;       /* default 1e-10 */
    int32_t reps;          /* default 2 */
    int32_t tune_sched;    /* default 1 */
} gc_autotune_opts;

#define GC_AUTOTUNE_MAX_CAND 48

typedef struct {
    double rtol;
    double h_max;
    double w_fallback;
    double ms;             /* best FP32 render time of the workload (HIP events) */
    int64_t steps;         /* FP32 accepted steps of the workload */
    double dir_p99, dir_max, changed, cc_err;   /* worst over the scenes */
    int32_t pass;          /* all bounds hold */
    int32_t reserved;
} gc_autotune_cand;

typedef struct {
    int32_t n_cand;
    int32_t chosen;        /* index of the candidate returned in opts_out: the fastest that
                              passed; if none passed, the fastest whose every measured error
                              (dir_p99, dir_max, changed, cc_err) is at most that of the options
                              as given (its pass stays 0); -1 if neither (opts_out = opts) */
    gc_autotune_cand cand[GC_AUTOTUNE_MAX_CAND];
    gc_tune tune;          /* installed scheduling */
    double tune_ms;        /* its best render time */
    double base_tune_ms;   /* the render time with the context's scheduling on entry */
    int64_t cal_rays;      /* rays of the direction check (all scenes) */
    int64_t ill_rays;      /* of them ill-conditioned in FP64 */
} gc_autotune_report;

void gc_default_autotune_opts(gc_autotune_opts* at);

/* Run the autotuner (see above) on n_scenes scenes and cameras with FP32
 * options `opts` (prec must be GC_F32).  Writes the tuned options to
 * opts_out (equal to opts but for rtol, atol, h_max and w_fallback) and, if `report` is non-null, the
 * measurements.  Device scratch for the calibration is allocated and freed
 * inside the call; the stream is synchronised.  GC_EINVAL for bad
 * arguments, GC_EUNSUPPORTED for prec != GC_F32. */
gc_status gc_autotune(gc_ctx* ctx, int32_t n_scenes, const gc_scene* scenes, const gc_camera* cameras,
                      const gc_opts* opts, const gc_autotune_opts* at, gc_opts* opts_out,
                      gc_autotune_report* report, hipStream_t stream);

/* Trace n rays (Sec. 3) from origins d_org and directions d_dir (n x 3
 * doubles, row-major; directions need not be unit) until they escape.
 * Outputs: exit point (where the ray left its last surface) and unit exit
 * direction (n x 3 doubles each), per-ray gc_ray_status (int32), accepted
 * steps (int64) and events (int32).  Any output pointer except d_out_dir may
 * be null.  Works in the precision opts->prec.  n = 0 is a no-op. */
gc_status gc_trace_rays(gc_ctx* ctx, const gc_scene* scene, const gc_opts* opts, int64_t n,
                        const double* d_org, const double* d_dir,
                        double* d_out_org, double* d_out_dir,
                        int32_t* d_status, int64_t* d_steps, int32_t* d_events,
                        hipStream_t stream);

/* Render one image (Sec. 4): d_rgb is height x width x 3 float32 (HWC, row
 * 0 at the top), each pixel the mean of its spp sky colours (failed samples
 * black).  With scene->mirror = 1 (flat mirror, cloak = 0) the reference
 * image is produced in closed form (FP64 direction and sky angles, FP32 tanh,
 * for either precision).
 * The FP32 pipeline looks the sky up in FP32 (the image is FP32).  `st` (host, may
 * be null) receives the counters and then the call synchronises the
 * stream. */
gc_status gc_render(gc_ctx* ctx, const gc_scene* scene, const gc_camera* camera,
                    const gc_opts* opts, float* d_rgb, gc_stats* st, hipStream_t stream);

/* Render n_scenes scenes in one launch of the FP32 pipeline (opts->prec
 * must be GC_F32): all samples of all scenes share the queues of the
 * persistent in-cloak kernel, so scenes of uneven resolution, amplitude,
 * cloak width and viewpoint keep the GPU busy together.  scenes[i] and
 * cameras[i] are host arrays of n_scenes entries; d_rgb[i] (host array of
 * device pointers) receives image i (height_i x width_i x 3 float32).  When
 * d_ref is non-null, d_ref[i] is the reference image of scene i and C0[i]
 * (host, n_scenes doubles) receives eq. (15) at zero shift for it.  `st`
 * (may be null) receives counters summed over all scenes.  Synchronises
 * the stream.  Reflection-only scenes (mirror = 1) are not accepted here. */
gc_status gc_render_batch(gc_ctx* ctx, int32_t n_scenes, const gc_scene* scenes, const gc_camera* cameras,
                          const gc_opts* opts, float* const* d_rgb, const float* const* d_ref, double* C0,
                          gc_stats* st, hipStream_t stream);

typedef enum {
    GC_LOSS_C0 = 0,     /* L = 1 - C0: eq. (15) at zero shift, sum f'g' / sum f'^2 */
    GC_LOSS_NCC = 1     /* L = 1 - NCC: sum f'g' / sqrt(sum f'^2 sum g'^2) */
} gc_loss;

/* Cloaking-quality loss L (gc_loss) of the image rendered as gc_render does,
 * against the reference d_ref, and its derivatives with respect to the
 * grating amplitude A (eq. (2)) and the cloak's half_width, by the discrete
 * adjoint of the RK4 tracer (opts->integ must be GC_RK4).  opts->prec
 * selects FP64 or FP32 in-cloak arithmetic; surface maps, sky and sums are
 * FP64.  In FP32 the samples whose derivative FP32 cannot resolve -- paths
 * of more than 8000 steps, or a sky parameter m more sensitive than 60 per
 * radian to the initial direction -- are traced and differentiated again
 * in FP64 (colour included).
 * Each sample is traced forward with its state recorded every
 * `checkpoint_every` steps (1..256; 64 is the usual choice) and at every
 * event, then reversed from dm = 1, where m is the sky's blend parameter
 * (colour = Cb + m (Ca - Cb)): segments are recomputed from their
 * checkpoint and the transposed step Jacobians applied, including the
 * derivative of every event time (partial steps ending on a face or on the
 * grating, straight flights ending on the grating or the box).  The
 * longest FP64 traces (256 or more records) apply each segment's transposed
 * map instead, formed for all their segments in parallel; the result is
 * the same up to rounding order and does not depend on scheduling.  The result
 * is the derivative of the discrete image, sample by sample; a sample
 * whose event sequence changes at the current parameters contributes its
 * one-sided value, and samples near grazing contacts or crests have large
 * derivatives that dominate the sum.
 * d_ref: height x width x 3 float32 (device, not constant).  Optional
 * outputs (null to skip): d_rgb receives the image (height x width x 3
 * float32); d_sample_dm the per-sample dm/dA and dm/dhw (width * height *
 * spp pairs of doubles, sample s of pixel (i, j) at ((j width + i) spp + s);
 * zero for failed samples); loss / dL_dA / dL_dhw (host) the results; st
 * the forward counters (rays, accepted_steps, events, failed; tail_rays =
 * samples differentiated again in FP64 with tapes long enough for any
 * trace the options allow -- tapes longer than 256 records, and in FP32 the
 * long or sensitive traces; the first pass stops a trace once its tape has
 * overflowed or, in FP32, once it has passed 8000 steps, and the counters
 * of such a sample come from the FP64 pass; rounds = the hand-overs of more
 * than 8000 steps, which
 * start first; hot_steps = steps reversed by the first pass;
 * first_pass_steps = forward steps the first pass took;
 * hot_ms / tail_ms / total_ms the device time of the first pass, of the
 * FP64 passes and of the call).  Device scratch (tapes of up to 8 GiB per
 * pass, and once a sample is handed over a pool of 1.9 GB for the longest
 * traces' tapes and segment maps) is owned by the context.  Synchronises the
 * stream.  GC_EUNSUPPORTED for DOPRI5, flat-mirror scenes or sky_K = inf;
 * GC_EINVAL for a constant reference (or, for NCC, a constant image). */
gc_status gc_render_grad(gc_ctx* ctx, const gc_scene* scene, const gc_camera* camera, const gc_opts* opts,
                         const float* d_ref, int32_t loss_kind, int32_t checkpoint_every, float* d_rgb,
                         double* d_sample_dm, double* loss, double* dL_dA, double* dL_dhw, gc_stats* st,
                         hipStream_t stream);

/* Zero-shift cross-correlation of eqs. (14)-(15) between d_img (g) and the
 * reference d_ref (f): both npix x nch float32, channel fastest.  Each
 * channel's mean is subtracted (eq. (14)) and the sums are pooled over
 * channels: *C0 = sum f'g' / sum f'^2 (eq. (15) at (0, 0)); *ncc = sum f'g'
 * / sqrt(sum f'^2 sum g'^2) (may be null).  Sums are formed in FP64.
 * Synchronises the stream.  GC_EINVAL if npix < 1, nch < 1 or the
 * reference is constant. */
gc_status gc_cross_correlate(gc_ctx* ctx, const float* d_img, const float* d_ref,
                             int64_t npix, int32_t nch, double* C0, double* ncc,
                             hipStream_t stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * zero-shift correlation as gc_cross_correlate, computed by the same
 * kernels, but with no allocation and no synchronisation: the block
 * partials live in a fixed scratch array compiled into the library (160 KiB
 * per GPU, held until the process ends; its device address is taken when the
 * first context on that GPU is created), and the results stay on the device.
 * d_img (g), d_ref (f): npix x nch float32, channel fastest.  d_out (device,
 * caller-owned, 12 doubles) receives { C0 = sum f'g' / sum f'^2 (eq. (15)
 * at (0, 0)), ncc, sum f'^2, sum g'^2, the 4 channel means of f, the 4
 * channel means of g } (unused channels 0); a constant reference gives
 * sum f'^2 = 0 and C0 = NaN.  Any npix >= 1 fits (the scratch holds 1024
 * block partials, and the blocks stride over the pixels); nch above 4 is
 * rejected with GC_EINVAL.  Every call on one GPU shares that GPU's scratch
 * (the last call's partials stay in it), so calls that overlap on one GPU --
 * on different streams, from different contexts or threads -- race and
 * must be ordered by the caller.  Asynchronous on `stream`; calls no
 * hipMalloc, hipFree or memset. */
gc_status gc_cross_correlate_noalloc(gc_ctx* ctx, const float* d_img, const float* d_ref, int64_t npix, int32_t nch,
                                     double* d_out, hipStream_t stream);

/* Correlation map: eq. (15) at every shift (Sec. 5), the "more generous"
 * measure of cloaking quality whose peak value and location also quantify
 * an image displacement.  d_img (g) and d_ref (f) are device windows of
 * height x width pixels, nch float32 channels each (channel fastest), whose
 * rows lie `pitch` pixels apart (pitch = width for a whole image; a column
 * window of a W-wide image is base + col0 * nch with pitch W).
 *   - eq. (14): each channel's mean over the window is subtracted;
 *   - C(dx, dy) = sum f'(j, i) g'(j + dy, i + dx) / sum f'^2, the
 *     numerator over the pixels whose shifted partner lies in the window (the
 *     photograph holds nothing outside it), pooled over channels; the
 *     denominator over the whole window.  dx is the shift along a row
 *     (columns, to the right), dy down the rows (row 0 at the top), in pixels;
 *     C(0, 0) is the zero-shift coefficient of gc_cross_correlate.
 * d_map (device, (2 ry + 1) x (2 rx + 1) doubles, caller-owned) receives
 * C(dx, dy) at (dy + ry) (2 rx + 1) + (dx + rx).  peak / peak_dx / peak_dy
 * (host, each may be null) receive the maximum of the map and its shift, the
 * first maximum in that row-major order on ties.  Sums in FP64.
 * Synchronises the stream.  GC_EINVAL for null pointers, height or width < 1,
 * pitch < width, nch outside 1..4, rx outside [0, width), ry outside
 * [0, height), or a constant reference window; GC_EUNSUPPORTED for
 * 2 rx + 1 > 1024 or (2 width + 2 rx) nch > 8192 (two rows of the window
 * are staged in 64 KiB of LDS).  Scratch (partial sums) is owned by the
 * context and grown on demand. */
gc_status gc_cross_correlate_map(gc_ctx* ctx, const float* d_img, const float* d_ref, int32_t height, int32_t width,
                                 int64_t pitch, int32_t nch, int32_t rx, int32_t ry, double* d_map, double* peak,
                                 int32_t* peak_dx, int32_t* peak_dy, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GCLOAK_H */
