/*
 * darts.h -- C ABI of libdarts, an MI355X (gfx950) implementation of the hot
 * path of DARTS (He, Du, Jiang, Jin, "DARTS: Diffusion Approximated Residual
 * Time Sampling for Time-of-flight Rendering in Homogeneous Scattering
 * Media", 2024): per-path transient volumetric path tracing in a homogeneous
 * medium with
 *   - free-flight distances resampled (RIS) against the transient diffusion
 *     fluence (Section IV, Eq. (9)-(15)),
 *   - scattering directions drawn from an offline-tabulated elliptical-DA
 *     density mixed with the phase function by one-sample MIS (Section V-A,
 *     Eq. (16)-(19)),
 *   - an elliptical control-vertex connection that closes the path inside a
 *     target path-length interval (Section V-B, Eq. (20)-(22)),
 *   - accumulation into path-length (time) bins on the sensor (Eq. (1), (4)).
 *
 * Units: speed of light and refractive index are 1; time and path length are
 * the same quantity (Eq. (3)).
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev are device pointers (hipMalloc'ed or torch CUDA
 *     tensors) owned by the caller; the library only writes the outputs
 *     named.  Apart from batch objects (darts_batch_*), which own their
 *     device memory from create to destroy, it never allocates, frees or
 *     keeps device memory across calls.
 *   - Host structs are read during the call only.
 *   - `stream` is a hipStream_t (NULL = default stream); all work is enqueued
 *     on it and the call returns without synchronising.
 *   - Return value: DARTS_OK (0) or a negative DARTS_ERR_* code; the message
 *     of the last failure on the calling thread is darts_last_error().
 *     Kernel faults are asynchronous and surface at the next synchronisation.
 */
#ifndef DARTS_H
#define DARTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DARTS_OK                  0
#define DARTS_ERR_INVALID_ARG    -1  /* bad sizes, parameters or null pointers  */
#define DARTS_ERR_DEVICE         -2  /* a HIP runtime call failed               */
#define DARTS_ERR_UNSUPPORTED    -3  /* valid request this library does not serve */
#define DARTS_ERR_TABLE_MISMATCH -4  /* table built for another medium / dims   */

#define DARTS_MAX_EMITTERS 8
#define DARTS_MAX_COS_BINS 1024

/* Homogeneous medium (Eq. (9)): sigma_s, sigma_a >= 0 in 1/length, with
 * sigma_s + sigma_a > 0; Henyey-Greenstein asymmetry |g| < 1. */
typedef struct { double sigma_s, sigma_a, g; } darts_medium;

/* Isotropic pulsed point emitter (Section III, Eq. (1)): the pulse leaves at
 * path-length offset `start`; radiant intensity power / (4 pi). */
typedef struct { float pos[3]; float start; float power; } darts_emitter;

/* Sensor.
 *   kind 0: point fluence detector at `origin` (ray directions uniform on the
 *           sphere, weight 4 pi); width = height = 1.
 *   kind 1: orthographic radiance sensor; pixel (px, py) covers
 *           origin + [px/width, (px+1)/width) du + [py/height, (py+1)/height) dv;
 *           rays travel along `dir` (need not be normalised).
 * width and height are at most 65535. */
typedef struct {
    int kind;
    float origin[3], dir[3], du[3], dv[3];
    int width, height;
} darts_sensor;

/* kind 0: infinite medium.  kind 1: the medium fills the axis-aligned box
 * [lo, hi] with an index-matched boundary (vacuum outside, no refraction).
 * kind 2: the box of kind 1 whose bottom face z = lo[2] is an opaque
 * Lambertian floor of albedo floor_albedo in [0, 1] (a fog layer over diffuse
 * ground; surface events and case II surface connections of Section V-B).
 * floor_albedo is ignored for kinds 0 and 1. */
typedef struct { int kind; float lo[3], hi[3]; float floor_albedo; } darts_geometry;

/* n_bins half-open bins of equal width over total path length [l_lo, l_hi),
 * measured from the sensor and including the emitter's start offset;
 * 1 <= n_bins < 2^29. */
typedef struct { float l_lo, l_hi; int n_bins; } darts_bins;

/* Sensor response W (Eq. (4)): NULL for a time-resolved image (W the
 * indicator of each bin), or a device table built by darts_build_response
 * holding a piecewise-constant W over the scene's bins.  With a response the
 * image has one value per pixel, [height][width], estimating the integral of
 * W(path length) times the path contribution; path id p maps to pixel
 * p mod (height * width) and, in the DARTS family, draws its target bin with
 * probability proportional to W (Section V-B: sampling the path length where
 * the sensor responds avoids rejected samples). */
typedef struct {
    darts_medium medium;
    darts_geometry geom;
    const darts_emitter *emitters;   /* host array of n_emitters entries */
    int n_emitters;                  /* 1 .. DARTS_MAX_EMITTERS          */
    darts_sensor sensor;
    darts_bins bins;
    const float *response_dev;       /* NULL or a table of bins.n_bins segments */
} darts_scene;

/* Elliptical-DA direction table (Section V-A): n_cs cells of C/S over [0,1),
 * n_s cells of S over [0, s_max), n_cos uniform cos(theta) bins over [-1,1].
 * The paper uses 256 cos bins; 32 is the default here (any table keeps the
 * estimator unbiased, only its variance changes). */
typedef struct { int n_cs, n_s, n_cos; float s_max; } darts_table_dims;

/* A built table: `cdf_dev` holds float[n_cs][n_s][n_cos + 1]; row (i, j) is
 * the cumulative distribution over cos-bins for C/S in cell i and S in cell
 * j, cdf[..][0] = 0, cdf[..][n_cos] = 1.  `medium` and `dims` must be the
 * values the table was built with; they are checked against the scene. */
typedef struct { darts_medium medium; darts_table_dims dims; const float *cdf_dev; } darts_table;

/* Sampling strategy bits (Section VI, ablation study):
 *   DARTS     = RIS_DIST | EDA_DIR | ELL_TEXP
 *   uniform   = ELL_UNIFORM            (temporally uniform connection, Section V-B)
 *   vanilla   = DIRECT_REUSE           (shadow connection, path binned by length)
 *   DA only   = RIS_DIST | ELL_UNIFORM,  EDA only = EDA_DIR | ELL_TEXP
 * Exactly one of ELL_TEXP / ELL_UNIFORM unless DIRECT_REUSE is set. */
#define DARTS_RIS_DIST      0x1u
#define DARTS_EDA_DIR       0x2u
#define DARTS_ELL_TEXP      0x4u
#define DARTS_ELL_UNIFORM   0x8u
#define DARTS_DIRECT_REUSE  0x10u

typedef struct {
    uint64_t n_paths;      /* paths in this call                                 */
    uint64_t path_offset;  /* first path id; ids drive the RNG and the cell map  */
    uint64_t seed;         /* Philox4x32-10 key                                  */
    int max_bounces;       /* >= 1; maximum scattering order                     */
    int n_ris;             /* RIS candidates; 8 (the paper's choice)             */
    float alpha;           /* Eq. (19) preference parameter, >= 0 (paper: 0.5)   */
    unsigned flags;        /* DARTS_* strategy bits                              */
} darts_params;

/* Statistics counters (uint64 each, accumulated with atomics): paths
 * started; vertices that reached the early-exit test; connections that added
 * a non-zero contribution; early exits (nothing reachable inside the gate);
 * walks that left the medium; RIS steps with no valid candidate; EDA-branch
 * direction samples; paths stopped at max_bounces; paths that contributed
 * nothing; early exits already at the path's first vertex; full path samples
 * (sensor-to-emitter paths a connection produced) and those the sensor
 * weights with zero (length outside the bins or W = 0: the rejected samples
 * of Section V-B; vanilla connects at every vertex whatever the length, the
 * DARTS family only inside the target bin). */
enum {
    DARTS_ST_PATHS = 0, DARTS_ST_VERTICES, DARTS_ST_CONNECTIONS, DARTS_ST_EARLY_EXIT,
    DARTS_ST_MEDIUM_EXIT, DARTS_ST_RIS_ALL_INVALID, DARTS_ST_EDA_BRANCH,
    DARTS_ST_TRUNCATED, DARTS_ST_ZERO_PATHS, DARTS_ST_SETUP_EXIT, DARTS_ST_SAMPLES,
    DARTS_ST_REJECTED, DARTS_ST_COUNT = 16
};

/* Size in bytes of the cdf array of a table of these dimensions.
 * Returns INVALID_ARG for non-positive dims, n_cos > DARTS_MAX_COS_BINS,
 * s_max <= 0, n_cs * n_s > 2^26 or more than 2^31 - 1 floats in all. */
int darts_table_bytes(const darts_table_dims *dims, size_t *bytes);

/* Build the elliptical-DA direction table of Section V-A (Eq. (16)-(18)).
 * Entry (i, j, k) integrates sigma_s exp(-sigma_t t) Phi(x + w t, S - t) over
 * t in [0, t_M(u)] (Eq. (18)) and u = cos(theta) in cos-bin k, with C/S and S
 * at the cell centres ((i + 1/2)/n_cs, (j + 1/2) s_max/n_s) and Phi the
 * transient diffusion fluence of Eq. (9).  Computed in FP64 on the device by
 * a fixed Gauss-Legendre rule (4 nodes per cos-bin in u; 64 nodes in
 * v = (1 - e^{-sigma_t t})/(1 - e^{-sigma_t t_M})); each row is normalised
 * and its cumulative sum stored as float.  Rows whose integral underflows are
 * uniform.  cdf_dev: device float[darts_table_bytes / 4], written in full. */
int darts_build_da_tables(const darts_medium *medium, const darts_table_dims *dims,
                          float *cdf_dev, void *stream);

/* Size in bytes of a sensor-response table for n_bins segments
 * ((2 n_bins + 1) floats).  INVALID_ARG for n_bins < 1. */
int darts_response_bytes(int n_bins, size_t *bytes);

/* Build a sensor-response table from W (host float[n_bins], W >= 0, finite,
 * not all zero): float cdf[n_bins + 1] (cdf[0] = 0, cdf[k+1] the running sum
 * of W_j / sum W accumulated in double and rounded to float, cdf[n_bins] = 1)
 * followed by float W[n_bins].  response_dev: device memory of
 * darts_response_bytes; the copy completes before the call returns. */
int darts_build_response(const float *w_host, int n_bins, float *response_dev, void *stream);

/* Render: accumulate raw path contributions into the time-resolved image.
 * Each path is the paper's estimator of the transient path integral
 * (Eq. (1); per pixel and bin, the box sensor response of Eq. (4), or a
 * general W): free flights by DA-RIS (Section IV, Eq. (9)-(15)), directions
 * by EDA/phase one-sample MIS (Section V-A, Eq. (16)-(19)) and an elliptical
 * control-vertex connection per vertex (Section V-B, Eq. (20)-(22)), or the
 * strategies the flags select.
 *   Path id p = path_offset + i (i < n_paths) belongs to cell
 *   c = p mod (n_bins * height * width); its pixel is c mod (height*width) and,
 *   except in vanilla mode, its target interval is bin c / (height*width).
 *   DARTS family: each path adds its estimate to its own cell; vanilla: each
 *   path adds to every bin of its pixel its length reaches.
 *   image_hi_dev, image_lo_dev: device float[n_bins][height][width]
 *     ([height][width] with a sensor response),
 *     accumulate-into; hi + lo is a compensated (two-float) sum.
 *   image_m2_dev (nullable): accumulate-into sums over paths of the square
 *     of each path's total contribution to the cell (the DARTS family adds
 *     to one cell per path; a vanilla path adds to every bin its length
 *     reaches, and each of those sums is squared once).
 *   stats_dev (nullable): accumulate-into uint64[DARTS_ST_COUNT].
 *   table: required when flags contain DARTS_EDA_DIR, else may be NULL.
 * The per-cell estimate is (hi + lo) / (number of paths mapped to the cell),
 * or per pixel for vanilla. */
int darts_render_transient(const darts_scene *scene, const darts_params *params,
                           const darts_table *table,
                           float *image_hi_dev, float *image_lo_dev, float *image_m2_dev,
                           uint64_t *stats_dev, void *stream);

/* Per-path estimates (DARTS family only), for parity checks and variance
 * studies: path_value_dev[i] = total contribution of path path_offset + i
 * to the estimate of Eq. (1) in its cell (Sections IV-V, as for
 * darts_render_transient; device float[n_paths], overwritten).  Same kernel
 * as the render.  A path's value is a function of its id, the seed and the
 * scene: it is bit-identical whatever work decomposition, knob setting or
 * kernel (single render, batch, adjoint replay) traces it; images differ
 * between such launches only in the order of their additions. */
int darts_render_paths(const darts_scene *scene, const darts_params *params,
                       const darts_table *table, float *path_value_dev, void *stream);

/* Differentiable rendering, which the paper names as future work (Section
 * VII): gradient of L = sum_c grad_image[c] * I[c] (I the raw per-cell sums
 * the render call would add) with respect to (sigma_s, sigma_a, g) of the
 * medium of Eq. (9) and the phase function, by replaying
 * the same paths (same ids, same Philox counters; nothing is stored between
 * the calls) and weighting each contribution with the derivative of the log
 * of its path throughput (detached sampling).  grad_image_dev: device
 * float[n_bins][height][width]; grad_out_dev: device double[3],
 * accumulate-into.  DARTS family only. */
int darts_render_transient_backward(const darts_scene *scene, const darts_params *params,
                                    const darts_table *table, const float *grad_image_dev,
                                    double *grad_out_dev, void *stream);

/* Forward mode of the same derivative (Section VII, as for the backward
 * call): tangent_dev[k][c] += the sum, over the paths mapped to cell c, of
 * each connection's contribution times the derivative of the log of its path
 * throughput with respect to theta_k, theta = (sigma_s, sigma_a, g): per-cell
 * images of dI_c/dtheta_k (I the raw per-cell sums the render call would
 * add; detached sampling, the same paths), whose sums weighted by a
 * grad_image are darts_render_transient_backward's gradient.  For
 * Gauss-Newton or Fisher-information computations that need the per-cell
 * Jacobian.  tangent_dev: device float[3][n_bins][height][width],
 * accumulate-into with plain FP32 atomics.  DARTS family only. */
int darts_render_transient_tangent(const darts_scene *scene, const darts_params *params,
                                   const darts_table *table, float *tangent_dev, void *stream);

/* ---------------------------------------------------------------------------
 * Batched persistent render: many independent scenes (media, tables,
 * sensors, bins, path budgets) rendered by one kernel launch.  Each scene is
 * the same estimator as darts_render_transient with the same path ids, so a
 * batch image equals the separate renders up to the order of the
 * floating-point additions.  The scenes' paths are cut into work units that a
 * grid sized to the device pulls from a device counter until none are left;
 * the counter rewinds itself at the end of the launch, so a launch can be
 * repeated and captured in a graph.  (This serves many-configuration sweeps
 * such as the scattering-coefficient study of Section VI.)
 * ------------------------------------------------------------------------- */
typedef struct {
    darts_scene scene;          /* read at create (emitters copied)                  */
    darts_params params;        /* DARTS family only (no DIRECT_REUSE)               */
    const darts_table *table;   /* required with EDA_DIR; its cdf_dev must stay valid
                                   while the batch is used                           */
} darts_batch_item;

/* Work decomposition (chosen by darts_batch_autotune or by hand):
 *   order DARTS_BATCH_TILES: units of 64 consecutive cells x a range of
 *     repetitions, per-cell sums privatised in LDS and flushed once per unit
 *     (many paths per cell);
 *   order DARTS_BATCH_IDS: units of consecutive path ids, each finished path
 *     added to the image with a global atomic (few paths per cell).
 * block_threads: 64 or 256; waves_per_cu: persistent grid = compute units x
 * waves_per_cu waves (1..64); unit_paths: paths per unit (>= 64; tile units
 * round it down to a multiple of 64). */
#define DARTS_BATCH_TILES 0
#define DARTS_BATCH_IDS   1
typedef struct {
    int order;
    int block_threads;
    int waves_per_cu;
    int64_t unit_paths;
} darts_batch_plan;

typedef struct darts_batch darts_batch;   /* opaque */

/* Default plan (tile order, 256 threads, 16 waves per CU, 8192-path units). */
int darts_batch_default_plan(darts_batch_plan *plan);

/* Validate the items (as darts_render_transient would; INVALID_ARG,
 * UNSUPPORTED or TABLE_MISMATCH name the first bad item) and build the batch
 * on the current device: device copies of the scene parameters, the unit list
 * of `plan` (NULL = default) and the unit counter.  *out receives the handle;
 * nothing is allocated when validation fails. */
int darts_batch_create(const darts_batch_item *items, int n_items, const darts_batch_plan *plan,
                       darts_batch **out);

/* Scene i's image is elements [offsets[i], offsets[i+1]) of the batch output,
 * laid out as darts_render_transient's.  offsets: host int64[n_items + 1]. */
int darts_batch_image_offsets(const darts_batch *batch, int64_t *offsets);

/* Replace the work decomposition (rebuilds the unit list; synchronous). */
int darts_batch_set_plan(darts_batch *batch, const darts_batch_plan *plan);
int darts_batch_get_plan(const darts_batch *batch, darts_batch_plan *plan);

/* One launch that accumulates every scene's raw sums into image_hi_dev /
 * image_lo_dev (device float[offsets[n_items]], compensated pair).  Calls on
 * one batch must not overlap (they share the unit counter). */
int darts_batch_render(darts_batch *batch, float *image_hi_dev, float *image_lo_dev, void *stream);

/* Clear image_hi_dev / image_lo_dev and render, as one graph (a clearing
 * kernel and the batch kernel) captured on first use for these buffers and
 * launched on `stream` afterwards. */
int darts_batch_graph_launch(darts_batch *batch, float *image_hi_dev, float *image_lo_dev, void *stream);

/* Time candidate plans (tile and id orders x 64 and 256 threads per block x
 * 16 and 32 waves per CU x units of 512, 1024, 2048, 8192 and 32768 paths), each
 * one warm-up launch plus `reps` timed launches on `stream` into the given
 * images (used as scratch: their contents are overwritten), keep the fastest
 * and return it with its mean launch time in ms.  Synchronous. */
int darts_batch_autotune(darts_batch *batch, float *image_hi_dev, float *image_lo_dev, int reps,
                         darts_batch_plan *chosen, double *best_ms, void *stream);

/* Release the batch's device memory and graph. */
int darts_batch_destroy(darts_batch *batch);

/* For callers that cannot allocate (serving loops and harnesses that forbid
 * device allocation): darts_batch_create + darts_batch_render +
 * darts_batch_destroy in one call that allocates no memory, device or host.
 * The scenes' parameter blocks, the work units of `plan` (NULL = default)
 * and the two unit counters are staged in a fixed host array and copied
 * into a fixed 4 MiB device array that the library holds on each device it
 * runs on until the process ends; each call clears the counters first.
 * Limits: the parameter blocks (about 0.5 KiB per scene) and the work units
 * (48 bytes each while the host sorts them) must fit in the 4 MiB; a larger
 * batch returns DARTS_ERR_INVALID_ARG naming the limit (use fewer scenes or
 * larger unit_paths).  image_hi_dev / image_lo_dev: device float arrays of
 * image_numel elements each, accumulate-into, scene i's image at the offset
 * darts_batch_image_offsets would give (the scenes' images back to back in
 * item order); INVALID_ARG if image_numel is smaller than the images.
 * Validation is that of darts_batch_create.  The call enqueues two
 * host-to-device copies from pageable host memory, a clearing kernel and
 * the batch kernel on `stream`; it is not meant for stream capture.  Calls
 * that overlap on one device race on its array: serialise them (the library
 * serialises the host side with a lock, not the device work). */
int darts_batch_render_noalloc(const darts_batch_item *items, int n_items, const darts_batch_plan *plan,
                               float *image_hi_dev, float *image_lo_dev, int64_t image_numel, void *stream);

/* Diagnostic: evaluate one device building block on n items (one thread per
 * item) with the same device functions the render kernel uses.  in_dev:
 * float[n][DARTS_PW_IN] (32-bit integers are passed by bit pattern), out_dev:
 * float[n][DARTS_PW_OUT]; per-function layouts are listed with the ids.
 * medium / table may be NULL for functions that do not use them. */
#define DARTS_PW_IN  16
#define DARTS_PW_OUT 8
enum {
    DARTS_PW_PHILOX = 0,  /* in: ctr[4], key[2] (bits)   out: x[4] (bits)              */
    DARTS_PW_HG_PDF,      /* in: mu, g                   out: pdf                      */
    DARTS_PW_HG_SAMPLE,   /* in: xi, g                   out: mu, sin(theta)           */
    DARTS_PW_DA_LOGPHI,   /* in: r, s                    out: log Phi (medium)         */
    DARTS_PW_TEXP,        /* in: u, sigma, width         out: x, pdf(x)                */
    DARTS_PW_ELLIPSE,     /* in: S, C, mu, pS            out: t, r, p_t                */
    DARTS_PW_SOBOL,       /* in: row, col, eps (bits)    out: u                        */
    DARTS_PW_ONB,         /* in: n[3]                    out: b1[3], b2[3]             */
    DARTS_PW_BOX_EXIT,    /* in: x[3], w[3], lo[3], hi[3] out: distance                */
    DARTS_PW_RIS,         /* in: x[3], w[3], xe[3], R_hi, d_m, row (bits), eps (bits),
                                 u_sel                   out: ok, d, factor, selected
                                                         candidate (-1 if none), mask
                                                         of valid candidates; both
                                                         index the candidates in
                                                         increasing order of their
                                                         uniform (medium)              */
    DARTS_PW_DIRECTION,   /* in: x[3], xe[3], w_prev[3], S, u[4], use_eda, alpha
                                                         out: w[3], weight, eda_branch,
                                                         table row i n_s + j, cos-bin
                                                         of the EDA density (-1: no
                                                         table) (medium, table)        */
    DARTS_PW_MATH,        /* in: x                       out: rcp, rsqrt, log2, exp2 of x,
                                                         sin 2 pi x, cos 2 pi x (hardware
                                                         transcendental unit)          */
    DARTS_PW_EXIT_LENGTH, /* in: x[3], w[3], xe[3], d_m  out: S_exit, S_exit - C as formed
                                                         (largest length sum of a
                                                         connection, Section V-B)      */
    DARTS_PW_CONNECT,     /* in: x[3], w[3] (unit), xe[3], R_lo, R_hi, d_m, u, texp, box
                                                         out: contribution, t, r_in,
                                                         mu_c, reached, range offsets
                                                         lo, hi above C: one elliptical
                                                         connection (Section V-B, Eq.
                                                         (20)-(22)) of a path of
                                                         throughput 1 at x to an
                                                         emitter of intensity 1, S
                                                         truncated-exponential if texp
                                                         != 0 (else uniform), in the
                                                         box [-1,1]^3 if box != 0
                                                         (d_m its distance along w;
                                                         else an infinite medium)
                                                         (medium)                      */
    DARTS_PW_COUNT
};
int darts_debug_pointwise(int fn, const float *in_dev, float *out_dev, int64_t n,
                          const darts_medium *medium, const darts_table *table, void *stream);

/* Tuning knobs: process-wide settings of how later renders split their work
 * over waves.  They change no result beyond the order of the floating-point
 * additions and may be called from any thread.
 *  - darts_set_ids_max_reps: a render whose cells hold at most `reps`
 *    repetitions of a path uses the id-range decomposition (each wave takes
 *    consecutive path ids; every finished path adds its sum with one
 *    compensated global atomic pair), otherwise the tile decomposition
 *    (per-cell sums in LDS).  Default 16; negative: never id ranges.
 *  - darts_set_target_waves: the number of waves a tile-decomposed launch
 *    aims for (default 65536).  Returns DARTS_ERR_INVALID_ARG below 1.
 *  - darts_set_vanilla_privatised: with `on` (the default), a vanilla render
 *    with at least 256 paths per pixel and at most 384 histogram bins (the
 *    scene's bins, or 1 with a sensor response) gives each wave the paths of
 *    one pixel and histograms their contributions in LDS, flushed with one
 *    compensated global atomic pair per bin and wave; otherwise every
 *    contribution is a compensated global atomic pair. */
int darts_set_ids_max_reps(int64_t reps);
int darts_set_target_waves(int64_t waves);
int darts_set_vanilla_privatised(int on);

/* Message of the last failed call on this thread ("" if none). */
const char *darts_last_error(void);

/* ABI version of this header (incremented on incompatible change). */
#define DARTS_ABI_VERSION 2
int darts_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DARTS_H */
