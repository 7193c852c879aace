/*
 * darts_ref.h -- FP64 CPU oracle for DARTS transient volumetric path tracing
 * (He, Du, Jiang, Jin, "DARTS: Diffusion Approximated Residual Time Sampling
 * for Time-of-flight Rendering in Homogeneous Scattering Media", 2024).
 *
 * TEST INFRASTRUCTURE. This library exists only to check the GPU library
 * against an independent, slow, obviously correct implementation. Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it. It shares no code, header, table or constant generator with the
 * GPU path; the structs below are declared here on their own, with the same
 * field meaning as the GPU library's public header so one set of Python
 * values can drive both.
 *
 * Units: the speed of light and the refractive index are 1, so time and
 * path length are the same quantity (Section III, Eq. (3)).
 */
#ifndef DARTS_REF_H
#define DARTS_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Homogeneous medium (Eq. (9)): scattering / absorption coefficients in
 * 1/length and the Henyey-Greenstein asymmetry g, |g| < 1. */
typedef struct { double sigma_s, sigma_a, g; } ref_medium;

/* Isotropic pulsed point emitter (Section III, Eq. (1)): emission starts at
 * path-length offset `start`; radiant intensity is power / (4 pi). */
typedef struct { double pos[3]; double start; double power; } ref_emitter;

/* kind 0: point fluence detector at origin (ray directions uniform on the
 *         sphere, weight 4 pi);  width = height = 1.
 * kind 1: orthographic radiance sensor: pixel (px,py) covers
 *         origin + [(px, px+1)/width] du + [(py, py+1)/height] dv,
 *         rays travel along dir (unit). */
typedef struct {
    int kind;
    double origin[3], dir[3], du[3], dv[3];
    int width, height;
} ref_sensor;

/* kind 0: infinite medium; kind 1: medium fills the box [lo, hi] with an
 * index-matched boundary (vacuum outside, no refraction); kind 2: the box of
 * kind 1 whose face z = lo[2] is an opaque Lambertian floor of albedo
 * floor_albedo (a fog layer over a diffuse ground; Section V-B, case II). */
typedef struct { int kind; double lo[3], hi[3]; double floor_albedo; } ref_geometry;

/* n_bins half-open path-length bins of equal width over [l_lo, l_hi). */
typedef struct { double l_lo, l_hi; int n_bins; } ref_bins;

typedef struct {
    ref_medium medium;
    ref_geometry geom;
    const ref_emitter *emitters;
    int n_emitters;
    ref_sensor sensor;
    ref_bins bins;
} ref_scene;

/* Elliptical-DA direction table (Section V-A): n_cs cells of C/S in [0,1),
 * n_s cells of S in [0, s_max), n_cos uniform bins of cos(theta) in [-1,1]. */
typedef struct { int n_cs, n_s, n_cos; double s_max; } ref_table_dims;

/* Sampling strategy bits (same values as the GPU library's). */
#define REF_RIS_DIST      0x1u  /* DA distance sampling by RIS, Section IV-C  */
#define REF_EDA_DIR       0x2u  /* EDA direction sampling + MIS, Section V-A  */
#define REF_ELL_TEXP      0x4u  /* truncated-exponential S, Section V-B       */
#define REF_ELL_UNIFORM   0x8u  /* uniform S (temporally uniform baseline)    */
#define REF_DIRECT_REUSE  0x10u /* vanilla: shadow connection + length reuse  */
#define REF_FORWARD       0x20u /* analog walk from the emitter (oracle only) */
#define REF_RESPONSE      0x40u /* general sensor response W (Eq. (4)); the
                                   image is per pixel, see `response`        */

typedef struct {
    uint64_t n_paths, path_offset, seed;
    int max_bounces, n_ris;
    double alpha;
    unsigned flags;
    int mutation; /* 0 in normal use; see REF_MUT_* (planted mistakes for tests) */
    /* With REF_RESPONSE: W(L) piecewise constant on the n_bins segments of the
     * scene's bins, response[k] >= 0, not all zero.  The DARTS family draws
     * each path's target segment with probability proportional to W (from
     * a float CDF: cdf[0] = 0, cdf[k+1] = sum_{j<=k} W_j / sum W accumulated
     * in double and rounded, cdf[n_bins] = 1) and weights it by W_k / (cdf[k+1]
     * - cdf[k]); vanilla weights every connection by W of its length.  Paths
     * map to pixels (id mod pixels) and the image is [height][width]. */
    const double *response;
    /* Test hook for the absorption-scaling invariant (DARTS family only; 0
     * in normal use): every connection's contribution is multiplied by
     * exp(-sigma_a_shift * in-medium length of the connected path), which
     * turns an estimate of the medium (sigma_s, sigma_a) into one of
     * (sigma_s, sigma_a + sigma_a_shift) with the first medium's sampling. */
    double sigma_a_shift;
} ref_params;

/* Planted mistakes. They exist so the test-suite can show that its pins
 * detect a plausible error in the oracle; never set outside tests. */
#define REF_MUT_NONE              0
#define REF_MUT_PRINTED_JACOBIAN  1 /* Eq. (22) Jacobian taken as printed     */
#define REF_MUT_RIS_NO_MEAN       2 /* RIS weight without the mean/selected   */
#define REF_MUT_EDA_PDF_UNSCALED  3 /* EDA pdf missing the solid-angle scale  */
#define REF_MUT_NO_EMITTER_TRANS  4 /* drop transmittance control->emitter    */
#define REF_MUT_HG_SAMPLE_FLIP    5 /* HG sample mirrored (cos -> -cos)       */
#define REF_MUT_GRAD_NO_COUNT     6 /* gradient: drop n / sigma_s              */
#define REF_MUT_RESPONSE_UNWEIGHTED 7 /* response: drop W_k / P(segment k)     */
#define REF_MUT_FLOOR_NO_COSINE   8 /* floor connection without its cosine      */
#define REF_MUT_TABLE_CELL_EDGE   9 /* table rows built at cell edges, not centres */
#define REF_MUT_TABLE_ROW_OFF_BY_ONE 10 /* direction lookup reads the next C/S row */

/* Statistics, uint64 counters. */
enum {
    REF_ST_PATHS = 0, REF_ST_VERTICES, REF_ST_CONNECTIONS, REF_ST_EARLY_EXIT,
    REF_ST_MEDIUM_EXIT, REF_ST_RIS_ALL_INVALID, REF_ST_EDA_BRANCH,
    REF_ST_TRUNCATED, REF_ST_ZERO_PATHS, REF_ST_RIS_INVALID_CANDS,
    /* full path samples (sensor-to-emitter paths produced by a connection)
     * and those the sensor weights with zero (length outside the bins, or
     * W = 0): vanilla connects at every vertex whatever its length; the
     * DARTS family only produces samples inside the target segment */
    REF_ST_SAMPLES, REF_ST_REJECTED,
    REF_ST_COUNT = 16
};

/* ---- pointwise functions (exported so tests can pin them) ---- */
void   ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double ref_u01(uint32_t x);
double ref_hg_pdf(double mu, double g);
double ref_hg_sample_mu(double xi, double g);
void   ref_onb(const double n[3], double b1[3], double b2[3]);
double ref_da_D(const ref_medium *m);
double ref_da_phi(const ref_medium *m, double r, double s);
double ref_da_log_phi(const ref_medium *m, double r, double s);
double ref_texp_sample(double u, double sigma, double width);
double ref_texp_pdf(double x, double sigma, double width);
double ref_ell_t(double S, double C, double mu);
double ref_ell_pdf_t(double pS, double S, double C, double mu, double t, int printed);
double ref_gamma(double kappa, double alpha);
/* Largest length sum S whose control vertex (Eq. (21)) on the ray x + t w
 * stays inside the medium: dm + |x + w dm - xe| (INFINITY for dm = INFINITY). */
double ref_exit_length(const double x[3], const double w[3], const double xe[3], double dm);
double ref_box_exit(const ref_geometry *g, const double x[3], const double w[3]);
/* 1 if the ray (x, w) leaves the medium through the Lambertian floor. */
int    ref_exits_through_floor(const ref_geometry *g, const double x[3], const double w[3]);
int    ref_box_entry(const ref_geometry *g, const double x[3], const double w[3],
                     double *t_in, double *t_out);
double ref_sobol_u(uint32_t row, uint32_t col, uint32_t eps_bits);

/* One elliptical connection (Section V-B, case I, Eq. (20)-(22)) for tests:
 * the ray (x, w unit) from a vertex with residual range [R_lo, R_hi) (target
 * interval minus the length so far) and distance d_m to the boundary along w
 * (INFINITY with geometry kind 0), an emitter of intensity 1 at xe, a path
 * throughput of 1, the uniform u for S, texp != 0 for the truncated
 * exponential S (else uniform).  Returns the contribution (0 when the
 * length-sum range is empty: *reached = 0) and, as the path tracer does,
 * the control vertex's polar distance *t, the in-medium length *r_in from it
 * to the emitter and the phase-function cosine *mu_c. */
double ref_connect(const ref_medium *m, const ref_geometry *g, const double x[3], const double w[3],
                   const double xe[3], double R_lo, double R_hi, double dm, double u, int texp,
                   double *t, double *r_in, double *mu_c, int *reached);

/* One RIS free-flight step (Section IV-C) for a medium event, for tests:
 * inputs x, w (unit), xe, R_hi, d_m; raw uniforms row bits, eps bits, u_sel.
 * Returns 1 and fills d, factor (sigma_s exp(-sigma_t d)/(p_c p(d)) estimate)
 * if a candidate is selected; 0 if all candidates are invalid. */
int ref_ris_step(const ref_medium *m, int n_ris, const double x[3], const double w[3],
                 const double xe[3], double R_hi, double d_m,
                 uint32_t row, uint32_t eps_bits, double u_sel,
                 double *d, double *factor, int mutation);

/* The same step with how close its discrete decisions sat to their
 * boundaries, for parity tests of an implementation in lower precision:
 * mask of valid candidates and selected candidate (-1: none), both indexed
 * in the order of increasing candidate uniform, the smallest
 * |s_i| or |s_i - r_i| over R_hi (validity), and the smallest distance of a
 * running weight sum from u_sel times the total, over the total (pick). */
typedef struct { unsigned mask; int sel; double valid_margin, pick_margin; } ref_ris_detail;
int ref_ris_step_detail(const ref_medium *m, int n_ris, const double x[3], const double w[3],
                        const double xe[3], double R_hi, double d_m,
                        uint32_t row, uint32_t eps_bits, double u_sel,
                        double *d, double *factor, ref_ris_detail *det, int mutation);

/* Integrand of the EDA table for one (C, S) cell (Eq. (17)), integrated over
 * each of n_cos cos-bins with the documented quadrature; out[n_cos]. */
void ref_eda_row_raw(const ref_medium *m, double C, double S, int n_cos, double *out);

/* Full table: pmf (double, [n_cs][n_s][n_cos]) and the float CDF the
 * sampler uses ([n_cs][n_s][n_cos+1]); either output may be NULL. */
int ref_build_da_tables(const ref_medium *m, const ref_table_dims *dims,
                        double *pmf, float *cdf, int n_threads, int mutation);

/* EDA/HG mixture direction sampling (Section V-A, Eq. (19)); for tests. */
void ref_sample_direction(const ref_medium *m, const ref_table_dims *dims, const float *cdf,
                          double alpha, int use_eda, const double x[3], const double xe[3],
                          const double w_prev[3], double S, const double u[4],
                          double w_out[3], double *weight, int *eda_branch, int *bin, int mutation);
/* (bin, may be NULL: the cos-bin whose mass enters the EDA density, -1 when
 * the EDA density is not used) */
/* Row index i n_s + j of the table cell holding (C/S, S). */
int ref_table_row(const ref_table_dims *dims, double C, double S, int mutation);
/* MIS weight phase / mixture density (Eq. (19)) of a given direction w;
 * cos-bin k of the EDA density (k < 0: the bin of w . a). */
double ref_direction_weight(const ref_medium *m, const ref_table_dims *dims, const float *cdf,
                            double alpha, int use_eda, const double x[3], const double xe[3],
                            const double w_prev[3], double S, const double w[3], int k);

/* Render: raw per-cell sums into image[n_bins][height][width] (+= semantics
 * are not used: the oracle writes, the caller accumulates); m2 (may be NULL)
 * receives per-cell sums of squared per-path contributions; stats (may be
 * NULL) receives REF_ST_COUNT counters. Returns 0 or a negative error. */
int ref_render_transient(const ref_scene *sc, const ref_params *pr,
                         const ref_table_dims *dims, const float *cdf,
                         double *image, double *m2, uint64_t *stats, int n_threads);

/* Per-path contributions (DARTS / uniform modes): path_value[i], path_cell[i]
 * for path id path_offset + i. */
int ref_render_paths(const ref_scene *sc, const ref_params *pr,
                     const ref_table_dims *dims, const float *cdf,
                     double *path_value, int64_t *path_cell, int n_threads);

/* Number of vertex steps (vertices that passed the early-exit test) of each
 * path, for work-distribution studies. */
int ref_render_paths_steps(const ref_scene *sc, const ref_params *pr,
                           const ref_table_dims *dims, const float *cdf,
                           int32_t *path_steps, int n_threads);

/* Per-path contributions for an explicit list of path ids. */
int ref_render_path_list(const ref_scene *sc, const ref_params *pr,
                         const ref_table_dims *dims, const float *cdf,
                         const uint64_t *ids, int64_t n, double *path_value, int n_threads);

/* Detached-sampling gradient of L = sum_cells grad_image[cell] * I[cell]
 * with respect to (sigma_s, sigma_a, g): raw sums over paths (divide by the
 * same per-cell path counts as the image). grad_out[3]. */
int ref_render_gradient(const ref_scene *sc, const ref_params *pr,
                        const ref_table_dims *dims, const float *cdf,
                        const double *grad_image, double *grad_out, int n_threads);

#ifdef __cplusplus
}
#endif
#endif
