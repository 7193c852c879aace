/*
 * darts_ref.c -- FP64 CPU oracle for DARTS transient path tracing.
 *
 * TEST INFRASTRUCTURE, not part of the product. It is the slow, plain,
 * double-precision statement of what the GPU library computes, written from
 * the paper (He et al., "DARTS", 2024) and from the published definitions of
 * the generic pieces it uses (Philox4x32-10: Salmon et al., SC'11; orthonormal
 * basis: Duff et al., JCGT 6(1), 2017; Henyey-Greenstein phase function and
 * its inverse CDF; Gauss-Legendre quadrature).  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load this library.
 *
 * Every function follows the steps of the paper in its order and notation.
 * Where the paper is ambiguous or garbled, the reading taken is stated in a
 * comment beside the code (and listed in the design notes of the repository).
 * The numbering of equations below is the order of appearance in the paper.
 *
 * Pinned by the test-suite against: published Philox known-answer vectors;
 * closed forms (diffusion normalisation and steady state, the truncated
 * exponential CDF, the ellipse identity, the analytic single-scattering
 * transient of an infinite isotropic medium); brute-force sampling
 * histograms; independent adaptive quadrature of the EDA integrand; and
 * agreement of independent estimators (DARTS, uniform-S, vanilla shadow
 * connection, forward analog walk).  Order >= 2 contributions have no closed
 * form; they are pinned only by agreement between those independent
 * estimators.
 */
#include "darts_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Small vector helpers                                                      */
/* ------------------------------------------------------------------------- */
static double dot3(const double a[3], const double b[3]) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
static double len3(const double a[3]) { return sqrt(dot3(a, a)); }
static void sub3(const double a[3], const double b[3], double o[3]) { o[0]=a[0]-b[0]; o[1]=a[1]-b[1]; o[2]=a[2]-b[2]; }
static void axpy3(const double x[3], const double w[3], double t, double o[3]) { o[0]=x[0]+w[0]*t; o[1]=x[1]+w[1]*t; o[2]=x[2]+w[2]*t; }
static double dist3(const double a[3], const double b[3]) { double d[3]; sub3(a, b, d); return len3(d); }

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                   */
/* ------------------------------------------------------------------------- */
void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   /* Weyl key schedule */
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 32-bit word -> uniform in [0,1): top 24 bits times 2^-24 (exact in both
 * float and double, so both implementations see the same number). */
double ref_u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* Random-number layout shared with the GPU library (an interface, not code):
 * key = (seed low 32, seed high 32); counter = (path low 32, path high 32,
 * vertex index, stream).  Stream 0 of vertex 0 (where no direction is
 * sampled) drives the camera set-up; stream 0 of vertex k >= 1 the direction
 * at vertex k; stream 1 of vertex k the connection and the free flight from
 * vertex k.  The forward walk uses stream 2 (0xFFFFFFFF for its set-up). */
static void draw(uint64_t seed, uint64_t path, uint32_t vertex, uint32_t stream, uint32_t out[4])
{
    uint32_t ctr[4] = { (uint32_t)path, (uint32_t)(path >> 32), vertex, stream };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    ref_philox4x32_10(ctr, key, out);
}
#define CAMERA_VERTEX 0xFFFFFFFFu

/* ------------------------------------------------------------------------- */
/* Henyey-Greenstein phase function (the paper's phase model, Section IV-B   */
/* and Section VII).                                                         */
/* ------------------------------------------------------------------------- */
double ref_hg_pdf(double mu, double g)
{
    double den = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * PI * den * sqrt(den));
}

/* Inverse of the HG cumulative distribution in mu = cos(theta), increasing
 * in xi, from mu = -1 at xi = 0 to mu = 1 at xi = 1. */
double ref_hg_sample_mu(double xi, double g)
{
    if (g == 0.0) return 2.0 * xi - 1.0;
    double q = (1.0 - g * g) / (1.0 - g + 2.0 * g * xi);
    double mu = (1.0 + g * g - q * q) / (2.0 * g);
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* d/dg of log f_HG(mu; g) = log(1 - g^2) - 1.5 log(1 + g^2 - 2 g mu) + const. */
static double dlog_hg_dg(double mu, double g)
{
    return -2.0 * g / (1.0 - g * g) + 3.0 * (mu - g) / (1.0 + g * g - 2.0 * g * mu);
}

/* Orthonormal basis (b1, b2) completing the unit vector n (Duff et al. 2017,
 * "Building an orthonormal basis, revisited", branchless form). */
void ref_onb(const double n[3], double b1[3], double b2[3])
{
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + sign * n[0] * n[0] * a; b1[1] = sign * b; b1[2] = -sign * n[0];
    b2[0] = b; b2[1] = sign + n[1] * n[1] * a; b2[2] = -n[1];
}

/* Direction with cosine mu to axis n and azimuth phi about it. */
static void from_frame(const double n[3], double mu, double phi, double w[3])
{
    double b1[3], b2[3];
    ref_onb(n, b1, b2);
    double s = sqrt(fmax(0.0, (1.0 - mu) * (1.0 + mu)));
    double cp = cos(phi), sp = sin(phi);
    for (int i = 0; i < 3; ++i) w[i] = s * cp * b1[i] + s * sp * b2[i] + mu * n[i];
}

/* ------------------------------------------------------------------------- */
/* Transient diffusion approximation (Section IV-B, Eq. (9)), c = 1.         */
/* ------------------------------------------------------------------------- */
double ref_da_D(const ref_medium *m)
{
    return 1.0 / (3.0 * (m->sigma_a + m->sigma_s * (1.0 - m->g)));
}

/* Fluence at distance r from the pulse, s = residual time since emission.
 * The Heaviside factor makes it zero for s <= 0 (causality). */
double ref_da_phi(const ref_medium *m, double r, double s)
{
    if (!(s > 0.0)) return 0.0;
    double D = ref_da_D(m);
    double fds = 4.0 * PI * D * s;
    return exp(-r * r / (4.0 * D * s) - m->sigma_a * s) / (fds * sqrt(fds));
}

double ref_da_log_phi(const ref_medium *m, double r, double s)
{
    if (!(s > 0.0)) return -INFINITY;
    double D = ref_da_D(m);
    return -1.5 * log(4.0 * PI * D * s) - r * r / (4.0 * D * s) - m->sigma_a * s;
}

/* ------------------------------------------------------------------------- */
/* Truncated exponential on [0, width) with rate sigma (Eq. (13)-(14); the   */
/* printed sample has the wrong sign, the inverse CDF is used).              */
/* ------------------------------------------------------------------------- */
double ref_texp_sample(double u, double sigma, double width)
{
    double pc = isinf(width) ? 1.0 : -expm1(-sigma * width);
    return -log1p(-pc * u) / sigma;
}

double ref_texp_pdf(double x, double sigma, double width)
{
    if (x < 0.0 || x >= width) return 0.0;
    double pc = isinf(width) ? 1.0 : -expm1(-sigma * width);
    return sigma * exp(-sigma * x) / pc;
}

/* ------------------------------------------------------------------------- */
/* Elliptical connection (Section V-B).                                      */
/* ------------------------------------------------------------------------- */
/* Polar distance from focus x to the ellipse of length sum S whose other
 * focus lies at distance C, along a direction at cosine mu to the focal axis
 * (Eq. (18) and Eq. (21)). */
double ref_ell_t(double S, double C, double mu)
{
    return (S * S - C * C) / (2.0 * S - 2.0 * C * mu);
}

/* Density of t when S has density pS (Eq. (22)).  The text defines it as
 * p(S) (dt/dS)^-1; since dt/dS = (S - t)/(S - C mu) this is
 * p(S) (S - C mu)/(S - t).  The expression printed in the paper is the
 * reciprocal Jacobian; `printed` selects it (only used to show that a test
 * catches it). */
double ref_ell_pdf_t(double pS, double S, double C, double mu, double t, int printed)
{
    if (printed) return pS * (S - t) / (S - C * mu);
    return pS * (S - C * mu) / (S - t);
}

/* Probability of choosing EDA over phase sampling (Eq. (19)). */
double ref_gamma(double kappa, double alpha)
{
    return kappa / (kappa + alpha);
}

/* ------------------------------------------------------------------------- */
/* Geometry: the index-matched box (or an infinite medium).                  */
/* ------------------------------------------------------------------------- */
double ref_box_exit(const ref_geometry *g, const double x[3], const double w[3])
{
    if (g->kind == 0) return INFINITY;
    double t = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (w[a] > 0.0) t = fmin(t, (g->hi[a] - x[a]) / w[a]);
        else if (w[a] < 0.0) t = fmin(t, (g->lo[a] - x[a]) / w[a]);
    }
    return t > 0.0 ? t : 0.0;
}

int ref_exits_through_floor(const ref_geometry *g, const double x[3], const double w[3])
{
    if (g->kind != 2 || !(w[2] < 0.0)) return 0;
    double tz = (g->lo[2] - x[2]) / w[2];
    for (int a = 0; a < 2; ++a) {
        if (w[a] > 0.0 && (g->hi[a] - x[a]) / w[a] < tz) return 0;
        if (w[a] < 0.0 && (g->lo[a] - x[a]) / w[a] < tz) return 0;
    }
    return 1;
}

/* Lambertian floor (normal +z), reached from x along w at distance t_s:
 * the contribution of the path that ends x -> floor point -> emitter
 * (Section V-B, case II: the control vertex is the surface point), with
 * transmittance along both segments, BRDF albedo/pi and the cosine at the
 * floor toward the emitter.  *L_out is the length x -> floor -> emitter and
 * *rin_out the in-medium part of the last segment. */
static double floor_connection(const ref_geometry *g, const double x[3], const double w[3], double t_s,
                               const double xe[3], double sigma_t, int mutation, double *L_out, double *rin_out)
{
    double xs[3], de[3], wc[3];
    axpy3(x, w, t_s, xs);
    xs[2] = g->lo[2];
    sub3(xe, xs, de);
    double r = len3(de);
    *L_out = t_s + r;
    *rin_out = 0.0;
    if (!(r > 0.0)) return 0.0;
    double cos_s = de[2] / r;
    if (!(cos_s > 0.0)) return 0.0;
    for (int i = 0; i < 3; ++i) wc[i] = de[i] / r;
    double r_in = fmin(r, ref_box_exit(g, xs, wc));
    *rin_out = r_in;
    double cosf = mutation == REF_MUT_FLOOR_NO_COSINE ? 1.0 : cos_s;
    return exp(-sigma_t * (t_s + r_in)) * (g->floor_albedo / PI) * cosf / (r * r);
}

int ref_box_entry(const ref_geometry *g, const double x[3], const double w[3],
                  double *t_in, double *t_out)
{
    if (g->kind == 0) { *t_in = 0.0; *t_out = INFINITY; return 1; }
    double tn = -INFINITY, tf = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (w[a] == 0.0) {
            if (x[a] < g->lo[a] || x[a] > g->hi[a]) return 0;
        } else {
            double t1 = (g->lo[a] - x[a]) / w[a], t2 = (g->hi[a] - x[a]) / w[a];
            tn = fmax(tn, fmin(t1, t2));
            tf = fmin(tf, fmax(t1, t2));
        }
    }
    *t_in = fmax(tn, 0.0);
    *t_out = tf;
    return tf > *t_in;
}

/* ------------------------------------------------------------------------- */
/* DA distance sampling by resampled importance sampling (Section IV-C).    */
/* ------------------------------------------------------------------------- */
static uint32_t bitrev32(uint32_t v)
{
    uint32_t r = 0;
    for (int i = 0; i < 32; ++i) { r = (r << 1) | (v & 1u); v >>= 1; }
    return r;
}

/* Candidate uniform: row `row` of the 32 x 8 table holds the base-2 radical
 * inverses (Sobol dimension 1) of indices 8*row .. 8*row+7, so one row hits
 * every eighth of [0,1); a shared random offset eps is added modulo 1.  The
 * sum is taken on 32-bit fixed point so that "modulo 1" is exact. */
double ref_sobol_u(uint32_t row, uint32_t col, uint32_t eps_bits)
{
    uint32_t v = bitrev32(8u * (row & 31u) + (col & 7u)) + eps_bits;
    return ref_u01(v);
}

int ref_ris_step(const ref_medium *m, int n_ris, const double x[3], const double w[3],
                 const double xe[3], double R_hi, double d_m,
                 uint32_t row, uint32_t eps_bits, double u_sel,
                 double *d, double *factor, int mutation)
{
    return ref_ris_step_detail(m, n_ris, x, w, xe, R_hi, d_m, row, eps_bits, u_sel, d, factor, NULL, mutation);
}

int ref_ris_step_detail(const ref_medium *m, int n_ris, const double x[3], const double w[3],
                        const double xe[3], double R_hi, double d_m,
                        uint32_t row, uint32_t eps_bits, double u_sel,
                        double *d, double *factor, ref_ris_detail *det, int mutation)
{
    double st = m->sigma_s + m->sigma_a;
    /* medium-event probability p_m (Eq. (12)); candidates follow the
     * truncated exponential on [0, d_m) (Eq. (13)-(14)). */
    double pc = isinf(d_m) ? 1.0 : -expm1(-st * d_m);
    double dc[8], lphi[8], us[8];
    int valid[8], any = 0;
    double lmax = -INFINITY;
    /* The candidates' uniforms, taken in increasing order: the selection
     * below walks the running weight sum in that order (any fixed order
     * gives the same categorical choice in distribution; this one is the
     * order of increasing distance). */
    for (int i = 0; i < n_ris; ++i) us[i] = ref_sobol_u(row, (uint32_t)i, eps_bits);
    for (int i = 1; i < n_ris; ++i) {
        double v = us[i];
        int j = i - 1;
        while (j >= 0 && us[j] > v) { us[j + 1] = us[j]; --j; }
        us[j + 1] = v;
    }
    for (int i = 0; i < n_ris; ++i) {
        double ui = us[i];
        dc[i] = -log1p(-pc * ui) / st;
        double si = R_hi - dc[i];                 /* upper residual time     */
        double p[3];
        axpy3(x, w, dc[i], p);
        double ri = dist3(p, xe);
        /* A candidate outside the residual-time ellipsoid, or with negative
         * residual, cannot reach the gate: weight zero (Section IV-C). */
        valid[i] = (si > 0.0) && (ri < si);
        /* Target: transmittance times the DA fluence at the upper residual
         * time (Eq. (10)); the candidate pdf cancels the transmittance, so
         * the resampling weight is proportional to the fluence. */
        lphi[i] = valid[i] ? ref_da_log_phi(m, ri, si) : -INFINITY;
        if (valid[i]) { any = 1; if (lphi[i] > lmax) lmax = lphi[i]; }
    }
    if (det) {
        /* how close each discrete decision sat to its boundary: validity
         * (s_i > 0 and r_i < s_i) relative to R_hi */
        det->mask = 0;
        det->valid_margin = INFINITY;
        for (int i = 0; i < n_ris; ++i) {
            double p[3];
            axpy3(x, w, dc[i], p);
            double si = R_hi - dc[i], ri = dist3(p, xe);
            double mg = fmin(fabs(si), fabs(si - ri)) / fabs(R_hi);
            if (mg < det->valid_margin) det->valid_margin = mg;
            if (valid[i]) det->mask |= 1u << i;
        }
        det->sel = -1;
        det->pick_margin = INFINITY;
    }
    if (!any) return 0;
    double wsum = 0.0, wi[8];
    for (int i = 0; i < n_ris; ++i) { wi[i] = valid[i] ? exp(lphi[i] - lmax) : 0.0; wsum += wi[i]; }
    /* Select the first candidate whose running sum exceeds u * total. */
    double target = u_sel * wsum, cum = 0.0;
    int sel = -1;
    for (int i = 0; i < n_ris; ++i) {
        cum += wi[i];
        if (det && fabs(cum - target) / wsum < det->pick_margin) det->pick_margin = fabs(cum - target) / wsum;
        if (cum > target && sel < 0) { sel = i; if (!det) break; }
    }
    if (sel < 0) { for (int i = n_ris - 1; i >= 0; --i) if (wi[i] > 0.0) { sel = i; break; } }
    if (det) det->sel = sel;
    *d = dc[sel];
    /* Unbiased contribution weight of the RIS estimator (Eq. (15), reading
     * p-hat as the numerator of Eq. (10) and summing over the candidates)
     * times sigma_s exp(-sigma_t d) / p_m:  albedo * mean(w) / w_selected. */
    double albedo = m->sigma_s / st;
    *factor = albedo * (wsum / n_ris) / wi[sel];
    if (mutation == REF_MUT_RIS_NO_MEAN) *factor = albedo;
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Elliptical DA direction table (Section V-A, Eq. (16)-(18)).               */
/* ------------------------------------------------------------------------- */
/* Quadrature (the paper integrates by Monte Carlo; a deterministic rule is
 * used instead so that any two implementations agree to rounding): in each
 * cos-bin an N_U-point Gauss-Legendre rule in u = cos(theta); along the ray
 * the substitution v = (1 - exp(-sigma_t t)) / (1 - exp(-sigma_t t_M)) turns
 * sigma_s exp(-sigma_t t) dt into albedo (1 - exp(-sigma_t t_M)) dv, and an
 * N_V-point Gauss-Legendre rule in v on [0,1] is used. */
#define N_U 4
#define N_V 64

/* Gauss-Legendre nodes/weights on [-1,1] by Newton iteration on P_n. */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;           /* P_0, P_1 */
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            /* p1 = P_n(z), p0 = P_{n-1}(z) */
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

void ref_eda_row_raw(const ref_medium *m, double C, double S, int n_cos, double *out)
{
    double xu[N_U], wu[N_U], xv[N_V], wv[N_V];
    gauss_legendre(N_U, xu, wu);
    gauss_legendre(N_V, xv, wv);
    double st = m->sigma_s + m->sigma_a, albedo = m->sigma_s / st;
    double h = 2.0 / n_cos;
    for (int k = 0; k < n_cos; ++k) {
        double lo = -1.0 + k * h, acc = 0.0;
        for (int a = 0; a < N_U; ++a) {
            double u = lo + 0.5 * h * (xu[a] + 1.0);
            double tM = ref_ell_t(S, C, u);          /* Eq. (18) */
            double pM = -expm1(-st * tM);
            double inner = 0.0;
            for (int b = 0; b < N_V; ++b) {
                double v = 0.5 * (xv[b] + 1.0);
                double t = -log1p(-v * pM) / st;
                double r2 = t * t + C * C - 2.0 * t * C * u;
                double r = sqrt(fmax(r2, 0.0));
                /* DA fluence at residual time S - t (Eq. (17)) */
                inner += 0.5 * wv[b] * ref_da_phi(m, r, S - t);
            }
            acc += 0.5 * h * wu[a] * albedo * pM * inner;
        }
        out[k] = acc;
    }
}

int ref_build_da_tables(const ref_medium *m, const ref_table_dims *dm,
                        double *pmf, float *cdf, int n_threads, int mutation)
{
    if (dm->n_cs <= 0 || dm->n_s <= 0 || dm->n_cos <= 0 || !(dm->s_max > 0.0)) return -1;
    int ncell = dm->n_cs * dm->n_s;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
    for (int cell = 0; cell < ncell; ++cell) {
        int i = cell / dm->n_s, j = cell % dm->n_s;
        /* cell centres in C/S and S */
        double off = mutation == REF_MUT_TABLE_CELL_EDGE ? 0.0 : 0.5;
        double kappa = (i + off) / dm->n_cs;
        double S = (j + off) * dm->s_max / dm->n_s;
        double *row = (double *)malloc(sizeof(double) * dm->n_cos);
        ref_eda_row_raw(m, kappa * S, S, dm->n_cos, row);
        double tot = 0.0;
        for (int k = 0; k < dm->n_cos; ++k) tot += row[k];
        int ok = isfinite(tot) && tot > 0.0;
        /* A row whose integrand underflows everywhere falls back to the
         * uniform distribution (any positive pdf keeps the MIS unbiased). */
        for (int k = 0; k < dm->n_cos; ++k) row[k] = ok ? row[k] / tot : 1.0 / dm->n_cos;
        if (pmf) memcpy(pmf + (size_t)cell * dm->n_cos, row, sizeof(double) * dm->n_cos);
        if (cdf) {
            float *c = cdf + (size_t)cell * (dm->n_cos + 1);
            double run = 0.0;
            c[0] = 0.0f;
            for (int k = 0; k < dm->n_cos; ++k) { run += row[k]; c[k + 1] = (float)run; }
            c[dm->n_cos] = 1.0f;
        }
        free(row);
    }
    (void)n_threads;
    return 0;
}

/* Mixture direction sampling at a medium vertex (Section V-A): with
 * probability gamma (Eq. (19)) draw cos(theta) about the axis to the emitter
 * from the table row of (C/S, S) by inverse transform, phi uniform; otherwise
 * draw from the phase function about the previous direction.  The returned
 * weight is phase / (one-sample MIS balance-heuristic pdf). */
/* Row of the direction table for the cell holding (C/S, S): nearest cell,
 * clamped to the table (Section V-A). */
int ref_table_row(const ref_table_dims *dm, double C, double S, int mutation)
{
    int i = (int)floor(C / S * dm->n_cs);
    int j = (int)floor(S / dm->s_max * dm->n_s);
    if (mutation == REF_MUT_TABLE_ROW_OFF_BY_ONE) ++i;
    if (i > dm->n_cs - 1) i = dm->n_cs - 1;
    if (i < 0) i = 0;
    if (j > dm->n_s - 1) j = dm->n_s - 1;
    if (j < 0) j = 0;
    return i * dm->n_s + j;
}

/* The one-sample MIS weight of Eq. (19) for a given direction w: the phase
 * function over the mixture density, with the EDA density of cos-bin k of the
 * table row of (C/S, S) (k < 0: the bin holding w . a). */
double ref_direction_weight(const ref_medium *m, const ref_table_dims *dm, const float *cdf,
                            double alpha, int use_eda, const double x[3], const double xe[3],
                            const double w_prev[3], double S, const double w[3], int k)
{
    double a[3];
    sub3(xe, x, a);
    double C = len3(a);
    for (int i = 0; i < 3; ++i) a[i] /= C;
    double gam = (use_eda && C > 0.0) ? ref_gamma(C / S, alpha) : 0.0;
    double p_hg = ref_hg_pdf(dot3(w_prev, w), m->g);
    if (!(gam > 0.0)) return 1.0;
    const float *row = cdf + (size_t)ref_table_row(dm, C, S, 0) * (dm->n_cos + 1);
    if (k < 0) {
        k = (int)floor((dot3(w, a) + 1.0) * 0.5 * dm->n_cos);
        if (k > dm->n_cos - 1) k = dm->n_cos - 1;
        if (k < 0) k = 0;
    }
    double p_eda = ((double)row[k + 1] - (double)row[k]) * dm->n_cos / (4.0 * PI);
    return p_hg / (gam * p_eda + (1.0 - gam) * p_hg);
}

void ref_sample_direction(const ref_medium *m, const ref_table_dims *dm, const float *cdf,
                          double alpha, int use_eda, const double x[3], const double xe[3],
                          const double w_prev[3], double S, const double u[4],
                          double w_out[3], double *weight, int *eda_branch, int *bin, int mutation)
{
    double a[3];
    sub3(xe, x, a);
    double C = len3(a);
    for (int i = 0; i < 3; ++i) a[i] /= C;
    double gam = (use_eda && C > 0.0) ? ref_gamma(C / S, alpha) : 0.0;
    const float *row = NULL;
    if (gam > 0.0) row = cdf + (size_t)ref_table_row(dm, C, S, mutation) * (dm->n_cos + 1);
    int k = -1;
    *eda_branch = 0;
    if (u[0] < gam) {
        /* inverse transform over the cos-bins: largest k with cdf[k] <= u */
        k = 0;
        while (k + 1 < dm->n_cos && (double)row[k + 1] <= u[1]) ++k;
        double mu = -1.0 + (k + u[3]) * (2.0 / dm->n_cos);
        from_frame(a, mu, 2.0 * PI * u[2], w_out);
        *eda_branch = 1;
    } else {
        double mu = ref_hg_sample_mu(u[1], m->g);
        if (mutation == REF_MUT_HG_SAMPLE_FLIP) mu = -mu;
        from_frame(w_prev, mu, 2.0 * PI * u[2], w_out);
        if (gam > 0.0) {
            k = (int)floor((dot3(w_out, a) + 1.0) * 0.5 * dm->n_cos);
            if (k > dm->n_cos - 1) k = dm->n_cos - 1;
            if (k < 0) k = 0;
        }
    }
    double p_hg = ref_hg_pdf(dot3(w_prev, w_out), m->g);
    double p_eda = 0.0;
    if (gam > 0.0) {
        double pk = (double)row[k + 1] - (double)row[k];
        /* cos(theta) uniform in a bin of width 2/n_cos, phi uniform: solid-angle
         * density pk * n_cos / (4 pi). */
        p_eda = (mutation == REF_MUT_EDA_PDF_UNSCALED) ? pk : pk * dm->n_cos / (4.0 * PI);
    }
    *weight = p_hg / (gam * p_eda + (1.0 - gam) * p_hg);
    if (bin) *bin = k;
}

/* ------------------------------------------------------------------------- */
/* Path construction                                                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    double x[3], w[3];   /* current vertex and walk direction            */
    double beta;         /* throughput / pdf so far                       */
    double Le;           /* path length from the sensor to x              */
    double G_lo, G_hi;   /* target interval of total path length          */
    const ref_emitter *em;
    double J;            /* 1 / probability of choosing this emitter       */
    int64_t cell, pixel;
    double dm0;          /* distance to the medium boundary along w at x  */
    int alive;
} path_state;

/* Segment k of a piecewise-constant sensor response drawn by inverse
 * transform from its float CDF (cdf[0] = 0, cdf[k+1] = running double sum of
 * W_j / sum W rounded to float, cdf[n] = 1): the largest k with cdf[k] <= u.
 * *weight = W_k / (cdf[k+1] - cdf[k]), the response over the probability. */
static int64_t response_segment(int n, const double *W, double u, double *weight)
{
    double tot = 0.0;
    for (int k = 0; k < n; ++k) tot += W[k];
    double run = 0.0;
    float lo = 0.0f;
    for (int k = 0; k < n; ++k) {
        run += W[k];
        float hi = (k == n - 1) ? 1.0f : (float)(run / tot);
        if (u < (double)hi && (double)lo <= u) {
            *weight = W[k] / ((double)hi - (double)lo);
            return k;
        }
        lo = hi;
    }
    *weight = 0.0;   /* not reached: u < 1 = cdf[n] */
    return n - 1;
}

/* Path set-up (Section III and Section V-A): stratified target interval,
 * camera ray, emitter choice, entry into the medium. */
static void setup_path(const ref_scene *sc, const ref_params *pr, uint64_t p, path_state *ps, int vanilla)
{
    const ref_sensor *sn = &sc->sensor;
    const int response = (pr->flags & REF_RESPONSE) != 0;
    int64_t npix = (int64_t)sn->width * sn->height;
    int64_t ncells = response ? npix : npix * sc->bins.n_bins;
    ps->cell = (int64_t)(p % (uint64_t)ncells);
    ps->pixel = ps->cell % npix;
    int64_t b = ps->cell / npix;
    uint32_t r[4];
    draw(pr->seed, p, 0u, 0, r);
    double u0 = ref_u01(r[0]), u1 = ref_u01(r[1]), u2 = ref_u01(r[2]);
    double resp_weight = 1.0;
    if (response && !vanilla) {
        /* target segment drawn with probability proportional to W (Eq. (4):
         * the estimator of the W-weighted integral picks the interval to
         * sample and divides by its probability) */
        b = response_segment(sc->bins.n_bins, pr->response, ref_u01(r[3]), &resp_weight);
        if (pr->mutation == REF_MUT_RESPONSE_UNWEIGHTED) resp_weight = 1.0;
    }
    double pos[3], w[3];
    if (sn->kind == 1) {
        int px = (int)(ps->pixel % sn->width), py = (int)(ps->pixel / sn->width);
        double fu = (px + u0) / sn->width, fv = (py + u1) / sn->height;
        for (int i = 0; i < 3; ++i) pos[i] = sn->origin[i] + fu * sn->du[i] + fv * sn->dv[i];
        double l = len3(sn->dir);
        for (int i = 0; i < 3; ++i) w[i] = sn->dir[i] / l;
        ps->beta = 1.0;                           /* radiance sensor        */
    } else {
        for (int i = 0; i < 3; ++i) pos[i] = sn->origin[i];
        double mu = 1.0 - 2.0 * u0, phi = 2.0 * PI * u1;
        double s = sqrt(fmax(0.0, (1.0 - mu) * (1.0 + mu)));
        w[0] = s * cos(phi); w[1] = s * sin(phi); w[2] = mu;
        ps->beta = 4.0 * PI;                      /* fluence: 1 / (1/4pi)   */
    }
    int j = (int)floor(u2 * sc->n_emitters);
    if (j > sc->n_emitters - 1) j = sc->n_emitters - 1;
    ps->em = &sc->emitters[j];
    ps->J = (double)sc->n_emitters * resp_weight;
    double delta = (sc->bins.l_hi - sc->bins.l_lo) / sc->bins.n_bins;
    if (vanilla) {
        ps->G_lo = sc->bins.l_lo - ps->em->start;
        ps->G_hi = sc->bins.l_hi - ps->em->start;
    } else {
        ps->G_lo = sc->bins.l_lo + b * delta - ps->em->start;
        ps->G_hi = sc->bins.l_lo + (b + 1) * delta - ps->em->start;
    }
    double t_in, t_out;
    ps->alive = ref_box_entry(&sc->geom, pos, w, &t_in, &t_out);
    if (!ps->alive) return;
    axpy3(pos, w, t_in, ps->x);
    for (int i = 0; i < 3; ++i) ps->w[i] = w[i];
    ps->Le = t_in;
    ps->dm0 = t_out - t_in;
}

typedef struct {
    uint64_t st[REF_ST_COUNT];
} ref_stats;

/* Largest reachable length sum (Section V-B, case II, boundary clipping S_M):
 * the control vertex must stay inside the medium, so the longest connected
 * path leaves the ray at the boundary point x + w d_m and goes straight to
 * the emitter: S_exit = d_m + |x + w d_m - x_e|.  Infinite for an unbounded
 * medium. */
double ref_exit_length(const double x[3], const double w[3], const double xe[3], double dm)
{
    if (isinf(dm)) return INFINITY;
    double pb[3];
    axpy3(x, w, dm, pb);
    return dm + dist3(pb, xe);
}

/* Generalised shadow connection through a control vertex on the current
 * ray (Section V-B, case I; Eq. (21)-(22)).  Returns the contribution. */
static double connect_elliptical(const ref_scene *sc, const ref_params *pr, const path_state *ps,
                                 double dm, double u4, double *t_out, double *rin_out, double *mu_c_out,
                                 int *reached)
{
    *t_out = 0.0; *rin_out = 0.0; *mu_c_out = 0.0; *reached = 0;
    const ref_medium *m = &sc->medium;
    double st = m->sigma_s + m->sigma_a;
    double de[3];
    sub3(ps->em->pos, ps->x, de);
    double C = len3(de);
    if (!(C > 0.0)) return 0.0;
    double mu = dot3(ps->w, de) / C;          /* cos to the focal axis */
    double R_lo = ps->G_lo - ps->Le, R_hi = ps->G_hi - ps->Le;
    double S_exit = ref_exit_length(ps->x, ps->w, ps->em->pos, dm);
    double S_lo = fmax(R_lo, C), S_hi = fmin(R_hi, S_exit);
    if (!(S_lo < S_hi)) return 0.0;
    *reached = 1;
    double width = S_hi - S_lo, S, pS;
    if (pr->flags & REF_ELL_TEXP) {
        S = S_lo + ref_texp_sample(u4, st, width);
        pS = ref_texp_pdf(S - S_lo, st, width);
    } else {
        S = S_lo + u4 * width;
        pS = 1.0 / width;
    }
    double t = ref_ell_t(S, C, mu);
    double r = S - t;
    double pt = ref_ell_pdf_t(pS, S, C, mu, t, pr->mutation == REF_MUT_PRINTED_JACOBIAN);
    double xc[3], wc[3], dv[3];
    axpy3(ps->x, ps->w, t, xc);
    sub3(ps->em->pos, xc, dv);
    double rv = len3(dv);                      /* equals r = S - t up to rounding */
    for (int i = 0; i < 3; ++i) wc[i] = dv[i] / rv;
    double r_in = fmin(r, ref_box_exit(&sc->geom, xc, wc));
    double Ie = ps->em->power / (4.0 * PI);
    double trans = exp(-st * t) * (pr->mutation == REF_MUT_NO_EMITTER_TRANS ? 1.0 : exp(-st * r_in));
    *t_out = t; *rin_out = r_in; *mu_c_out = dot3(ps->w, wc);
    return ps->beta * ps->J * m->sigma_s * ref_hg_pdf(dot3(ps->w, wc), m->g) * trans * Ie / (r * r * pt);
}

/* One connection through the same code, for tests: a scene holding the
 * medium, the geometry and one emitter of power 4 pi (intensity 1) at xe, a
 * path of throughput 1 and emitter weight 1 at x heading along w with length
 * 0 so far and target interval [R_lo, R_hi). */
double ref_connect(const ref_medium *m, const ref_geometry *g, const double x[3], const double w[3],
                   const double xe[3], double R_lo, double R_hi, double dm, double u, int texp,
                   double *t, double *r_in, double *mu_c, int *reached)
{
    ref_emitter em;
    for (int i = 0; i < 3; ++i) em.pos[i] = xe[i];
    em.start = 0.0;
    em.power = 4.0 * PI;
    ref_scene sc;
    memset(&sc, 0, sizeof sc);
    sc.medium = *m;
    sc.geom = *g;
    sc.emitters = &em;
    sc.n_emitters = 1;
    ref_params pr;
    memset(&pr, 0, sizeof pr);
    pr.flags = texp ? REF_ELL_TEXP : REF_ELL_UNIFORM;
    path_state ps;
    memset(&ps, 0, sizeof ps);
    for (int i = 0; i < 3; ++i) { ps.x[i] = x[i]; ps.w[i] = w[i]; }
    ps.beta = 1.0;
    ps.Le = 0.0;
    ps.G_lo = R_lo;
    ps.G_hi = R_hi;
    ps.em = &em;
    ps.J = 1.0;
    ps.dm0 = dm;
    ps.alive = 1;
    return connect_elliptical(&sc, &pr, &ps, dm, u, t, r_in, mu_c, reached);
}

/* Direction leaving the Lambertian floor: cosine-weighted about +z
 * (cos theta = sqrt(u1), phi = 2 pi u2); the BRDF-to-pdf ratio is the albedo. */
static void floor_direction(double u1, double u2, double w[3])
{
    double ct = sqrt(u1), sn = sqrt(fmax(0.0, 1.0 - u1)), phi = 2.0 * PI * u2;
    w[0] = sn * cos(phi); w[1] = sn * sin(phi); w[2] = ct;
}

/* DARTS family (DARTS, uniform-S baseline and the ablation arms): one path,
 * following the recursive residual-time estimator (Eq. (6)-(7)): at every
 * vertex a control-vertex connection, then a free flight. */
/* When grad is not NULL, grad[0..2] receives the sum over the path's
 * connections of contribution x d log f / d(sigma_s, sigma_a, g), f the
 * throughput of the connected path (sigma_s per scattering vertex,
 * exp(-sigma_t x in-medium length), one phase function per scattering
 * vertex): the detached-sampling derivative of the estimate. */
static double trace_darts(const ref_scene *sc, const ref_params *pr, const ref_table_dims *dm_t,
                          const float *cdf, uint64_t p, int64_t *cell, ref_stats *S, double *grad)
{
    double L_med = 0.0, dlg = 0.0;   /* in-medium walk length; sum of dlog f_HG/dg */
    if (grad) { grad[0] = grad[1] = grad[2] = 0.0; }
    const ref_medium *m = &sc->medium;
    double st = m->sigma_s + m->sigma_a;
    path_state ps;
    setup_path(sc, pr, p, &ps, 0);
    *cell = ps.cell;
    S->st[REF_ST_PATHS]++;
    double acc = 0.0;
    if (!ps.alive) { S->st[REF_ST_ZERO_PATHS]++; return 0.0; }
    double dm = ps.dm0;
    const ref_geometry *geo = &sc->geom;
    int on_floor = 0, n_surf = 0;   /* current vertex on the floor; floor vertices so far */
    double Ie = ps.em->power / (4.0 * PI);
    for (int k = 0; k < pr->max_bounces; ++k) {
        S->st[REF_ST_VERTICES]++;
        double C = dist3(ps.em->pos, ps.x);
        double R_hi = ps.G_hi - ps.Le;
        /* early exit: nothing on or beyond the current vertex can close a
         * path shorter than the gate's upper end (Section V-B). */
        if (R_hi <= C) { S->st[REF_ST_EARLY_EXIT]++; break; }
        if (k >= 1) {
            uint32_t r0[4];
            draw(pr->seed, p, (uint32_t)k, 0, r0);
            double u[4] = { ref_u01(r0[0]), ref_u01(r0[1]), ref_u01(r0[2]), ref_u01(r0[3]) };
            double wn[3], weight;
            if (on_floor) {
                floor_direction(u[1], u[2], wn);
                weight = geo->floor_albedo;
                on_floor = 0;
            } else {
                int eb;
                ref_sample_direction(m, dm_t, cdf, pr->alpha, (pr->flags & REF_EDA_DIR) != 0,
                                     ps.x, ps.em->pos, ps.w, R_hi, u, wn, &weight, &eb, NULL, pr->mutation);
                S->st[REF_ST_EDA_BRANCH] += (uint64_t)eb;
                dlg += dlog_hg_dg(dot3(ps.w, wn), m->g);
            }
            for (int i = 0; i < 3; ++i) ps.w[i] = wn[i];
            ps.beta *= weight;
            dm = ref_box_exit(&sc->geom, ps.x, ps.w);
        }
        uint32_t r1[4];
        draw(pr->seed, p, (uint32_t)k, 1, r1);
        double tc, rin, muc;
        int reached;
        double c = connect_elliptical(sc, pr, &ps, dm, ref_u01(r1[0]), &tc, &rin, &muc, &reached);
        /* a full path sample exists when a control vertex can close the
         * path; its length lies in the target segment, where W > 0 */
        if (reached) S->st[REF_ST_SAMPLES]++;
        if (pr->sigma_a_shift != 0.0) c *= exp(-pr->sigma_a_shift * (L_med + tc + rin));
        if (c != 0.0) {
            S->st[REF_ST_CONNECTIONS]++;
            if (grad) {
                double Lm = L_med + tc + rin;
                /* medium scattering vertices: the walk's (floor vertices
                 * excluded) plus the control vertex */
                double n_sc = pr->mutation == REF_MUT_GRAD_NO_COUNT ? 0.0 : (double)(k + 1 - n_surf);
                grad[0] += c * (n_sc / m->sigma_s - Lm);
                grad[1] += c * (-Lm);
                grad[2] += c * (dlg + dlog_hg_dg(muc, m->g));
            }
        }
        acc += c;
        if (ref_exits_through_floor(geo, ps.x, ps.w)) {
            /* case II: the ray meets the floor at t_s = dm; the floor point
             * closes a path of fixed length, which counts if it falls in
             * the target interval */
            double Lp, rin_s;
            double fc = floor_connection(geo, ps.x, ps.w, dm, ps.em->pos, st, pr->mutation, &Lp, &rin_s);
            double L = ps.Le + Lp;
            S->st[REF_ST_SAMPLES]++;
            if (L >= ps.G_lo && L < ps.G_hi) {
                double cs = ps.beta * ps.J * Ie * fc;
                if (pr->sigma_a_shift != 0.0) cs *= exp(-pr->sigma_a_shift * (L_med + dm + rin_s));
                if (cs != 0.0) {
                    S->st[REF_ST_CONNECTIONS]++;
                    if (grad) {
                        double Lm = L_med + dm + rin_s;
                        double n_sc = pr->mutation == REF_MUT_GRAD_NO_COUNT ? 0.0 : (double)(k - n_surf);
                        grad[0] += cs * (n_sc / m->sigma_s - Lm);
                        grad[1] += cs * (-Lm);
                        grad[2] += cs * dlg;
                    }
                }
                acc += cs;
            } else {
                S->st[REF_ST_REJECTED]++;
            }
        }
        if (k == pr->max_bounces - 1) { S->st[REF_ST_TRUNCATED]++; break; }
        /* free flight: medium-event Bernoulli (Eq. (12)) */
        double pc = isinf(dm) ? 1.0 : -expm1(-st * dm);
        double u5 = ref_u01(r1[1]);
        if (!(u5 < pc)) {
            if (!ref_exits_through_floor(geo, ps.x, ps.w)) { S->st[REF_ST_MEDIUM_EXIT]++; break; }
            /* surface event (probability e^{-sigma_t d_m}, equal to the
             * transmittance: the throughput is unchanged) */
            axpy3(ps.x, ps.w, dm, ps.x);
            ps.x[2] = geo->lo[2];
            ps.Le += dm;
            L_med += dm;
            on_floor = 1;
            ++n_surf;
            continue;
        }
        double d, factor;
        if (pr->flags & REF_RIS_DIST) {
            if (!ref_ris_step(m, pr->n_ris, ps.x, ps.w, ps.em->pos, R_hi, dm,
                              r1[1] & 31u, r1[2], ref_u01(r1[3]), &d, &factor, pr->mutation)) {
                S->st[REF_ST_RIS_ALL_INVALID]++;
                break;
            }
        } else {
            /* plain exponential free flight given a medium event */
            d = -log1p(-u5) / st;
            factor = m->sigma_s / st;
        }
        axpy3(ps.x, ps.w, d, ps.x);
        ps.Le += d;
        L_med += d;
        ps.beta *= factor;
        dm = ref_box_exit(&sc->geom, ps.x, ps.w);
    }
    if (acc == 0.0) S->st[REF_ST_ZERO_PATHS]++;
    return acc;
}

/* Per-path sparse histogram for modes whose path scatters into many bins. */
typedef struct { double *val; unsigned char *mark; int *touched; int n_touched; } bin_scratch;

static void scratch_add(bin_scratch *bs, int bin, double v)
{
    if (!bs->mark[bin]) { bs->mark[bin] = 1; bs->touched[bs->n_touched++] = bin; }
    bs->val[bin] += v;
}

/* Vanilla transient path tracing (Section V-B "vanilla", Section VI):
 * exponential free flight, phase sampling, a shadow connection to the
 * emitter at every medium vertex, the path binned by its length. */
static void trace_vanilla(const ref_scene *sc, const ref_params *pr, uint64_t p,
                          bin_scratch *bs, int64_t *pixel, ref_stats *S)
{
    const ref_medium *m = &sc->medium;
    double st = m->sigma_s + m->sigma_a;
    path_state ps;
    setup_path(sc, pr, p, &ps, 1);
    *pixel = ps.pixel;
    S->st[REF_ST_PATHS]++;
    if (!ps.alive) { S->st[REF_ST_ZERO_PATHS]++; return; }
    double delta = (sc->bins.l_hi - sc->bins.l_lo) / sc->bins.n_bins;
    double Ie = ps.em->power / (4.0 * PI);
    double dm = ps.dm0;
    int any = 0;
    const int response = (pr->flags & REF_RESPONSE) != 0;
    const ref_geometry *geo = &sc->geom;
    int on_floor = 0;   /* current vertex on the Lambertian floor */
    for (int k = 0; k <= pr->max_bounces; ++k) {
        S->st[REF_ST_VERTICES]++;
        if (k >= 1) {
            double de[3];
            sub3(ps.em->pos, ps.x, de);
            double r = len3(de), wc[3];
            for (int i = 0; i < 3; ++i) wc[i] = de[i] / r;
            double r_in = fmin(r, ref_box_exit(&sc->geom, ps.x, wc));
            /* local scattering toward the emitter: phase function in the
             * medium, BRDF times cosine on the floor */
            double fl = on_floor ? (wc[2] > 0.0 ? geo->floor_albedo / PI *
                                    (pr->mutation == REF_MUT_FLOOR_NO_COSINE ? 1.0 : wc[2]) : 0.0)
                                 : ref_hg_pdf(dot3(ps.w, wc), m->g);
            double L = ps.Le + r + ps.em->start;       /* arrival time */
            int bin = (int)floor((L - sc->bins.l_lo) / delta);
            S->st[REF_ST_SAMPLES]++;
            if (L >= sc->bins.l_lo && bin >= 0 && bin < sc->bins.n_bins) {
                /* sensor weight: the bin indicator, or W of the length */
                double wsens = response ? pr->response[bin] : 1.0;
                double v = wsens * ps.beta * ps.J * fl * exp(-st * r_in) * Ie / (r * r);
                if (wsens > 0.0) {
                    scratch_add(bs, response ? 0 : bin, v);
                    S->st[REF_ST_CONNECTIONS]++;
                    any = 1;
                } else {
                    S->st[REF_ST_REJECTED]++;
                }
            } else {
                S->st[REF_ST_REJECTED]++;
            }
        }
        if (k == pr->max_bounces) { S->st[REF_ST_TRUNCATED]++; break; }
        double C = dist3(ps.em->pos, ps.x);
        if (ps.G_hi - ps.Le <= C) { S->st[REF_ST_EARLY_EXIT]++; break; }
        uint32_t r1[4];
        if (k >= 1) {
            uint32_t r0[4];
            draw(pr->seed, p, (uint32_t)k, 0, r0);
            double wn[3];
            if (on_floor) {
                floor_direction(ref_u01(r0[1]), ref_u01(r0[2]), wn);
                ps.beta *= geo->floor_albedo;
                on_floor = 0;
            } else {
                double mu = ref_hg_sample_mu(ref_u01(r0[1]), m->g);
                from_frame(ps.w, mu, 2.0 * PI * ref_u01(r0[2]), wn);
            }
            for (int i = 0; i < 3; ++i) ps.w[i] = wn[i];
            dm = ref_box_exit(&sc->geom, ps.x, ps.w);
        }
        draw(pr->seed, p, (uint32_t)k, 1, r1);
        double pc = isinf(dm) ? 1.0 : -expm1(-st * dm);
        double u5 = ref_u01(r1[1]);
        if (!(u5 < pc)) {
            if (!ref_exits_through_floor(geo, ps.x, ps.w)) { S->st[REF_ST_MEDIUM_EXIT]++; break; }
            axpy3(ps.x, ps.w, dm, ps.x);     /* surface event on the floor */
            ps.x[2] = geo->lo[2];
            ps.Le += dm;
            on_floor = 1;
            continue;
        }
        double d = -log1p(-u5) / st;
        axpy3(ps.x, ps.w, d, ps.x);
        ps.Le += d;
        ps.beta *= m->sigma_s / st;
        dm = ref_box_exit(&sc->geom, ps.x, ps.w);
    }
    if (!any) S->st[REF_ST_ZERO_PATHS]++;
}

/* Forward analog walk from the emitter with a point-detector estimate at
 * every collision (independent of all sampling above; point detector only). */
static void trace_forward(const ref_scene *sc, const ref_params *pr, uint64_t p,
                          bin_scratch *bs, ref_stats *S)
{
    const ref_medium *m = &sc->medium;
    double st = m->sigma_s + m->sigma_a, albedo = m->sigma_s / st;
    double delta = (sc->bins.l_hi - sc->bins.l_lo) / sc->bins.n_bins;
    const double *xd = sc->sensor.origin;
    uint32_t r[4];
    draw(pr->seed, p, CAMERA_VERTEX, 2, r);
    int j = (int)floor(ref_u01(r[2]) * sc->n_emitters);
    if (j > sc->n_emitters - 1) j = sc->n_emitters - 1;
    const ref_emitter *em = &sc->emitters[j];
    double x[3], w[3];
    double mu0 = 1.0 - 2.0 * ref_u01(r[0]), phi0 = 2.0 * PI * ref_u01(r[1]);
    double s0 = sqrt(fmax(0.0, (1.0 - mu0) * (1.0 + mu0)));
    w[0] = s0 * cos(phi0); w[1] = s0 * sin(phi0); w[2] = mu0;
    double wt = em->power * sc->n_emitters;
    double ell = 0.0, t_in, t_out;
    S->st[REF_ST_PATHS]++;
    if (!ref_box_entry(&sc->geom, em->pos, w, &t_in, &t_out)) { S->st[REF_ST_ZERO_PATHS]++; return; }
    axpy3(em->pos, w, t_in, x);
    ell = t_in;
    double dm = t_out - t_in;
    for (int k = 1; k <= pr->max_bounces; ++k) {
        S->st[REF_ST_VERTICES]++;
        draw(pr->seed, p, (uint32_t)k, 2, r);
        double d = -log1p(-ref_u01(r[0])) / st;
        if (d >= dm) { S->st[REF_ST_MEDIUM_EXIT]++; break; }
        axpy3(x, w, d, x);
        ell += d;
        double dd[3];
        sub3(xd, x, dd);
        double rr = len3(dd);
        if (ell + rr + em->start >= sc->bins.l_hi) { S->st[REF_ST_EARLY_EXIT]++; break; }
        double wd[3];
        for (int i = 0; i < 3; ++i) wd[i] = dd[i] / rr;
        double r_in = fmin(rr, ref_box_exit(&sc->geom, x, wd));
        double L = ell + rr + em->start;
        if (L >= sc->bins.l_lo) {
            int bin = (int)floor((L - sc->bins.l_lo) / delta);
            if (bin >= 0 && bin < sc->bins.n_bins) {
                scratch_add(bs, bin, wt * albedo * ref_hg_pdf(dot3(w, wd), m->g) * exp(-st * r_in) / (rr * rr));
                S->st[REF_ST_CONNECTIONS]++;
            }
        }
        wt *= albedo;
        double mu = ref_hg_sample_mu(ref_u01(r[1]), m->g), wn[3];
        from_frame(w, mu, 2.0 * PI * ref_u01(r[2]), wn);
        for (int i = 0; i < 3; ++i) w[i] = wn[i];
        dm = ref_box_exit(&sc->geom, x, w);
        if (k == pr->max_bounces) S->st[REF_ST_TRUNCATED]++;
    }
}

/* ------------------------------------------------------------------------- */
/* Entry points                                                               */
/* ------------------------------------------------------------------------- */
static int check_args(const ref_scene *sc, const ref_params *pr)
{
    const ref_medium *m = &sc->medium;
    if (!(m->sigma_s >= 0.0) || !(m->sigma_a >= 0.0) || !(m->sigma_s + m->sigma_a > 0.0)) return -1;
    if (!(fabs(m->g) < 1.0)) return -1;
    if (sc->n_emitters <= 0 || !sc->emitters) return -1;
    if (sc->bins.n_bins <= 0 || !(sc->bins.l_hi > sc->bins.l_lo)) return -1;
    if (sc->sensor.width <= 0 || sc->sensor.height <= 0) return -1;
    if (pr->max_bounces <= 0 || pr->n_ris < 1 || pr->n_ris > 8) return -1;
    if (sc->geom.kind < 0 || sc->geom.kind > 2) return -1;
    if (sc->geom.kind == 2 && !(sc->geom.floor_albedo >= 0.0 && sc->geom.floor_albedo <= 1.0)) return -1;
    unsigned f = pr->flags;
    if ((f & REF_FORWARD) && sc->geom.kind == 2) return -1;   /* the analog walk has no floor */
    if (f & REF_RESPONSE) {
        if (!pr->response || (f & REF_FORWARD)) return -1;
        double tot = 0.0;
        for (int k = 0; k < sc->bins.n_bins; ++k) {
            if (!(pr->response[k] >= 0.0) || isinf(pr->response[k])) return -1;
            tot += pr->response[k];
        }
        if (!(tot > 0.0)) return -1;
        f &= ~REF_RESPONSE;
    }
    if (f & REF_FORWARD) { if (sc->sensor.kind != 0) return -1; return 0; }
    if (f & REF_DIRECT_REUSE) return 0;
    if (((f & REF_ELL_TEXP) != 0) == ((f & REF_ELL_UNIFORM) != 0)) return -1;
    return 0;
}

static int nthreads_eff(int n)
{
#ifdef _OPENMP
    return n > 0 ? n : omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

int ref_render_paths_steps(const ref_scene *sc, const ref_params *pr,
                           const ref_table_dims *dims, const float *cdf,
                           int32_t *path_steps, int n_threads)
{
    if (check_args(sc, pr)) return -1;
    if (pr->flags & (REF_DIRECT_REUSE | REF_FORWARD)) return -1;
    int nt = nthreads_eff(n_threads);
    int64_t n = (int64_t)pr->n_paths;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i) {
        ref_stats S;
        memset(&S, 0, sizeof S);
        int64_t cell;
        trace_darts(sc, pr, dims, cdf, pr->path_offset + (uint64_t)i, &cell, &S, NULL);
        path_steps[i] = (int32_t)(S.st[REF_ST_VERTICES] - S.st[REF_ST_EARLY_EXIT]);
    }
    (void)nt;
    return 0;
}

int ref_render_paths(const ref_scene *sc, const ref_params *pr,
                     const ref_table_dims *dims, const float *cdf,
                     double *path_value, int64_t *path_cell, int n_threads)
{
    if (check_args(sc, pr)) return -1;
    if (pr->flags & (REF_DIRECT_REUSE | REF_FORWARD)) return -1;
    if ((pr->flags & REF_EDA_DIR) && (!cdf || !dims)) return -1;
    int nt = nthreads_eff(n_threads);
    int64_t n = (int64_t)pr->n_paths;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i) {
        ref_stats S;
        memset(&S, 0, sizeof S);
        int64_t cell;
        path_value[i] = trace_darts(sc, pr, dims, cdf, pr->path_offset + (uint64_t)i, &cell, &S, NULL);
        path_cell[i] = cell;
    }
    (void)nt;
    return 0;
}

int ref_render_path_list(const ref_scene *sc, const ref_params *pr,
                         const ref_table_dims *dims, const float *cdf,
                         const uint64_t *ids, int64_t n, double *path_value, int n_threads)
{
    if (check_args(sc, pr)) return -1;
    if (pr->flags & (REF_DIRECT_REUSE | REF_FORWARD)) return -1;
    if ((pr->flags & REF_EDA_DIR) && (!cdf || !dims)) return -1;
    int nt = nthreads_eff(n_threads);
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        ref_stats S;
        memset(&S, 0, sizeof S);
        int64_t cell;
        path_value[i] = trace_darts(sc, pr, dims, cdf, ids[i], &cell, &S, NULL);
    }
    (void)nt;
    return 0;
}

int ref_render_transient(const ref_scene *sc, const ref_params *pr,
                         const ref_table_dims *dims, const float *cdf,
                         double *image, double *m2, uint64_t *stats, int n_threads)
{
    if (check_args(sc, pr)) return -1;
    if ((pr->flags & REF_EDA_DIR) && !(pr->flags & (REF_DIRECT_REUSE | REF_FORWARD)) && (!cdf || !dims)) return -1;
    int nt = nthreads_eff(n_threads);
    int64_t npix = (int64_t)sc->sensor.width * sc->sensor.height;
    int B = sc->bins.n_bins;
    int64_t ncells = (pr->flags & REF_RESPONSE) ? npix : npix * B;   /* response: one value per pixel */
    int64_t n = (int64_t)pr->n_paths;
    memset(image, 0, sizeof(double) * (size_t)ncells);
    if (m2) memset(m2, 0, sizeof(double) * (size_t)ncells);
    ref_stats tot;
    memset(&tot, 0, sizeof tot);

    if (!(pr->flags & (REF_DIRECT_REUSE | REF_FORWARD))) {
        /* one contribution per path into its own cell: per-path values, then
         * a serial sum in path order (independent of the thread count) */
        double *pv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        int64_t *pc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        ref_stats *ts = (ref_stats *)calloc((size_t)nt, sizeof(ref_stats));
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
            for (int64_t i = 0; i < n; ++i)
                pv[i] = trace_darts(sc, pr, dims, cdf, pr->path_offset + (uint64_t)i, &pc[i], &ts[tid], NULL);
        }
        for (int64_t i = 0; i < n; ++i) {
            image[pc[i]] += pv[i];
            if (m2) m2[pc[i]] += pv[i] * pv[i];
        }
        for (int t = 0; t < nt; ++t)
            for (int c = 0; c < REF_ST_COUNT; ++c) tot.st[c] += ts[t].st[c];
        free(pv); free(pc); free(ts);
    } else {
        /* many bins per path: per-thread images merged in thread order */
        double *timg = (double *)calloc((size_t)nt * (size_t)ncells * 2, sizeof(double));
        ref_stats *ts = (ref_stats *)calloc((size_t)nt, sizeof(ref_stats));
        if (!timg || !ts) { free(timg); free(ts); return -2; }
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double *img = timg + (size_t)tid * (size_t)ncells * 2, *mm = img + ncells;
            bin_scratch bs;
            bs.val = (double *)calloc((size_t)B, sizeof(double));
            bs.mark = (unsigned char *)calloc((size_t)B, 1);
            bs.touched = (int *)malloc(sizeof(int) * (size_t)B);
#ifdef _OPENMP
#pragma omp for schedule(static, 1024)
#endif
            for (int64_t i = 0; i < n; ++i) {
                bs.n_touched = 0;
                int64_t pixel = 0;
                uint64_t p = pr->path_offset + (uint64_t)i;
                if (pr->flags & REF_FORWARD) trace_forward(sc, pr, p, &bs, &ts[tid]);
                else trace_vanilla(sc, pr, p, &bs, &pixel, &ts[tid]);
                for (int q = 0; q < bs.n_touched; ++q) {
                    int b = bs.touched[q];
                    double v = bs.val[b];
                    img[(int64_t)b * npix + pixel] += v;
                    mm[(int64_t)b * npix + pixel] += v * v;
                    bs.val[b] = 0.0;
                    bs.mark[b] = 0;
                }
            }
            free(bs.val); free(bs.mark); free(bs.touched);
        }
        for (int t = 0; t < nt; ++t) {
            const double *img = timg + (size_t)t * (size_t)ncells * 2, *mm = img + ncells;
            for (int64_t c = 0; c < ncells; ++c) {
                image[c] += img[c];
                if (m2) m2[c] += mm[c];
            }
            for (int c = 0; c < REF_ST_COUNT; ++c) tot.st[c] += ts[t].st[c];
        }
        free(timg); free(ts);
    }
    if (stats) memcpy(stats, tot.st, sizeof tot.st);
    return 0;
}

/* Detached-sampling gradient of L = sum_c grad_image[c] I[c] (I the raw
 * per-cell sums) with respect to (sigma_s, sigma_a, g), path by path, then a
 * serial sum in path order. */
int ref_render_gradient(const ref_scene *sc, const ref_params *pr,
                        const ref_table_dims *dims, const float *cdf,
                        const double *grad_image, double *grad_out, int n_threads)
{
    if (check_args(sc, pr)) return -1;
    if (pr->flags & (REF_DIRECT_REUSE | REF_FORWARD)) return -1;
    if ((pr->flags & REF_EDA_DIR) && (!cdf || !dims)) return -1;
    int nt = nthreads_eff(n_threads);
    int64_t n = (int64_t)pr->n_paths;
    double *pg = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!pg) return -2;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i) {
        ref_stats S;
        memset(&S, 0, sizeof S);
        int64_t cell;
        double g[3];
        trace_darts(sc, pr, dims, cdf, pr->path_offset + (uint64_t)i, &cell, &S, g);
        for (int a = 0; a < 3; ++a) pg[3 * i + a] = grad_image[cell] * g[a];
    }
    grad_out[0] = grad_out[1] = grad_out[2] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) grad_out[a] += pg[3 * i + a];
    free(pg);
    (void)nt;
    return 0;
}
