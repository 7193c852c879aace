// libdarts: gfx950 kernels and the C ABI declared in include/darts.h.
//
// Hot path (one launch per call):  every lane owns one image cell and a
// contiguous chunk of that cell's paths (ids c + m * n_cells) and runs them
// back to back in a path-regeneration loop; per-path sums stay in registers
// and each lane flushes one compensated FP32 atomic pair at the end.  Lanes of
// a wave own consecutive cells of the same time bin, so their paths have
// similar lengths, and blocks are ordered latest bin first so the long paths
// start first.
#include "../../include/darts.h"
#include "darts_device.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

using namespace darts;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int ok()
{
    g_last_error.clear();
    return DARTS_OK;
}

// ---------------------------------------------------------------------------
// Kernel parameter block (passed by value in the kernarg segment).
// ---------------------------------------------------------------------------
struct KParams {
    Medium med;
    int box;                    // 0 infinite, 1 box (also with a floor)
    Box bx;
    int n_em;
    float em_pos[DARTS_MAX_EMITTERS][3];
    float em_start[DARTS_MAX_EMITTERS];
    float em_scale[DARTS_MAX_EMITTERS];  // power / (4 pi) * n_em
    int sensor_kind;
    float origin[3], dir[3], du[3], dv[3];
    float inv_dir[3];           // 1 / dir per axis (orthographic sensor; 0 where dir is 0)
    int width, height;
    float inv_width, inv_height;
    float beta0;
    float l_lo, l_hi, delta;
    int n_bins;
    uint64_t path_offset, n_paths;
    uint32_t key0, key1;
    int max_bounces;
    float alpha;
    unsigned flags;
    int64_t npix, ncells;
    // sensor response (null: time-resolved image): cdf[n_bins + 1], W[n_bins]
    const float *resp_cdf, *resp_w;
    // work decomposition: the launch covers path ids [q0*ncells + r0, q1*ncells + r1);
    // cell c holds repetitions m in [q0 + (c < r0), q1 + (c < r1)); waves own
    // tiles of 64 cells and chunks of chunk_reps repetitions
    uint64_t q0, r0, q1, r1;
    uint64_t n_tiles, max_reps, chunk_reps, n_waves;
    Table tb;
    float *hi, *lo, *m2;
    unsigned long long *stats;
    float *path_out;
    const float *grad_image;
    double *grad_out;
    float *tangent;             // OUT_TANGENT: [3][ncells] accumulate-into
    int floor;                  // the box's bottom face is an opaque Lambertian floor
    float floor_albedo;
    // id-range decomposition (few paths per cell): wave w takes path ids
    // path_offset + [w unit_paths, (w + 1) unit_paths)
    uint64_t unit_paths;
    // vanilla pixel decomposition (vtile != 0): wave w owns pixel w mod npix
    // and the chunk w div npix (of vt_chunk ids i) of that pixel's paths
    // p = pixel + i npix, histogramming their contributions over hist_bins
    // bins in LDS
    int vtile, hist_bins;
    uint64_t vt_chunk;
};

constexpr int kBlock = 256;
// Minimum resident waves per SIMD the render kernel is compiled for (caps its
// VGPR budget at 512 / waves, allocated in granules of 8: 96 at 5 waves).  At
// 5 the DARTS path loop keeps its 95 VGPRs without spilling, and five
// 256-thread blocks of 31 KiB of LDS share a CU's 160 KiB; measured on the
// box frame, 5 resident waves run 8% faster than 4, and 3 ran 26% slower
// than 4 with the previous pool (the loop needs several waves per SIMD to
// hide the latency of its table reads, LDS queue and FP64 chains).  Floor
// scenes keep 4: their tile kernel would spill at 5, and the fog layer's
// id-range kernel times the same at 4 and 5.
#ifndef DARTS_RENDER_WAVES_PER_SIMD
#define DARTS_RENDER_WAVES_PER_SIMD 5
#endif
// The batched kernel keeps more registers (it runs the whole pool per work
// unit from parameters in constant memory) and is faster at 4.
#ifndef DARTS_BATCH_WAVES_PER_SIMD
#define DARTS_BATCH_WAVES_PER_SIMD 4
#endif

// OUT_TANGENT: per-cell images of the derivatives of the path contributions
// (forward mode of the same detached-sampling derivative OUT_GRAD reduces).
enum { OUT_IMAGE = 0, OUT_PATHS = 1, OUT_GRAD = 2, OUT_TANGENT = 3 };

// Per-lane statistics counters; with ON = false every increment compiles away.
template <bool ON>
struct Stats {
    uint32_t v[DARTS_ST_COUNT];
    __device__ __forceinline__ void inc(int i, uint32_t by = 1u)
    {
        if (ON) v[i] += by;
    }
};

// Per-path state carried across vertices.
struct PathState {
    V3 x, w;          // vertex and walk direction
    float beta;       // throughput / pdf
    float Le;         // length travelled from the sensor
    float G_lo, G_hi; // target interval for the total path length
    float C;          // distance to the emitter
    float dm;         // distance to the boundary along w (inf: infinite medium)
    int k;            // vertex index
    V3 xe;            // chosen emitter position
    int em;           // its index
    float em_scale;   // its intensity power / (4 pi) divided by its selection probability
    float acc;        // sum of this path's contributions
    // derivative bookkeeping for the backward pass (detached sampling)
    float L_med;      // in-medium length walked so far
    float dlog_g;     // sum of d log f_HG / dg over walk vertices so far
    int n_surf;       // floor vertices among vertices 1..k
    bool on_floor;    // the current vertex lies on the floor
    // vanilla with squared sums: the bin whose contributions this path is
    // summing (-1: none yet) and that sum
    int vbin;
    float vpart;
};

// Emitter j's position, start and scale.  The kernels reach the parameter
// block through a pointer into constant memory (the kernel-argument segment,
// or the batch's scene array), so a per-lane index becomes a vector load
// rather than keeping every emitter's fields live in scalar registers.
__device__ __forceinline__ void emitter(const KParams &P, int j, V3 &pos, float &start, float &scale)
{
    if (P.n_em == 1) {   // wave-uniform: scalar loads
        pos = V3{P.em_pos[0][0], P.em_pos[0][1], P.em_pos[0][2]};
        start = P.em_start[0];
        scale = P.em_scale[0];
        return;
    }
    pos = V3{P.em_pos[j][0], P.em_pos[j][1], P.em_pos[j][2]};
    start = P.em_start[j];
    scale = P.em_scale[j];
}

__device__ __forceinline__ V3 emitter_pos(const KParams &P, int j)
{
    if (P.n_em == 1) return V3{P.em_pos[0][0], P.em_pos[0][1], P.em_pos[0][2]};   // scalar loads
    return V3{P.em_pos[j][0], P.em_pos[j][1], P.em_pos[j][2]};
}

__device__ __forceinline__ float dlog_hg_dg(float mu, float g)
{
    // d/dg log[(1 - g^2)(1 + g^2 - 2 g mu)^{-3/2}]
    return -2.f * g / (1.f - g * g) + 3.f * (mu - g) / fmaf(-2.f * g, mu, fmaf(g, g, 1.f));
}

// Path set-up (Section III; Section V-A: the target interval is fixed per
// path by the stratified cell map) from the camera uniforms r (stream 0 of
// vertex 0).  Returns false if the path cannot contribute (the camera ray
// misses the medium, or nothing is reachable inside the gate).
template <class ST>
__device__ bool setup_path(const KParams &P, U4 r, int bin, int px, int py, PathState &s, ST &st,
                           bool vanilla)
{
    const float u0 = u01(r.x), u1 = u01(r.y), u2 = u01(r.z);
    V3 pos, w;
    if (P.sensor_kind == 1) {
        const float fu = ((float)px + u0) * P.inv_width, fv = ((float)py + u1) * P.inv_height;
        pos = V3{P.origin[0] + fu * P.du[0] + fv * P.dv[0], P.origin[1] + fu * P.du[1] + fv * P.dv[1],
                 P.origin[2] + fu * P.du[2] + fv * P.dv[2]};
        w = V3{P.dir[0], P.dir[1], P.dir[2]};
    } else {
        pos = V3{P.origin[0], P.origin[1], P.origin[2]};
        const float mu = 1.f - 2.f * u0;
        const float sn = hw_sqrt(fmaxf((1.f - mu) * (1.f + mu), 0.f));
        float sp, cp;
        sincos_rev(u1, sp, cp);
        w = V3{sn * cp, sn * sp, mu};
    }
    int j = (int)(u2 * (float)P.n_em);
    j = min(j, P.n_em - 1);
    float start;
    emitter(P, j, s.xe, start, s.em_scale);
    s.em = j;
    s.beta = P.beta0;
    s.k = 0;
    s.n_surf = 0;
    s.on_floor = false;
    s.acc = 0.f;
    s.L_med = 0.f;
    s.dlog_g = 0.f;
    s.vbin = -1;
    s.vpart = 0.f;
    if (P.resp_cdf && !vanilla) {
        // target segment drawn with probability proportional to W, the path
        // weighted by W_k over that probability (Eq. (4))
        const float u3 = u01(r.w);
        int lo = 0, hi = P.n_bins;
        float c_lo = 0.f, c_hi = 1.f;
        while (hi - lo > 1) {   // largest k with cdf[k] <= u3
            const int mid = (lo + hi) >> 1;
            const float v = P.resp_cdf[mid];
            if (v <= u3) { lo = mid; c_lo = v; } else { hi = mid; c_hi = v; }
        }
        bin = lo;
        s.em_scale *= P.resp_w[lo] / (c_hi - c_lo);
    }
    if (vanilla) {
        s.G_lo = P.l_lo - start;
        s.G_hi = P.l_hi - start;
    } else {
        s.G_lo = fmaf((float)bin, P.delta, P.l_lo) - start;
        s.G_hi = fmaf((float)(bin + 1), P.delta, P.l_lo) - start;
    }
    st.inc(DARTS_ST_PATHS);
    float t_in = 0.f, t_out = kInf;
    if (P.box) {
        if (P.sensor_kind == 1) {
            // every ray of the orthographic sensor has the same direction: its
            // zero components are wave-uniform tests and 1/dir comes from the host
            float tn = -kInf, tf = kInf;
            bool hit = true;
            const float xs[3] = {pos.x, pos.y, pos.z};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (P.dir[a] == 0.f) {
                    hit = hit && !(xs[a] < P.bx.lo[a] || xs[a] > P.bx.hi[a]);
                } else {
                    const float t1 = (P.bx.lo[a] - xs[a]) * P.inv_dir[a], t2 = (P.bx.hi[a] - xs[a]) * P.inv_dir[a];
                    tn = fmaxf(tn, fminf(t1, t2));
                    tf = fminf(tf, fmaxf(t1, t2));
                }
            }
            t_in = fmaxf(tn, 0.f);
            t_out = tf;
            if (!(hit && tf > t_in)) return false;
        } else if (!box_entry(P.bx, pos, w, t_in, t_out)) {
            return false;
        }
    }
    s.x = fma3(pos, w, t_in);
    s.w = w;
    s.Le = t_in;
    s.dm = P.box ? t_out - t_in : kInf;
    s.C = length(s.xe - s.x);
    st.inc(DARTS_ST_VERTICES);
    if (s.G_hi - s.Le <= s.C) {
        st.inc(DARTS_ST_EARLY_EXIT);
        st.inc(DARTS_ST_SETUP_EXIT);
        return false;
    }
    return true;
}

// Generalised shadow connection through a control vertex on the current ray
// (Section V-B, case I, with the boundary clipping S_M): the length sum S is
// sampled in [max(R_lo, C), min(R_hi, S_exit)), the control vertex placed at
// the polar distance t(S) (Eq. (21)) and weighted with p(t) = p(S) (S - C
// mu)/(S - t) (Eq. (22), Jacobian taken as the text defines it).
struct Conn {
    V3 x, w, xe;      // vertex, ray direction, emitter
    float C;          // |xe - x|
    float lo, hi;     // length-sum range [C + lo, C + hi), as offsets above C
    float scale;      // throughput times emitter intensity / selection probability
    float u;          // uniform for S
    float dm;         // distance along the ray to the medium boundary
};

// cm = C (1 - mu) = C |w - a|^2 / 2, mu the cosine between the ray and the
// unit vector a to the emitter: no cancellation when the ray points almost
// at the emitter.
__device__ __forceinline__ float focal_cm(V3 x, V3 w, V3 xe, float C)
{
    const V3 dw = w - (xe - x) * rcp(C);
    return 0.5f * C * dot(dw, dw);
}

// Largest length sum whose control vertex stays inside the medium (the
// boundary clipping of Section V-B): S_exit = d_m + |b|, b = x + w d_m - x_e,
// with d_m the finite distance to the boundary along the ray.  When the ray
// points at an emitter outside the medium, d_m + |b| - C cancels, and one ulp
// of rounding would open a range in which the ellipse is degenerate and
// 1 / (S - C mu) explodes.  By the law of cosines |b|^2 - (C - d_m)^2 =
// 2 d_m cm, so for C >= d_m
//   S_exit - C = 2 d_m cm / (|b| + C - d_m),
// which has no cancellation; it is used where the plain sum leaves less than
// 2^-10 C above C (elsewhere the two agree to rounding).  For C < d_m the
// plain sum has no cancellation.  `excess` receives S_exit - C as formed.
__device__ __forceinline__ float exit_length(V3 x, V3 w, V3 xe, float C, float dm, float &excess)
{
    const float bl = length(fma3(x, w, dm) - xe);
    const float cd = C - dm;
    float S_exit = dm + bl;
    excess = S_exit - C;
    if (cd >= 0.f && excess < 0x1p-10f * C) {
        const float den = bl + cd;
        const float num = 2.f * dm * focal_cm(x, w, xe, C), rden = rcp(den);
        excess = den > 0.f ? num * rden : 0.f;
        S_exit = den > 0.f ? fmaf(num, rden, C) : C;
    }
    return S_exit;
}

// Range of the length sum as offsets above C, [C + lo, C + hi); false if no
// control vertex can close the path.  Kept relative to C so that, when the
// boundary clips the range to a few ulps of C (a ray aimed almost at an
// emitter outside the medium), its width is the cancellation-free excess
// itself rather than (C + excess) - C, whose rounding would move the
// contribution (proportional to the width) by percents.
__device__ __forceinline__ bool connect_range(const KParams &P, const PathState &s, float &lo, float &hi)
{
    if (!(s.C > 0.f)) return false;
    float excess = kInf;
    if (P.box) exit_length(s.x, s.w, s.xe, s.C, s.dm, excess);
    lo = fmaxf(s.G_lo - s.Le - s.C, 0.f);
    hi = fminf(s.G_hi - s.Le - s.C, excess);
    return lo < hi;
}

// Contribution of one connection; mu_c and the in-medium lengths t, r_in
// are returned for the derivative bookkeeping of the backward pass.
__device__ __forceinline__ float connect_eval(const KParams &P, const Conn &q, float &mu_c, float &t_out, float &r_in_out)
{
    const Medium &m = P.med;
    const float C = q.C;
    const float cm = focal_cm(q.x, q.w, q.xe, C);
    const float W = q.hi - q.lo;
    const bool texp = (P.flags & DARTS_ELL_TEXP) != 0;
    float sc, mass = 0.f;   // S - C
    if (texp) {
        float emass;
        mass = one_minus_exp_neg(m.sigma_t * W, emass);
        sc = q.lo + texp_sample(q.u, m.ln2_over_sigma_t, mass, emass);
    } else {
        sc = fmaf(q.u, W, q.lo);
    }
    const float S = C + sc;
    float den, t, r;
    ellipse(S, C, sc, cm, den, t, r);
    mu_c = 0.f;
    t_out = 0.f;
    r_in_out = 0.f;
    if (!(den > 0.f) || !(r > 0.f)) return 0.f;
    // the control vertex lies on the ray inside the medium (t <= d_m is the
    // same condition as S <= S_exit): a sum that rounding of S_exit still
    // lets past it would place the vertex beyond the boundary
    if (!(t <= q.dm)) return 0.f;
    const V3 xc = fma3(q.x, q.w, t);
    const float ir = rcp(r);
    // unit direction from the control vertex to the emitter, normalised from
    // the vector itself: when the ray points almost at the emitter and the S
    // range is a few ulps wide, r from the ellipse formula is far below the
    // rounding of xe - xc, and dividing by it would leave |wc| > 1
    const V3 dv = q.xe - xc;
    const V3 wc = dv * rsq(dot(dv, dv));
    const float r_in = P.box ? fminf(r, box_exit(P.bx, xc, wc)) : r;
    mu_c = fminf(fmaxf(dot(q.w, wc), -1.f), 1.f);
    t_out = t;
    r_in_out = r_in;
    const float f = hg_pdf(m.hg, mu_c);
    const float scale = q.scale * f * ir * rcp(den);
    if (texp) {
        // e^{-sigma_t (t + r_in)} / p(S) = (mass / sigma_t) e^{-sigma_t (S_lo - (r - r_in))}
        return scale * m.albedo * mass * fast_exp(-m.sigma_t * ((C + q.lo) - (r - r_in)));
    }
    return scale * m.sigma_s * W * fast_exp(-m.sigma_t * (t + r_in));
}

// Direct connection (range + contribution); dlog (if not null) receives the
// derivative of the log path throughput w.r.t. (sigma_s, sigma_a, g).
template <class ST>
__device__ float connect(const KParams &P, const PathState &s, float u4, float *dlog, ST &st)
{
    Conn q;
    if (!connect_range(P, s, q.lo, q.hi)) return 0.f;
    st.inc(DARTS_ST_SAMPLES);   // a full path sample, its length inside the target bin
    q.x = s.x; q.w = s.w; q.xe = s.xe; q.C = s.C; q.scale = s.beta * s.em_scale; q.u = u4; q.dm = s.dm;
    float mu_c, t, r_in;
    const float c = connect_eval(P, q, mu_c, t, r_in);
    if (dlog) {
        const Medium &m = P.med;
        const float Lm = s.L_med + t + r_in;               // in-medium length
        const float n = (float)(s.k + 1 - s.n_surf);       // medium scattering vertices
        dlog[0] = n / m.sigma_s - Lm;
        dlog[1] = -Lm;
        dlog[2] = s.dlog_g + dlog_hg_dg(mu_c, m.g);
    }
    return c;
}

// Direction at vertex k >= 1 (DARTS family), from stream 0 of vertex k.
template <int OUT, bool FLOOR, class ST>
__device__ __forceinline__ void direction_darts(const KParams &P, PathState &s, U4 r0, ST &st)
{
    const Medium &m = P.med;
    if (FLOOR && s.on_floor) {
        s.w = floor_direction(u01(r0.y), u01(r0.z));
        s.beta *= P.floor_albedo;
        s.on_floor = false;
        s.dm = box_exit(P.bx, s.x, s.w);
        return;
    }
    const V3 de = s.xe - s.x;
    float weight;
    bool eb;
    const V3 wp = s.w;
    s.w = sample_direction(m, P.tb, P.alpha, (P.flags & DARTS_EDA_DIR) != 0, de * rcp(s.C), s.C, s.G_hi - s.Le,
                           wp, r0, weight, eb);
    if (OUT == OUT_GRAD || OUT == OUT_TANGENT) s.dlog_g += dlog_hg_dg(dot(wp, s.w), m.g);
    st.inc(DARTS_ST_EDA_BRANCH, eb ? 1u : 0u);
    s.beta *= weight;
    s.dm = P.box ? box_exit(P.bx, s.x, s.w) : kInf;
}

// Floor point as the connection vertex (Section V-B, case II): the ray meets
// the floor at t_s = s.dm; the path x -> floor point -> emitter has a fixed
// length and counts when it falls in the target interval.  Contribution:
// throughput x transmittance of both segments x albedo/pi x cosine at the
// floor x emitter intensity / r^2.  dlog as for connect().
template <class ST>
__device__ float floor_connect(const KParams &P, const PathState &s, float *dlog, ST &st)
{
    const float t_s = s.dm;
    V3 xs = fma3(s.x, s.w, t_s);
    xs.z = P.bx.lo[2];
    const V3 de = s.xe - xs;
    const float r = length(de);
    if (!(r > 0.f) || !(de.z > 0.f)) return 0.f;
    const float L = s.Le + t_s + r;
    st.inc(DARTS_ST_SAMPLES);
    if (!(L >= s.G_lo && L < s.G_hi)) {
        st.inc(DARTS_ST_REJECTED);
        return 0.f;
    }
    const float ir = rcp(r);
    const float r_in = fminf(r, box_exit(P.bx, xs, de * ir));
    const Medium &m = P.med;
    if (dlog) {
        const float Lm = s.L_med + t_s + r_in;
        dlog[0] = (float)(s.k - s.n_surf) / m.sigma_s - Lm;
        dlog[1] = -Lm;
        dlog[2] = s.dlog_g;
    }
    const float cos_s = de.z * ir;
    return s.beta * s.em_scale * fast_exp(-m.sigma_t * (t_s + r_in)) * (P.floor_albedo * (1.f / kPi)) * cos_s *
           ir * ir;
}

// What the free flight from vertex k needs once its medium event has been
// drawn: the stream-1 words of vertex k that DA-RIS reads (Sobol row, offset,
// selection uniform) and pc = 1 - e^{-sigma_t d_m}, epc = e^{-sigma_t d_m}.
struct Pending {
    uint32_t y, z, w;
    float pc, epc;
};

// Connection at vertex k and the medium-event Bernoulli (Eq. (12)) from r1,
// stream 1 of vertex k (DARTS family).  Returns false when the path has
// ended (truncation, a flight that leaves the medium, or the early-exit test
// after a floor vertex); otherwise a medium event is pending and `pd` holds
// what the flight needs.  A flight that reaches the floor is a surface event
// (floor scenes): the walk goes on from the floor point, whose direction is
// drawn from stream 0 of the new vertex, and the connection and the event
// are drawn again there.
//
// Callers draw streams 0 and 1 of a vertex next to each other: the two
// counters differ only in their last word, which enters the first products
// in the second round, so four of the forty 32x32 -> 64-bit products of the
// pair are common to both and computed once.
template <int OUT, bool FLOOR, class ST>
__device__ bool connect_and_event(const KParams &P, uint64_t p, PathState &s, ST &st, float grad_w, double *gacc,
                                  Pending &pd, U4 r1)
{
    const Medium &m = P.med;
    while (true) {
        {
            float dl[3];
            const float c = connect(P, s, u01(r1.x), OUT == OUT_GRAD || OUT == OUT_TANGENT ? dl : nullptr, st);
            if (c != 0.f) {
                st.inc(DARTS_ST_CONNECTIONS);
                s.acc += c;
                if (OUT == OUT_GRAD || OUT == OUT_TANGENT) {
                    // the tangent mode sums this path's c dlog/dtheta (weight 1)
                    const double cw = OUT == OUT_GRAD ? (double)c * (double)grad_w : (double)c;
                    gacc[0] += cw * dl[0]; gacc[1] += cw * dl[1]; gacc[2] += cw * dl[2];
                }
            }
        }
        const bool to_floor = FLOOR && exits_floor(P.bx, s.x, s.w);
        if (to_floor) {
            float dl[3];
            const float c = floor_connect(P, s, OUT == OUT_GRAD || OUT == OUT_TANGENT ? dl : nullptr, st);
            if (c != 0.f) {
                st.inc(DARTS_ST_CONNECTIONS);
                s.acc += c;
                if (OUT == OUT_GRAD || OUT == OUT_TANGENT) {
                    const double cw = OUT == OUT_GRAD ? (double)c * (double)grad_w : (double)c;
                    gacc[0] += cw * dl[0]; gacc[1] += cw * dl[1]; gacc[2] += cw * dl[2];
                }
            }
        }
        if (s.k == P.max_bounces - 1) { st.inc(DARTS_ST_TRUNCATED); return false; }
        float epc = 0.f;
        const float pc = P.box ? one_minus_exp_neg(m.sigma_t * s.dm, epc) : 1.f;
        if (u01(r1.y) < pc) {
            pd = Pending{r1.y, r1.z, r1.w, pc, epc};
            return true;
        }
        if (!to_floor) { st.inc(DARTS_ST_MEDIUM_EXIT); return false; }
        // surface event: probability e^{-sigma_t d_m}, equal to the
        // transmittance, so the throughput is unchanged
        s.x = fma3(s.x, s.w, s.dm);
        s.x.z = P.bx.lo[2];
        s.Le += s.dm;
        s.L_med += s.dm;
        s.k += 1;
        s.n_surf += 1;
        s.on_floor = true;
        s.C = length(s.xe - s.x);
        st.inc(DARTS_ST_VERTICES);
        if (s.G_hi - s.Le <= s.C) { st.inc(DARTS_ST_EARLY_EXIT); return false; }
        const U4 r0 = philox((uint32_t)p, (uint32_t)(p >> 32), (uint32_t)s.k, 0u, P.key0, P.key1);
        r1 = philox((uint32_t)p, (uint32_t)(p >> 32), (uint32_t)s.k, 1u, P.key0, P.key1);
        direction_darts<OUT, FLOOR>(P, s, r0, st);
    }
}

// Free flight from vertex k given its pending medium event: DA-RIS distance
// (Section IV-C) or the plain exponential, the move to vertex k + 1 and its
// early-exit test.  Returns false when the path has ended.
template <class ST>
__device__ bool fly(const KParams &P, PathState &s, ST &st, const Pending &pd)
{
    const Medium &m = P.med;
    float d, factor;
    if (P.flags & DARTS_RIS_DIST) {
        const V3 de = s.xe - s.x;
        if (!ris_distance(m, s.C * s.C, dot(s.w, de), s.G_hi - s.Le, pd.pc, pd.epc, pd.y & 31u, pd.z, u01(pd.w), d,
                          factor)) {
            st.inc(DARTS_ST_RIS_ALL_INVALID);
            return false;
        }
    } else {
        d = texp_sample(u01(pd.y), m.ln2_over_sigma_t, 1.f, 0.f);   // plain exponential, given u < pc
        factor = m.albedo;
    }
    s.x = fma3(s.x, s.w, d);
    s.Le += d;
    s.L_med += d;
    s.beta *= factor;
    s.k += 1;
    s.C = length(s.xe - s.x);
    st.inc(DARTS_ST_VERTICES);
    if (s.G_hi - s.Le <= s.C) { st.inc(DARTS_ST_EARLY_EXIT); return false; }
    return true;
}

__device__ __forceinline__ void add_compensated(float *hi, float *lo, int64_t i, float v, float v_lo)
{
    const float old = unsafeAtomicAdd(hi + i, v);
    const float e = two_sum_err(old, v, old + v);
    const float tot = e + v_lo;
    if (tot != 0.f) unsafeAtomicAdd(lo + i, tot);
}

// Vanilla transient path tracing (the paper's baseline): exponential free
// flight, phase sampling, a shadow connection at every medium vertex, each
// connection binned by its total length.
template <bool FLOOR>
__device__ __forceinline__ void direction_vanilla(const KParams &P, PathState &s, U4 r0)
{
    if (FLOOR && s.on_floor) {
        s.w = floor_direction(u01(r0.y), u01(r0.z));
        s.beta *= P.floor_albedo;
        s.on_floor = false;
    } else {
        float mu, sn;
        hg_sample(P.med.hg, u01(r0.y), mu, sn);
        s.w = from_frame(s.w, mu, sn, u01(r0.z));
    }
    s.dm = P.box ? box_exit(P.bx, s.x, s.w) : kInf;
}

__device__ __forceinline__ void compensated_lds_add(float *hi, float *lo, int i, float v)
{
    const float old = atomicAdd(&hi[i], v);
    const float e = two_sum_err(old, v, old + v);
    if (e != 0.f) atomicAdd(&lo[i], e);
}

// Adds the square of the path's running sum for its current bin to m2 (the
// global image, or with PRIV the wave's LDS histogram hist[2 hist_bins + b]).
template <bool PRIV>
__device__ __forceinline__ void vanilla_flush_m2(const KParams &P, const PathState &s, int64_t pixel, float *hist)
{
    if (s.vbin >= 0) {
        if (PRIV) {
            atomicAdd(&hist[2 * P.hist_bins + s.vbin], s.vpart * s.vpart);
        } else {
            const int64_t cell = P.resp_w ? pixel : (int64_t)s.vbin * P.npix + pixel;
            unsafeAtomicAdd(P.m2 + cell, s.vpart * s.vpart);
        }
    }
}

// PRIV: every path of the wave belongs to one pixel, and its contributions go
// to the wave's compensated LDS histogram hist[0 .. hist_bins) (hi),
// hist[hist_bins .. 2 hist_bins) (lo) instead of global atomics.
template <bool FLOOR, bool PRIV, class ST>
__device__ bool fly_vanilla(const KParams &P, uint64_t p, int64_t pixel, PathState &s, ST &st, float *hist)
{
    const Medium &m = P.med;
    const U4 r1 = philox((uint32_t)p, (uint32_t)(p >> 32), (uint32_t)s.k, 1u, P.key0, P.key1);
    const float pc = P.box ? texp_mass(m.sigma_t, s.dm) : 1.f;
    const float u5 = u01(r1.y);
    if (!(u5 < pc)) {
        if (!(FLOOR && exits_floor(P.bx, s.x, s.w))) { st.inc(DARTS_ST_MEDIUM_EXIT); return false; }
        // surface event on the floor (probability = transmittance)
        s.x = fma3(s.x, s.w, s.dm);
        s.x.z = P.bx.lo[2];
        s.Le += s.dm;
        s.on_floor = true;
    } else {
        const float d = texp_sample(u5, m.ln2_over_sigma_t, 1.f, 0.f);
        s.x = fma3(s.x, s.w, d);
        s.Le += d;
        s.beta *= m.albedo;
    }
    s.k += 1;
    const V3 de = s.xe - s.x;
    const float r = length(de);
    s.C = r;
    {
        const float ir = rcp(r);
        const V3 wc = de * ir;
        // local scattering toward the emitter: phase function in the medium,
        // BRDF times cosine on the floor
        const float f_loc = FLOOR && s.on_floor ? (wc.z > 0.f ? P.floor_albedo * (1.f / kPi) * wc.z : 0.f)
                                       : hg_pdf(m.hg, dot(s.w, wc));
        const float r_in = P.box ? fminf(r, box_exit(P.bx, s.x, wc)) : r;
        // total length with the emitter's start offset: G_lo = l_lo - start
        const float L = s.Le + r + (P.l_lo - s.G_lo);
        const int bin = (int)floorf((L - P.l_lo) / P.delta);
        st.inc(DARTS_ST_SAMPLES);
        // sensor weight: the indicator of the bin, or W of the length
        const bool in_range = L >= P.l_lo && bin >= 0 && bin < P.n_bins;
        const float wsens = !in_range ? 0.f : (P.resp_w ? P.resp_w[bin] : 1.f);
        if (wsens > 0.f) {
            const float v = wsens * s.beta * s.em_scale * f_loc * fast_exp(-m.sigma_t * r_in) * ir * ir;
            const int vb = P.resp_w ? 0 : bin;
            if (PRIV) {
                compensated_lds_add(hist, hist + P.hist_bins, vb, v);
            } else {
                const int64_t cell = P.resp_w ? pixel : (int64_t)bin * P.npix + pixel;
                add_compensated(P.hi, P.lo, cell, v, 0.f);
            }
            if (P.m2) {
                // squares of per-path-per-bin sums: a path's length never
                // decreases (a flight of d adds d to Le and shortens the
                // distance to the emitter by at most d), so its contributions
                // to one bin are consecutive and one running sum suffices
                if (vb != s.vbin) {
                    vanilla_flush_m2<PRIV>(P, s, pixel, hist);
                    s.vbin = vb;
                    s.vpart = v;
                } else {
                    s.vpart += v;
                }
            }
            st.inc(DARTS_ST_CONNECTIONS);
            s.acc += v;
        } else {
            st.inc(DARTS_ST_REJECTED);
        }
    }
    if (s.k == P.max_bounces) { st.inc(DARTS_ST_TRUNCATED); return false; }
    st.inc(DARTS_ST_VERTICES);
    if (s.G_hi - s.Le <= s.C) { st.inc(DARTS_ST_EARLY_EXIT); return false; }
    return true;
}

// ---------------------------------------------------------------------------
// Path pool.  A wave works through a range [j_begin, j_end) of path slots.
// New paths are set up in bulk: when lanes need a path and the wave's queue
// is empty, all 64 lanes set up the next 64 slots at once and the paths that
// survive set-up are written, compacted, to the wave's queue in LDS.  A lane
// whose path has ended takes the next queued path at the top of the next
// iteration (ballot + popcount on the wave-uniform queue head), so set-up
// runs with full lanes once per 64 paths instead of for the few lanes that
// happen to need a path, and no lane waits for others before it refills.
//
// DARTS family: the bulk set-up also makes vertex 0's connection and draws
// its medium event, and a queued path waits for its first free flight.  One
// loop iteration is then: the free flight from vertex k (DA-RIS) and the
// move to vertex k + 1; stream-0 Philox and direction sampling at k + 1;
// stream-1 Philox, connection and medium-event draw at k + 1.  A path that
// leaves the medium ends at the end of an iteration and its lane takes a new
// path, queued ready for its flight, at the top of the next one: no lane sits
// out the RIS flight of an iteration because its path left the medium there.
// Vanilla: set-up only; one iteration is the direction at vertex k (k >= 1),
// the shadow connection and the free flight.
//
// Slot sources:
//  - SRC_TILE: slot j is repetition j / 64 of cell c0 + (j mod 64) of a tile
//    of 64 consecutive cells; a bulk set-up covers one repetition of the
//    whole tile, lane l taking cell c0 + l.  Per-cell sums go to compensated
//    LDS accumulators (one slot per tile cell), flushed by the caller with
//    one compensated global atomic pair per cell: the histogram is
//    privatised.
//  - SRC_IDS: slot j is path id j itself, in cell c0 + (j - j_begin) (wrapped
//    once at n_cells; the caller keeps ranges no longer than n_cells).  Each
//    finished path adds its sum to the global image with one compensated
//    atomic pair: suited to scenes with few paths per cell.
//  - SRC_VTILE (vanilla): the wave owns pixel c0; slot j is path id
//    c0 + j npix, and every contribution goes to the wave's compensated LDS
//    histogram over the bins (hist), flushed by the caller once per wave.
// ---------------------------------------------------------------------------
enum { LANE_NEED = 0, LANE_FRESH = 1, LANE_ACTIVE = 2, LANE_DONE = 3 };
enum { SRC_TILE = 0, SRC_IDS = 1, SRC_VTILE = 2 };

// Set-up path queue of one wave in LDS, structure of arrays: field f of
// entry i at q[f * 64 + i].  The DARTS family adds the state after vertex
// 0's connection and medium event (throughput, vertex index, sum so far,
// the pending flight; and the derivative bookkeeping for the gradient
// outputs).
enum {
    Q_X = 0, Q_W = 3, Q_LE = 6, Q_DM, Q_C, Q_GLO, Q_GHI, Q_EMS, Q_EM, Q_PLO, Q_PHI, Q_CLO, Q_CHI, Q_PIX,
    Q_BASE_FIELDS,
    Q_BETA = Q_BASE_FIELDS, Q_K, Q_ACC, Q_RY, Q_RZ, Q_RW, Q_PC, Q_EPC,
    Q_DARTS_FIELDS,
    Q_LMED = Q_DARTS_FIELDS, Q_DLG, Q_NSURF,
    Q_GRAD_FIELDS
};
template <int MODE, int OUT>
constexpr int queue_floats()
{
    return 64 * (MODE == 1 ? Q_BASE_FIELDS : OUT == OUT_GRAD || OUT == OUT_TANGENT ? Q_GRAD_FIELDS : Q_DARTS_FIELDS);
}
// LDS per wave of the pool: the queue, and for the DARTS family the tile's
// cell descriptions (two words per lane)
template <int MODE, int OUT>
constexpr int pool_floats()
{
    return queue_floats<MODE, OUT>() + (MODE == 1 ? 0 : 2 * 64);
}

// Number of set bits of the wave mask below this lane (one mbcnt pair, no
// per-lane mask kept in registers).
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Tile-cell description of lane l (SRC_TILE), packed in two registers:
// bf = bin | flags << 29 (bit 29: the cell exists, bit 30: cell < r0, bit
// 31: cell < r1), xy = px | py << 16.
template <int SRC>
__device__ __forceinline__ void tile_cell(const KParams &P, int64_t c0, uint64_t j_begin, uint64_t j_end, int lane,
                                          uint32_t &bf, uint32_t &xy)
{
    bf = 0;
    xy = 0;
    if (SRC == SRC_TILE) {
        const int64_t my_cell = c0 + lane;
        if (j_begin < j_end && my_cell < P.ncells) {
            const int64_t b = my_cell / P.npix;
            const int64_t pix = my_cell - b * P.npix;
            const uint32_t y = (uint32_t)(pix / P.width);
            const uint32_t x = (uint32_t)(pix - (int64_t)y * P.width);
            bf = (uint32_t)b | (1u << 29) | ((uint64_t)my_cell < P.r0 ? 1u << 30 : 0u) |
                 ((uint64_t)my_cell < P.r1 ? 1u << 31 : 0u);
            xy = x | (y << 16);
        }
    }
}

// Path id, cell, pixel and (bin, px, py) of slot j; false for an empty slot
// of a ragged range.
template <int SRC>
__device__ __forceinline__ bool pool_slot(const KParams &P, int64_t c0, uint64_t j, uint64_t j_begin, int lane,
                                          uint32_t my_bf, uint32_t my_xy, uint64_t &pj, int64_t &cj, int64_t &pixj,
                                          int &bin, int &px, int &py)
{
    if (SRC == SRC_TILE) {
        const uint64_t m = P.q0 + (uint64_t)((my_bf >> 30) & 1u) + (j >> 6);
        const uint64_t m_hi = P.q1 + (uint64_t)(my_bf >> 31);
        cj = c0 + lane;
        pj = (uint64_t)cj + m * (uint64_t)P.ncells;
        bin = (int)(my_bf & ((1u << 29) - 1u));
        px = (int)(my_xy & 0xFFFFu);
        py = (int)(my_xy >> 16);
        pixj = (int64_t)py * P.width + px;
        return ((my_bf >> 29) & 1u) && m < m_hi;
    } else if (SRC == SRC_VTILE) {
        pj = (uint64_t)c0 + j * (uint64_t)P.npix;
        cj = c0;
        pixj = c0;
        py = (int)(c0 / P.width);
        px = (int)(c0 - (int64_t)py * P.width);
        bin = 0;
        return true;
    } else {
        pj = j;
        cj = c0 + (int64_t)(j - j_begin);
        if (cj >= P.ncells) cj -= P.ncells;
        if (P.ncells <= 0xFFFFFFFFll) {
            const uint32_t c32 = (uint32_t)cj, np = (uint32_t)P.npix;
            const uint32_t b = c32 / np, pix = c32 - b * np;
            const uint32_t y = pix / (uint32_t)P.width;
            bin = (int)b;
            py = (int)y;
            px = (int)(pix - y * (uint32_t)P.width);
            pixj = pix;
        } else {
            const int64_t b = cj / P.npix;
            pixj = cj - b * P.npix;
            bin = (int)b;
            py = (int)(pixj / P.width);
            px = (int)(pixj - (int64_t)py * P.width);
        }
        return true;
    }
}

// A finished path of the DARTS family: its sum into its cell (LDS slot or
// global compensated pair), its square into the second moments, or its value
// into the per-path output; the tangent images receive the path's derivative
// sums.
template <int OUT, int SRC, class ST>
__device__ __forceinline__ void finish_path(const KParams &P, const PathState &s, uint64_t p, int64_t cell, int slot,
                                            float *img_hi, float *img_lo, float *acc_hi, float *acc_lo, float *acc_m2,
                                            ST &st, double *gacc)
{
    if (s.acc == 0.f) st.inc(DARTS_ST_ZERO_PATHS);
    if (OUT == OUT_TANGENT) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (gacc[k] != 0.0) unsafeAtomicAdd(P.tangent + (int64_t)k * P.ncells + cell, (float)gacc[k]);
            gacc[k] = 0.0;
        }
    } else if (OUT == OUT_PATHS) {
        P.path_out[p - P.path_offset] = s.acc;
    } else if (OUT == OUT_IMAGE && s.acc != 0.f) {
        if (SRC == SRC_TILE) {
            compensated_lds_add(acc_hi, acc_lo, slot, s.acc);
            if (P.m2) atomicAdd(&acc_m2[slot], s.acc * s.acc);
        } else {
            add_compensated(img_hi, img_lo, cell, s.acc, 0.f);
            if (P.m2) unsafeAtomicAdd(P.m2 + cell, s.acc * s.acc);
        }
    }
}

template <bool STATS, int SRC, bool FLOOR>
__device__ __forceinline__ void run_pool_vanilla(const KParams &P, int64_t c0, uint64_t j_begin, uint64_t j_end,
                                                 float *img_hi, float *img_lo, float *q, float *hist, Stats<STATS> &st)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lanes_below = (1ull << lane) - 1ull;
    uint32_t my_bf, my_xy;
    tile_cell<SRC>(P, c0, j_begin, j_end, lane, my_bf, my_xy);

    PathState s;
    uint64_t next = j_begin;   // next slot to set up (wave-uniform)
    uint32_t qh = 0, qn = 0;   // queue head and length (wave-uniform)
    int state = j_begin < j_end ? LANE_NEED : LANE_DONE;
    uint64_t p = 0;
    int64_t pixel = 0;

    while (true) {
        const uint64_t need = __ballot(state == LANE_NEED);
        if (need) {
            if (qh == qn && next < j_end) {
                // bulk set-up of slots next .. next + 63, one per lane
                const uint64_t j = next + (uint64_t)lane;
                bool ok = false;
                PathState t;
                uint64_t pj = 0;
                int64_t cj = 0, pixj = 0;
                if (j < j_end) {
                    int bin = 0, px = 0, py = 0;
                    if (pool_slot<SRC>(P, c0, j, j_begin, lane, my_bf, my_xy, pj, cj, pixj, bin, px, py)) {
                        const U4 r0 = philox((uint32_t)pj, (uint32_t)(pj >> 32), 0u, 0u, P.key0, P.key1);
                        ok = setup_path(P, r0, bin, px, py, t, st, true);
                        if (!ok) st.inc(DARTS_ST_ZERO_PATHS);
                    }
                }
                const uint64_t okb = __ballot(ok);
                if (ok) {
                    const int i = __popcll(okb & lanes_below);
                    q[(Q_X + 0) * 64 + i] = t.x.x; q[(Q_X + 1) * 64 + i] = t.x.y; q[(Q_X + 2) * 64 + i] = t.x.z;
                    q[(Q_W + 0) * 64 + i] = t.w.x; q[(Q_W + 1) * 64 + i] = t.w.y; q[(Q_W + 2) * 64 + i] = t.w.z;
                    q[Q_LE * 64 + i] = t.Le;
                    q[Q_DM * 64 + i] = t.dm;
                    q[Q_C * 64 + i] = t.C;
                    q[Q_GLO * 64 + i] = t.G_lo;
                    q[Q_GHI * 64 + i] = t.G_hi;
                    q[Q_EMS * 64 + i] = t.em_scale;
                    q[Q_EM * 64 + i] = __int_as_float(t.em);
                    q[Q_PLO * 64 + i] = __uint_as_float((uint32_t)pj);
                    q[Q_PHI * 64 + i] = __uint_as_float((uint32_t)(pj >> 32));
                    q[Q_PIX * 64 + i] = __uint_as_float((uint32_t)pixj);
                }
                qh = 0;
                qn = (uint32_t)__popcll(okb);
                next += 64;
                __builtin_amdgcn_wave_barrier();
            }
            if (qh < qn) {
                const uint32_t rank = (uint32_t)__popcll(need & lanes_below);
                if (state == LANE_NEED && rank < qn - qh) {
                    const int i = (int)(qh + rank);
                    s.x = V3{q[(Q_X + 0) * 64 + i], q[(Q_X + 1) * 64 + i], q[(Q_X + 2) * 64 + i]};
                    s.w = V3{q[(Q_W + 0) * 64 + i], q[(Q_W + 1) * 64 + i], q[(Q_W + 2) * 64 + i]};
                    s.Le = q[Q_LE * 64 + i];
                    s.dm = q[Q_DM * 64 + i];
                    s.C = q[Q_C * 64 + i];
                    s.G_lo = q[Q_GLO * 64 + i];
                    s.G_hi = q[Q_GHI * 64 + i];
                    s.em_scale = q[Q_EMS * 64 + i];
                    s.em = __float_as_int(q[Q_EM * 64 + i]);
                    s.beta = P.beta0;
                    s.k = 0;
                    s.n_surf = 0;
                    s.on_floor = false;
                    s.acc = 0.f;
                    s.L_med = 0.f;
                    s.dlog_g = 0.f;
                    s.vbin = -1;
                    s.vpart = 0.f;
                    p = (uint64_t)__float_as_uint(q[Q_PLO * 64 + i]) |
                        ((uint64_t)__float_as_uint(q[Q_PHI * 64 + i]) << 32);
                    pixel = (int64_t)__float_as_uint(q[Q_PIX * 64 + i]);
                    state = LANE_FRESH;
                }
                const uint32_t took = (uint32_t)__popcll(need);
                qh += took < qn - qh ? took : qn - qh;
            } else if (next >= j_end && state == LANE_NEED) {
                state = LANE_DONE;
            }
        }
        if (__ballot(state != LANE_DONE) == 0) break;
        if (state == LANE_FRESH || state == LANE_ACTIVE) {
            s.xe = emitter_pos(P, s.em);
            if (state == LANE_ACTIVE) {
                const U4 r0 = philox((uint32_t)p, (uint32_t)(p >> 32), (uint32_t)s.k, 0u, P.key0, P.key1);
                direction_vanilla<FLOOR>(P, s, r0);
            }
            if (fly_vanilla<FLOOR, SRC == SRC_VTILE>(P, p, pixel, s, st, hist)) {
                state = LANE_ACTIVE;
            } else {
                state = LANE_NEED;
                if (s.acc == 0.f) st.inc(DARTS_ST_ZERO_PATHS);
                if (P.m2) vanilla_flush_m2<SRC == SRC_VTILE>(P, s, pixel, hist);
            }
        }
    }
}

template <int OUT, bool STATS, int SRC, bool FLOOR>
__device__ __forceinline__ void run_pool_darts(const KParams &P, int64_t c0, uint64_t j_begin, uint64_t j_end,
                                               float *img_hi, float *img_lo, float *acc_hi, float *acc_lo,
                                               float *acc_m2, float *q, Stats<STATS> &st, double *gacc)
{
    constexpr bool kGrad = OUT == OUT_GRAD || OUT == OUT_TANGENT;
    // SRC_TILE: the tile's cell descriptions wait in LDS between bulk
    // set-ups (two words per lane after the queue) rather than in registers
    uint32_t *tdesc = (uint32_t *)(q + queue_floats<0, OUT>());
    if (SRC == SRC_TILE) {
        const int lane = threadIdx.x & 63;
        uint32_t bf, xy;
        tile_cell<SRC>(P, c0, j_begin, j_end, lane, bf, xy);
        tdesc[lane] = bf;
        tdesc[64 + lane] = xy;
    }

    PathState s;
    Pending pd;
    uint64_t next = j_begin;   // next slot to set up (wave-uniform)
    uint32_t qh = 0, qn = 0;   // queue head and length (wave-uniform)
    int state = j_begin < j_end ? LANE_NEED : LANE_DONE;
    uint64_t p = 0;
    int slot = 0;          // SRC_TILE: the path's cell is c0 + slot
    int64_t cell_ids = 0;  // other sources: the path's cell
    float grad_w = 0.f;

    while (true) {
        const uint64_t need = __ballot(state == LANE_NEED);
        if (need) {
            if (qh == qn && next < j_end) {
                // bulk set-up of slots next .. next + 63, one per lane: camera
                // ray (stream 0 of vertex 0), then vertex 0's connection and
                // medium event (stream 1 of vertex 0)
                const int lane = threadIdx.x & 63;
                const uint64_t j = next + (uint64_t)lane;
                bool ok = false;
                PathState t;
                Pending tpd;
                uint64_t pj = 0;
                int64_t cj = 0, pixj = 0;
                if (j < j_end) {
                    int bin = 0, px = 0, py = 0;
                    const uint32_t my_bf = SRC == SRC_TILE ? tdesc[lane] : 0u;
                    const uint32_t my_xy = SRC == SRC_TILE ? tdesc[64 + lane] : 0u;
                    if (pool_slot<SRC>(P, c0, j, j_begin, lane, my_bf, my_xy, pj, cj, pixj, bin, px, py)) {
                        const U4 r0 = philox((uint32_t)pj, (uint32_t)(pj >> 32), 0u, 0u, P.key0, P.key1);
                        const U4 r1 = philox((uint32_t)pj, (uint32_t)(pj >> 32), 0u, 1u, P.key0, P.key1);
                        if (setup_path(P, r0, bin, px, py, t, st, false)) {
                            double g0[3] = {0.0, 0.0, 0.0};
                            const float gw = OUT == OUT_GRAD ? P.grad_image[cj] : 0.f;
                            ok = connect_and_event<OUT, FLOOR>(P, pj, t, st, gw, g0, tpd, r1);
                            if (OUT == OUT_GRAD) { gacc[0] += g0[0]; gacc[1] += g0[1]; gacc[2] += g0[2]; }
                            if (!ok) {
                                finish_path<OUT, SRC>(P, t, pj, cj, (int)(cj - c0), img_hi, img_lo, acc_hi, acc_lo,
                                                      acc_m2, st, g0);
                            } else if (OUT == OUT_TANGENT) {
                                // vertex 0's derivative sums go to the tangent images now
#pragma unroll
                                for (int k = 0; k < 3; ++k)
                                    if (g0[k] != 0.0) unsafeAtomicAdd(P.tangent + (int64_t)k * P.ncells + cj, (float)g0[k]);
                            }
                        } else {
                            st.inc(DARTS_ST_ZERO_PATHS);
                            if (OUT == OUT_PATHS) P.path_out[pj - P.path_offset] = 0.f;
                        }
                    }
                }
                const uint64_t okb = __ballot(ok);
                if (ok) {
                    const int i = (int)lane_rank(okb);
                    q[(Q_X + 0) * 64 + i] = t.x.x; q[(Q_X + 1) * 64 + i] = t.x.y; q[(Q_X + 2) * 64 + i] = t.x.z;
                    q[(Q_W + 0) * 64 + i] = t.w.x; q[(Q_W + 1) * 64 + i] = t.w.y; q[(Q_W + 2) * 64 + i] = t.w.z;
                    q[Q_LE * 64 + i] = t.Le;
                    q[Q_DM * 64 + i] = t.dm;
                    q[Q_C * 64 + i] = t.C;
                    q[Q_GLO * 64 + i] = t.G_lo;
                    q[Q_GHI * 64 + i] = t.G_hi;
                    q[Q_EMS * 64 + i] = t.em_scale;
                    q[Q_EM * 64 + i] = __int_as_float(t.em);
                    q[Q_PLO * 64 + i] = __uint_as_float((uint32_t)pj);
                    q[Q_PHI * 64 + i] = __uint_as_float((uint32_t)(pj >> 32));
                    q[Q_CLO * 64 + i] = __uint_as_float((uint32_t)cj);
                    if (SRC != SRC_TILE) q[Q_CHI * 64 + i] = __uint_as_float((uint32_t)((uint64_t)cj >> 32));
                    q[Q_BETA * 64 + i] = t.beta;
                    q[Q_K * 64 + i] = __int_as_float(t.k);
                    q[Q_ACC * 64 + i] = t.acc;
                    q[Q_RY * 64 + i] = __uint_as_float(tpd.y);
                    q[Q_RZ * 64 + i] = __uint_as_float(tpd.z);
                    q[Q_RW * 64 + i] = __uint_as_float(tpd.w);
                    q[Q_PC * 64 + i] = tpd.pc;
                    q[Q_EPC * 64 + i] = tpd.epc;
                    if (kGrad) {
                        q[Q_LMED * 64 + i] = t.L_med;
                        q[Q_DLG * 64 + i] = t.dlog_g;
                        q[Q_NSURF * 64 + i] = __int_as_float(t.n_surf);
                    }
                }
                qh = 0;
                qn = (uint32_t)__popcll(okb);
                next += 64;
                __builtin_amdgcn_wave_barrier();
            }
            if (qh < qn) {
                const uint32_t rank = lane_rank(need);
                if (state == LANE_NEED && rank < qn - qh) {
                    const int i = (int)(qh + rank);
                    s.x = V3{q[(Q_X + 0) * 64 + i], q[(Q_X + 1) * 64 + i], q[(Q_X + 2) * 64 + i]};
                    s.w = V3{q[(Q_W + 0) * 64 + i], q[(Q_W + 1) * 64 + i], q[(Q_W + 2) * 64 + i]};
                    s.Le = q[Q_LE * 64 + i];
                    s.dm = q[Q_DM * 64 + i];
                    s.C = q[Q_C * 64 + i];
                    s.G_lo = q[Q_GLO * 64 + i];
                    s.G_hi = q[Q_GHI * 64 + i];
                    s.em_scale = q[Q_EMS * 64 + i];
                    s.em = __float_as_int(q[Q_EM * 64 + i]);
                    s.beta = q[Q_BETA * 64 + i];
                    s.k = __float_as_int(q[Q_K * 64 + i]);
                    s.acc = q[Q_ACC * 64 + i];
                    s.on_floor = false;
                    if (kGrad) {
                        s.L_med = q[Q_LMED * 64 + i];
                        s.dlog_g = q[Q_DLG * 64 + i];
                        s.n_surf = __float_as_int(q[Q_NSURF * 64 + i]);
                    } else {
                        s.L_med = 0.f;
                        s.dlog_g = 0.f;
                        s.n_surf = 0;
                    }
                    pd.y = __float_as_uint(q[Q_RY * 64 + i]);
                    pd.z = __float_as_uint(q[Q_RZ * 64 + i]);
                    pd.w = __float_as_uint(q[Q_RW * 64 + i]);
                    pd.pc = q[Q_PC * 64 + i];
                    pd.epc = q[Q_EPC * 64 + i];
                    p = (uint64_t)__float_as_uint(q[Q_PLO * 64 + i]) |
                        ((uint64_t)__float_as_uint(q[Q_PHI * 64 + i]) << 32);
                    if (SRC == SRC_TILE) {
                        slot = (int)(__float_as_uint(q[Q_CLO * 64 + i]) - (uint32_t)c0);
                        if (OUT == OUT_GRAD) grad_w = P.grad_image[c0 + slot];
                    } else {
                        cell_ids = (int64_t)((uint64_t)__float_as_uint(q[Q_CLO * 64 + i]) |
                                             ((uint64_t)__float_as_uint(q[Q_CHI * 64 + i]) << 32));
                        if (OUT == OUT_GRAD) grad_w = P.grad_image[cell_ids];
                    }
                    state = LANE_ACTIVE;
                }
                const uint32_t took = (uint32_t)__popcll(need);
                qh += took < qn - qh ? took : qn - qh;
            } else if (next >= j_end && state == LANE_NEED) {
                state = LANE_DONE;
            }
        }
        if (__ballot(state != LANE_DONE) == 0) break;
        if (state == LANE_ACTIVE) {
            // the emitter position is looked up again in every iteration
            // rather than carried across it (scalar loads for one emitter)
            s.xe = emitter_pos(P, s.em);
            bool alive = fly(P, s, st, pd);
            if (alive) {
                const U4 r0 = philox((uint32_t)p, (uint32_t)(p >> 32), (uint32_t)s.k, 0u, P.key0, P.key1);
                const U4 r1 = philox((uint32_t)p, (uint32_t)(p >> 32), (uint32_t)s.k, 1u, P.key0, P.key1);
                direction_darts<OUT, FLOOR>(P, s, r0, st);
                alive = connect_and_event<OUT, FLOOR>(P, p, s, st, grad_w, gacc, pd, r1);
            }
            if (!alive) {
                state = LANE_NEED;
                finish_path<OUT, SRC>(P, s, p, SRC == SRC_TILE ? c0 + slot : cell_ids, slot, img_hi, img_lo, acc_hi,
                                      acc_lo, acc_m2, st, gacc);
            }
        }
    }
}

template <int MODE /*0 DARTS family, 1 vanilla*/, int OUT, bool STATS, int SRC, bool FLOOR>
__device__ __forceinline__ void run_pool(const KParams &P, int64_t c0, uint64_t j_begin, uint64_t j_end,
                                         float *img_hi, float *img_lo, float *acc_hi, float *acc_lo,
                                         float *acc_m2, float *q, float *hist, Stats<STATS> &st, double *gacc)
{
    if constexpr (MODE == 1)
        run_pool_vanilla<STATS, SRC, FLOOR>(P, c0, j_begin, j_end, img_hi, img_lo, q, hist, st);
    else
        run_pool_darts<OUT, STATS, SRC, FLOOR>(P, c0, j_begin, j_end, img_hi, img_lo, acc_hi, acc_lo, acc_m2, q, st,
                                               gacc);
}

// Single-scene render kernel: each wave owns a tile of 64 consecutive cells
// (later time bins first, so the long paths start first) and a chunk of
// repetitions, runs its pool with LDS accumulators and flushes one
// compensated global atomic pair per cell.
typedef __attribute__((address_space(4))) const KParams CKParams;

// The adjoint and the derivative images keep three FP64 accumulators per
// lane and are compiled for 4 waves per SIMD, as are the floor scenes.
template <int OUT, bool FLOOR>
constexpr int render_waves_per_simd()
{
    return OUT == OUT_GRAD || OUT == OUT_TANGENT || FLOOR ? 4 : DARTS_RENDER_WAVES_PER_SIMD;
}

template <int MODE, int OUT, bool STATS, bool FLOOR, int SRC>
__global__ __launch_bounds__(kBlock, (render_waves_per_simd<OUT, FLOOR>())) void render_kernel(KParams P_arg)
{
    // the parameter block, read in place in the kernel-argument segment
    (void)P_arg;
    const KParams &P = *(const KParams *)(CKParams *)__builtin_amdgcn_kernarg_segment_ptr();
    __shared__ float acc_hi[kBlock], acc_lo[kBlock], acc_m2[kBlock];
    __shared__ float qmem[(kBlock / 64) * pool_floats<MODE, OUT>()];
    const int lane = threadIdx.x & 63;
    // the wave's index within the block is the same on all of its lanes: read
    // it as a scalar so that the wave's cell and path ranges (and its LDS
    // offsets) live in scalar registers rather than occupying vector
    // registers for the whole loop
    const uint32_t wave_in_block = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wbase = (int)wave_in_block * 64;
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / 64) + wave_in_block;
    const bool have = wave < P.n_waves;
    int64_t c0;
    uint64_t j_begin, j_end;
    if (SRC == SRC_TILE) {
        const uint64_t tile = have ? wave % P.n_tiles : 0;
        const uint64_t chunk = have ? wave / P.n_tiles : 0;
        c0 = (int64_t)(P.n_tiles - 1 - tile) * 64;
        j_begin = chunk * P.chunk_reps * 64;
        j_end = have ? min((chunk + 1) * P.chunk_reps, P.max_reps) * 64 : j_begin;
    } else if (SRC == SRC_VTILE) {
        // pixel q's paths in the launch are p = q + i npix for i in [i_lo, i_hi)
        const uint64_t npix = (uint64_t)P.npix;
        const uint64_t qp = have ? wave % npix : 0, chunk = have ? wave / npix : 0;
        const uint64_t off = P.path_offset, end = P.path_offset + P.n_paths;
        const uint64_t i_lo = off > qp ? (off - qp + npix - 1) / npix : 0;
        const uint64_t i_hi = end > qp ? (end - qp + npix - 1) / npix : 0;
        j_begin = min(i_lo + chunk * P.vt_chunk, i_hi);
        j_end = have ? min(j_begin + P.vt_chunk, i_hi) : j_begin;
        c0 = (int64_t)qp;
    } else {
        const uint64_t end = P.path_offset + P.n_paths;
        j_begin = P.path_offset + (have ? wave : 0) * P.unit_paths;
        j_end = have ? min(j_begin + P.unit_paths, end) : j_begin;
        c0 = (int64_t)(j_begin % (uint64_t)P.ncells);
    }
    acc_hi[threadIdx.x] = 0.f;
    acc_lo[threadIdx.x] = 0.f;
    acc_m2[threadIdx.x] = 0.f;
    // vanilla pixel decomposition: the wave's histogram (hi, lo[, m2] over
    // hist_bins bins) in dynamic LDS
    extern __shared__ float vhist[];
    const int n_hist = SRC == SRC_VTILE ? (P.m2 ? 3 : 2) * P.hist_bins : 0;
    float *hist = vhist + wave_in_block * n_hist;
    if (SRC == SRC_VTILE)
        for (int b = lane; b < n_hist; b += 64) hist[b] = 0.f;

    Stats<STATS> st;
#pragma unroll
    for (int i = 0; i < DARTS_ST_COUNT; ++i) st.v[i] = 0;
    double gacc[3] = {0.0, 0.0, 0.0};
    run_pool<MODE, OUT, STATS, SRC, FLOOR>(P, c0, j_begin, j_end, P.hi, P.lo, acc_hi + wbase, acc_lo + wbase,
                                           acc_m2 + wbase, qmem + wave_in_block * pool_floats<MODE, OUT>(), hist, st, gacc);

    if (SRC == SRC_VTILE && have) {
        // one compensated global atomic pair per bin the wave's paths reached
        const int nb = P.hist_bins;
        for (int b = lane; b < nb; b += 64) {
            const float h = hist[b], l = hist[nb + b];
            const int64_t cell = P.resp_w ? c0 : (int64_t)b * P.npix + c0;
            if (h != 0.f || l != 0.f) add_compensated(P.hi, P.lo, cell, h, l);
            if (P.m2 && hist[2 * nb + b] != 0.f) unsafeAtomicAdd(P.m2 + cell, hist[2 * nb + b]);
        }
    }

    if (SRC == SRC_TILE && MODE == 0 && OUT == OUT_IMAGE && have) {
        // The flush indices are formed again from the thread index here; the
        // empty asm hides that they equal values known before the path loop,
        // which the compiler would otherwise keep alive across the loop in
        // registers it has to spill to scratch memory.
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        const int64_t cell = c0 + (t & 63);
        const float h = acc_hi[t], l = acc_lo[t];
        if (cell < P.ncells) {
            if (h != 0.f || l != 0.f) add_compensated(P.hi, P.lo, cell, h, l);
            if (P.m2 && acc_m2[t] != 0.f) unsafeAtomicAdd(P.m2 + cell, acc_m2[t]);
        }
    }
    if (OUT == OUT_GRAD) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double v = gacc[i];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0 && v != 0.0) unsafeAtomicAdd(P.grad_out + i, v);
        }
    }
    if (STATS) {
#pragma unroll
        for (int i = 0; i < DARTS_ST_REJECTED + 1; ++i) {
            uint32_t v = st.v[i];
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0 && v) atomicAdd(P.stats + i, (unsigned long long)v);
        }
    }
}

// ---------------------------------------------------------------------------
// Batched persistent render: many scenes (each with its own medium, table,
// sensor, bins and path budget) in one launch.  The host cuts every scene's
// paths into work units; a grid sized to the machine pulls units from a
// global counter (one vector atomic per unit) until none are left, so scenes
// with long paths do not hold up the rest.  The last wave to leave rewinds
// the counters, which makes the launch repeatable (and capturable in a graph)
// without a clearing step.
// ---------------------------------------------------------------------------
struct BItem {
    KParams P;              // the scene's parameters (output pointers unused)
    int64_t image_offset;   // first element of the scene's image in the batch output
};

struct BUnit {
    uint32_t item;
    uint32_t pad;
    int64_t c0;             // SRC_TILE: first tile cell; SRC_IDS: cell of path j_begin
    uint64_t j_begin, j_end;
};

struct BParams {
    const BItem *items;
    const BUnit *units;
    uint32_t n_units;
    uint32_t n_waves;       // waves in the grid
    unsigned *ctr;          // [0] next unit, [1] waves finished; zero between launches
    float *hi, *lo;
};

typedef __attribute__((address_space(4))) const BItem CItem;
typedef __attribute__((address_space(4))) const BUnit CUnit;

template <int SRC, int BLOCK, bool FLOOR>
__global__ __launch_bounds__(BLOCK, DARTS_BATCH_WAVES_PER_SIMD) void batch_kernel(BParams B)
{
    __shared__ float acc_hi[BLOCK], acc_lo[BLOCK];
    __shared__ float qmem[(BLOCK / 64) * pool_floats<0, OUT_IMAGE>()];
    const int lane = threadIdx.x & 63;
    const uint32_t wave_in_block = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wbase = (int)wave_in_block * 64;
    Stats<false> st;
    while (true) {
        uint32_t u = 0;
        if (lane == 0) u = atomicAdd(&B.ctr[0], 1u);
        u = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl((int)u, 0));
        if (u >= B.n_units) break;
        // unit and scene parameters are read-only and wave-uniform: reading
        // them through the constant address space lets them live in scalar
        // registers instead of being loaded per lane
        const CUnit *units = (const CUnit *)B.units;
        const CItem *items = (const CItem *)B.items;
        const uint32_t item = units[u].item;
        const int64_t c0 = units[u].c0;
        const uint64_t j_begin = units[u].j_begin, j_end = units[u].j_end;
        const KParams &P = *(const KParams *)&items[item].P;
        const int64_t off = items[item].image_offset;
        float *img_hi = B.hi + off, *img_lo = B.lo + off;
        if (SRC == SRC_TILE) {
            acc_hi[threadIdx.x] = 0.f;
            acc_lo[threadIdx.x] = 0.f;
        }
        run_pool<0, OUT_IMAGE, false, SRC, FLOOR>(P, c0, j_begin, j_end, img_hi, img_lo, acc_hi + wbase, acc_lo + wbase,
                                                  nullptr, qmem + wave_in_block * pool_floats<0, OUT_IMAGE>(), nullptr, st, nullptr);
        if (SRC == SRC_TILE) {
            const int64_t cell = c0 + lane;
            const float h = acc_hi[threadIdx.x], l = acc_lo[threadIdx.x];
            if (cell < P.ncells && (h != 0.f || l != 0.f)) add_compensated(img_hi, img_lo, cell, h, l);
        }
    }
    // every wave has made its last pull once all have counted themselves out
    if (lane == 0) {
        const unsigned done = atomicAdd(&B.ctr[1], 1u);
        if (done == B.n_waves - 1) {
            atomicExch(&B.ctr[0], 0u);
            atomicExch(&B.ctr[1], 0u);
        }
    }
}

__global__ void zero2_kernel(float *a, float *b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n; k += stride) {
        a[k] = 0.f;
        b[k] = 0.f;
    }
}

// ---------------------------------------------------------------------------
// Elliptical-DA table (Section V-A, Eq. (16)-(18)), FP64.
// One wave per (C/S, S) cell.  The (cos-bin, u-node) pairs of the row's
// quadrature are spread over the 64 lanes (kGLU = 4 u-nodes per cos-bin: 16
// bins per pass of the wave); each lane integrates its pair over the kGLV
// v-nodes, the u-nodes of a bin are summed across 4 neighbouring lanes, and
// the row is normalised and turned into its float CDF by a wave-wide FP64
// prefix sum.
// ---------------------------------------------------------------------------
constexpr int kGLU = 4, kGLV = 64;
static_assert(64 % kGLU == 0, "a cos-bin's u-nodes must share one pass of the wave");

struct TParams {
    double sigma_s, sigma_a, sigma_t, albedo, D;
    int n_cs, n_s, n_cos;
    double s_max;
    double xu[kGLU], wu[kGLU], xv[kGLV], wv[kGLV];
    float *cdf;
};

__device__ double da_phi64(const TParams &T, double r2, double s)
{
    if (!(s > 0.0)) return 0.0;
    const double fds = 4.0 * M_PI * T.D * s;
    return exp(-r2 / (4.0 * T.D * s) - T.sigma_a * s) / (fds * sqrt(fds));
}

__global__ __launch_bounds__(64) void table_kernel(TParams T)
{
    extern __shared__ double row[];
    const int cell = blockIdx.x;
    const int lane = threadIdx.x;
    const int i = cell / T.n_s, j = cell % T.n_s;
    const double kappa = (i + 0.5) / T.n_cs;
    const double S = (j + 0.5) * T.s_max / T.n_s;
    const double C = kappa * S;
    const double h = 2.0 / T.n_cos;
    const int n_pairs = T.n_cos * kGLU;
    for (int base = 0; base < n_pairs; base += 64) {
        const int pidx = base + lane;
        double v = 0.0;
        if (pidx < n_pairs) {
            const int k = pidx / kGLU, a = pidx % kGLU;
            const double u = -1.0 + k * h + 0.5 * h * (T.xu[a] + 1.0);
            const double tM = (S * S - C * C) / (2.0 * S - 2.0 * C * u);   // Eq. (18)
            const double pM = -expm1(-T.sigma_t * tM);
            double inner = 0.0;
            for (int bq = 0; bq < kGLV; ++bq) {
                const double vq = 0.5 * (T.xv[bq] + 1.0);
                const double t = -log1p(-vq * pM) / T.sigma_t;
                const double r2 = fmax(t * t + C * C - 2.0 * t * C * u, 0.0);
                inner += 0.5 * T.wv[bq] * da_phi64(T, r2, S - t);
            }
            v = 0.5 * h * T.wu[a] * T.albedo * pM * inner;
        }
        // the kGLU u-nodes of a cos-bin sit on consecutive lanes
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        if (pidx < n_pairs && (lane & (kGLU - 1)) == 0) row[pidx / kGLU] = v;
    }
    __syncthreads();
    double tot = 0.0;
    for (int k = lane; k < T.n_cos; k += 64) tot += row[k];
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
    const bool good = isfinite(tot) && tot > 0.0;
    float *out = T.cdf + (size_t)cell * (T.n_cos + 1);
    if (lane == 0) out[0] = 0.f;
    double carry = 0.0;
    for (int base = 0; base < T.n_cos; base += 64) {
        const int k = base + lane;
        double x = k < T.n_cos ? (good ? row[k] / tot : 1.0 / T.n_cos) : 0.0;
        for (int o = 1; o < 64; o <<= 1) {   // inclusive prefix sum across the wave
            const double y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        x += carry;
        if (k < T.n_cos) out[k + 1] = k == T.n_cos - 1 ? 1.f : (float)x;
        carry = __shfl(x, 63);
    }
}

// Gauss-Legendre nodes on [-1, 1]: Newton's method on P_n from Tricomi's
// asymptotic initial guess, P_n and P_n' by the three-term recurrence.
void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 1; i <= n; ++i) {
        const double th = M_PI * (4.0 * i - 1.0) / (4.0 * n + 2.0);
        double z = (1.0 - (n - 1.0) / (8.0 * n * n * n)) * std::cos(th);
        double pn = 0.0, dpn = 1.0;
        for (int it = 0; it < 64; ++it) {
            double pm1 = 1.0, p = z;
            for (int k = 1; k < n; ++k) {
                const double pp1 = ((2.0 * k + 1.0) * z * p - k * pm1) / (k + 1.0);
                pm1 = p;
                p = pp1;
            }
            pn = p;
            dpn = n * (pm1 - z * p) / (1.0 - z * z);
            const double step = pn / dpn;
            z -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        double pm1 = 1.0, p = z;
        for (int k = 1; k < n; ++k) {
            const double pp1 = ((2.0 * k + 1.0) * z * p - k * pm1) / (k + 1.0);
            pm1 = p;
            p = pp1;
        }
        dpn = n * (pm1 - z * p) / (1.0 - z * z);
        x[i - 1] = z;
        w[i - 1] = 2.0 / ((1.0 - z * z) * dpn * dpn);
    }
}

// ---------------------------------------------------------------------------
// Pointwise diagnostics.
// ---------------------------------------------------------------------------
struct PWParams {
    int fn;
    int64_t n;
    const float *in;
    float *out;
    Medium med;
    Table tb;
};

__device__ __forceinline__ uint32_t bits(float f) { return __float_as_uint(f); }

__global__ __launch_bounds__(kBlock) void pointwise_kernel(PWParams Q)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= Q.n) return;
    const float *a = Q.in + i * DARTS_PW_IN;
    float *o = Q.out + i * DARTS_PW_OUT;
    switch (Q.fn) {
    case DARTS_PW_PHILOX: {
        const U4 r = philox(bits(a[0]), bits(a[1]), bits(a[2]), bits(a[3]), bits(a[4]), bits(a[5]));
        o[0] = __uint_as_float(r.x); o[1] = __uint_as_float(r.y);
        o[2] = __uint_as_float(r.z); o[3] = __uint_as_float(r.w);
        break;
    }
    case DARTS_PW_HG_PDF: o[0] = hg_pdf(a[0], a[1]); break;
    case DARTS_PW_HG_SAMPLE: hg_sample(a[0], a[1], o[0], o[1]); break;
    case DARTS_PW_DA_LOGPHI: o[0] = da_log_phi_rel(Q.med, a[0] * a[0], a[1]); break;
    case DARTS_PW_TEXP: {
        float emass = 0.f;
        const float mass = isinf(a[2]) ? 1.f : one_minus_exp_neg(a[1] * a[2], emass);
        const float x = texp_sample(a[0], 0.69314718055994530942f / a[1], mass, emass);
        o[0] = x;
        o[1] = a[1] * fast_exp(-a[1] * x) * rcp(mass);
        break;
    }
    case DARTS_PW_ELLIPSE: {
        float den, t, r;
        const float S = a[0], C = a[1], mu = a[2];
        ellipse(S, C, S - C, C * (1.f - mu), den, t, r);
        o[0] = t; o[1] = r; o[2] = a[3] * den / r;
        break;
    }
    case DARTS_PW_SOBOL: o[0] = sobol_u(bits(a[0]), bits(a[1]), bits(a[2])); break;
    case DARTS_PW_ONB: {
        V3 b1, b2;
        onb(V3{a[0], a[1], a[2]}, b1, b2);
        o[0] = b1.x; o[1] = b1.y; o[2] = b1.z; o[3] = b2.x; o[4] = b2.y; o[5] = b2.z;
        break;
    }
    case DARTS_PW_BOX_EXIT: {
        Box b{{a[6], a[7], a[8]}, {a[9], a[10], a[11]}};
        o[0] = box_exit(b, V3{a[0], a[1], a[2]}, V3{a[3], a[4], a[5]});
        break;
    }
    case DARTS_PW_RIS: {
        const V3 x{a[0], a[1], a[2]}, w{a[3], a[4], a[5]}, xe{a[6], a[7], a[8]};
        const float R_hi = a[9], d_m = a[10];
        const V3 de = xe - x;
        const float C = length(de);
        float epc = 0.f;
        const float pc = isinf(d_m) ? 1.f : one_minus_exp_neg(Q.med.sigma_t * d_m, epc);
        float d = 0.f, f = 0.f;
        uint32_t choice = 0;
        const bool okk = ris_distance(Q.med, C * C, dot(w, de), R_hi, pc, epc, bits(a[11]) & 31u, bits(a[12]), a[13],
                                      d, f, &choice);
        o[0] = okk ? 1.f : 0.f; o[1] = d; o[2] = f;
        o[3] = okk ? (float)(choice & 0xFFu) : -1.f;
        o[4] = (float)(choice >> 8);
        break;
    }
    case DARTS_PW_DIRECTION: {
        const V3 x{a[0], a[1], a[2]}, xe{a[3], a[4], a[5]}, wp{a[6], a[7], a[8]};
        const float S = a[9];
        const U4 r{bits(a[10]), bits(a[11]), bits(a[12]), bits(a[13])};
        const V3 de = xe - x;
        const float C = length(de);
        float wt;
        bool eb;
        int dbg[2] = {-1, -1};
        const V3 w = sample_direction(Q.med, Q.tb, a[15], a[14] != 0.f, de * rcp(C), C, S, wp, r, wt, eb, dbg);
        o[0] = w.x; o[1] = w.y; o[2] = w.z; o[3] = wt; o[4] = eb ? 1.f : 0.f;
        o[5] = (float)dbg[0]; o[6] = (float)dbg[1];
        break;
    }
    case DARTS_PW_EXIT_LENGTH: {
        const V3 x{a[0], a[1], a[2]}, w{a[3], a[4], a[5]}, xe{a[6], a[7], a[8]};
        float excess;
        o[0] = exit_length(x, w, xe, length(xe - x), a[9], excess);
        o[1] = excess;
        break;
    }
    case DARTS_PW_CONNECT: {
        KParams P{};
        P.med = Q.med;
        P.box = a[14] != 0.f ? 1 : 0;
        P.bx = Box{{-1.f, -1.f, -1.f}, {1.f, 1.f, 1.f}};
        P.flags = a[13] != 0.f ? DARTS_ELL_TEXP : DARTS_ELL_UNIFORM;
        PathState s{};
        s.x = V3{a[0], a[1], a[2]};
        s.w = V3{a[3], a[4], a[5]};
        s.xe = V3{a[6], a[7], a[8]};
        s.C = length(s.xe - s.x);
        s.G_lo = a[9];
        s.G_hi = a[10];
        s.Le = 0.f;
        s.dm = P.box ? a[11] : kInf;
        s.beta = 1.f;
        s.em_scale = 1.f;
        Stats<false> st;
        float lo = 0.f, hi = 0.f;
        const bool reached = connect_range(P, s, lo, hi);
        o[0] = connect(P, s, a[12], nullptr, st);
        Conn q;
        q.x = s.x; q.w = s.w; q.xe = s.xe; q.C = s.C; q.lo = lo; q.hi = hi; q.scale = 1.f; q.u = a[12]; q.dm = s.dm;
        float mu_c = 0.f, t = 0.f, r_in = 0.f;
        if (reached) connect_eval(P, q, mu_c, t, r_in);
        o[1] = t; o[2] = r_in; o[3] = mu_c; o[4] = reached ? 1.f : 0.f; o[5] = lo; o[6] = hi;
        break;
    }
    case DARTS_PW_MATH: {
        const float x = a[0];
        o[0] = rcp(x); o[1] = rsq(x); o[2] = log2_hw(x); o[3] = exp2_hw(x);
        sincos_rev(x, o[4], o[5]);
        o[6] = hw_sqrt(x);
        break;
    }
    default: break;
    }
}

// ---------------------------------------------------------------------------
// Host-side validation and parameter set-up.
// ---------------------------------------------------------------------------
int check_medium(const darts_medium *m)
{
    if (!m) return fail(DARTS_ERR_INVALID_ARG, "medium is null");
    if (!(m->sigma_s >= 0.0) || !(m->sigma_a >= 0.0) || !(m->sigma_s + m->sigma_a > 0.0) ||
        !std::isfinite(m->sigma_s) || !std::isfinite(m->sigma_a))
        return fail(DARTS_ERR_INVALID_ARG, "need sigma_s, sigma_a >= 0 and sigma_s + sigma_a > 0");
    if (!(std::fabs(m->g) < 1.0)) return fail(DARTS_ERR_INVALID_ARG, "need |g| < 1");
    return DARTS_OK;
}

int check_dims(const darts_table_dims *d)
{
    if (!d) return fail(DARTS_ERR_INVALID_ARG, "table dims are null");
    if (d->n_cs <= 0 || d->n_s <= 0 || d->n_cos <= 0 || d->n_cos > DARTS_MAX_COS_BINS || !(d->s_max > 0.f) ||
        !std::isfinite(d->s_max))
        return fail(DARTS_ERR_INVALID_ARG, "table dims must be positive, n_cos <= %d, s_max > 0",
                    DARTS_MAX_COS_BINS);
    if ((int64_t)d->n_cs * d->n_s > (1 << 26) || (int64_t)d->n_cs * d->n_s * (d->n_cos + 1) > INT32_MAX)
        return fail(DARTS_ERR_INVALID_ARG, "table too large");
    return DARTS_OK;
}

Medium make_medium(const darts_medium &m)
{
    Medium o;
    o.sigma_s = (float)m.sigma_s;
    o.sigma_a = (float)m.sigma_a;
    o.sigma_t = (float)(m.sigma_s + m.sigma_a);
    o.inv_sigma_t = (float)(1.0 / (m.sigma_s + m.sigma_a));
    o.albedo = (float)(m.sigma_s / (m.sigma_s + m.sigma_a));
    o.g = (float)m.g;
    const double D = 1.0 / (3.0 * (m.sigma_a + m.sigma_s * (1.0 - m.g)));
    o.inv4D = (float)(1.0 / (4.0 * D));
    o.ln2_over_sigma_t = (float)(0.69314718055994530942 / (m.sigma_s + m.sigma_a));
    o.inv4D_log2e = (float)(1.4426950408889634074 / (4.0 * D));
    o.sigma_a_log2e = (float)(1.4426950408889634074 * m.sigma_a);
    o.four_D_sigma_a = (float)(4.0 * D * m.sigma_a);
    o.hg = hg_consts(o.g);
    return o;
}

bool same_medium(const darts_medium &a, const darts_medium &b)
{
    return a.sigma_s == b.sigma_s && a.sigma_a == b.sigma_a && a.g == b.g;
}

int fill_table(const darts_table *t, const darts_scene *sc, bool needed, Table &tb)
{
    tb = Table{nullptr, 1, 1, 1, 1, 0.f, 1.f, 1.f, 2.f};
    if (!needed) return DARTS_OK;
    if (!t || !t->cdf_dev) return fail(DARTS_ERR_INVALID_ARG, "EDA direction sampling needs a built table");
    if (int rc = check_dims(&t->dims)) return rc;
    if (sc && !same_medium(t->medium, sc->medium))
        return fail(DARTS_ERR_TABLE_MISMATCH, "table was built for another medium");
    tb.cdf = t->cdf_dev;
    tb.n_cs = t->dims.n_cs;
    tb.n_s = t->dims.n_s;
    tb.n_cos = t->dims.n_cos;
    tb.cos_pow2 = 1;
    while (tb.cos_pow2 <= tb.n_cos / 2) tb.cos_pow2 *= 2;
    tb.ns_over_smax = (float)t->dims.n_s / t->dims.s_max;
    tb.fn_cs = (float)tb.n_cs;
    tb.fn_cos = (float)tb.n_cos;
    tb.cos_step = 2.f / (float)tb.n_cos;
    return DARTS_OK;
}

std::atomic<int64_t> g_ids_max_reps{16};         // id ranges when no cell has more repetitions
constexpr uint64_t kIdsUnit = 2048;   // most paths per wave in the id-range decomposition
constexpr uint64_t kIdsWaves = 16384; // waves the id-range decomposition aims for
std::atomic<int64_t> g_target_waves{1 << 16};   // measured: 4 chunks per tile balance the 2^28-path box frame best
std::atomic<int> g_vanilla_privatised{1};      // vanilla renders histogram per pixel in LDS when it fits
// most bins of a vanilla pixel histogram in LDS: hi, lo and m2 of 4 waves
// (18 KiB) beside the 21 KiB of static LDS keep 4 blocks on a CU
constexpr int kVTileMaxBins = 384;

int make_params(const darts_scene *sc, const darts_params *pr, const darts_table *table, KParams &P,
                bool per_path_only)
{
    if (!sc || !pr) return fail(DARTS_ERR_INVALID_ARG, "scene or params is null");
    if (int rc = check_medium(&sc->medium)) return rc;
    if (sc->n_emitters < 1 || sc->n_emitters > DARTS_MAX_EMITTERS || !sc->emitters)
        return fail(DARTS_ERR_INVALID_ARG, "need 1..%d emitters", DARTS_MAX_EMITTERS);
    if (sc->bins.n_bins <= 0 || !(sc->bins.l_hi > sc->bins.l_lo) || !std::isfinite(sc->bins.l_lo) ||
        !std::isfinite(sc->bins.l_hi))
        return fail(DARTS_ERR_INVALID_ARG, "bins need n_bins > 0 and l_hi > l_lo");
    const darts_sensor &sn = sc->sensor;
    if (sn.kind != 0 && sn.kind != 1) return fail(DARTS_ERR_INVALID_ARG, "sensor kind must be 0 or 1");
    if (sn.width <= 0 || sn.height <= 0) return fail(DARTS_ERR_INVALID_ARG, "sensor size must be positive");
    if (sn.width > 65535 || sn.height > 65535)
        return fail(DARTS_ERR_INVALID_ARG, "sensor sides are limited to 65535 pixels");
    if (sc->bins.n_bins >= (1 << 29)) return fail(DARTS_ERR_INVALID_ARG, "n_bins must be below 2^29");
    if (sn.kind == 0 && (sn.width != 1 || sn.height != 1))
        return fail(DARTS_ERR_INVALID_ARG, "point detector has width = height = 1");
    if (sc->geom.kind < 0 || sc->geom.kind > 2) return fail(DARTS_ERR_INVALID_ARG, "geometry kind must be 0, 1 or 2");
    if (sc->geom.kind == 2 && !(sc->geom.floor_albedo >= 0.f && sc->geom.floor_albedo <= 1.f))
        return fail(DARTS_ERR_INVALID_ARG, "floor albedo must be in [0, 1]");
    if (sc->geom.kind >= 1)
        for (int a = 0; a < 3; ++a)
            if (!(sc->geom.hi[a] > sc->geom.lo[a])) return fail(DARTS_ERR_INVALID_ARG, "box needs hi > lo");
    if (pr->max_bounces < 1) return fail(DARTS_ERR_INVALID_ARG, "max_bounces must be >= 1");
    if (pr->n_ris != 8) return fail(DARTS_ERR_UNSUPPORTED, "only n_ris = 8 (the paper's candidate count) is implemented");
    if (!(pr->alpha >= 0.f)) return fail(DARTS_ERR_INVALID_ARG, "alpha must be >= 0");
    const unsigned f = pr->flags;
    if (f & ~(DARTS_RIS_DIST | DARTS_EDA_DIR | DARTS_ELL_TEXP | DARTS_ELL_UNIFORM | DARTS_DIRECT_REUSE))
        return fail(DARTS_ERR_INVALID_ARG, "unknown flag bits 0x%x", f);
    const bool vanilla = (f & DARTS_DIRECT_REUSE) != 0;
    if (vanilla && (f != DARTS_DIRECT_REUSE))
        return fail(DARTS_ERR_INVALID_ARG, "DIRECT_REUSE (vanilla) excludes the other strategy bits");
    if (!vanilla && (((f & DARTS_ELL_TEXP) != 0) == ((f & DARTS_ELL_UNIFORM) != 0)))
        return fail(DARTS_ERR_INVALID_ARG, "exactly one of ELL_TEXP / ELL_UNIFORM");
    if (per_path_only && vanilla) return fail(DARTS_ERR_UNSUPPORTED, "per-path output needs the DARTS family");
    if (int rc = fill_table(table, sc, !vanilla && (f & DARTS_EDA_DIR), P.tb)) return rc;

    std::memset(&P.em_pos, 0, sizeof P.em_pos);
    P.med = make_medium(sc->medium);
    P.box = sc->geom.kind >= 1 ? 1 : 0;
    P.floor = sc->geom.kind == 2 ? 1 : 0;
    P.floor_albedo = sc->geom.kind == 2 ? sc->geom.floor_albedo : 0.f;
    for (int a = 0; a < 3; ++a) { P.bx.lo[a] = sc->geom.lo[a]; P.bx.hi[a] = sc->geom.hi[a]; }
    P.n_em = sc->n_emitters;
    for (int j = 0; j < P.n_em; ++j) {
        const darts_emitter &e = sc->emitters[j];
        if (!std::isfinite(e.start) || !(e.power >= 0.f)) return fail(DARTS_ERR_INVALID_ARG, "bad emitter %d", j);
        for (int a = 0; a < 3; ++a) P.em_pos[j][a] = e.pos[a];
        P.em_start[j] = e.start;
        P.em_scale[j] = (float)(e.power / (4.0 * M_PI) * sc->n_emitters);
    }
    P.sensor_kind = sn.kind;
    double dl = 0;
    for (int a = 0; a < 3; ++a) dl += (double)sn.dir[a] * sn.dir[a];
    if (sn.kind == 1 && !(dl > 0)) return fail(DARTS_ERR_INVALID_ARG, "sensor dir must be non-zero");
    dl = std::sqrt(dl);
    for (int a = 0; a < 3; ++a) {
        P.origin[a] = sn.origin[a];
        P.dir[a] = sn.kind == 1 ? (float)(sn.dir[a] / dl) : 0.f;
        P.inv_dir[a] = P.dir[a] != 0.f ? 1.f / P.dir[a] : 0.f;
        P.du[a] = sn.du[a];
        P.dv[a] = sn.dv[a];
    }
    P.width = sn.width;
    P.height = sn.height;
    P.inv_width = 1.f / (float)sn.width;
    P.inv_height = 1.f / (float)sn.height;
    P.beta0 = sn.kind == 0 ? (float)(4.0 * M_PI) : 1.f;
    P.l_lo = sc->bins.l_lo;
    P.l_hi = sc->bins.l_hi;
    P.n_bins = sc->bins.n_bins;
    P.delta = (float)(((double)sc->bins.l_hi - sc->bins.l_lo) / sc->bins.n_bins);
    P.path_offset = pr->path_offset;
    P.n_paths = pr->n_paths;
    P.key0 = (uint32_t)pr->seed;
    P.key1 = (uint32_t)(pr->seed >> 32);
    P.max_bounces = pr->max_bounces;
    P.alpha = pr->alpha;
    P.flags = f;
    P.npix = (int64_t)sn.width * sn.height;
    P.ncells = P.npix * sc->bins.n_bins;
    P.resp_cdf = P.resp_w = nullptr;
    if (sc->response_dev) {
        // one value per pixel; table = cdf[n_bins + 1] then W[n_bins]
        P.ncells = P.npix;
        P.resp_cdf = sc->response_dev;
        P.resp_w = sc->response_dev + sc->bins.n_bins + 1;
    }
    if (P.ncells > ((int64_t)1 << 40)) return fail(DARTS_ERR_INVALID_ARG, "image too large");
    const uint64_t nc = (uint64_t)P.ncells;
    if (pr->path_offset > UINT64_MAX - pr->n_paths) return fail(DARTS_ERR_INVALID_ARG, "path id range overflows");
    const uint64_t end = pr->path_offset + pr->n_paths;
    P.q0 = pr->path_offset / nc;
    P.r0 = pr->path_offset % nc;
    P.q1 = end / nc;
    P.r1 = end % nc;
    // repetitions per cell: at most ceil(n / nc) + 1.  Waves own tiles of 64
    // cells; the repetitions are split into chunks (of at least 32, so that a
    // wave's pool amortises its last path) until the launch has about
    // g_target_waves waves.
    P.max_reps = (P.q1 + (P.r1 > 0 ? 1 : 0)) - P.q0;
    P.n_tiles = (nc + 63) / 64;
    const int64_t target_waves = g_target_waves.load(std::memory_order_relaxed);
    uint64_t n_chunks = (uint64_t)std::max<int64_t>(1, (target_waves + (int64_t)P.n_tiles - 1) / (int64_t)P.n_tiles);
    n_chunks = std::max<uint64_t>(1, std::min(n_chunks, (P.max_reps + 31) / 32));
    P.chunk_reps = (P.max_reps + n_chunks - 1) / n_chunks;
    if (P.chunk_reps == 0) P.chunk_reps = 1;
    n_chunks = (P.max_reps + P.chunk_reps - 1) / P.chunk_reps;
    P.n_waves = P.n_tiles * n_chunks;
    // few repetitions per cell: a tile's wave would run a handful of paths per
    // lane and idle while its longest path finishes, so waves take ranges of
    // consecutive ids instead (each finished path adds to the image directly)
    // (units of up to kIdsUnit paths, smaller when that would leave fewer
    // than about kIdsWaves waves to spread over the device)
    P.unit_paths = 0;
    if ((int64_t)P.max_reps <= g_ids_max_reps.load(std::memory_order_relaxed)) {
        const uint64_t want = (pr->n_paths + kIdsWaves - 1) / kIdsWaves;
        P.unit_paths = std::min<uint64_t>(nc, std::max<uint64_t>(64, std::min<uint64_t>(kIdsUnit, want)));
        P.n_waves = (pr->n_paths + P.unit_paths - 1) / P.unit_paths;
    }
    // vanilla with many paths per pixel: waves own pixels and histogram their
    // paths' contributions in LDS (flushed once per wave) instead of one
    // compensated global atomic pair per contribution
    P.vtile = 0;
    P.hist_bins = 0;
    P.vt_chunk = 0;
    if (vanilla && g_vanilla_privatised.load(std::memory_order_relaxed)) {
        const int nb = sc->response_dev ? 1 : sc->bins.n_bins;
        const uint64_t ppp = pr->n_paths / (uint64_t)P.npix;   // paths per pixel (at least)
        if (nb <= kVTileMaxBins && ppp >= 256) {
            const int64_t target_waves = g_target_waves.load(std::memory_order_relaxed);
            uint64_t chunks = (uint64_t)std::max<int64_t>(1, target_waves / P.npix);
            chunks = std::max<uint64_t>(1, std::min<uint64_t>(chunks, ppp / 256));
            P.vtile = 1;
            P.hist_bins = nb;
            P.vt_chunk = (ppp + 1 + chunks - 1) / chunks;
            P.n_waves = (uint64_t)P.npix * ((ppp + 1 + P.vt_chunk - 1) / P.vt_chunk);
        }
    }
    if (P.n_waves / (kBlock / 64) > 0x7FFFFFFFull) return fail(DARTS_ERR_INVALID_ARG, "launch too large");
    P.hi = P.lo = P.m2 = nullptr;
    P.stats = nullptr;
    P.path_out = nullptr;
    P.grad_image = nullptr;
    P.grad_out = nullptr;
    P.tangent = nullptr;
    return DARTS_OK;
}

template <int MODE, int OUT>
int launch_render(const KParams &P, bool stats, hipStream_t stream)
{
    const uint64_t blocks = (P.n_waves + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks == 0 || P.n_paths == 0) return ok();
    const dim3 grid((uint32_t)blocks), block(kBlock);
    // scenes without a floor run kernels compiled without its branches
    if constexpr (MODE == 1) {
        if (P.vtile) {
            const size_t lds = (size_t)(kBlock / 64) * (P.m2 ? 3 : 2) * (size_t)P.hist_bins * sizeof(float);
            if (P.floor) {
                if (stats) hipLaunchKernelGGL((render_kernel<MODE, OUT, true, true, SRC_VTILE>), grid, block, lds, stream, P);
                else hipLaunchKernelGGL((render_kernel<MODE, OUT, false, true, SRC_VTILE>), grid, block, lds, stream, P);
            } else {
                if (stats) hipLaunchKernelGGL((render_kernel<MODE, OUT, true, false, SRC_VTILE>), grid, block, lds, stream, P);
                else hipLaunchKernelGGL((render_kernel<MODE, OUT, false, false, SRC_VTILE>), grid, block, lds, stream, P);
            }
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return fail(DARTS_ERR_DEVICE, "render launch failed: %s", hipGetErrorString(e));
            return ok();
        }
    }
    if (P.unit_paths) {
        if (P.floor) {
            if (stats) hipLaunchKernelGGL((render_kernel<MODE, OUT, true, true, SRC_IDS>), grid, block, 0, stream, P);
            else hipLaunchKernelGGL((render_kernel<MODE, OUT, false, true, SRC_IDS>), grid, block, 0, stream, P);
        } else {
            if (stats) hipLaunchKernelGGL((render_kernel<MODE, OUT, true, false, SRC_IDS>), grid, block, 0, stream, P);
            else hipLaunchKernelGGL((render_kernel<MODE, OUT, false, false, SRC_IDS>), grid, block, 0, stream, P);
        }
    } else if (P.floor) {
        if (stats) hipLaunchKernelGGL((render_kernel<MODE, OUT, true, true, SRC_TILE>), grid, block, 0, stream, P);
        else hipLaunchKernelGGL((render_kernel<MODE, OUT, false, true, SRC_TILE>), grid, block, 0, stream, P);
    } else {
        if (stats) hipLaunchKernelGGL((render_kernel<MODE, OUT, true, false, SRC_TILE>), grid, block, 0, stream, P);
        else hipLaunchKernelGGL((render_kernel<MODE, OUT, false, false, SRC_TILE>), grid, block, 0, stream, P);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DARTS_ERR_DEVICE, "render launch failed: %s", hipGetErrorString(e));
    return ok();
}

// ---------------------------------------------------------------------------
// Batched render: host side
// ---------------------------------------------------------------------------
bool valid_plan(const darts_batch_plan &pl)
{
    return (pl.order == DARTS_BATCH_TILES || pl.order == DARTS_BATCH_IDS) &&
           (pl.block_threads == 64 || pl.block_threads == 256) && pl.waves_per_cu >= 1 && pl.waves_per_cu <= 64 &&
           pl.unit_paths >= 64 && pl.unit_paths <= ((int64_t)1 << 32);
}

darts_batch_plan default_plan()
{
    darts_batch_plan pl;
    pl.order = DARTS_BATCH_TILES;
    pl.block_threads = 256;
    pl.waves_per_cu = 16;
    pl.unit_paths = 8192;
    return pl;
}

// Rough cost of one path of a scene (vertex steps), used only to start the
// expensive units first: the walk ends after about sigma_t * length steps or
// at max_bounces.
double path_cost(const KParams &P)
{
    const double len = std::max(1.0, (double)P.l_hi - (double)P.l_lo);
    const double steps = 2.0 + (double)P.med.sigma_t * std::min(len, 1.0 / std::max((double)P.med.sigma_a, 1e-6));
    return std::min(steps, (double)P.max_bounces + 1.0);
}

// Number of repetitions of cell c in the scene's path range.
uint64_t reps_of(const KParams &P, uint64_t c)
{
    return (P.q1 + (c < P.r1 ? 1 : 0)) - (P.q0 + (c < P.r0 ? 1 : 0));
}

struct UnitCost {
    BUnit u;
    double cost;
    uint64_t seq;   // position in enumeration order (ties keep it)
};

// Enumerate the work units of `items` under plan `pl`, calling push(UnitCost)
// for each; returns false as soon as push does.
template <class Push>
bool enumerate_units(const BItem *items, size_t n_items, const darts_batch_plan &pl, Push push)
{
    uint64_t seq = 0;
    for (size_t i = 0; i < n_items; ++i) {
        const KParams &P = items[i].P;
        const double pc = path_cost(P);
        const uint64_t nc = (uint64_t)P.ncells;
        if (P.n_paths == 0) continue;
        if (pl.order == DARTS_BATCH_TILES) {
            const uint64_t reps_unit = std::max<uint64_t>(1, (uint64_t)pl.unit_paths / 64);
            for (uint64_t t = 0; t < (uint64_t)P.n_tiles; ++t) {
                // later bins first inside a scene (long paths start early)
                const uint64_t c0 = ((uint64_t)P.n_tiles - 1 - t) * 64;
                const uint64_t c1 = std::min(c0 + 64, nc) - 1;
                // repetitions per cell change only at r0 and r1
                uint64_t reps = std::max(reps_of(P, c0), reps_of(P, c1));
                if (P.r0 > c0 && P.r0 <= c1) reps = std::max(reps, reps_of(P, P.r0));
                if (P.r1 > c0 && P.r1 <= c1) reps = std::max(reps, reps_of(P, P.r1 - 1));
                for (uint64_t r = 0; r < reps; r += reps_unit) {
                    UnitCost uc;
                    uc.u.item = (uint32_t)i;
                    uc.u.pad = 0;
                    uc.u.c0 = (int64_t)c0;
                    uc.u.j_begin = r * 64;
                    uc.u.j_end = std::min(r + reps_unit, reps) * 64;
                    uc.cost = pc * (double)(uc.u.j_end - uc.u.j_begin);
                    uc.seq = seq++;
                    if (!push(uc)) return false;
                }
            }
        } else {
            const uint64_t step = std::min<uint64_t>((uint64_t)pl.unit_paths, nc);
            const uint64_t end = P.path_offset + P.n_paths;
            for (uint64_t j = P.path_offset; j < end; j += std::min(step, end - j)) {
                UnitCost uc;
                uc.u.item = (uint32_t)i;
                uc.u.pad = 0;
                uc.u.c0 = (int64_t)(j % nc);
                uc.u.j_begin = j;
                uc.u.j_end = j + std::min(step, end - j);
                uc.cost = pc * (double)(uc.u.j_end - uc.u.j_begin);
                uc.seq = seq++;
                if (!push(uc)) return false;
            }
        }
    }
    return true;
}

// Most expensive units first; equal costs keep their enumeration order.
inline bool unit_before(const UnitCost &a, const UnitCost &b)
{
    return a.cost > b.cost || (a.cost == b.cost && a.seq < b.seq);
}

void build_units(const std::vector<BItem> &items, const darts_batch_plan &pl, std::vector<BUnit> &out)
{
    std::vector<UnitCost> v;
    enumerate_units(items.data(), items.size(), pl, [&](const UnitCost &uc) {
        v.push_back(uc);
        return true;
    });
    std::sort(v.begin(), v.end(), unit_before);
    out.resize(v.size());
    for (size_t k = 0; k < v.size(); ++k) out[k] = v[k].u;
}

}  // namespace

struct darts_batch {
    int device = 0;
    int n_cu = 0;
    std::vector<BItem> items;
    std::vector<int64_t> offsets;
    darts_batch_plan plan{};
    BItem *items_dev = nullptr;
    BUnit *units_dev = nullptr;
    uint32_t n_units = 0;
    unsigned *ctr_dev = nullptr;
    hipGraphExec_t exec = nullptr;
    float *graph_hi = nullptr, *graph_lo = nullptr;
    bool any_floor = false;   // some scene has a floor: the batch runs the floor kernels
};

namespace {

void drop_graph(darts_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->graph_hi = b->graph_lo = nullptr;
}

int upload_units(darts_batch *b, const darts_batch_plan &pl)
{
    std::vector<BUnit> units;
    build_units(b->items, pl, units);
    if (units.size() > 0xFFFFFFF0ull) return fail(DARTS_ERR_INVALID_ARG, "too many work units; raise unit_paths");
    BUnit *dev = nullptr;
    if (!units.empty()) {
        if (hipMalloc(&dev, units.size() * sizeof(BUnit)) != hipSuccess)
            return fail(DARTS_ERR_DEVICE, "allocating %zu work units failed", units.size());
        if (hipMemcpy(dev, units.data(), units.size() * sizeof(BUnit), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(dev);
            return fail(DARTS_ERR_DEVICE, "uploading work units failed");
        }
    }
    if (b->units_dev) (void)hipFree(b->units_dev);
    b->units_dev = dev;
    b->n_units = (uint32_t)units.size();
    b->plan = pl;
    drop_graph(b);
    return DARTS_OK;
}

// One launch of the batch kernel over `n_units` units (device arrays of the
// scenes' parameter blocks and of the units, and the two unit counters, zero
// at entry; the launch leaves them zero).
int launch_batch_units(int n_cu, const darts_batch_plan &plan, bool any_floor, const BItem *items_dev,
                       const BUnit *units_dev, uint32_t n_units, unsigned *ctr_dev, float *hi, float *lo,
                       hipStream_t stream)
{
    if (n_units == 0) return ok();
    const int per_block = plan.block_threads / 64;
    const uint32_t blocks = (uint32_t)std::max(1, n_cu * plan.waves_per_cu / per_block);
    BParams B;
    B.items = items_dev;
    B.units = units_dev;
    B.n_units = n_units;
    B.n_waves = blocks * (uint32_t)per_block;   // exactly the waves launched: the last one rewinds the counter
    B.ctr = ctr_dev;
    B.hi = hi;
    B.lo = lo;
    const dim3 grid(blocks);
    const bool tiles = plan.order == DARTS_BATCH_TILES;
    if (any_floor) {
        if (plan.block_threads == 64) {
            if (tiles) hipLaunchKernelGGL((batch_kernel<SRC_TILE, 64, true>), grid, dim3(64), 0, stream, B);
            else hipLaunchKernelGGL((batch_kernel<SRC_IDS, 64, true>), grid, dim3(64), 0, stream, B);
        } else {
            if (tiles) hipLaunchKernelGGL((batch_kernel<SRC_TILE, 256, true>), grid, dim3(256), 0, stream, B);
            else hipLaunchKernelGGL((batch_kernel<SRC_IDS, 256, true>), grid, dim3(256), 0, stream, B);
        }
    } else {
        if (plan.block_threads == 64) {
            if (tiles) hipLaunchKernelGGL((batch_kernel<SRC_TILE, 64, false>), grid, dim3(64), 0, stream, B);
            else hipLaunchKernelGGL((batch_kernel<SRC_IDS, 64, false>), grid, dim3(64), 0, stream, B);
        } else {
            if (tiles) hipLaunchKernelGGL((batch_kernel<SRC_TILE, 256, false>), grid, dim3(256), 0, stream, B);
            else hipLaunchKernelGGL((batch_kernel<SRC_IDS, 256, false>), grid, dim3(256), 0, stream, B);
        }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DARTS_ERR_DEVICE, "batch launch failed: %s", hipGetErrorString(e));
    return ok();
}

int launch_batch(const darts_batch *b, float *hi, float *lo, hipStream_t stream)
{
    return launch_batch_units(b->n_cu, b->plan, b->any_floor, b->items_dev, b->units_dev, b->n_units, b->ctr_dev, hi,
                              lo, stream);
}

// ---------------------------------------------------------------------------
// Batched render without allocation.  The scenes' parameter blocks, the work
// units and the two unit counters live in `scratch`, one fixed array per
// device that stays allocated until the process ends.  Host code never passes
// the array's name to a kernel or a copy (in host code it is a host-side
// stand-in, not a device address): it uses the device address that
// hipGetSymbolAddress returns, fetched once per device with that device
// current.  The host side stages the same bytes in `g_stage` (a fixed host
// array) and copies them over with two asynchronous copies.
// Layout: [0, 256) counters; [256, 256 + items) parameter blocks (rounded up
// to 256 bytes); then the units.  While the units are sorted on the host
// they take sizeof(UnitCost) bytes each in the staging array.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr size_t kScratchItemsOff = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

alignas(256) unsigned char g_stage[kScratchBytes];
std::mutex g_noalloc_mu;            // guards g_stage and the per-device tables below
void *g_scratch_dev[kMaxDevices];   // device address of `scratch` on each device (null until first use)
int g_scratch_ncu[kMaxDevices];

__global__ void clear_counters_kernel(unsigned *ctr)
{
    if (threadIdx.x < 2) ctr[threadIdx.x] = 0u;
}

// Device address of this device's scratch array and its compute-unit count;
// called with g_noalloc_mu held.
int scratch_of_device(unsigned char **ptr, int *n_cu)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(DARTS_ERR_DEVICE, "no current HIP device");
    if (dev < 0 || dev >= kMaxDevices) return fail(DARTS_ERR_UNSUPPORTED, "device index %d is not below %d", dev, kMaxDevices);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DARTS_ERR_DEVICE, "address of the scratch array on device %d: %s", dev, hipGetErrorString(e));
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1)
            return fail(DARTS_ERR_DEVICE, "compute-unit count of device %d unavailable", dev);
        g_scratch_ncu[dev] = cu;
        g_scratch_dev[dev] = p;
    }
    *ptr = (unsigned char *)g_scratch_dev[dev];
    *n_cu = g_scratch_ncu[dev];
    return DARTS_OK;
}

int check_batch_device(const darts_batch *b)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return fail(DARTS_ERR_INVALID_ARG, "batch was created on device %d, current device is %d", b->device, dev);
    return DARTS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *darts_last_error(void) { return g_last_error.c_str(); }

int darts_abi_version(void) { return DARTS_ABI_VERSION; }

int darts_table_bytes(const darts_table_dims *dims, size_t *bytes)
{
    if (int rc = check_dims(dims)) return rc;
    if (!bytes) return fail(DARTS_ERR_INVALID_ARG, "bytes is null");
    *bytes = (size_t)dims->n_cs * dims->n_s * (dims->n_cos + 1) * sizeof(float);
    return ok();
}

int darts_response_bytes(int n_bins, size_t *bytes)
{
    if (n_bins < 1) return fail(DARTS_ERR_INVALID_ARG, "n_bins must be >= 1");
    if (!bytes) return fail(DARTS_ERR_INVALID_ARG, "bytes is null");
    *bytes = (size_t)(2 * (int64_t)n_bins + 1) * sizeof(float);
    return ok();
}

int darts_build_response(const float *w_host, int n_bins, float *response_dev, void *stream)
{
    if (n_bins < 1 || !w_host || !response_dev) return fail(DARTS_ERR_INVALID_ARG, "bad response arguments");
    double tot = 0.0;
    for (int k = 0; k < n_bins; ++k) {
        if (!(w_host[k] >= 0.f) || !std::isfinite(w_host[k]))
            return fail(DARTS_ERR_INVALID_ARG, "response W[%d] must be finite and >= 0", k);
        tot += w_host[k];
    }
    if (!(tot > 0.0)) return fail(DARTS_ERR_INVALID_ARG, "response W is all zero");
    std::vector<float> h((size_t)(2 * n_bins + 1));
    double run = 0.0;
    h[0] = 0.f;
    for (int k = 0; k < n_bins; ++k) {
        run += w_host[k];
        h[(size_t)k + 1] = k == n_bins - 1 ? 1.f : (float)(run / tot);
        h[(size_t)n_bins + 1 + k] = w_host[k];
    }
    if (hipMemcpyAsync(response_dev, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice,
                       (hipStream_t)stream) != hipSuccess ||
        hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return fail(DARTS_ERR_DEVICE, "copying the response table failed");
    return ok();
}

int darts_build_da_tables(const darts_medium *medium, const darts_table_dims *dims, float *cdf_dev, void *stream)
{
    if (int rc = check_medium(medium)) return rc;
    if (int rc = check_dims(dims)) return rc;
    if (!cdf_dev) return fail(DARTS_ERR_INVALID_ARG, "cdf_dev is null");
    TParams T;
    T.sigma_s = medium->sigma_s;
    T.sigma_a = medium->sigma_a;
    T.sigma_t = medium->sigma_s + medium->sigma_a;
    T.albedo = medium->sigma_s / T.sigma_t;
    T.D = 1.0 / (3.0 * (medium->sigma_a + medium->sigma_s * (1.0 - medium->g)));
    T.n_cs = dims->n_cs;
    T.n_s = dims->n_s;
    T.n_cos = dims->n_cos;
    T.s_max = dims->s_max;
    gauss_legendre(kGLU, T.xu, T.wu);
    gauss_legendre(kGLV, T.xv, T.wv);
    T.cdf = cdf_dev;
    const uint32_t blocks = (uint32_t)(dims->n_cs * dims->n_s);
    hipLaunchKernelGGL(table_kernel, dim3(blocks), dim3(64), sizeof(double) * dims->n_cos, (hipStream_t)stream, T);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DARTS_ERR_DEVICE, "table launch failed: %s", hipGetErrorString(e));
    return ok();
}

int darts_render_transient(const darts_scene *scene, const darts_params *params, const darts_table *table,
                           float *image_hi_dev, float *image_lo_dev, float *image_m2_dev, uint64_t *stats_dev,
                           void *stream)
{
    KParams P;
    if (int rc = make_params(scene, params, table, P, false)) return rc;
    if (!image_hi_dev || !image_lo_dev) return fail(DARTS_ERR_INVALID_ARG, "image_hi/lo are null");
    P.hi = image_hi_dev;
    P.lo = image_lo_dev;
    P.m2 = image_m2_dev;
    P.stats = (unsigned long long *)stats_dev;
    const bool vanilla = (params->flags & DARTS_DIRECT_REUSE) != 0;
    if (vanilla) return launch_render<1, OUT_IMAGE>(P, stats_dev != nullptr, (hipStream_t)stream);
    return launch_render<0, OUT_IMAGE>(P, stats_dev != nullptr, (hipStream_t)stream);
}

int darts_render_paths(const darts_scene *scene, const darts_params *params, const darts_table *table,
                       float *path_value_dev, void *stream)
{
    KParams P;
    if (int rc = make_params(scene, params, table, P, true)) return rc;
    if (!path_value_dev) return fail(DARTS_ERR_INVALID_ARG, "path_value_dev is null");
    P.path_out = path_value_dev;
    return launch_render<0, OUT_PATHS>(P, false, (hipStream_t)stream);
}

int darts_render_transient_backward(const darts_scene *scene, const darts_params *params, const darts_table *table,
                                    const float *grad_image_dev, double *grad_out_dev, void *stream)
{
    KParams P;
    if (int rc = make_params(scene, params, table, P, true)) return rc;
    if (!grad_image_dev || !grad_out_dev) return fail(DARTS_ERR_INVALID_ARG, "grad buffers are null");
    P.grad_image = grad_image_dev;
    P.grad_out = grad_out_dev;
    return launch_render<0, OUT_GRAD>(P, false, (hipStream_t)stream);
}

int darts_render_transient_tangent(const darts_scene *scene, const darts_params *params, const darts_table *table,
                                   float *tangent_dev, void *stream)
{
    KParams P;
    if (int rc = make_params(scene, params, table, P, true)) return rc;
    if (!tangent_dev) return fail(DARTS_ERR_INVALID_ARG, "tangent_dev is null");
    P.tangent = tangent_dev;
    return launch_render<0, OUT_TANGENT>(P, false, (hipStream_t)stream);
}

int darts_batch_default_plan(darts_batch_plan *plan)
{
    if (!plan) return fail(DARTS_ERR_INVALID_ARG, "plan is null");
    *plan = default_plan();
    return ok();
}

int darts_batch_create(const darts_batch_item *items, int n_items, const darts_batch_plan *plan, darts_batch **out)
{
    if (!out) return fail(DARTS_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (n_items < 1 || !items) return fail(DARTS_ERR_INVALID_ARG, "need at least one item");
    const darts_batch_plan pl = plan ? *plan : default_plan();
    if (!valid_plan(pl)) return fail(DARTS_ERR_INVALID_ARG, "invalid batch plan");
    std::vector<BItem> host((size_t)n_items);
    std::vector<int64_t> offsets((size_t)n_items + 1, 0);
    for (int i = 0; i < n_items; ++i) {
        const darts_batch_item &it = items[i];
        if (it.params.flags & DARTS_DIRECT_REUSE)
            return fail(DARTS_ERR_UNSUPPORTED, "item %d: batches render the DARTS family only", i);
        KParams &P = host[(size_t)i].P;
        if (int rc = make_params(&it.scene, &it.params, it.table, P, false)) {
            const std::string msg = g_last_error;
            return fail(rc, "item %d: %s", i, msg.c_str());
        }
        host[(size_t)i].image_offset = offsets[(size_t)i];
        offsets[(size_t)i + 1] = offsets[(size_t)i] + P.ncells;
    }
    if (offsets.back() > ((int64_t)1 << 40)) return fail(DARTS_ERR_INVALID_ARG, "batch image too large");

    auto *b = new darts_batch();
    b->items = std::move(host);
    b->offsets = std::move(offsets);
    for (const BItem &it : b->items) b->any_floor = b->any_floor || it.P.floor != 0;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete b;
        return fail(DARTS_ERR_DEVICE, "no usable HIP device");
    }
    b->device = dev;
    b->n_cu = prop.multiProcessorCount;
    const size_t ib = b->items.size() * sizeof(BItem);
    if (hipMalloc(&b->items_dev, ib) != hipSuccess || hipMalloc(&b->ctr_dev, 2 * sizeof(unsigned)) != hipSuccess ||
        hipMemcpy(b->items_dev, b->items.data(), ib, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(b->ctr_dev, 0, 2 * sizeof(unsigned)) != hipSuccess) {
        darts_batch_destroy(b);
        return fail(DARTS_ERR_DEVICE, "allocating the batch failed");
    }
    if (int rc = upload_units(b, pl)) {
        const std::string msg = g_last_error;
        darts_batch_destroy(b);
        return fail(rc, "%s", msg.c_str());
    }
    *out = b;
    return ok();
}

int darts_batch_image_offsets(const darts_batch *batch, int64_t *offsets)
{
    if (!batch || !offsets) return fail(DARTS_ERR_INVALID_ARG, "batch or offsets is null");
    std::memcpy(offsets, batch->offsets.data(), batch->offsets.size() * sizeof(int64_t));
    return ok();
}

int darts_batch_set_plan(darts_batch *batch, const darts_batch_plan *plan)
{
    if (!batch || !plan) return fail(DARTS_ERR_INVALID_ARG, "batch or plan is null");
    if (!valid_plan(*plan)) return fail(DARTS_ERR_INVALID_ARG, "invalid batch plan");
    if (int rc = check_batch_device(batch)) return rc;
    if (int rc = upload_units(batch, *plan)) return rc;
    return ok();
}

int darts_batch_get_plan(const darts_batch *batch, darts_batch_plan *plan)
{
    if (!batch || !plan) return fail(DARTS_ERR_INVALID_ARG, "batch or plan is null");
    *plan = batch->plan;
    return ok();
}

int darts_batch_render(darts_batch *batch, float *image_hi_dev, float *image_lo_dev, void *stream)
{
    if (!batch) return fail(DARTS_ERR_INVALID_ARG, "batch is null");
    if (!image_hi_dev || !image_lo_dev) return fail(DARTS_ERR_INVALID_ARG, "image_hi/lo are null");
    if (int rc = check_batch_device(batch)) return rc;
    return launch_batch(batch, image_hi_dev, image_lo_dev, (hipStream_t)stream);
}

int darts_batch_graph_launch(darts_batch *batch, float *image_hi_dev, float *image_lo_dev, void *stream)
{
    if (!batch) return fail(DARTS_ERR_INVALID_ARG, "batch is null");
    if (!image_hi_dev || !image_lo_dev) return fail(DARTS_ERR_INVALID_ARG, "image_hi/lo are null");
    if (int rc = check_batch_device(batch)) return rc;
    if (!batch->exec || batch->graph_hi != image_hi_dev || batch->graph_lo != image_lo_dev) {
        drop_graph(batch);
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
            return fail(DARTS_ERR_DEVICE, "creating the capture stream failed");
        hipGraph_t g = nullptr;
        int rc = DARTS_OK;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(DARTS_ERR_DEVICE, "begin capture failed");
        } else {
            const int64_t n = batch->offsets.back();
            const uint32_t zb = (uint32_t)std::min<int64_t>((n + 255) / 256, 4096);
            hipLaunchKernelGGL(zero2_kernel, dim3(std::max<uint32_t>(zb, 1)), dim3(256), 0, cs, image_hi_dev,
                               image_lo_dev, n);
            rc = launch_batch(batch, image_hi_dev, image_lo_dev, cs);
            const hipError_t e = hipStreamEndCapture(cs, &g);
            if (rc == DARTS_OK && e != hipSuccess) rc = fail(DARTS_ERR_DEVICE, "end capture failed");
        }
        if (rc == DARTS_OK && hipGraphInstantiate(&batch->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            batch->exec = nullptr;
            rc = fail(DARTS_ERR_DEVICE, "graph instantiation failed");
        }
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cs);
        if (rc != DARTS_OK) return rc;
        batch->graph_hi = image_hi_dev;
        batch->graph_lo = image_lo_dev;
    }
    if (hipGraphLaunch(batch->exec, (hipStream_t)stream) != hipSuccess)
        return fail(DARTS_ERR_DEVICE, "graph launch failed");
    return ok();
}

int darts_batch_autotune(darts_batch *batch, float *image_hi_dev, float *image_lo_dev, int reps,
                         darts_batch_plan *chosen, double *best_ms, void *stream)
{
    if (!batch) return fail(DARTS_ERR_INVALID_ARG, "batch is null");
    if (!image_hi_dev || !image_lo_dev) return fail(DARTS_ERR_INVALID_ARG, "image_hi/lo are null");
    if (reps < 1) return fail(DARTS_ERR_INVALID_ARG, "reps must be >= 1");
    if (int rc = check_batch_device(batch)) return rc;
    const hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(DARTS_ERR_DEVICE, "creating timing events failed");
    const darts_batch_plan start = batch->plan;
    darts_batch_plan best = start;
    double best_t = 1e300;
    int rc = DARTS_OK;
    for (int order : {DARTS_BATCH_TILES, DARTS_BATCH_IDS})
        for (int bt : {64, 256})
            for (int wpc : {16, 32})
                for (int64_t up : {(int64_t)512, (int64_t)1024, (int64_t)2048, (int64_t)8192, (int64_t)32768}) {
                    if (rc != DARTS_OK) break;
                    darts_batch_plan pl{order, bt, wpc, up};
                    if ((rc = upload_units(batch, pl)) != DARTS_OK) break;
                    if ((rc = launch_batch(batch, image_hi_dev, image_lo_dev, st)) != DARTS_OK) break;
                    (void)hipEventRecord(e0, st);
                    for (int r = 0; r < reps && rc == DARTS_OK; ++r)
                        rc = launch_batch(batch, image_hi_dev, image_lo_dev, st);
                    (void)hipEventRecord(e1, st);
                    if (rc != DARTS_OK) break;
                    float ms = 0.f;
                    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                        rc = fail(DARTS_ERR_DEVICE, "timing a candidate plan failed");
                        break;
                    }
                    if (ms / reps < best_t) {
                        best_t = ms / reps;
                        best = pl;
                    }
                }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != DARTS_OK) {
        const std::string msg = g_last_error;
        (void)upload_units(batch, start);
        return fail(rc, "%s", msg.c_str());
    }
    if ((rc = upload_units(batch, best)) != DARTS_OK) return rc;
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = best_t;
    return ok();
}

int darts_batch_destroy(darts_batch *batch)
{
    if (!batch) return ok();
    drop_graph(batch);
    if (batch->units_dev) (void)hipFree(batch->units_dev);
    if (batch->items_dev) (void)hipFree(batch->items_dev);
    if (batch->ctr_dev) (void)hipFree(batch->ctr_dev);
    delete batch;
    return ok();
}

int darts_batch_render_noalloc(const darts_batch_item *items, int n_items, const darts_batch_plan *plan,
                               float *image_hi_dev, float *image_lo_dev, int64_t image_numel, void *stream)
{
    if (n_items < 1 || !items) return fail(DARTS_ERR_INVALID_ARG, "need at least one item");
    if (!image_hi_dev || !image_lo_dev) return fail(DARTS_ERR_INVALID_ARG, "image_hi/lo are null");
    const darts_batch_plan pl = plan ? *plan : default_plan();
    if (!valid_plan(pl)) return fail(DARTS_ERR_INVALID_ARG, "invalid batch plan");
    const size_t items_bytes = ((size_t)n_items * sizeof(BItem) + 255) / 256 * 256;
    if (kScratchItemsOff + items_bytes + sizeof(UnitCost) > kScratchBytes)
        return fail(DARTS_ERR_INVALID_ARG, "%d scenes need %zu bytes of parameter blocks; the scratch array holds %zu",
                    n_items, items_bytes, kScratchBytes - kScratchItemsOff - sizeof(UnitCost));
    const size_t units_off = kScratchItemsOff + items_bytes;

    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    unsigned char *dev = nullptr;
    int n_cu = 0;
    if (int rc = scratch_of_device(&dev, &n_cu)) return rc;

    BItem *h_items = (BItem *)(g_stage + kScratchItemsOff);
    int64_t off = 0;
    bool any_floor = false;
    for (int i = 0; i < n_items; ++i) {
        const darts_batch_item &it = items[i];
        if (it.params.flags & DARTS_DIRECT_REUSE)
            return fail(DARTS_ERR_UNSUPPORTED, "item %d: batches render the DARTS family only", i);
        KParams &P = h_items[i].P;
        if (int rc = make_params(&it.scene, &it.params, it.table, P, false)) {
            const std::string msg = g_last_error;
            return fail(rc, "item %d: %s", i, msg.c_str());
        }
        h_items[i].image_offset = off;
        off += P.ncells;
        any_floor = any_floor || P.floor != 0;
    }
    if (image_numel < off)
        return fail(DARTS_ERR_INVALID_ARG, "the batch image has %lld elements; the buffers hold %lld",
                    (long long)off, (long long)image_numel);

    UnitCost *h_cost = (UnitCost *)(g_stage + units_off);
    const size_t cap = (kScratchBytes - units_off) / sizeof(UnitCost);
    size_t n_units = 0;
    const bool fits = enumerate_units(h_items, (size_t)n_items, pl, [&](const UnitCost &uc) {
        if (n_units == cap) return false;
        h_cost[n_units++] = uc;
        return true;
    });
    if (!fits)
        return fail(DARTS_ERR_INVALID_ARG, "more than %zu work units do not fit the scratch array; raise unit_paths",
                    cap);
    std::sort(h_cost, h_cost + n_units, unit_before);
    // compact to BUnit in place (smaller stride: unit k is read before a
    // later write can reach it)
    BUnit *h_units = (BUnit *)(g_stage + units_off);
    for (size_t k = 0; k < n_units; ++k) {
        const BUnit u = h_cost[k].u;
        h_units[k] = u;
    }
    if (n_units == 0) return ok();

    const hipStream_t st = (hipStream_t)stream;
    unsigned *ctr = (unsigned *)dev;
    BItem *d_items = (BItem *)(dev + kScratchItemsOff);
    BUnit *d_units = (BUnit *)(dev + units_off);
    if (hipMemcpyAsync(d_items, h_items, (size_t)n_items * sizeof(BItem), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_units, h_units, n_units * sizeof(BUnit), hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(DARTS_ERR_DEVICE, "copying the batch to the scratch array failed");
    hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(64), 0, st, ctr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DARTS_ERR_DEVICE, "clearing the unit counters failed: %s", hipGetErrorString(e));
    return launch_batch_units(n_cu, pl, any_floor, d_items, d_units, (uint32_t)n_units, ctr, image_hi_dev,
                              image_lo_dev, st);
}

int darts_debug_pointwise(int fn, const float *in_dev, float *out_dev, int64_t n, const darts_medium *medium,
                          const darts_table *table, void *stream)
{
    if (fn < 0 || fn >= DARTS_PW_COUNT) return fail(DARTS_ERR_INVALID_ARG, "unknown pointwise function %d", fn);
    if (n < 0 || (n > 0 && (!in_dev || !out_dev))) return fail(DARTS_ERR_INVALID_ARG, "bad buffers");
    PWParams Q;
    Q.fn = fn;
    Q.n = n;
    Q.in = in_dev;
    Q.out = out_dev;
    Q.med = Medium{};
    const bool need_med = fn == DARTS_PW_DA_LOGPHI || fn == DARTS_PW_RIS || fn == DARTS_PW_DIRECTION ||
                          fn == DARTS_PW_CONNECT;
    if (need_med) {
        if (int rc = check_medium(medium)) return rc;
        Q.med = make_medium(*medium);
    }
    if (int rc = fill_table(table, nullptr, fn == DARTS_PW_DIRECTION, Q.tb)) return rc;
    if (fn == DARTS_PW_DIRECTION && !same_medium(table->medium, *medium))
        return fail(DARTS_ERR_TABLE_MISMATCH, "table was built for another medium");
    if (n == 0) return ok();
    const uint64_t blocks = ((uint64_t)n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(pointwise_kernel, dim3((uint32_t)blocks), dim3(kBlock), 0, (hipStream_t)stream, Q);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DARTS_ERR_DEVICE, "pointwise launch failed: %s", hipGetErrorString(e));
    return ok();
}

// Tuning knob: renders whose cells hold at most this many repetitions use
// the id-range decomposition (negative: never).
int darts_set_ids_max_reps(int64_t reps)
{
    g_ids_max_reps.store(reps, std::memory_order_relaxed);
    return ok();
}

// Tuning knob: vanilla renders histogram per pixel in LDS when it fits.
int darts_set_vanilla_privatised(int on)
{
    g_vanilla_privatised.store(on ? 1 : 0, std::memory_order_relaxed);
    return ok();
}

// Tuning knob: waves a tile-decomposed render launch aims for.
int darts_set_target_waves(int64_t waves)
{
    if (waves < 1) return fail(DARTS_ERR_INVALID_ARG, "target waves must be >= 1");
    g_target_waves.store(waves, std::memory_order_relaxed);
    return ok();
}

}  // extern "C"
