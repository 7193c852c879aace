// Device building blocks of the DARTS path kernel (gfx950, wave64, FP32 path
// arithmetic).  Every function here is also reachable one item per thread
// through darts_debug_pointwise, so it can be checked on its own.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace darts {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInv4Pi = 0.0795774715459476679f;   // 1 / (4 pi)
constexpr float kInf = __builtin_huge_valf();
constexpr float kLog2e = 1.44269504088896341f;

// Hardware transcendental helpers (gfx950 VALU transcendental unit):
// v_rcp_f32, v_rsq_f32 and v_sqrt_f32 (1 ulp), v_log_f32 / v_exp_f32 (base 2), and
// v_sin_f32 / v_cos_f32, whose argument is in revolutions.  Their accuracy on
// the ranges used here is checked against FP64 by the diagnostics tests.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float log2_hw(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_log(float x) { return log2_hw(x) * 0.693147180559945309f; }
__device__ __forceinline__ float fast_exp(float x) { return exp2_hw(x * 1.44269504088896341f); }
__device__ __forceinline__ void sincos_rev(float u, float &s, float &c)   // sin, cos of 2 pi u
{
    s = __builtin_amdgcn_sinf(u);
    c = __builtin_amdgcn_cosf(u);
}

struct V3 { float x, y, z; };
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return V3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float length(V3 a) { return hw_sqrt(dot(a, a)); }
__device__ __forceinline__ V3 fma3(V3 x, V3 w, float t) { return V3{fmaf(w.x, t, x.x), fmaf(w.y, t, x.y), fmaf(w.z, t, x.z)}; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// with a Weyl-sequence key schedule.  Counter layout of this library:
// (path id low, path id high, vertex index k, stream), key = seed; stream 0
// of vertex 0 is the camera set-up, stream 0 of vertex k >= 1 the direction
// sample, stream 1 of vertex k the connection and free flight.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

// a ^ b ^ c in one gfx950 three-input bit operation (truth table 0x96: the
// parity of the three input bits)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;   // one 32x32->64 multiply each
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0), n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// 24-bit uniform in [0,1): exact in float and double.
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

// RIS candidate uniform: base-2 radical inverse of 8*row + col (row of the
// 32x8 Sobol table, Section IV-C) plus a random offset, modulo 1 on 32-bit
// fixed point.
__device__ __forceinline__ float sobol_u(uint32_t row, uint32_t col, uint32_t eps)
{
    return u01(__builtin_bitreverse32(8u * row + col) + eps);
}

// ---------------------------------------------------------------------------
// Henyey-Greenstein phase function.
// ---------------------------------------------------------------------------
// Constants of the phase function for one g, formed once per medium (on the
// host for a render, so the path loop reads them as scalars).
struct HG {
    float g, c0, c1, s;   // den = c0 + c1 (1 - s mu): c0 = (1 - |g|)^2, c1 = 2 |g|, s = sign g
    float omg, opg;       // 1 - g, 1 + g
    float two_g, norm;    // 2 g, (1 - g)(1 + g) / (4 pi)
};
__host__ __device__ inline HG hg_consts(float g)
{
    HG h;
    const float ag = g >= 0.f ? g : -g;
    h.g = g;
    h.c0 = (1.f - ag) * (1.f - ag);
    h.c1 = 2.f * ag;
    h.s = g >= 0.f ? 1.f : -1.f;
    h.omg = 1.f - g;
    h.opg = 1.f + g;
    h.two_g = 2.f * g;
    h.norm = h.omg * h.opg * kInv4Pi;
    return h;
}

// 1 + g^2 - 2 g mu is evaluated as a sum of non-negative terms,
// (1 - g)^2 + 2 g (1 - mu) for g >= 0 and (1 + g)^2 + 2 |g| (1 + mu) for g < 0,
// so the forward peak keeps full relative precision.
__device__ __forceinline__ float hg_pdf(const HG &h, float mu)
{
    const float den = fmaf(h.c1, fmaf(-h.s, mu, 1.f), h.c0);
    const float r = rsq(den);
    return h.norm * (r * r * r);
}
__device__ __forceinline__ float hg_pdf(float mu, float g) { return hg_pdf(hg_consts(g), mu); }

// Inverse CDF of HG in mu, rewritten without cancellation: with
// t = 1 - g + 2 g xi and q = (1 - g^2)/t,
//   1 - mu = (1 - g)(1 - xi)(q + 1 - g)/t,   1 + mu = (1 + g) xi (q + 1 + g)/t,
// both products of non-negative terms for every |g| < 1 (g = 0 gives
// mu = 2 xi - 1).
__device__ __forceinline__ void hg_sample(const HG &h, float xi, float &mu, float &sin_t)
{
    const float t = fmaf(h.two_g, xi, h.omg);
    const float it = rcp(t);
    const float q = h.omg * h.opg * it;
    const float omu = h.omg * (1.f - xi) * (q + 1.f - h.g) * it;
    const float opu = h.opg * xi * (q + 1.f + h.g) * it;
    mu = fminf(fmaxf(0.5f * (opu - omu), -1.f), 1.f);
    sin_t = hw_sqrt(fmaxf(omu * opu, 0.f));
}
__device__ __forceinline__ void hg_sample(float xi, float g, float &mu, float &sin_t)
{
    hg_sample(hg_consts(g), xi, mu, sin_t);
}

// Orthonormal basis completing unit n (Duff et al., JCGT 2017, branchless).
__device__ __forceinline__ void onb(V3 n, V3 &b1, V3 &b2)
{
    const float sign = copysignf(1.f, n.z);
    const float a = -rcp(sign + n.z);
    const float b = n.x * n.y * a;
    b1 = V3{fmaf(sign * n.x * n.x, a, 1.f), sign * b, -sign * n.x};
    b2 = V3{b, fmaf(n.y * n.y, a, sign), -n.y};
}

// Direction at cosine mu (sine s) to axis n, azimuth 2 pi u.
__device__ __forceinline__ V3 from_frame(V3 n, float mu, float s, float u)
{
    V3 b1, b2;
    onb(n, b1, b2);
    float sp, cp;
    sincos_rev(u, sp, cp);
    const float a1 = s * cp, a2 = s * sp;
    return V3{fmaf(a1, b1.x, fmaf(a2, b2.x, mu * n.x)),
              fmaf(a1, b1.y, fmaf(a2, b2.y, mu * n.y)),
              fmaf(a1, b1.z, fmaf(a2, b2.z, mu * n.z))};
}

// ---------------------------------------------------------------------------
// Truncated exponential on [0, width) (Eq. (13)-(14)).
// ---------------------------------------------------------------------------
// 1 - e^{-x} for x >= 0 without cancellation: for small x Kahan's rescaling
// (1 - u) x / (-log u) with u the rounded e^{-x} (1 - u exact).
__device__ __forceinline__ float one_minus_exp_neg(float x, float &emx)
{
    const float u = fast_exp(-x);
    emx = u;
    if (x > 0.5f) return 1.f - u;
    if (u == 1.f) return x;
    return (1.f - u) * x * rcp(-fast_log(u));
}
__device__ __forceinline__ float texp_mass(float sigma, float width)   // 1 - e^{-sigma width}
{
    float e;
    return one_minus_exp_neg(sigma * width, e);
}

// x = -log(1 - mass u) / sigma with mass = 1 - emass, emass = e^{-sigma width},
// without cancellation: for y = mass u < 1/100 the series
// y + y^2/2 + y^3/3 (relative error < y^3/4 < 2.5e-7), taken in base 2; for
// 1/100 <= y < 1/2 the logarithm of the rounded 1 - y (relative error
// < 6e-6); otherwise 1 - mass u = (1 - u) + u emass, a sum of non-negative
// terms with 1 - u exact (u >= 1/2).  ln2_over_sigma = ln 2 / sigma (the
// hardware logarithm is base 2).
__device__ __forceinline__ float texp_sample(float u, float ln2_over_sigma, float mass, float emass)
{
    const float y = mass * u;
    const float v = y < 0.5f ? 1.f - y : fmaf(u, emass, 1.f - u);
    const float L = log2_hw(v);
    const float series = y * fmaf(y, fmaf(y, kLog2e / 3.f, kLog2e / 2.f), kLog2e);
    const float nl = y < 0.01f ? series : -L;
    return nl * ln2_over_sigma;
}

// ---------------------------------------------------------------------------
// Index-matched box.
// ---------------------------------------------------------------------------
struct Box { float lo[3], hi[3]; };

// Distance from x (inside) along w to the boundary, iw = componentwise 1/w.
// Per axis the face ahead is chosen by the sign bit of w, so a zero
// component (iw = +inf for +0, -inf for -0) gives +inf, or NaN for a point
// on that face, which the minimum ignores.
__device__ __forceinline__ float box_exit_inv(const Box &b, V3 x, V3 w, V3 iw)
{
    const float tx = ((__float_as_int(w.x) < 0 ? b.lo[0] : b.hi[0]) - x.x) * iw.x;
    const float ty = ((__float_as_int(w.y) < 0 ? b.lo[1] : b.hi[1]) - x.y) * iw.y;
    const float tz = ((__float_as_int(w.z) < 0 ? b.lo[2] : b.hi[2]) - x.z) * iw.z;
    return fmaxf(fminf(fminf(tx, ty), tz), 0.f);
}
__device__ __forceinline__ float box_exit(const Box &b, V3 x, V3 w)
{
    return box_exit_inv(b, x, w, V3{rcp(w.x), rcp(w.y), rcp(w.z)});
}

// True if the ray from x (inside) along w leaves the box through its bottom
// face z = lo[2] (the opaque floor, when the geometry has one).
__device__ __forceinline__ bool exits_floor(const Box &b, V3 x, V3 w)
{
    if (!(w.z < 0.f)) return false;
    const float tz = (b.lo[2] - x.z) / w.z;
    const float tx = w.x > 0.f ? (b.hi[0] - x.x) / w.x : (w.x < 0.f ? (b.lo[0] - x.x) / w.x : kInf);
    const float ty = w.y > 0.f ? (b.hi[1] - x.y) / w.y : (w.y < 0.f ? (b.lo[1] - x.y) / w.y : kInf);
    return !(tx < tz) && !(ty < tz);
}

// Direction leaving a Lambertian floor (normal +z), cosine-weighted:
// cos theta = sqrt(u1), phi = 2 pi u2.  The BRDF-to-pdf ratio is the albedo.
__device__ __forceinline__ V3 floor_direction(float u1, float u2)
{
    const float ct = hw_sqrt(u1), sn = hw_sqrt(fmaxf(1.f - u1, 0.f));
    float sp, cp;
    sincos_rev(u2, sp, cp);
    return V3{sn * cp, sn * sp, ct};
}

// Slab test for a ray from x along w; returns false on a miss.
__device__ __forceinline__ bool box_entry(const Box &b, V3 x, V3 w, float &t_in, float &t_out)
{
    float tn = -kInf, tf = kInf;
    const float xs[3] = {x.x, x.y, x.z}, ws[3] = {w.x, w.y, w.z};
    bool hit = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (ws[a] == 0.f) {
            hit = hit && !(xs[a] < b.lo[a] || xs[a] > b.hi[a]);
        } else {
            const float iw = rcp(ws[a]);
            const float t1 = (b.lo[a] - xs[a]) * iw, t2 = (b.hi[a] - xs[a]) * iw;
            tn = fmaxf(tn, fminf(t1, t2));
            tf = fminf(tf, fmaxf(t1, t2));
        }
    }
    t_in = fmaxf(tn, 0.f);
    t_out = tf;
    return hit && tf > t_in;
}

// ---------------------------------------------------------------------------
// Medium constants (FP32) derived once on the host.
// ---------------------------------------------------------------------------
struct Medium {
    float sigma_s, sigma_a, sigma_t, inv_sigma_t, albedo, g;
    float inv4D;      // 1 / (4 D), D = 1 / (3 (sigma_a + sigma_s (1 - g)))  (Eq. (9))
    float ln2_over_sigma_t;
    float inv4D_log2e, sigma_a_log2e;   // the exponent of Eq. (9) in base 2
    float four_D_sigma_a;               // 4 D sigma_a = sigma_a_log2e / inv4D_log2e
    HG hg;
};

// log of the DA fluence without its constant -1.5 log(4 pi D) (Eq. (9));
// s > 0 is the residual time, r2 the squared distance to the emitter.
__device__ __forceinline__ float da_log_phi_rel(const Medium &m, float r2, float s)
{
    const float is = rcp(s);
    return fmaf(-1.5f * 0.693147180559945309f, log2_hw(s), -fmaf(r2 * m.inv4D, is, m.sigma_a * s));
}

// ---------------------------------------------------------------------------
// Elliptical connection geometry (Eq. (18), (21), (22)).  For a length sum S,
// focal distance C, the excess sc = S - C (passed as the caller formed it,
// not recomputed from S, which may have rounded it away) and cm = C (1 - mu) >= 0 (mu the cosine of
// the direction to the focal axis):  den = S - C mu, t the polar distance,
// r = S - t the distance from the control vertex to the emitter, written so
// that nothing cancels when S ~ C or mu ~ 1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ellipse(float S, float C, float sc, float cm, float &den, float &t, float &r)
{
    den = sc + cm;
    const float ih = 0.5f * rcp(den);
    t = sc * (S + C) * ih;
    r = fmaf(sc, sc, 2.f * S * cm) * ih;
}

// ---------------------------------------------------------------------------
// DA distance sampling by RIS with 8 candidates (Section IV-C).  Candidates
// follow the truncated exponential on [0, d_m) (pc = 1 - e^{-sigma_t d_m});
// weights are the DA fluence at the upper residual time R_hi - d (zero
// outside the residual-time ellipsoid); the normalisation and the selection
// run in FP64.  On success returns the distance and the factor
// albedo * mean(w) / w_selected that multiplies the path throughput.
// b_dot = dot(w, x_e - x), C2 = |x_e - x|^2, epc = 1 - pc = e^{-sigma_t d_m}.
// ---------------------------------------------------------------------------
// choice (diagnostics only; null in the kernels): selected candidate in bits
// 0-7, mask of the valid candidates in bits 8-15, candidates indexed in
// increasing order of their uniform.
__device__ __forceinline__ bool ris_distance(const Medium &m, float C2, float b_dot, float R_hi, float pc,
                                             float epc, uint32_t row, uint32_t eps, float u_sel,
                                             float &d_out, float &factor, uint32_t *choice = nullptr)
{
    // Phi_i = (4 pi D s_i)^{-3/2} exp(E_i),  E_i = -r_i^2 / (4 D s_i) - sigma_a s_i
    // = -(r_i^2 + 4 D sigma_a s_i^2) / (4 D s_i): with F_i = (r_i^2 + 4 D
    // sigma_a s_i^2) / s_i the weights s_i^{-3/2} 2^{(F_min - F_i) log2 e / (4 D)}
    // share one rsq per candidate (1/s_i = rsq^2, s_i^{-3/2} = rsq^3) and
    // cannot underflow for the candidate with the smallest F.
    //
    // Candidate uniforms: row `row` of the 32 x 8 Sobol table (the radical
    // inverses of 8 row .. 8 row + 7) plus the offset eps, on 32-bit fixed
    // point.  The radical inverse of 8 row + i is that of 8 row (bits 0-28)
    // plus that of i (the top three bits), so each candidate keeps the low
    // 29 bits of base = bitrev(8 row) + eps and has (top3(base) + bitrev3(i))
    // mod 8 as its top three: one candidate per eighth of [0,1).  Taken in
    // increasing order (the order of the selection below), the candidate in
    // eighth s has the 24-bit integer k = s 2^21 + b of u = k 2^-24, with
    // b = (base mod 2^29) >> 8: one exact float add per candidate.
    //
    // Candidate distance d = -ln(1 - pc u) / sigma_t (Eq. (14)) without
    // cancellation:
    //  - eighths 0-3 (u < 1/2, so pc u < 1/2): v = fl(1 - pc u) >= 1/2 from
    //    one fma, its rounding error e = (1 - v) - pc u from a second (1 - v
    //    is exact there), and ln(1 - pc u) = ln(v + e) = ln v + e (error
    //    below 2^-24 of the result, also for pc u -> 0, where ln v alone
    //    would lose the low bits);
    //  - eighths 4-7 (u >= 1/2): 1 - pc u = (1 - u) + u e^{-sigma_t d_m}, a
    //    sum of non-negative terms with 1 - u exact, rounded once.
    const uint32_t base = __builtin_bitreverse32(8u * row) + eps;
    float b = (float)((base & 0x1FFFFFFFu) >> 8);
    // b < 2^21 is hidden from the compiler, which would otherwise rewrite
    // each exact add b + s 2^21 as an integer or plus a conversion
    asm volatile("" : "+v"(b));
    const float pc24 = pc * 0x1p-24f, em24 = epc * 0x1p-24f;
    float dc[8], q[8], F[8];
    float fmin = kInf;
    const float two_b = 2.f * b_dot;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float k = b + (float)(i << 21);
        float L;   // log2(1 - pc u)
        if (i < 4) {
            const float va = fmaf(-pc24, k, 1.f);
            const float ea = fmaf(-pc24, k, 1.f - va);
            L = fmaf(ea, kLog2e, log2_hw(va));
        } else {
            L = log2_hw(fmaf(k, em24, fmaf(k, -0x1p-24f, 1.f)));
        }
        const float di = -L * m.ln2_over_sigma_t;
        const float si = R_hi - di;
        const float r2 = fmaf(di, di - two_b, C2);
        const float si2 = si * si;
        const bool valid = (si > 0.f) && (r2 < si2);   // inside the residual-time ellipsoid
        const float rq = rsq(si), rq2 = rq * rq;
        const float f = fmaf(si2, m.four_D_sigma_a, r2) * rq2;
        dc[i] = di;
        q[i] = valid ? rq2 * rq : 0.f;
        F[i] = valid ? f : kInf;
        fmin = fminf(fmin, F[i]);
        if (choice) *choice = (i == 0 ? 0u : *choice) | (valid ? 1u << (8 + i) : 0u);
    }
    if (!(fmin < kInf)) return false;
    const float cmin = m.inv4D_log2e * fmin;
    // running sums of the weights in FP64; the first term starts them (the
    // weights are >= +0, so this equals 0 + w_0)
    float wv[8];
    double cs[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        wv[i] = q[i] * exp2_hw(fmaf(-m.inv4D_log2e, F[i], cmin));
        cs[i] = i == 0 ? (double)wv[0] : cs[i - 1] + (double)wv[i];
    }
    const double wsum = cs[7];
    const double target = (double)u_sel * wsum;
    float dsel = dc[7], wsel = wv[7];
    uint32_t isel = 7;
    bool found = false;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double cum = cs[i];
        const bool take = !found && (cum > target);
        dsel = take ? dc[i] : dsel;
        wsel = take ? wv[i] : wsel;
        if (choice) isel = take ? (uint32_t)i : isel;
        found = found || take;
    }
    if (!found) {  // only reachable through rounding: take the last positive weight
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (wv[i] > 0.f) { dsel = dc[i]; wsel = wv[i]; if (choice) isel = (uint32_t)i; }
    }
    if (choice) *choice |= isel;
    d_out = dsel;
    factor = m.albedo * ((float)wsum * 0.125f) * rcp(wsel);
    return true;
}

// ---------------------------------------------------------------------------
// EDA direction sampling with one-sample MIS (Section V-A, Eq. (19)).
// With probability gamma = kappa/(kappa + alpha) (kappa = C/S) cos(theta) to
// the axis towards the emitter is drawn from the table row of (C/S, S) by
// inverse transform (cos uniform inside the chosen bin, phi uniform);
// otherwise from the phase function about the previous direction.  The
// throughput is multiplied by phase / (gamma p_EDA + (1 - gamma) p_HG).
// ---------------------------------------------------------------------------
// A built direction table as the kernels read it: the float constants are
// formed once on the host (fn_cs = n_cs, fn_cos = n_cos, cos_step =
// 2 / n_cos, ns_over_smax = n_s / s_max, cos_pow2); offsets fit 32 bits.
struct Table {
    const float *cdf;
    int n_cs, n_s, n_cos;
    int cos_pow2;   // the largest power of two <= n_cos
    float ns_over_smax, fn_cs, fn_cos, cos_step;
};

// dbg (diagnostics only; null in the kernels): [0] table row i n_s + j
// (-1 without the table), [1] the cos-bin whose EDA density enters the
// weight (-1 without the table).
__device__ __forceinline__ V3 sample_direction(const Medium &m, const Table &tb, float alpha, bool use_eda,
                                               V3 a /*unit, to emitter*/, float C, float S, V3 w_prev,
                                               U4 r, float &weight, bool &eda_branch, int *dbg = nullptr)
{
    const float u0 = u01(r.x), u1 = u01(r.y), u2 = u01(r.z), u3 = u01(r.w);
    float gam = 0.f;
    const float *row = nullptr;
    if (use_eda && C > 0.f) {
        const float kappa = C * rcp(S);
        gam = kappa * rcp(kappa + alpha);
        const int i = min(max((int)(kappa * tb.fn_cs), 0), tb.n_cs - 1);
        const int j = min(max((int)(S * tb.ns_over_smax), 0), tb.n_s - 1);
        row = tb.cdf + (uint32_t)(i * tb.n_s + j) * (uint32_t)(tb.n_cos + 1);
        if (dbg) dbg[0] = i * tb.n_s + j;
    }
    eda_branch = u0 < gam;
    V3 axis;
    float mu, s, c_lo = 0.f, c_hi = 0.f;
    int k = 0;
    if (eda_branch) {
        // largest k < n_cos with cdf[k] <= u1 (cdf[0] = 0 <= u1 < 1 =
        // cdf[n_cos], nondecreasing) by a binary search whose probes depend
        // on n_cos alone: with P the largest power of two <= n_cos, one probe
        // at n_cos - P, then steps P/2, ..., 1 (lo + step <= n_cos - 1), so
        // every lane makes the same number of probes and the loop stays
        // uniform across the wave.
        int lo = 0;
        const int first = tb.n_cos - tb.cos_pow2;
        if (first > 0 && row[first] <= u1) lo = first;
        for (int step = tb.cos_pow2 >> 1; step > 0; step >>= 1)
            lo = row[lo + step] <= u1 ? lo + step : lo;
        k = lo;
        c_lo = row[k];
        c_hi = row[k + 1];
        // cos(theta) = -1 + (k + u3) 2/n_cos; sin(theta) from 1 + cos and
        // 1 - cos = (n_cos - k - u3) 2/n_cos, formed without going through
        // cos itself: its FP32 rounding near +-1 (steps of 2^-24) quantises
        // the angle to the emitter, and at 1 - cos ~ 1e-7 a connection whose
        // control vertex lands ~1e-4 from the emitter changed by up to 14%
        const float kf = (float)k;
        mu = fmaf(kf + u3, tb.cos_step, -1.f);
        const float opmu = (kf + u3) * tb.cos_step;
        const float omu = ((tb.fn_cos - kf) - u3) * tb.cos_step;
        s = hw_sqrt(omu * opmu);
        axis = a;
    } else {
        hg_sample(m.hg, u1, mu, s);
        axis = w_prev;
    }
    const V3 w = from_frame(axis, mu, s, u2);
    const float p_hg = hg_pdf(m.hg, dot(w_prev, w));
    float p_mix = p_hg;
    if (gam > 0.f) {
        if (!eda_branch) {
            k = (int)floorf((dot(w, a) + 1.f) * 0.5f * tb.fn_cos);
            k = min(max(k, 0), tb.n_cos - 1);
            c_lo = row[k];
            c_hi = row[k + 1];
        }
        const float p_eda = (c_hi - c_lo) * tb.fn_cos * kInv4Pi;
        p_mix = fmaf(gam, p_eda - p_hg, p_hg);
        if (dbg) dbg[1] = k;
    }
    weight = p_hg * rcp(p_mix);
    return w;
}

// Compensated addition: s + e == a + b exactly (Knuth TwoSum).
__device__ __forceinline__ float two_sum_err(float a, float b, float s)
{
#pragma clang fp contract(off)
    const float bb = s - a;
    return (a - (s - bb)) + (b - bb);
}

}  // namespace darts
