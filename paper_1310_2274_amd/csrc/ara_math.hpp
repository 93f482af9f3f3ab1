// ara_math.hpp -- device numerics for aggregate risk analysis with secondary
// uncertainty on gfx950: counter-based uniforms, the log Beta function, the
// regularised incomplete beta and its inverse (section 3.3 of Varghese &
// Rau-Chaplin, WHPCF'13), and the normal transforms of section 3.2.
//
// Functions are __host__ __device__ so the same source can be exercised on
// the host during development; the product path runs them on the GPU only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ara {

// ---------------------------------------------------------------------------
// Per-entry record of a loaded XELT, derived on the device at load time from
// (mean, sigma_I + sigma_C, max_l) by the moment matching of section 3.3.
// 32 bytes: one aligned vector load per draw.
// ---------------------------------------------------------------------------
struct alignas(16) EntryRec {
    double a;      // alpha; 0 marks a degenerate entry (sigma = 0: loss = mean)
    double b;      // beta
    double lnB;    // ln B(alpha, beta); the mean loss for a degenerate entry
    float us;      // I_ts(alpha, beta) at ts = (alpha+1)/(alpha+beta+2)
    float maxl;    // max_l
};
static_assert(sizeof(EntryRec) == 32, "EntryRec must stay 32 bytes");

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products; the key advances by the golden-ratio Weyl
// constants between rounds.  Only the first output word is used here.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t philox_word0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
    constexpr uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;
    constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)MA * c0;
        const uint64_t pb = (uint64_t)MB * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += WA;
        k1 += WB;
    }
    return c0;
}

// 32-bit word -> odd multiple of 2^-24 in (0,1): exact in FP32, symmetric
// about 1/2, never 0 or 1.
__host__ __device__ inline float u01(uint32_t w)
{
    return (float)(2u * (w >> 9) + 1u) * 0x1p-24f;
}

// ---------------------------------------------------------------------------
// ln B(a, b).  lnGamma(b) - lnGamma(a+b) cancels badly when a << b, which is
// exactly where the quantile is most sensitive (relative error / a), so the
// difference D(a,b) = lnGamma(a+b) - lnGamma(b) is formed directly:
//   D(a,b) = D(a,b+1) - log1p(a/b)                     (shift b to >= 16)
//   D(a,b) = (b-1/2) log1p(a/b) + a ln(a+b) - a + w(a+b) - w(b)
// with w the remainder of Stirling's series, w(z) = sum B_2k/(2k(2k-1) z^(2k-1)).
// ---------------------------------------------------------------------------
__host__ __device__ inline double stirling_remainder(double z)
{
    const double r = 1.0 / z, r2 = r * r;
    return r * (1.0 / 12.0 + r2 * (-1.0 / 360.0 + r2 * (1.0 / 1260.0 + r2 * (-1.0 / 1680.0
           + r2 * (1.0 / 1188.0 + r2 * (-691.0 / 360360.0 + r2 * (1.0 / 156.0)))))));
}

__host__ __device__ inline double lgamma_shift(double a, double b)
{
    double s = 0.0;
    while (b < 16.0) {
        s -= log1p(a / b);
        b += 1.0;
    }
    const double c = a + b;
    return s + (b - 0.5) * log1p(a / b) + a * log(c) - a + (stirling_remainder(c) - stirling_remainder(b));
}

__host__ __device__ inline double log_beta(double a, double b)
{
    const double s = a < b ? a : b, l = a < b ? b : a;
    return lgamma(s) - lgamma_shift(s, l);
}

// ---------------------------------------------------------------------------
// Continued fraction of the incomplete beta (DLMF 8.17.22):
//   I_t(A,B) = t^A (1-t)^B / (A B(A,B)) / T,   T = 1 + d1/(1 + d2/(1 + ...))
//   d_{2m+1} = -(A+m)(A+B+m) t / ((A+2m)(A+2m+1)),
//   d_{2m}   =  m(B-m) t / ((A+2m-1)(A+2m)),
// fast for t <= (A+1)/(A+B+2).  With d_n = p_n / q_n, q_n = (A+n-1)(A+n), the
// equivalent fraction with partial denominators q_n and numerators q_{n-1} p_n
// needs no division: the convergents follow X_n = q_n X_{n-1} + q_{n-1} p_n X_{n-2}
// for numerators and denominators alike, rescaled by exact powers of two.
// Returns T as num/den.
// ---------------------------------------------------------------------------
template <typename R>
__host__ __device__ inline void beta_cf(R t, R A, R B, R eps, int max_pairs, R& num, R& den)
{
    R n2 = 1, n1 = 1;     // numerators   X_{-1}, X_0
    R d2 = 0, d1 = 1;     // denominators X_{-1}, X_0
    R qprev = 1;
    const R apb = A + B;
    R fm = 0;                              // m, carried in R (no integer conversions)
    for (int m = 0; m < max_pairs; ++m, fm += 1) {
        // n = 2m+1
        const R qo = (A + 2 * fm) * (A + 2 * fm + 1);
        const R po = -(A + fm) * (apb + fm) * t;
        const R co = qprev * po;
        const R no = qo * n1 + co * n2;
        const R dd = qo * d1 + co * d2;
        // n = 2m+2
        const R qe = (A + 2 * fm + 1) * (A + 2 * fm + 2);
        const R pe = (fm + 1) * (B - fm - 1) * t;
        const R ce = qo * pe;
        const R ne = qe * no + ce * n1;
        const R de = qe * dd + ce * d1;
        int ex;
        frexp(fabs(de) > fabs(ne) ? de : ne, &ex);
        n2 = ldexp(no, -ex);
        d2 = ldexp(dd, -ex);
        n1 = ldexp(ne, -ex);
        d1 = ldexp(de, -ex);
        qprev = qe;
        const R x = n1 * d2, y = n2 * d1;
        if (fabs(x - y) <= eps * fabs(x)) break;
    }
    num = n1;
    den = d1;
}

// I_t(A, B) for t <= ~(A+1)/(A+B+2), FP64; lnB = ln B(A, B).
__host__ __device__ inline double beta_inc_lower(double t, double A, double B, double lnB)
{
    if (t <= 0.0) return 0.0;
    double num, den;
    beta_cf<double>(t, A, B, 1e-16, 400, num, den);
    return exp(A * log(t) + B * log1p(-t) - lnB) / A * (den / num);
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// I_t(a, b) in FP64 for any t: the lower fraction below t_s, the reflection
// I_t(a, b) = 1 - I_{1-t}(b, a) above it.
__host__ __device__ inline double beta_inc(double t, const EntryRec& E)
{
    if (t <= 0.0) return 0.0;
    if (t >= 1.0) return 1.0;
    const double ts = (E.a + 1.0) / (E.a + E.b + 2.0);
    return t <= ts ? beta_inc_lower(t, E.a, E.b, E.lnB) : 1.0 - beta_inc_lower(1.0 - t, E.b, E.a, E.lnB);
}

// Term thresholds of one packed entry in 16 bits: lo and hi as 8-bit codes
// in steps of 1/255.  thr_lo <= lo and thr_hi >= hi hold with a relative
// margin of 1e-6, far above the rounding of the float decode, so
// z <= thr_lo implies z <= lo and z >= thr_hi implies z >= hi.  A code of 255
// decodes to 1: as lo it skips every draw (z < 1), as hi none.
typedef uint16_t TermThr;
__host__ __device__ inline float thr_lo(TermThr t) { return (float)(t & 0xFFu) * (1.0f / 255.0f); }
__host__ __device__ inline float thr_hi(TermThr t) { return (float)(t >> 8) * (1.0f / 255.0f); }

// The draws of an entry whose per-XELT term does not depend on the quantile
// (section 2.3's financial terms I on the sampled loss of section 3.3): a
// loss l = max_l x at most the retention nets to 0, one at least retention +
// limit nets to the limit, and x <= t  <=>  z <= I_t(alpha, beta).  From the
// FP64 probabilities lo = I_{ret/max_l} and hi = I_{(ret+lim)/max_l},
// widened by 1e-10 relative (far above their rounding) and coded outward, a
// draw is skipped only where its loss certainly lies beyond a threshold; the
// draws within one code step (1/255) of it are solved.  A degenerate
// entry's loss is its mean (lnB): always one side or never.  Two bytes per
// entry keep the table small enough to stay in L2 beside the layer rows.
__host__ __device__ inline TermThr term_thresholds(const EntryRec& E, double ret, double lim)
{
    double lo = 0.0, hi = 2.0;                         // never: z > 0 and z < 1
    if (E.a == 0.0) {
        if (E.lnB <= ret) lo = 1.0;
        else if (E.lnB >= ret + lim) hi = 0.0;
    } else {
        const double m = (double)E.maxl;
        const double tl = ret / m, th = (ret + lim) / m;
        if (tl >= 1.0) lo = 1.0;                          // every loss is within the retention
        else if (tl > 0.0) lo = beta_inc(tl, E) * (1.0 - 1e-10);
        if (th < 1.0) {
            const double I = beta_inc(th, E);
            hi = I + (1.0 - I) * 1e-10;
        }
    }
    const uint32_t cl = lo >= 1.0 ? 255u : (uint32_t)floor(lo * 255.0 * (1.0 - 1e-6));
    const uint32_t ch = hi <= 0.0 ? 0u : hi >= 1.0 ? 255u : (uint32_t)fmin(ceil(hi * 255.0 * (1.0 + 1e-6)), 255.0);
    return (TermThr)(cl | (ch << 8));
}

// ---------------------------------------------------------------------------
// Inverse of the regularised incomplete beta: x with I_x(a,b) = z.
//
// The root lies below ts = (a+1)/(a+b+2) iff z <= us = I_ts(a,b) (stored per
// entry).  Above it the reflection I_x(a,b) = 1 - I_{1-x}(b,a) turns the
// problem into the same lower-tail one for t = 1-x, p = 1-z and swapped
// shapes, so one solver covers both sides and the fraction always converges
// quickly.  The solver works on y = ln t, where
//   f(y) = ln I_t(A,B) - ln p = A y + B ln(1-t) - lnB - ln A - ln T - ln p,
//   f'(y) = A T / (1 - t),
// which is close to linear in the tails (I ~ t^A / (A B)), so Newton's method
// converges in a few steps from the leading-term start y0 = (ln p + ln A +
// lnB)/A even for shape parameters of 1e-6.  Both stages take Halley's steps
// (the second derivative costs a few operations in this form, see newton32).
// An FP32 stage brings y within ~1e-3, then FP64 steps finish it (cubic
// convergence, one step nearly always): the FP64 pass is what keeps tiny
// shapes, whose quantile amplifies any error in ln I by 1/A, accurate to well
// below the YLT tolerance.
// ---------------------------------------------------------------------------
struct InvBetaStats {
    int it32, it64;
};

// FP32 helpers of the solver's first stage: the hardware log2 / exp2 /
// reciprocal (1 ulp each) in device code, the C library on the host.
__host__ __device__ inline float f32_ln(float x)        // x > 0 and normal
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_logf(x) * 0.6931471805599453f;
#else
    return logf(x);
#endif
}
__host__ __device__ inline float f32_exp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __expf(x);
#else
    return expf(x);
#endif
}
__host__ __device__ inline float f32_rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
// e with x = m 2^e, 1/2 <= |m| < 1 (0 for x = 0)
__host__ __device__ inline int f32_frexp_exp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_frexp_expf(x);
#else
    int e;
    frexpf(x, &e);
    return e;
#endif
}
// ln(1 - t) for 0 <= t < 1: with w = fl(1 - t), ln(w) * t / (1 - w) corrects
// the rounding of w (Goldberg's log1p), a few ulps without extended precision.
__host__ __device__ inline float f32_log1m(float t, float w)
{
    return (w == 1.0f) ? -t : f32_ln(w) * (t * f32_rcp(1.0f - w));
}

// ---------------------------------------------------------------------------
// Per-entry start table of the FP32 solve.  On each side of t_s (the lower
// side solves for t = x, the upper for t = 1 - x with the shapes swapped and
// p = 1 - z) the solution y = ln t is written as the leading term plus a
// residual, y = (ln p - c0)/A + r, where r vanishes as p -> 0.  r is tabulated
// at five knots u_k = k/4 of a variable u in [0, 1], with its exact
// derivative (stored times the knot spacing h), for cubic Hermite
// interpolation.  The variable depends on the side's leading shape A:
//  * A < kVmapShape: u = (p/p_s)^(1/A) (p_s = I_{t_s} on that side).  The
//    series of I_t about t = 0 makes r a power series in t0 u (t0 the leading
//    term's root at p_s), so r is smooth in u from u = 0, where it vanishes
//    with slope (B-1)/(A+1) t0;
//  * otherwise u = (ln(p/p_s) / ln(p_min/p_s))^(1/3) (p_min = 2^-24, the
//    smallest p a draw takes): for large A the draws crowd towards t_s, where
//    the first variable would pile them up at u = 1.
// Built in FP64 from the solver itself and kept in half precision: the
// interpolated start is within about 1e-3 of the root (1e-2 at worst), so one
// Halley step settles nearly every draw.
// ---------------------------------------------------------------------------
constexpr int kKnots = 5;
constexpr float kLnPmin = -16.635532333438686f;      // ln 2^-24
constexpr float kVmapShape = 3.0f;


// One entry's record for the FP32 solve: the shapes and constants in FP32 and
// both sides' start tables, one 64-byte line per draw.  Small-shape entries
// (pol) carry tables too: they start the series form of the solve.
struct alignas(64) SolveRec {
    float a, b;                   // alpha, beta
    float lam;                    // ln B(alpha, beta) + ln min(alpha, beta), formed in FP64
    float us;                     // I_ts, as in EntryRec
    float maxl;                   // max_l
    uint32_t pol;                 // 1: a small shape (is_small_shape): its draws are deferred
    half2_t knot[2][kKnots];      // side 0 lower, 1 upper: (r_k, h * dr/du at u_k)
};
static_assert(sizeof(SolveRec) == 64, "SolveRec must stay one 64-byte line");


// The tabulated residual r at p on one side (cubic Hermite between the two
// knots around u); A is that side's leading shape, lnps = ln p_s and rA = 1/A.
// A side without a table has all knots zero: r = 0.
__host__ __device__ inline float table_residual(const SolveRec& R, bool lower, float A, float lnp, float lnps, float rA)
{
    const half2_t* K = R.knot[lower ? 0 : 1];
    const float q = fmaxf((lnp - lnps) * f32_rcp(kLnPmin - lnps), 0.0f);
    const float u = fminf(A < kVmapShape ? f32_exp((lnp - lnps) * rA)                          // (p/p_s)^(1/A)
                                         : f32_exp(f32_ln(q) * (1.0f / 3.0f)),                // q^(1/3)
                          1.0f);
    const float g = u * (float)(kKnots - 1);
    const int j = g < (float)(kKnots - 2) ? (int)g : kKnots - 2;
    const float w = g - (float)j, w1 = 1.0f - w;
    const half2_t k0 = K[j], k1 = K[j + 1];
    return (1.0f + 2.0f * w) * w1 * w1 * (float)k0.x + w * w1 * w1 * (float)k0.y +
           w * w * (3.0f - 2.0f * w) * (float)k1.x - w * w * w1 * (float)k1.y;
}

__host__ __device__ inline double inv_beta(double z, const EntryRec& E, InvBetaStats* st = nullptr,
                                            const SolveRec* R = nullptr)
{
    const bool lower = z <= (double)E.us;
    const double A = lower ? E.a : E.b;
    const double B = lower ? E.b : E.a;
    const double p = lower ? z : 1.0 - z;
    const double lnB = E.lnB;

    // ---- FP32 stage
    const float Af = (float)A, Bf = (float)B;
    const float lnpf = f32_ln((float)p);
    const float rA = f32_rcp(Af);
    const float ts = (Af + 1.0f) * f32_rcp(Af + Bf + 2.0f);
    const float ymax = f32_ln(fminf(1.1f * ts, 0.5f * (1.0f + ts)));
    // the leading term and the constants are formed in FP64: for tiny A the
    // two logs cancel to O(A) and the FP32 difference would be noise
    const double lnA = log(A), lnp = log(p);
    const float c0f = (float)(-(lnB + lnA));
    float y = (float)((lnp + lnA + lnB) / A);
    if (R && y > -1e30f) y += table_residual(*R, lower, Af, lnpf, f32_ln(lower ? E.us : 1.0f - E.us), rA);
    y = fmaxf(fminf(y, f32_ln(ts)), -1e30f);
    // below these t the loss rounds to 0 (lower side, FP32 loss) or x to 1
    // (upper side, FP64): no need to iterate further
    const float yfloor = lower ? -110.0f : -40.0f;
    int it32 = 0;
    for (; it32 < 12 && y > yfloor; ++it32) {
        const float t = f32_exp(y);
        const float w = 1.0f - t;
        const float l1t = f32_log1m(t, w);
        float num, den;
        beta_cf<float>(t, Af, Bf, 2e-7f, 48, num, den);
        const float rnum = f32_rcp(num);
        const float f = Af * y + Bf * l1t + c0f + f32_ln(den * rnum) - lnpf;   // ln(1/T) = ln(den/num)
        float dy = -(f * w * den) * (rA * rnum);
        // Halley's correction (f''/f' = A - (B-1) t/(1-t) - f', see newton32)
        const float hc = 0.5f * ((Af - (Bf - 1.0f) * t * f32_rcp(w)) * dy + f);
        if (fabsf(hc) < 0.5f) dy *= f32_rcp(1.0f + hc);
        const float yn = fmaxf(fminf(y + dy, ymax), -1e30f);
        const float step = yn - y;
        y = yn;
        if (fabsf(step) <= 2e-3f * fmaxf(1.0f, fabsf(y))) break;
    }

    // ---- FP64 polish
    const double ts64 = (A + 1.0) / (A + B + 2.0);
    const double ymax64 = log(fmin(1.1 * ts64, 0.5 * (1.0 + ts64)));
    double yd = (double)y;
    int it64 = 0;
    for (; it64 < 6 && yd > (double)yfloor; ++it64) {
        const double t = exp(yd);
        const double l1t = log1p(-t);
        double num, den;
        beta_cf<double>(t, A, B, 1e-13, 200, num, den);
        const double T = num / den;
        const double f = A * yd + B * l1t - lnB - lnA - log(T) - lnp;
        double dy = -f * (1.0 - t) / (A * T);
        const double hc = 0.5 * ((A - (B - 1.0) * t / (1.0 - t)) * dy + f);
        if (fabs(hc) < 0.5) dy /= 1.0 + hc;
        const double yn = fmax(fmin(yd + dy, ymax64), -1e300);
        const double step = yn - yd;
        yd = yn;
        // cubic convergence: after a step below 1e-4 the error is of order 1e-12
        if (fabs(step) <= 1e-4) break;
    }
    if (st) {
        st->it32 = it32;
        st->it64 = it64;
    }
    return lower ? exp(yd) : -expm1(yd);
}

// Draws of entries whose smaller shape parameter is below this are small-shape
// draws: on the side whose leading shape is below it they take the series
// form of the solve (inv_beta32_any), deferred in the plain kernel so that the
// two forms do not split a solve wave.  At or above it the continued-fraction
// FP32 solve, with c0 formed in FP64, is within 1e-5 relative of the FP64
// inverse (5e-6 at worst, 2e-6 in 99 of 100 draws); the quantile's
// sensitivity to an error in ln I grows like 1/shape, most of all near t_s,
// where the terms of ln I cancel in that form (1e-5 is reached near 0.15).
constexpr double kSmallShape = 0.2;
// Below this the surrogate kernel's exact fallback, which solves from the
// entry record (c0 in FP32, whose error the quantile divides by the shape),
// takes the FP64 polish of inv_beta.
constexpr double kPolishShapeEntry = 0.2;

__host__ __device__ inline bool is_small_shape(const EntryRec& E)
{
    return (E.a < E.b ? E.a : E.b) < kSmallShape;
}

// Knots of one side, nk of them at u_k = k/(nk-1): out[2k] = r_k and
// out[2k+1] = h * dr/du at u_k (h = 1/(nk-1)).  A side no draw reaches, or one
// whose knots leave FP64 or half range, is left zero (the start is then the
// leading term alone).
__host__ __device__ inline void knot_side_n(const EntryRec& E, bool lower, int nk, float* out)
{
    for (int k = 0; k < 2 * nk; ++k) out[k] = 0.0f;
    if (E.a == 0.0) return;                                // degenerate entry: no draws solve
    const double A = lower ? E.a : E.b, B = lower ? E.b : E.a;
    const double ps = lower ? (double)E.us : 1.0 - (double)E.us;
    if (!(ps > 0.0)) return;
    const double lnps = log(ps);
    const double smin = (double)kLnPmin - lnps;
    if (!(smin < 0.0)) return;                             // no p on the 2^-24 grid reaches this side
    const double c0 = -(E.lnB + log(A));
    const double h = 1.0 / (nk - 1);
    const bool vmap = (float)A < kVmapShape;               // the same test the solve makes
    EntryRec S = E;                                        // the side's own problem: shapes (A, B), I_ts = p_s
    S.a = A;
    S.b = B;
    S.us = (float)ps;
    const double ts = (A + 1.0) / (A + B + 2.0);
    for (int k = 0; k < nk; ++k) {
        const double u = k * h;
        double r, d;
        if (vmap && k == 0) {
            r = 0.0;
            d = (B - 1.0) / (A + 1.0) * exp((lnps - c0) / A);
        } else {
            // ln(p/p_s) at the knot, and d ln(p/p_s)/du there
            const double sk = vmap ? A * log(u) : smin * u * u * u;
            const double dsdu = vmap ? A / u : smin * 3.0 * u * u;
            const double p = (k == nk - 1 && vmap) || (k == 0) ? ps : ps * exp(sk);
            const double t = (p == ps) ? ts : inv_beta(p, S);
            if (!(t > 0.0)) {                              // below FP64 range: leave the side empty
                for (int q = 0; q < 2 * nk; ++q) out[q] = 0.0f;
                return;
            }
            double num, den;
            beta_cf<double>(t, A, B, 1e-15, 400, num, den);
            const double dyds = (1.0 - t) * den / (A * num);   // 1 / (d ln I / d ln t)
            r = log(t) - (log(p) - c0) / A;
            d = (dyds - 1.0 / A) * dsdu;
        }
        if (!(fabs(r) < 1e4)) {                            // beyond half precision: no table
            for (int q = 0; q < 2 * nk; ++q) out[q] = 0.0f;
            return;
        }
        if (!(fabs(d) < 1e4)) d = 0.0;
        out[2 * k] = (float)r;
        out[2 * k + 1] = (float)(d * h);
    }
}

__host__ __device__ inline void knot_side(const EntryRec& E, bool lower, float* out)
{
    knot_side_n(E, lower, kKnots, out);
}

__host__ __device__ inline SolveRec make_solve_rec(const EntryRec& E)
{
    SolveRec R;
    R.a = (float)E.a;
    R.b = (float)E.b;
    R.lam = E.a == 0.0 ? 0.0f : (float)(E.lnB + log(E.a < E.b ? E.a : E.b));
    R.us = E.us;
    R.maxl = E.maxl;
    R.pol = is_small_shape(E) ? 1u : 0u;
    for (int side = 0; side < 2; ++side) {
        float v[2 * kKnots];
        knot_side(E, side == 0, v);
        for (int k = 0; k < kKnots; ++k) {
            half2_t q;
            q.x = (_Float16)v[2 * k];
            q.y = (_Float16)v[2 * k + 1];
            R.knot[side][k] = q;
        }
    }
    return R;
}

// The continued fraction F = 1/(1 + d1/(1 + d2/(1 + ...))) of DLMF 8.17.22
// in FP32 (I_t = t^A (1-t)^B / (A B(A, B)) F), as the ratio P/Q of the
// continuants of that normalized form (every partial denominator 1):
//   X_n = X_{n-1} + d_n X_{n-2},
//   d_{2m+1} = -(A+m)(A+B+m) t / ((A+2m)(A+2m+1)),
//   d_{2m+2} = (m+1)(B-m-1) t / ((A+2m+1)(A+2m+2)).
// The continuants stay near order one, so a power-of-two rescale every two
// pairs of terms keeps them in range; the two denominators of a pair share
// one reciprocal.  Convergence (successive approximants within eps) is tested
// after every two pairs; at most 48 pairs.
__host__ __device__ inline void beta_cf32(float t, float A, float B, float eps, float& P, float& Q)
{
    float P2 = 0.0f, P1 = 1.0f, Q2 = 1.0f, Q1 = 1.0f;     // X_{n-2}, X_{n-1} from n = 2
    const float apb = A + B, bm1 = B - 1.0f;
    float fm = 0.0f;                                      // m, carried as a float
    for (int k = 0; k < 24; ++k) {
        for (int h = 0; h < 2; ++h, fm += 1.0f) {
            const float a2 = fmaf(2.0f, fm, A), a21 = a2 + 1.0f;
            const float Do = a2 * a21, De = a21 * (a2 + 2.0f);
            const float r = f32_rcp(Do * De);
            const float d_o = -(A + fm) * (apb + fm) * t * (De * r);
            const float d_e = (fm + 1.0f) * (bm1 - fm) * t * (Do * r);
            const float Po = fmaf(d_o, P2, P1), Qo = fmaf(d_o, Q2, Q1);
            P1 = fmaf(d_e, P1, Po);
            Q1 = fmaf(d_e, Q1, Qo);
            P2 = Po;
            Q2 = Qo;
        }
        const int ex = -f32_frexp_exp(Q1);
        P2 = ldexpf(P2, ex);
        Q2 = ldexpf(Q2, ex);
        P1 = ldexpf(P1, ex);
        Q1 = ldexpf(Q1, ex);
        const float x = P1 * Q2;
        if (fabsf(x - P2 * Q1) <= eps * fabsf(x)) break;
    }
    P = P1;
    Q = Q1;
}

// Halley iteration of the FP32 solve from the start y, on f(y) = ln I_t - ln p
// with t = e^y.  f'(y) = 1/(dy/d ln I) is what the Newton step divides by, and
// f''/f' = A - (B-1) t/(1-t) - f', so the cubic correction costs a few
// operations: with the Newton step d = -f/f', Halley's step is
// d / (1 + d f''/(2 f')), taken while that factor stays within (1/2, 3/2).
// From a rough start (ROUGH) the first step only has to land near the root: a
// continued fraction good to 1e-2 suffices there, and that step never ends the
// loop.  The loop stops once a step moves the quantile x by less than 1e-2
// relative: cubic convergence leaves far less than the FP32 evaluation noise
// in ln I, which sets the error in x on the shapes this path takes
// (min(a, b) >= kSmallShape): below 1e-5 against the FP64 inverse.
constexpr float kStopX = 1e-2f;

template <bool ROUGH>
__device__ inline float newton32(float y, bool lower, float A, float B, float lnp, float c0, float rA, float ymax)
{
    const float yfloor = lower ? -110.0f : -40.0f;
    for (int it = 0; it < 10 && y > yfloor; ++it) {
        const float t = __expf(y);
        const float w = 1.0f - t;
        const float l1t = f32_log1m(t, w);
        const float tw = t * f32_rcp(w);
        float P, Q;
        const bool rough = ROUGH && it == 0;
        beta_cf32(t, A, B, rough ? 1e-2f : 2e-7f, P, Q);
        const float F = P * f32_rcp(Q);
        const float f = A * y + B * l1t + c0 + f32_ln(F) - lnp;
        float dy = -(f * w * F) * rA;                                      // Newton: -f/f', f' = A/((1-t) F)
        const float hc = 0.5f * ((A - (B - 1.0f) * tw) * dy + f);          // d f''/(2 f')
        if (fabsf(hc) < 0.5f) dy *= f32_rcp(1.0f + hc);
        const float yn = fminf(y + dy, ymax);
        const float step = yn - y;
        y = yn;
        // a step dy moves x by dy (lower side, x = t) or by dy * t / (1 - t)
        // relative to x (upper side, x = 1 - t)
        if (!rough && fabsf(step) * (lower ? 1.0f : tw) <= kStopX) break;
    }
    return lower ? __expf(y) : -expm1f(y);
}

// A draw's z in FP64 (the correlated draws of section 3.2) as the FP32 solves
// take it: z itself at or below 1/2, minus (1 - z) above, with 1 - z formed in
// FP64 before rounding, so either tail keeps its relative accuracy in one
// float (rounding z itself would turn any z above 1 - 2^-25 into 1).  Draws on
// the 2^-24 grid code exactly.
__host__ __device__ inline float tail_code(double z)
{
    return z <= 0.5 ? (float)z : -(float)(1.0 - z);
}

// The side of t_s a coded draw falls on (lower: z <= I_ts = us) and that
// side's probability p (z on the lower side, 1 - z on the upper).
__host__ __device__ inline void tail_side(float code, float us, bool& lower, float& p)
{
    if (code > 0.0f) {
        lower = code <= us;
        p = lower ? code : 1.0f - code;
    } else {
        const float q = -code;                 // 1 - z
        lower = q >= 1.0f - us;
        p = lower ? 1.0f - q : q;
    }
}

// FP32-only inverse for well-conditioned shapes (min(a, b) >= kSmallShape),
// started from the entry's table: inv_beta's log-space iteration with Halley's
// correction and the hardware helpers above, given the draw's side and that
// side's probability.  Device only.
__device__ inline float inv_beta32_side(bool lower, float p, const SolveRec& R)
{
    const float A = lower ? R.a : R.b;
    const float B = lower ? R.b : R.a;
    const float lnp = f32_ln(p);
    const float rA = f32_rcp(A);
    // c0 = -(ln B + ln A).  For a small shape the two logs cancel to O(A),
    // and the quantile moves by the error of c0 over A, so the smaller side's
    // c0 comes formed in FP64 (-lam); the other side adds ln(A / min(a, b)).
    const float mn = fminf(R.a, R.b);
    const float c0 = A == mn ? -R.lam : -(R.lam + f32_ln(A * f32_rcp(mn)));
    const float ts = (A + 1.0f) * f32_rcp(A + B + 2.0f);
    const float ymax = f32_ln(fminf(1.1f * ts, 0.5f * (1.0f + ts)));
    const float lnps = f32_ln(lower ? R.us : 1.0f - R.us);
    const float r = table_residual(R, lower, A, lnp, lnps, rA);
    return newton32<false>(fminf((lnp - c0) * rA + r, ymax), lower, A, B, lnp, c0, rA, ymax);
}

// The same for a draw on the 2^-24 grid (p = 1 - z is exact there).
__device__ inline float inv_beta32(float z, const SolveRec& R)
{
    const bool lower = z <= R.us;
    return inv_beta32_side(lower, lower ? z : 1.0f - z, R);
}

// The same for a coded draw (tail_code).
__device__ inline float inv_beta32_code(float code, const SolveRec& R)
{
    bool lower;
    float p;
    tail_side(code, R.us, lower, p);
    return inv_beta32_side(lower, p, R);
}

// ---------------------------------------------------------------------------
// Small leading shape.  The hypergeometric form of I_t (DLMF 8.17(ii)),
//   I_t(A, B) = t^A / (A B(A, B)) (1 + A S(t)),
//   S(t) = sum_{n>=1} (1-B)(2-B)...(n-B) t^n / (n! (A+n)),
// writes ln I_t - ln p = A y + c0 + ln(1 + A S) - ln p with every term of
// order A near the root, where the continued-fraction form subtracts two
// terms of order B t (B ln(1-t) and ln T) to leave that remainder: in FP32
// their rounding, divided by the slope A, swamps the quantile near t_s.  With
// the series, c0 formed in FP64 and ln p and the sum taken in FP64, the FP32
// solve holds 1e-5 relative for any shape.  The series converges like t^n
// (t <= 1.1 t_s on this side, and t_s <= 1/2 once A <= B).
// ---------------------------------------------------------------------------
__device__ inline float ln1p_as(float t, float A, float B)       // ln(1 + A S(t))
{
    float c = 1.0f, S = 0.0f;                                      // c = (1-B)_n t^n / n!
    for (int n = 1; n <= 64; ++n) {
        const float fn = (float)n;
        c *= (fn - B) * t * f32_rcp(fn);
        const float term = c * f32_rcp(A + fn);
        S += term;
        if (fabsf(term) <= 3e-8f * fabsf(S)) break;
    }
    return log1pf(A * S);
}

// Halley's iteration on y = ln t with that form: f' = A (1-t)^(B-1) / (1 + A S)
// and f''/f' = A - (B-1) t/(1-t) - f' as in newton32.
__device__ inline float newton32_small(float y, bool lower, float A, float B, double lnp, double c0, float ymax)
{
    const float yfloor = lower ? -110.0f : -40.0f;
    for (int it = 0; it < 12 && y > yfloor; ++it) {
        const float t = __expf(y);
        const float w = 1.0f - t;
        const float l1t = f32_log1m(t, w);
        const float tw = t * f32_rcp(w);
        const float lg = ln1p_as(t, A, B);
        const float f = (float)(((double)A * (double)y + c0 - lnp) + (double)lg);
        float dy = -f * f32_rcp(A * __expf((B - 1.0f) * l1t - lg));
        const float hc = 0.5f * ((A - (B - 1.0f) * tw) * dy + f);
        if (fabsf(hc) < 0.5f) dy *= f32_rcp(1.0f + hc);
        const float yn = fminf(y + dy, ymax);
        const float step = yn - y;
        y = yn;
        if (fabsf(step) * (lower ? 1.0f : tw) <= kStopX) break;
    }
    // the quantile itself through the accurate exp: __expf scales y by log2(e)
    // in FP32 first, a relative error of |y| 2^-24 in x
    return lower ? expf(y) : -expm1f(y);
}

// The solve of a draw with z in FP64 (any shape): the side's leading shape at
// or above kSmallShape takes inv_beta32_side, a smaller one the series form,
// with c0 from the entry's FP64 ln B (for two tiny shapes c0 is of order one
// while the slope A is tiny, so even its FP32 rounding would show).
__device__ inline float inv_beta32_any(double z, const EntryRec& E, const SolveRec& R)
{
    const bool lower = z <= (double)R.us;
    const double p = lower ? z : 1.0 - z;
    const float A = lower ? R.a : R.b;
    if (A >= (float)kSmallShape) return inv_beta32_side(lower, (float)p, R);
    const float B = lower ? R.b : R.a;
    const double c0 = -(E.lnB + log(lower ? E.a : E.b));
    const double lnp = log(p);
    const float rA = f32_rcp(A);
    const float ts = (A + 1.0f) * f32_rcp(A + B + 2.0f);
    const float ymax = f32_ln(fminf(1.1f * ts, 0.5f * (1.0f + ts)));
    const float lnpf = (float)lnp;
    const float lnps = f32_ln(lower ? R.us : 1.0f - R.us);
    const float r = table_residual(R, lower, A, lnpf, lnps, rA);
    return newton32_small(fminf((lnpf - (float)c0) * rA + r, ymax), lower, A, B, lnp, c0, ymax);
}

// The same solve started from a corrected leading term, for callers that hold
// only the entry record.  ln I_t = A y + c0 + g(t) with g(t) = B ln(1-t) -
// ln T(t), which vanishes at t = 0 and equals ln I_ts - A ln ts - c0 at ts (I_ts
// is stored).  Taking g linear in t and evaluating it at the leading-term root
// gives one cheap fixed-point step that brings the draws near ts, where the
// leading term alone is worst, within one Newton step.  Device only.
__device__ inline float inv_beta32_side(bool lower, float p, const EntryRec& E)
{
    const float A = (float)(lower ? E.a : E.b);
    const float B = (float)(lower ? E.b : E.a);
    const float lnp = f32_ln(p);
    const float rA = f32_rcp(A);
    const float c0 = -((float)E.lnB + f32_ln(A));
    const float ts = (A + 1.0f) * f32_rcp(A + B + 2.0f);
    const float lts = f32_ln(ts);
    const float ymax = f32_ln(fminf(1.1f * ts, 0.5f * (1.0f + ts)));
    const float lnps = f32_ln(lower ? E.us : 1.0f - E.us);
    float y = fminf((lnp - c0) * rA, lts);
    const float gs = lnps - A * lts - c0;
    y = fminf((lnp - c0 - gs * __expf(y) * f32_rcp(ts)) * rA, lts);
    return newton32<true>(y, lower, A, B, lnp, c0, rA, ymax);
}

__device__ inline float inv_beta32_code(float code, const EntryRec& E)
{
    bool lower;
    float p;
    tail_side(code, E.us, lower, p);
    return inv_beta32_side(lower, p, E);
}

// ---------------------------------------------------------------------------
// Tabulated inverse (the table mode, a third sampling form beside the exact
// solve and the surrogate): the same residual representation as the start
// tables, y = (ln p - c0)/A + r(u), with the same variable u per side, but
// seventeen FP32 knots per side and no iteration afterwards.  The leading
// term carries the quantile's p^(1/A) behaviour in the lower tail, so the
// interpolated part stays smooth; x = e^y (lower side) or 1 - e^y (upper).
// Against the FP64 inverse on the paper's shapes: relative error below 1e-4
// for every draw (1.3e-5 at the 99th percentile), absolute error in x below
// 1e-5.  Built in FP64 at load; 320 bytes per entry, of which a draw reads the
// 32-byte head and two adjacent knots.
// ---------------------------------------------------------------------------
constexpr int kTabKnots = 17;

struct alignas(64) TabRec {
    float a, b;                      // alpha, beta
    float lnB;                       // ln B(alpha, beta)
    float us;                        // I_ts
    float maxl;                      // max_l; the mean loss of a degenerate entry
    uint32_t deg;                    // 1: degenerate (sigma = 0): the loss is maxl itself
    float c0[2];                     // -(ln B + ln A) per side, formed in FP64 (for tiny A the
                                     // two logs cancel to O(A): FP32 would leave noise / A in y)
    float2 knot[2][kTabKnots];       // side 0 lower, 1 upper: (r_k, h * dr/du at u_k)
};
static_assert(sizeof(TabRec) == 320, "TabRec must stay 320 bytes");

__host__ __device__ inline TabRec make_tab_rec(const EntryRec& E)
{
    TabRec T;
    T.a = (float)E.a;
    T.b = (float)E.b;
    T.lnB = (float)E.lnB;
    T.us = E.us;
    T.deg = E.a == 0.0 ? 1u : 0u;
    T.maxl = T.deg ? (float)E.lnB : E.maxl;
    T.c0[0] = T.deg ? 0.0f : (float)(-(E.lnB + log(E.a)));
    T.c0[1] = T.deg ? 0.0f : (float)(-(E.lnB + log(E.b)));
    for (int side = 0; side < 2; ++side) {
        float v[2 * kTabKnots];
        knot_side_n(E, side == 0, kTabKnots, v);
        for (int k = 0; k < kTabKnots; ++k) {
            T.knot[side][k].x = v[2 * k];
            T.knot[side][k].y = v[2 * k + 1];
        }
    }
    return T;
}

// x = I^-1(z) from the entry's table (1 for a degenerate entry, whose loss is
// maxl).
__host__ __device__ inline float tab_inverse_side(bool lower, float p, const TabRec& T)
{
    if (T.deg) return 1.0f;
    const float A = lower ? T.a : T.b;
    const float lnp = f32_ln(p);
    const float rA = f32_rcp(A);
    const float c0 = T.c0[lower ? 0 : 1];
    const float lnps = f32_ln(lower ? T.us : 1.0f - T.us);
    const float2* K = T.knot[lower ? 0 : 1];
    const float q = fmaxf((lnp - lnps) * f32_rcp(kLnPmin - lnps), 0.0f);
    const float u = fminf(A < kVmapShape ? f32_exp((lnp - lnps) * rA) : f32_exp(f32_ln(q) * (1.0f / 3.0f)), 1.0f);
    const float g = u * (float)(kTabKnots - 1);
    const int j = g < (float)(kTabKnots - 2) ? (int)g : kTabKnots - 2;
    const float w = g - (float)j, w1 = 1.0f - w;
    const float2 k0 = K[j], k1 = K[j + 1];
    const float r = (1.0f + 2.0f * w) * w1 * w1 * k0.x + w * w1 * w1 * k0.y + w * w * (3.0f - 2.0f * w) * k1.x -
                    w * w * w1 * k1.y;
    const float ts = (A + 1.0f) * f32_rcp(A + (lower ? T.b : T.a) + 2.0f);
    const float y = fminf((lnp - c0) * rA + r, f32_ln(ts));
    return lower ? f32_exp(y) : -expm1f(y);
}

// The same for a draw on the 2^-24 grid, and for a coded draw (tail_code).
__host__ __device__ inline float tab_inverse(float z, const TabRec& T)
{
    const bool lower = z <= T.us;
    return tab_inverse_side(lower, lower ? z : 1.0f - z, T);
}
__host__ __device__ inline float tab_inverse_code(float code, const TabRec& T)
{
    bool lower;
    float p;
    tail_side(code, T.us, lower, p);
    return tab_inverse_side(lower, p, T);
}

// The inverse the plain layer kernel applies to one draw of z (FP64: any z in
// (0, 1), not only the 2^-24 grid, reaches the FP32 solve as its tail code).
__device__ inline double inv_beta_layer(double z, const EntryRec& E, const SolveRec& R)
{
    if (R.pol) return E.a == 0.0 ? E.lnB / E.maxl : (double)inv_beta32_any(z, E, R);
    return (double)inv_beta32_code(tail_code(z), R);
}

// Sampled loss of one draw: max_l * InvCDF_beta(z; alpha, beta) (section 3.3).
__host__ __device__ inline float sample_loss(double z, const EntryRec& E)
{
    if (E.a == 0.0) return (float)E.lnB;       // degenerate: the mean loss
    return E.maxl * (float)inv_beta(z, E);
}

// ---------------------------------------------------------------------------
// Normal quantile Phi^-1(p) for 0 < p < 1, FP64: Wichura's algorithm AS 241
// (PPND16, Applied Statistics 37, 1988), relative accuracy about 1e-16.  A
// rational function of degree 7 in r = 0.180625 - q^2 around the centre
// (|q| = |p - 1/2| <= 0.425); in the tails, of r = sqrt(-ln min(p, 1 - p))
// shifted by 1.6 (r <= 5) or by 5.  The correlated draws of section 3.2 need
// two per draw, so this replaces the general library routine, which is an
// order of magnitude longer.
// ---------------------------------------------------------------------------
__host__ __device__ inline double poly7(double x, double c0, double c1, double c2, double c3, double c4, double c5,
                                        double c6, double c7)
{
    return ((((((c7 * x + c6) * x + c5) * x + c4) * x + c3) * x + c2) * x + c1) * x + c0;
}

__host__ __device__ inline double normal_quantile(double p)
{
    const double q = p - 0.5;
    if (fabs(q) <= 0.425) {
        const double r = 0.180625 - q * q;
        return q *
               poly7(r, 3.3871328727963666080e0, 1.3314166789178437745e+2, 1.9715909503065514427e+3,
                     1.3731693765509461125e+4, 4.5921953931549871457e+4, 6.7265770927008700853e+4,
                     3.3430575583588128105e+4, 2.5090809287301226727e+3) /
               poly7(r, 1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2, 5.3941960214247511077e+3,
                     2.1213794301586595867e+4, 3.9307895800092710610e+4, 2.8729085735721942674e+4,
                     5.2264952788528545610e+3);
    }
    double r = sqrt(-log(q < 0.0 ? p : 1.0 - p));
    double x;
    if (r <= 5.0) {
        r -= 1.6;
        x = poly7(r, 1.42343711074968357734e0, 4.63033784615654529590e0, 5.76949722146069140550e0,
                  3.64784832476320460504e0, 1.27045825245236838258e0, 2.41780725177450611770e-1,
                  2.27238449892691845833e-2, 7.74545014278341407640e-4) /
            poly7(r, 1.0, 2.05319162663775882187e0, 1.67638483018380384940e0, 6.89767334985100004550e-1,
                  1.48103976427480074590e-1, 1.51986665636164571966e-2, 5.47593808499534494600e-4,
                  1.05075007164441684324e-9);
    } else {
        r -= 5.0;
        x = poly7(r, 6.65790464350110377720e0, 5.46378491116411436990e0, 1.78482653991729133580e0,
                  2.96560571828504891230e-1, 2.65321895265761230930e-2, 1.24266094738807843860e-3,
                  2.71155556874348757815e-5, 2.01033439929228813265e-7) /
            poly7(r, 1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1, 1.48753612908506148525e-2,
                  7.86869131145613259100e-4, 1.84631831751005468180e-5, 1.42151175831644588870e-7,
                  2.04426310338993978564e-15);
    }
    return q < 0.0 ? -x : x;
}

// Financial terms: min(max(l - retention, 0), limit).
__host__ __device__ inline float xl(float l, float retention, float limit)
{
    return fminf(fmaxf(l - retention, 0.0f), limit);
}

}  // namespace ara
