// ara_mlp.hpp -- the sampling surrogate: a 3 -> 64 -> 64 -> 1 multilayer
// perceptron approximating the inverse Beta CDF of section 3.3, evaluated and
// trained with gfx950 matrix cores (v_mfma_f32_16x16x32_f16).
//
// Model.  For a draw with shapes (a, b) and uniform u, with v = Phi^-1(u):
//   features  f = (ln a / 2, ln b / 2, v / 3)
//   base      logit-normal approximation of the quantile in logit space:
//             m + s v,  m = psi(a) - psi(b),  s = sqrt(psi'(a) + psi'(b))
//             (ln(X/(1-X)) for X ~ Beta(a,b) is a difference of log-gamma
//             variates with exactly this mean and variance)
//   network   o = w3 . g(W2 g(W1 f + b1) + b2) + b3,  g(z) = z S(z), with S a
//             piecewise-cubic stand-in for the Gaussian CDF of GELU:
//             S(z) = smoothstep(clamp(z/5 + 1/2, 0, 1)) = u^2 (3 - 2u)
//   output    x = sigmoid(m + s v + o)
// so the network learns a residual in logit space.  Weights are kept in FP32
// (training master copy) and used rounded to BF16; activations are FP16 and
// every product accumulates in FP32.  A BF16 value is exact in FP16 when its
// magnitude lies in FP16's normal range [2^-14, 65504] (8-bit significand
// inside an 11-bit one); the MFMAs run in FP16 on the BF16-rounded weights,
// so a weight below 2^-14 lands on an FP16 subnormal, within 2^-25 of its
// BF16 value (the tests check that trained weights stay below 65504).
#pragma once

#include "ara_math.hpp"

namespace ara {

constexpr int kHid = 64;
// flat FP32 parameter vector
constexpr int kOffW1 = 0;                  // [64][3]
constexpr int kOffB1 = 192;                // [64]
constexpr int kOffW2 = 256;                // [64 out][64 in]
constexpr int kOffB2 = 256 + 4096;         // [64]
constexpr int kOffW3 = kOffB2 + 64;        // [64]
constexpr int kOffB3 = kOffW3 + 64;        // [1]
constexpr int kNumParams = kOffB3 + 1;     // 4481

// Surrogate domain and region grid of the error table.
constexpr float kSurLo = 0.2f, kSurHi = 50.0f;
constexpr int kCellsA = 16, kCellsB = 16, kCellsV = 16;
constexpr int kCells = kCellsA * kCellsB * kCellsV;
constexpr float kVLim = 5.5f;              // |Phi^-1(u)| < 5.34 on the 2^-24 grid
// Calibration: per-cell error sums in units of 2^-36 (|error| <= 1, so 10^7
// points stay below 2^63); a cell answers by the surrogate only when it saw at
// least kCalibMinCount held-out points and kCalibMargin times its largest
// error after the bias correction is within the tolerance.
constexpr double kCalibScale = 68719476736.0;   // 2^36
constexpr unsigned kCalibMinCount = 64;
constexpr double kCalibMargin = 1.5;

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// activation g(z) = z S(z) and its derivative S(z) + z S'(z), in FP32 (training)
__host__ __device__ inline float gelu_s(float z)
{
    const float u = fminf(fmaxf(z * 0.2f + 0.5f, 0.0f), 1.0f);
    return z * (u * u * (3.0f - 2.0f * u));
}
__host__ __device__ inline float gelu_s_grad(float z)
{
    const float u = fminf(fmaxf(z * 0.2f + 0.5f, 0.0f), 1.0f);
    return u * u * (3.0f - 2.0f * u) + z * (1.2f * u * (1.0f - u));
}

// the same activation on two FP16 values at once (inference)
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
__device__ inline h2 gelu_h2(h2 z)
{
    const h2 half = {(_Float16)0.5f, (_Float16)0.5f}, fifth = {(_Float16)0.2f, (_Float16)0.2f};
    const h2 zero = {(_Float16)0.0f, (_Float16)0.0f}, one = {(_Float16)1.0f, (_Float16)1.0f};
    const h2 three = {(_Float16)3.0f, (_Float16)3.0f}, mtwo = {(_Float16)-2.0f, (_Float16)-2.0f};
    h2 u = z * fifth + half;
    u = __builtin_elementwise_min(__builtin_elementwise_max(u, zero), one);
    return z * (u * u * (u * mtwo + three));
}

// ---- digamma and trigamma (asymptotic series after the recurrences
// psi(x) = psi(x+1) - 1/x and psi'(x) = psi'(x+1) + 1/x^2, x shifted to >= 8)
__host__ __device__ inline double digamma(double x)
{
    double r = 0.0;
    while (x < 8.0) {
        r -= 1.0 / x;
        x += 1.0;
    }
    const double i2 = 1.0 / (x * x);
    return r + log(x) - 0.5 / x - i2 * (1.0 / 12 - i2 * (1.0 / 120 - i2 * (1.0 / 252 - i2 * (1.0 / 240 - i2 / 132))));
}

__host__ __device__ inline double trigamma(double x)
{
    double r = 0.0;
    while (x < 8.0) {
        r += 1.0 / (x * x);
        x += 1.0;
    }
    const double i = 1.0 / x, i2 = i * i;
    return r + i + 0.5 * i2 + i * i2 * (1.0 / 6 - i2 * (1.0 / 30 - i2 * (1.0 / 42 - i2 * (1.0 / 30 - i2 * 5.0 / 66))));
}

// Per-entry surrogate record (derived at table build from the entry's shapes).
struct alignas(16) SurEntry {
    float f0, f1;       // ln a / 2, ln b / 2
    float m, s;         // logit-normal base
};

__host__ __device__ inline SurEntry sur_entry(double a, double b)
{
    SurEntry S;
    S.f0 = (float)(0.5 * log(a));
    S.f1 = (float)(0.5 * log(b));
    S.m = (float)(digamma(a) - digamma(b));
    S.s = (float)sqrt(trigamma(a) + trigamma(b));
    return S;
}

__host__ __device__ inline bool sur_in_domain(double a, double b)
{
    return a >= kSurLo && a <= kSurHi && b >= kSurLo && b <= kSurHi;
}

__host__ __device__ inline int sur_bin(float x, float lo, float hi, int n)
{
    int i = (int)floorf((x - lo) / (hi - lo) * (float)n);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__host__ __device__ inline int sur_cell(float f0, float f1, float v)
{
    const float lo = 0.5f * logf(kSurLo), hi = 0.5f * logf(kSurHi);
    return (sur_bin(f0, lo, hi, kCellsA) * kCellsB + sur_bin(f1, lo, hi, kCellsB)) * kCellsV +
           sur_bin(v, -kVLim, kVLim, kCellsV);
}

// Round an FP32 weight to the nearest BF16 value (returned as FP16, exact).
__host__ __device__ inline _Float16 bf16_round_to_h(float w)
{
    uint32_t u;
    __builtin_memcpy(&u, &w, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
    float r;
    __builtin_memcpy(&r, &u, 4);
    return (_Float16)r;
}

// ---------------------------------------------------------------------------
// Inference fragments.  The network is evaluated transposed (hidden units as
// rows, draws as columns) on 16-draw tiles.  For v_mfma_f32_16x16x32_f16 lane
// l (q = l/16) holds A[l%16][8q+t], B[8q+t][l%16] and D[4q+r][l%16].  The
// K-order of the second and third products is permuted so that the FP32
// accumulators of the previous layer, passed through g and packed to FP16,
// are the next B operand without any data movement: K slot 8q+t of K-step s
// is hidden unit 16(2s) + 4q + t for t < 4 and 16(2s+1) + 4q + t-4 for t >= 4.
// ---------------------------------------------------------------------------
struct MlpFrag {
    h8 w1[4][64];        // A of layer 1, per hidden tile; K slots 0..2 features, 3 the bias
    h8 w2[4][2][64];     // A of layer 2, per output tile and K-step
    h8 w3[2][64];        // A of layer 3 (row 0 only)
    f4 b2[4][64];        // accumulator start of layer 2
    float b3;
};

__host__ __device__ inline int perm_hidden(int s, int q, int t)
{
    return t < 4 ? 16 * (2 * s) + 4 * q + t : 16 * (2 * s + 1) + 4 * q + (t - 4);
}

// Build lane `l`'s fragments from the flat FP32 parameters.
__device__ inline void mlp_build_frag_lane(const float* __restrict__ P, MlpFrag& F, int l)
{
    const int q = l >> 4, i = l & 15;
    for (int I = 0; I < 4; ++I) {
        h8 a;
        for (int t = 0; t < 8; ++t) {
            float w = 0.0f;
            if (q == 0 && t < 3) w = P[kOffW1 + (16 * I + i) * 3 + t];
            if (q == 0 && t == 3) w = P[kOffB1 + 16 * I + i];
            a[t] = bf16_round_to_h(w);
        }
        F.w1[I][l] = a;
        for (int s = 0; s < 2; ++s) {
            h8 w;
            for (int t = 0; t < 8; ++t) w[t] = bf16_round_to_h(P[kOffW2 + (16 * I + i) * kHid + perm_hidden(s, q, t)]);
            F.w2[I][s][l] = w;
        }
        f4 bb;
        for (int r = 0; r < 4; ++r) bb[r] = (float)bf16_round_to_h(P[kOffB2 + 16 * I + 4 * q + r]);
        F.b2[I][l] = bb;
    }
    for (int s = 0; s < 2; ++s) {
        h8 w;
        for (int t = 0; t < 8; ++t) w[t] = (i == 0) ? bf16_round_to_h(P[kOffW3 + perm_hidden(s, q, t)]) : (_Float16)0.0f;
        F.w3[s][l] = w;
    }
    if (l == 0) F.b3 = (float)bf16_round_to_h(P[kOffB3]);
}

// g applied to two FP32 accumulator quads, packed as the 8 FP16 K slots of
// the next B operand (first quad -> slots 0..3, second -> 4..7)
__device__ inline h8 act_pack(const f4& a, const f4& b)
{
    h2 p[4];
    p[0] = h2{(_Float16)a[0], (_Float16)a[1]};
    p[1] = h2{(_Float16)a[2], (_Float16)a[3]};
    p[2] = h2{(_Float16)b[0], (_Float16)b[1]};
    p[3] = h2{(_Float16)b[2], (_Float16)b[3]};
    h8 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const h2 g = gelu_h2(p[i]);
        r[2 * i] = g[0];
        r[2 * i + 1] = g[1];
    }
    return r;
}

// Residual o for the 64 draws of a wave: lane L supplies draw L's features
// and receives draw L's output.  F lives in LDS.
__device__ inline float mlp_forward64(const MlpFrag& F, float f0, float f1, float f2)
{
    const int l = threadIdx.x & 63, q = l >> 4;
    float out = 0.0f;
#pragma unroll
    for (int J = 0; J < 4; ++J) {
        // B operand of layer 1: lanes 0..15 carry the features of draw 16J + l
        const int src = 16 * J + (l & 15);
        const float g0 = __shfl(f0, src, 64), g1 = __shfl(f1, src, 64), g2 = __shfl(f2, src, 64);
        h8 x = {0, 0, 0, 0, 0, 0, 0, 0};
        if (q == 0) {
            x[0] = (_Float16)g0;
            x[1] = (_Float16)g1;
            x[2] = (_Float16)g2;
            x[3] = (_Float16)1.0f;
        }
        h8 h1[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const f4 z0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(F.w1[2 * s][l], x, f4{0, 0, 0, 0}, 0, 0, 0);
            const f4 z1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(F.w1[2 * s + 1][l], x, f4{0, 0, 0, 0}, 0, 0, 0);
            h1[s] = act_pack(z0, z1);
        }
        f4 z2[4];
#pragma unroll
        for (int I = 0; I < 4; ++I) {
            f4 acc = F.b2[I][l];
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(F.w2[I][0][l], h1[0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(F.w2[I][1][l], h1[1], acc, 0, 0, 0);
            z2[I] = acc;
        }
        h8 hb[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) hb[s] = act_pack(z2[2 * s], z2[2 * s + 1]);
        f4 o = {F.b3, F.b3, F.b3, F.b3};
        o = __builtin_amdgcn_mfma_f32_16x16x32_f16(F.w3[0][l], hb[0], o, 0, 0, 0);
        o = __builtin_amdgcn_mfma_f32_16x16x32_f16(F.w3[1][l], hb[1], o, 0, 0, 0);
        // row 0 of the output tile sits in register 0 of lanes 0..15
        const float oj = __shfl(o[0], l & 15, 64);
        if ((l >> 4) == J) out = oj;
    }
    return out;
}

// Surrogate quantile for one draw (all 64 lanes must call it together).
// Subtract a region's calibrated mean error, keeping x inside [0, 1].
__host__ __device__ inline float sur_debias(float x, float bias)
{
    return fminf(fmaxf(x - bias, 0.0f), 1.0f);
}

__device__ inline float sur_quantile64(const MlpFrag& F, const SurEntry& S, float v)
{
    const float o = mlp_forward64(F, S.f0, S.f1, v * (1.0f / 3.0f));
    const float lg = S.m + S.s * v + o;
    return 1.0f / (1.0f + expf(-lg));
}

}  // namespace ara
