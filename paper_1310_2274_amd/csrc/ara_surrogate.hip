// ara_surrogate.hip -- the sampling surrogate on gfx950: training-tuple
// generation labelled by the plain inverse, MFMA forward/backward with Adam,
// the per-region error table that decides fallback to the exact inverse, and
// the layer kernel that samples with the network.
#include "ara_internal.hpp"
#include "ara_mlp.hpp"
#include "ara_wave.hpp"
#include "ara_surrogate.hpp"

namespace ara {

// ===========================================================================
// Training tuples: (a, b) log-uniform on [0.2, 50]^2; u on the 2^-24 grid,
// even tuples uniform, odd tuples logit-uniform (tail emphasis); label x =
// the plain inverse Beta (FP32 Newton + FP64 polish).
// Tuple layout: f0, f1, f2, base, x (5 floats).
// ===========================================================================
__global__ void k_tuplegen(int64_t n, uint32_t seed, float* __restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t ci = (uint32_t)i, ch = (uint32_t)(i >> 32);
    const uint32_t w0 = philox_word0(ci, ch, 0u, 2u, seed, 0xA5A5A5A5u);
    const uint32_t w1 = philox_word0(ci, ch, 1u, 2u, seed, 0xA5A5A5A5u);
    const uint32_t w2 = philox_word0(ci, ch, 2u, 2u, seed, 0xA5A5A5A5u);
    const double lo = log((double)kSurLo), hi = log((double)kSurHi);
    const double a = exp(lo + (hi - lo) * (double)u01(w0));
    const double b = exp(lo + (hi - lo) * (double)u01(w1));
    double u;
    if ((i & 1) == 0) {
        u = (double)u01(w2);
    } else {
        const double L = -16.6 + 33.2 * (double)u01(w2);
        const double p = 1.0 / (1.0 + exp(-L));
        double k = floor(p * 8388608.0);
        k = fmin(fmax(k, 0.0), 8388607.0);
        u = (2.0 * k + 1.0) * 0x1p-24;
    }
    EntryRec E;
    E.a = a;
    E.b = b;
    E.lnB = log_beta(a, b);
    E.us = (float)beta_inc_lower((a + 1.0) / (a + b + 2.0), a, b, E.lnB);
    E.maxl = 1.0f;
    const double x = inv_beta(u, E);
    const SurEntry S = sur_entry(a, b);
    const float v = (float)normcdfinv(u);
    float* o = out + i * 5;
    o[0] = S.f0;
    o[1] = S.f1;
    o[2] = v * (1.0f / 3.0f);
    o[3] = S.m + S.s * v;
    o[4] = (float)x;
}

// ===========================================================================
// Training step, one wave per 64 tuples (rows of a batch).  Layers are
// evaluated transposed (hidden x draws) with MFMA on FP16 operands held in
// LDS; the backward pass forms dW2 = dZ2 H1^T and dH1 = W2^T dZ2 with MFMA,
// the rank-3 and rank-1 pieces on the VALU.  Each wave writes its partial
// gradient (kNumParams floats) and partial loss.
// ===========================================================================
template <typename TA, typename TB, int NT, int K>
__device__ inline void lds_gemm(const TA* As, int am, int ak, const TB* Bs, int bk, int bn, f4 (&C)[4][NT])
{
    const int l = threadIdx.x & 63, q = l >> 4, i = l & 15;
    for (int ks = 0; ks < K / 32; ++ks) {
        h8 b[NT];
        for (int J = 0; J < NT; ++J)
            for (int t = 0; t < 8; ++t) b[J][t] = (_Float16)Bs[(ks * 32 + 8 * q + t) * bk + (16 * J + i) * bn];
        for (int I = 0; I < 4; ++I) {
            h8 a;
            for (int t = 0; t < 8; ++t) a[t] = (_Float16)As[(16 * I + i) * am + (ks * 32 + 8 * q + t) * ak];
            for (int J = 0; J < NT; ++J) C[I][J] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b[J], C[I][J], 0, 0, 0);
        }
    }
}

struct TrainLds {
    _Float16 X[32 * 64];      // [k][d]: features, ones row, zeros
    _Float16 W1[64 * 32];     // [h][k]
    _Float16 W2[64 * 64];     // [h'][h]
    float Z1[64 * 64];        // [h][d], later dZ1
    _Float16 H1[64 * 64];
    float Z2[64 * 64];        // [h][d], later dZ2
    _Float16 H2[64 * 64];
    float w3[64];
    float dout[64];
};

__global__ __launch_bounds__(64) void k_train_fwd_bwd(const float* __restrict__ tuples, int64_t n_tuples,
                                                     int64_t perm_a, int64_t perm_c, int64_t row0, int32_t batch,
                                                     const float* __restrict__ P, float* __restrict__ gpart,
                                                     float* __restrict__ lpart)
{
    __shared__ TrainLds S;
    const int l = threadIdx.x;
    const int q = l >> 4, i16 = l & 15;
    // ---- operands
    for (int e = l; e < 64 * 32; e += 64) {
        const int h = e / 32, k = e % 32;
        float w = 0.0f;
        if (k < 3) w = P[kOffW1 + h * 3 + k];
        else if (k == 3) w = P[kOffB1 + h];
        S.W1[e] = bf16_round_to_h(w);
    }
    for (int e = l; e < 64 * 64; e += 64) S.W2[e] = bf16_round_to_h(P[kOffW2 + e]);
    S.w3[l] = (float)bf16_round_to_h(P[kOffW3 + l]);
    const float b3 = (float)bf16_round_to_h(P[kOffB3]);
    // this lane's tuple: row r of the epoch permutation
    const int64_t r = row0 + (int64_t)blockIdx.x * 64 + l;
    const int64_t idx = (int64_t)(((uint64_t)r * (uint64_t)perm_a + (uint64_t)perm_c) % (uint64_t)n_tuples);
    const float* T = tuples + idx * 5;
    const float f0 = T[0], f1 = T[1], f2 = T[2], base = T[3], xt = T[4];
    for (int k = 0; k < 32; ++k) {
        float v = 0.0f;
        if (k == 0) v = f0;
        else if (k == 1) v = f1;
        else if (k == 2) v = f2;
        else if (k == 3) v = 1.0f;
        S.X[k * 64 + l] = (_Float16)v;
    }
    __syncthreads();
    // ---- forward
    {
        f4 C[4][4];
        for (int I = 0; I < 4; ++I)
            for (int J = 0; J < 4; ++J) C[I][J] = f4{0, 0, 0, 0};
        lds_gemm<_Float16, _Float16, 4, 32>(S.W1, 32, 1, S.X, 64, 1, C);
        for (int I = 0; I < 4; ++I)
            for (int J = 0; J < 4; ++J)
                for (int rr = 0; rr < 4; ++rr) {
                    const int h = 16 * I + 4 * q + rr, d = 16 * J + i16;
                    S.Z1[h * 64 + d] = C[I][J][rr];
                    S.H1[h * 64 + d] = (_Float16)gelu_s(C[I][J][rr]);
                }
    }
    __syncthreads();
    {
        f4 C[4][4];
        for (int I = 0; I < 4; ++I) {
            f4 bb;
            for (int rr = 0; rr < 4; ++rr) bb[rr] = (float)bf16_round_to_h(P[kOffB2 + 16 * I + 4 * q + rr]);
            for (int J = 0; J < 4; ++J) C[I][J] = bb;
        }
        lds_gemm<_Float16, _Float16, 4, 64>(S.W2, 64, 1, S.H1, 64, 1, C);
        for (int I = 0; I < 4; ++I)
            for (int J = 0; J < 4; ++J)
                for (int rr = 0; rr < 4; ++rr) {
                    const int h = 16 * I + 4 * q + rr, d = 16 * J + i16;
                    S.Z2[h * 64 + d] = C[I][J][rr];
                    S.H2[h * 64 + d] = (_Float16)gelu_s(C[I][J][rr]);
                }
    }
    __syncthreads();
    // output, loss and dL/do for draw l
    float o = b3;
    for (int h = 0; h < 64; ++h) o += S.w3[h] * (float)S.H2[h * 64 + l];
    const float xh = 1.0f / (1.0f + expf(-(base + o)));
    const float err = xh - xt;
    // backward values carry a factor kLossScale (FP16 MFMA operands would
    // underflow otherwise); partial gradients divide it out with the batch
    constexpr float kLossScale = 1024.0f;
    const float dout = 2.0f * err * xh * (1.0f - xh) * kLossScale;
    const float inv = 1.0f / (kLossScale * (float)batch);
    S.dout[l] = dout;
    // partial loss (sum of squared errors)
    float se = err * err;
    for (int m = 32; m >= 1; m >>= 1) se += __shfl_xor(se, m, 64);
    if (l == 0) lpart[blockIdx.x] = se;
    __syncthreads();
    // dZ2 = w3 dout g'(Z2), in place of Z2 (lane = draw column)
    for (int h = 0; h < 64; ++h) {
        const float z = S.Z2[h * 64 + l];
        S.Z2[h * 64 + l] = S.w3[h] * dout * gelu_s_grad(z);
    }
    __syncthreads();
    float* G = gpart + (int64_t)blockIdx.x * kNumParams;
    // dw3, db2 (lane = hidden unit), db3
    {
        float a3 = 0.0f, a2 = 0.0f;
        for (int d = 0; d < 64; ++d) {
            a3 += (float)S.H2[l * 64 + d] * S.dout[d];
            a2 += S.Z2[l * 64 + d];
        }
        G[kOffW3 + l] = a3 * inv;
        G[kOffB2 + l] = a2 * inv;
        float s3 = dout;
        for (int m = 32; m >= 1; m >>= 1) s3 += __shfl_xor(s3, m, 64);
        if (l == 0) G[kOffB3] = s3 * inv;
    }
    // dW2 = dZ2 (h' x d) . H1^T (d x h)
    {
        f4 C[4][4];
        for (int I = 0; I < 4; ++I)
            for (int J = 0; J < 4; ++J) C[I][J] = f4{0, 0, 0, 0};
        lds_gemm<float, _Float16, 4, 64>(S.Z2, 64, 1, S.H1, 1, 64, C);
        for (int I = 0; I < 4; ++I)
            for (int J = 0; J < 4; ++J)
                for (int rr = 0; rr < 4; ++rr) G[kOffW2 + (16 * I + 4 * q + rr) * 64 + 16 * J + i16] = C[I][J][rr] * inv;
    }
    // dH1 = W2^T (h x h') . dZ2 (h' x d);  dZ1 = dH1 g'(Z1), in place of Z1
    {
        f4 C[4][4];
        for (int I = 0; I < 4; ++I)
            for (int J = 0; J < 4; ++J) C[I][J] = f4{0, 0, 0, 0};
        lds_gemm<_Float16, float, 4, 64>(S.W2, 1, 64, S.Z2, 64, 1, C);
        __syncthreads();
        for (int I = 0; I < 4; ++I)
            for (int J = 0; J < 4; ++J)
                for (int rr = 0; rr < 4; ++rr) {
                    const int h = 16 * I + 4 * q + rr, d = 16 * J + i16;
                    S.Z1[h * 64 + d] = C[I][J][rr] * gelu_s_grad(S.Z1[h * 64 + d]);
                }
    }
    __syncthreads();
    // dW1, db1 (lane = hidden unit): rank-3 plus bias, on the VALU
    {
        float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, gb = 0.0f;
        for (int d = 0; d < 64; ++d) {
            const float dz = S.Z1[l * 64 + d];
            g0 += dz * (float)S.X[0 * 64 + d];
            g1 += dz * (float)S.X[1 * 64 + d];
            g2 += dz * (float)S.X[2 * 64 + d];
            gb += dz;
        }
        G[kOffW1 + l * 3 + 0] = g0 * inv;
        G[kOffW1 + l * 3 + 1] = g1 * inv;
        G[kOffW1 + l * 3 + 2] = g2 * inv;
        G[kOffB1 + l] = gb * inv;
    }
}

// Sum of the per-wave partial gradients, in wave order (deterministic).
__global__ void k_grad_reduce(const float* __restrict__ gpart, int32_t nparts, float* __restrict__ grad,
                              const float* __restrict__ lpart, float* __restrict__ loss_acc)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNumParams) {
        float s = 0.0f;
        for (int b = 0; b < nparts; ++b) s += gpart[(int64_t)b * kNumParams + p];
        grad[p] = s;
    }
    if (p == 0) {
        double s = 0.0;
        for (int b = 0; b < nparts; ++b) s += (double)lpart[b];
        loss_acc[0] += (float)s;
    }
}

__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNumParams) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    P[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_init_params(float* __restrict__ P, uint32_t seed)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNumParams) return;
    const float u = 2.0f * u01(philox_word0((uint32_t)p, 0u, 0u, 3u, seed, 0x5EED5EEDu)) - 1.0f;
    float w = 0.0f;
    if (p < kOffB1) w = u * sqrtf(6.0f / (3.0f + 64.0f));
    else if (p >= kOffW2 && p < kOffB2) w = u * sqrtf(6.0f / 128.0f);
    else if (p >= kOffW3 && p < kOffB3) w = 0.1f * u * sqrtf(6.0f / 65.0f);
    P[p] = w;
}

__global__ void k_build_frag(const float* __restrict__ P, MlpFrag* __restrict__ F)
{
    mlp_build_frag_lane(P, *F, threadIdx.x);
}

// ===========================================================================
// Inference for arbitrary (a, b, u): calibration of the region table and the
// evaluation entry point share it.  Cell statistics: count, sum of errors in
// fixed point (kCalibScale units; integer sums do not depend on the order of
// the atomic adds, so the table is reproducible), max |error| (as float bits:
// non-negative floats order like integers).
// ===========================================================================
__device__ inline void copy_frag_to_lds(const MlpFrag* __restrict__ Fg, MlpFrag& Fs)
{
    const uint32_t* src = reinterpret_cast<const uint32_t*>(Fg);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&Fs);
    for (int w = threadIdx.x; w < (int)(sizeof(MlpFrag) / 4); w += blockDim.x) dst[w] = src[w];
}

__global__ __launch_bounds__(256) void k_sur_calib(const float* __restrict__ tuples, int64_t n,
                                                   const MlpFrag* __restrict__ Fg, const float* __restrict__ bias,
                                                   unsigned int* __restrict__ cnt,
                                                   unsigned long long* __restrict__ sum,
                                                   unsigned int* __restrict__ maxbits)
{
    __shared__ MlpFrag F;
    copy_frag_to_lds(Fg, F);
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool ok = i < n;
    const float* T = tuples + (ok ? i : 0) * 5;
    const float f0 = T[0], f1 = T[1], f2 = T[2], base = T[3], xt = T[4];
    const float o = mlp_forward64(F, f0, f1, f2);
    if (!ok) return;
    const int c = sur_cell(f0, f1, 3.0f * f2);
    const float xh = sur_debias(1.0f / (1.0f + expf(-(base + o))), bias ? bias[c] : 0.0f);
    const float e = xh - xt;
    atomicAdd(&cnt[c], 1u);
    atomicAdd(&sum[c], (unsigned long long)llrint((double)e * kCalibScale));   // two's complement sum
    atomicMax(&maxbits[c], __float_as_uint(fabsf(e)));
}

// x = surrogate quantile where (a, b) lies in the domain and the region is not
// marked for fallback, else the plain inverse.
__global__ __launch_bounds__(256) void k_sur_eval(const double* __restrict__ a, const double* __restrict__ b,
                                                  const double* __restrict__ u, int64_t n,
                                                  const MlpFrag* __restrict__ Fg, const uint32_t* __restrict__ mask,
                                                  const float* __restrict__ bias, double* __restrict__ x,
                                                  int32_t* __restrict__ used)
{
    __shared__ MlpFrag F;
    copy_frag_to_lds(Fg, F);
    __syncthreads();
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool ok = i < n;
    const double ai = ok ? a[i] : 1.0, bi = ok ? b[i] : 1.0, ui = ok ? u[i] : 0.5;
    const SurEntry S = sur_entry(ai, bi);
    const float v = (float)normcdfinv(ui);
    const int c = sur_cell(S.f0, S.f1, v);
    const bool sur = sur_in_domain(ai, bi) && !((mask[c >> 5] >> (c & 31)) & 1u);
    const float xs = sur_debias(sur_quantile64(F, S, v), bias[c]);
    if (!ok) return;
    if (sur) {
        x[i] = (double)xs;
    } else {
        EntryRec E;
        E.a = ai;
        E.b = bi;
        E.lnB = log_beta(ai, bi);
        E.us = (float)beta_inc_lower((ai + 1.0) / (ai + bi + 2.0), ai, bi, E.lnB);
        E.maxl = 1.0f;
        x[i] = inv_beta(ui, E);
    }
    used[i] = sur ? 1 : 0;
}

// Per packed entry of a layer: the surrogate's features and base.
__global__ void k_sur_entries(const EntryRec* __restrict__ pent, int64_t n, SurEntry* __restrict__ psur)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const EntryRec E = pent[i];
    SurEntry S;
    if (E.a > 0.0 && sur_in_domain(E.a, E.b)) {
        S = sur_entry(E.a, E.b);
    } else {
        S.f0 = -INFINITY;      // outside the trained domain: always the exact inverse
        S.f1 = 0.0f;
        S.m = 0.0f;
        S.s = 0.0f;
    }
    psur[i] = S;
}

// ===========================================================================
// Layer kernel, surrogate mode.  As the plain kernel, with each drain round
// split in passes over the queued draws: (A) draw u, decide
// surrogate-or-exact from the entry's domain and the error table, and
// compact the draws into three lists -- surrogate, exact FP32 solve, exact
// FP32 + FP64 polish; (B) evaluate the surrogate 64 draws at a time on the
// matrix cores and subtract the region's calibrated bias; (C) run the exact
// inverse on the rest, each cost class in waves of its own.  Every draw's net
// loss lands at its queue position, so the per-event sums keep the XELT order
// and the result stays a function of the trial.
// ===========================================================================
// The exact inverse for the draws the surrogate does not answer, out of line
// so its registers stay out of the MLP kernel's allocation.
static __device__ __attribute__((noinline)) float exact_loss32(float code, EntryRec E)
{
    return E.maxl * inv_beta32_code(code, E);
}
static __device__ __attribute__((noinline)) float exact_loss64(double z, EntryRec E)
{
    return sample_loss(z, E);
}
// z of a draw; the correlated form (two normal quantiles and a CDF in FP64) out of line.
static __device__ __attribute__((noinline)) double corr_draw_z(uint32_t trial, uint32_t slot, uint32_t j,
                                                               uint32_t seed, uint32_t prog, const float2* pcw,
                                                               uint32_t pi)
{
    return draw_z<true>(trial, slot, j, seed, prog, pcw, pi);
}
template <bool HAS_CORR>
__device__ __forceinline__ double sur_draw_z(uint32_t trial, uint32_t slot, uint32_t j, uint32_t seed, uint32_t prog,
                                             const float2* pcw, uint32_t pi)
{
    return HAS_CORR ? corr_draw_z(trial, slot, j, seed, prog, pcw, pi)
                    : draw_z<false>(trial, slot, j, seed, prog, nullptr, pi);
}

constexpr int kSurRound = 8;
constexpr int kSurQueue = 64 * kSurRound;

template <bool HAS_CORR, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_layer_surrogate(YetDev y, int64_t t0, int64_t t1,
                                                              const LayerDev* __restrict__ layers, int32_t n_layers,
                                                              const MlpFrag* __restrict__ Fg,
                                                              const uint32_t* __restrict__ gmask,
                                                              const float* __restrict__ gbias)
{
    __shared__ MlpFrag F;
    __shared__ uint32_t mask[kCells / 32];
    __shared__ uint32_t qidx[WPB][kSurQueue];
    __shared__ uint32_t qmeta[WPB][kSurQueue];
    __shared__ float qv[WPB][kSurQueue];
    __shared__ uint16_t lst[WPB][3][kSurQueue];
    copy_frag_to_lds(Fg, F);
    for (int w = threadIdx.x; w < kCells / 32; w += blockDim.x) mask[w] = gmask[w];
    __syncthreads();
    const float* __restrict__ bias = gbias;     // 16 KB, read through the L1 cache
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const int64_t trial = t0 + (int64_t)blockIdx.x * WPB + w;
    // waves past the end take part in no block-wide barrier below
    if (trial >= t1) return;
    uint32_t* QI = qidx[w];
    uint32_t* QM = qmeta[w];
    float* QV = qv[w];
    uint16_t* LS = lst[w][0];
    uint16_t* LF = lst[w][1];        // exact, FP32 solve alone
    uint16_t* LP = lst[w][2];        // exact, FP32 solve + FP64 polish (and degenerate entries)
    int64_t row;
    int32_t len;
    trial_range(y, trial, row, len);
    const uint32_t tr = (uint32_t)trial;
    const float flo = 0.5f * logf(kSurLo), fhi = 0.5f * logf(kSurHi);

    for (int32_t l = 0; l < n_layers; ++l) {
        const LayerDev& L = layers[l];
        float S = 0.0f, Sc = 0.0f, omax = 0.0f;
        for (int32_t base = 0; base < len; base += 64) {
            const int32_t k = base + lane;
            const bool valid = k < len;
            uint4 r = make_uint4(0, 0, 0, 0);
            if (valid) r = layer_row(L, y.ev[row + k]);
            uint64_t msk = (uint64_t)r.x | ((uint64_t)r.y << 32);
            const uint32_t off = r.z;
            int remaining = row_count(r.w);
            int rank = 0;
            float c = 0.0f;
            while (true) {
                const int take = remaining < kSurRound ? remaining : kSurRound;
                const int incl = wave_incl_scan(take);
                const int total = __builtin_amdgcn_readlane(incl, 63);     // wave-uniform (scalar)
                if (total == 0) break;
                const int pos = incl - take;
                for (int i = 0; i < take; ++i) {
                    const int j = __ffsll((unsigned long long)msk) - 1;
                    msk &= msk - 1;
                    QI[pos + i] = off + (uint32_t)(rank + i);
                    QM[pos + i] = (uint32_t)lane | ((uint32_t)j << 8);
                }
                wave_sync();
                // (A) classify
                int ns = 0, nf = 0, np = 0;
                for (int b0 = 0; b0 < total; b0 += 64) {
                    const int q = b0 + lane;
                    const bool in = q < total;
                    bool is_sur = false, pol = false, keep = in;
                    if (in) {
                        const uint32_t pi = QI[q], meta = QM[q];
                        const uint32_t slot = (uint32_t)base + (meta & 63u), j = meta >> 8;
                        const double z = sur_draw_z<HAS_CORR>(tr, slot, j, L.seed, L.prog, L.pcw, pi);
                        // a draw whose XELT term the quantile cannot change takes it here
                        // (term_thresholds): no network and no exact inverse
                        const TermThr th = L.pthr[pi];
                        const SurEntry SE = L.psur[pi];
                        if (z <= (double)thr_lo(th)) {
                            QV[q] = 0.0f;
                            keep = false;
                        } else if (z >= (double)thr_hi(th)) {
                            const float4 jt = L.jt[j];
                            QV[q] = jt.z * jt.y;
                            keep = false;
                        } else if (SE.f0 >= flo && SE.f0 <= fhi && SE.f1 >= flo && SE.f1 <= fhi) {
                            // Phi^-1 of the draw from its tail code (1 - z formed in FP64 for correlated draws)
                            const float zc = tail_code(z);
                            const float v = zc > 0.0f ? normcdfinvf(zc) : -normcdfinvf(-zc);
                            const int cell = sur_cell(SE.f0, SE.f1, v);
                            is_sur = !((mask[cell >> 5] >> (cell & 31)) & 1u);
                            QV[q] = v;
                        } else {
                            const EntryRec& E = L.pent[pi];
                            pol = fmin(E.a, E.b) < kPolishShapeEntry;
                        }
                    }
                    const uint64_t bs = __ballot(keep && is_sur);
                    const uint64_t bf = __ballot(keep && !is_sur && !pol);
                    const uint64_t bp = __ballot(keep && pol);
                    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
                    if (keep) {
                        if (is_sur) LS[ns + __popcll(bs & below)] = (uint16_t)q;
                        else if (pol) LP[np + __popcll(bp & below)] = (uint16_t)q;
                        else LF[nf + __popcll(bf & below)] = (uint16_t)q;
                    }
                    ns += __popcll(bs);
                    nf += __popcll(bf);
                    np += __popcll(bp);
                }
                wave_sync();
                // (B) surrogate, 64 draws per MLP evaluation
                for (int b0 = 0; b0 < ns; b0 += 64) {
                    const int idx = b0 + lane;
                    const bool act = idx < ns;
                    const int q = LS[act ? idx : b0];
                    const uint32_t pi = QI[q], meta = QM[q];
                    const SurEntry SE = L.psur[pi];
                    const float v = QV[q];
                    const float xs = sur_quantile64(F, SE, v);
                    if (act) {
                        const uint32_t j = meta >> 8;
                        const float loss = L.pent[pi].maxl * sur_debias(xs, bias[sur_cell(SE.f0, SE.f1, v)]);
                        const float4 jt = L.jt[j];
                        QV[q] = jt.z * xl(loss, jt.x, jt.y);
                    }
                }
                // (C) the exact inverse for the rest: FP32 solve alone ...
                for (int b0 = 0; b0 < nf; b0 += 64) {
                    const int idx = b0 + lane;
                    if (idx < nf) {
                        const int q = LF[idx];
                        const uint32_t pi = QI[q], meta = QM[q];
                        const uint32_t slot = (uint32_t)base + (meta & 63u), j = meta >> 8;
                        const EntryRec E = L.pent[pi];
                        const double z = sur_draw_z<HAS_CORR>(tr, slot, j, L.seed, L.prog, L.pcw, pi);
                        const float loss = exact_loss32(tail_code(z), E);
                        const float4 jt = L.jt[j];
                        QV[q] = jt.z * xl(loss, jt.x, jt.y);
                    }
                }
                // ... and with the FP64 polish for small shapes and degenerate entries
                for (int b0 = 0; b0 < np; b0 += 64) {
                    const int idx = b0 + lane;
                    if (idx < np) {
                        const int q = LP[idx];
                        const uint32_t pi = QI[q], meta = QM[q];
                        const uint32_t slot = (uint32_t)base + (meta & 63u), j = meta >> 8;
                        const EntryRec E = L.pent[pi];
                        const double z = sur_draw_z<HAS_CORR>(tr, slot, j, L.seed, L.prog, L.pcw, pi);
                        const float loss = exact_loss64(z, E);
                        const float4 jt = L.jt[j];
                        QV[q] = jt.z * xl(loss, jt.x, jt.y);
                    }
                }
                wave_sync();
                for (int i = 0; i < take; ++i) c += QV[pos + i];
                rank += take;
                remaining -= take;
                wave_sync();
            }
            if (valid) {
                const float o = xl(c, L.occR, L.occL);
                omax = fmaxf(omax, o);
                neumaier_add(S, Sc, o);
                if (L.yelt) L.yelt[row + k - L.yelt_base] = o;
            }
        }
        wave_sum_pair(S, Sc);
        omax = wave_max(omax);
        if (lane == 0) {
            L.ylt[trial - t0] = fminf(fmaxf((S - L.aggR) + Sc, 0.0f), L.aggL);
            if (L.omax) L.omax[trial - t0] = omax;
        }
    }
}

// ===========================================================================
// Launchers
// ===========================================================================
static inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_sur_entries(const EntryRec* pent, int64_t n, SurEntry* psur, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_sur_entries, dim3(grid_for(n, 256)), dim3(256), 0, s, pent, n, psur);
    return hipGetLastError();
}

template <int WPB>
static void launch_sur_wpb(bool has_corr, const YetDev& y, int64_t t0, int64_t t1, const LayerDev* layers,
                           int32_t n_layers, const MlpFrag* frag, const uint32_t* cellmask, const float* bias,
                           hipStream_t s)
{
    const dim3 grid(grid_for(t1 - t0, WPB)), block(64 * WPB);
    if (has_corr)
        hipLaunchKernelGGL((k_layer_surrogate<true, WPB>), grid, block, 0, s, y, t0, t1, layers, n_layers, frag, cellmask,
                           bias);
    else
        hipLaunchKernelGGL((k_layer_surrogate<false, WPB>), grid, block, 0, s, y, t0, t1, layers, n_layers, frag,
                           cellmask, bias);
}

hipError_t launch_layers_surrogate(bool has_corr, const YetDev& y, int64_t t0, int64_t t1, const LayerDev* layers,
                                   int32_t n_layers, const MlpFrag* frag, const uint32_t* cellmask,
                                   const float* bias, int32_t wpb, hipStream_t s)
{
    if (t1 - t0 <= 0 || n_layers <= 0) return hipSuccess;
    switch (wpb) {
        case 1: launch_sur_wpb<1>(has_corr, y, t0, t1, layers, n_layers, frag, cellmask, bias, s); break;
        case 2: launch_sur_wpb<2>(has_corr, y, t0, t1, layers, n_layers, frag, cellmask, bias, s); break;
        default: launch_sur_wpb<4>(has_corr, y, t0, t1, layers, n_layers, frag, cellmask, bias, s); break;
    }
    return hipGetLastError();
}

hipError_t sur_launch_tuplegen(int64_t n, uint32_t seed, float* out, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_tuplegen, dim3(grid_for(n, 128)), dim3(128), 0, s, n, seed, out);
    return hipGetLastError();
}

hipError_t sur_launch_init(float* P, uint32_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_params, dim3(grid_for(kNumParams, 256)), dim3(256), 0, s, P, seed);
    return hipGetLastError();
}

hipError_t sur_launch_train_step(const float* tuples, int64_t n_tuples, int64_t pa, int64_t pc, int64_t row0,
                                 int32_t batch, float* P, float* m, float* v, float* gpart, float* lpart, float* grad,
                                 float* loss_acc, float lr, int64_t step, bool update, hipStream_t s)
{
    const int nw = batch / 64;
    hipLaunchKernelGGL(k_train_fwd_bwd, dim3(nw), dim3(64), 0, s, tuples, n_tuples, pa, pc, row0, batch,
                       (const float*)P, gpart, lpart);
    hipLaunchKernelGGL(k_grad_reduce, dim3(grid_for(kNumParams, 256)), dim3(256), 0, s, (const float*)gpart, nw, grad,
                       (const float*)lpart, loss_acc);
    if (update) {
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
        hipLaunchKernelGGL(k_adam, dim3(grid_for(kNumParams, 256)), dim3(256), 0, s, P, m, v, (const float*)grad, lr, b1,
                           b2, 1e-8f, c1, c2);
    }
    return hipGetLastError();
}

hipError_t sur_launch_build_frag(const float* P, MlpFrag* F, hipStream_t s)
{
    hipLaunchKernelGGL(k_build_frag, dim3(1), dim3(64), 0, s, P, F);
    return hipGetLastError();
}

hipError_t sur_launch_calib(const float* tuples, int64_t n, const MlpFrag* F, const float* bias, unsigned int* cnt,
                            unsigned long long* sum, unsigned int* maxbits, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_sur_calib, dim3(grid_for(n, 256)), dim3(256), 0, s, tuples, n, F, bias, cnt, sum, maxbits);
    return hipGetLastError();
}

hipError_t sur_launch_eval(const double* a, const double* b, const double* u, int64_t n, const MlpFrag* F,
                           const uint32_t* mask, const float* bias, double* x, int32_t* used, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(k_sur_eval, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, u, n, F, mask, bias, x, used);
    return hipGetLastError();
}

}  // namespace ara
