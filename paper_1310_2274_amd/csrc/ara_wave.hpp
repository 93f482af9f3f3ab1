// ara_wave.hpp -- 64-lane wavefront helpers shared by the layer kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "ara_internal.hpp"

namespace ara {

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// inclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// (hi, lo) compensated pair: error-free sum of the high parts, low parts added
__device__ __forceinline__ void two_sum_merge(float& hi, float& lo, float ohi, float olo)
{
    const float s = hi + ohi;
    const float bb = s - hi;
    const float err = (hi - (s - bb)) + (ohi - bb);
    hi = s;
    lo = (lo + olo) + err;
}

__device__ __forceinline__ void neumaier_add(float& s, float& c, float x)
{
    const float t = s + x;
    if (fabsf(s) >= fabsf(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

// Sum of (hi, lo) over the wave; every lane ends with the same pair.
__device__ __forceinline__ void wave_sum_pair(float& hi, float& lo)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const float oh = __shfl_xor(hi, m, 64);
        const float ol = __shfl_xor(lo, m, 64);
        two_sum_merge(hi, lo, oh, ol);
    }
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    return v;
}

__device__ __forceinline__ void trial_range(const YetDev& y, int64_t i, int64_t& row, int32_t& len)
{
    if (y.offs) {
        row = y.offs[i];
        len = (int32_t)(y.offs[i + 1] - row);
    } else {
        row = i * (int64_t)y.K;
        len = y.K;
    }
}

// The layer-table row of event e: direct access, or a probe of the hashed
// table (multiplicative hash, linear probing; at most half the slots are
// taken, so a probe ends at the event's slot or at an empty one).  A slot
// keeps the key beside its row in one 32-byte line, so a probe that finds
// the event costs one line.
__device__ __forceinline__ uint32_t layer_hash(int32_t e, uint32_t bits)
{
    return ((uint32_t)e * 0x9E3779B1u) >> (32u - bits);
}

__device__ __forceinline__ uint4 layer_row(const LayerDev& L, int32_t e)
{
    if (L.hbits == 0u) return L.rows[e];
    const uint32_t m = (1u << L.hbits) - 1u;
    for (uint32_t h = layer_hash(e, L.hbits);; h = (h + 1u) & m) {
        const uint4 a = L.rows[2u * h];
        const uint4 b = L.rows[2u * h + 1u];
        if ((int32_t)a.x == e) return make_uint4(a.y, a.z, a.w, b.x);
        if ((int32_t)a.x < 0) return make_uint4(0u, 0u, 0u, 0u);
    }
}

// Draw z for one (trial, slot, XELT) hit: section 3.1 uniforms, section 3.2
// combination when the entry has a correlated part.
template <bool HAS_CORR>
__device__ __forceinline__ double draw_z(uint32_t trial, uint32_t slot, uint32_t j, uint32_t seed, uint32_t prog,
                                         const float2* pcw, uint32_t pi)
{
    const double ui = (double)u01(philox_word0(trial, slot, j, 0u, seed, prog));
    if (!HAS_CORR || !pcw) return ui;
    const float2 w = pcw[pi];
    if (w.y == 0.0f) return ui;
    const double uc = (double)u01(philox_word0(trial, slot, 0xFFFFFFFFu, 1u, seed, 0xFFFFFFFFu));
    if (w.x == 0.0f) return uc;
    return normcdf((double)w.x * normal_quantile(ui) + (double)w.y * normal_quantile(uc));
}

}  // namespace ara
