// Device helpers shared by the inference kernels (kernels.hip) and the
// training kernels (train.hip): wave reductions, elementwise functions,
// LayerNorm statistics and bf16 conversion.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

namespace boa {

#define DEVI __device__ __forceinline__

// ============================================================== wave helpers
DEVI float wave_sum(float v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}
DEVI float wave_max(float v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    return v;
}
DEVI int wave_sum_i(int v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}
// inclusive prefix sum over the 64 lanes (integers: exact)
DEVI int wave_incl_scan_i(int v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// ============================================================== elementwise
DEVI float silu_f(float v) { return v / (1.0f + expf(-v)); }
DEVI float softplus_f(float v) { return v > 20.0f ? v : log1pf(expf(v)); }
DEVI float exp2_hw(float v) { return __builtin_amdgcn_exp2f(v); }

// LayerNorm statistics of one row of length D, computed by one full wave.
DEVI void ln_stats(const float* __restrict__ row, int D, int lane, float& mu, float& rstd) {
    float s = 0.0f;
    for (int k = lane; k < D; k += 64) s += row[k];
    s = wave_sum(s);
    mu = s / (float)D;
    float q = 0.0f;
    for (int k = lane; k < D; k += 64) {
        float c = row[k] - mu;
        q = fmaf(c, c, q);
    }
    q = wave_sum(q);
    rstd = 1.0f / sqrtf(q / (float)D + 1e-5f);
}
// The same statistics from values already in registers: v[j] = row[lane + 64 j]
// for j < NV = D / 64 (identical operations and order to ln_stats).
template <int NV>
DEVI void ln_stats_v(const float (&v)[NV], int D, float& mu, float& rstd) {
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < NV; ++j) s += v[j];
    s = wave_sum(s);
    mu = s / (float)D;
    float q = 0.0f;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        float c = v[j] - mu;
        q = fmaf(c, c, q);
    }
    q = wave_sum(q);
    rstd = 1.0f / sqrtf(q / (float)D + 1e-5f);
}
DEVI float ln_apply(float v, float mu, float rstd, float g, float b) {
    return fmaf((v - mu) * rstd, g, b);
}

DEVI float bf16r(float v) {   // round to bfloat16 (nearest-even) and back
    return __bfloat162float(__float2bfloat16(v));
}
DEVI float bf16_bits_to_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }


}  // namespace boa
