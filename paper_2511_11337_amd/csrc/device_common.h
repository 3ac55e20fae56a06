// Device helpers shared by the inference kernels (kernels.hip) and the
// training kernels (train.hip): wave reductions, elementwise functions,
// LayerNorm statistics and bf16 conversion.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

namespace boa {

#define DEVI __device__ __forceinline__

// ============================================================== wave helpers
// All-lane reductions over a full wave (every lane active).  The value is the
// xor butterfly over partner distances 1, 2, 4, 8, 16, 32: after the steps
// for 1 and 2 every lane of a quad holds the quad's result, so the partner at
// distance 4 (8) holds the same value as the lane mirrored within its half
// row (row); the steps for 1, 2, 4, 8 therefore run as DPP moves
// (quad_perm, row_half_mirror, row_mirror) and the last two as reads of
// lanes 0, 16, 32, 48 combined as (r0 + r1) + (r2 + r3) -- the same operands
// in the same order as the butterfly, with no LDS permutes.
template <int CTRL>
DEVI int dpp_i(int v) { return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false); }
template <int CTRL>
DEVI float dpp_f(float v) { return __int_as_float(dpp_i<CTRL>(__float_as_int(v))); }
constexpr int DPP_XOR1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;
DEVI float lane_f(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }

DEVI float wave_sum(float v) {
    v = v + dpp_f<DPP_XOR1>(v);
    v = v + dpp_f<DPP_XOR2>(v);
    v = v + dpp_f<DPP_HALF_MIRROR>(v);
    v = v + dpp_f<DPP_MIRROR>(v);
    return (lane_f(v, 0) + lane_f(v, 16)) + (lane_f(v, 32) + lane_f(v, 48));
}
DEVI float wave_max(float v) {
    v = fmaxf(v, dpp_f<DPP_XOR1>(v));
    v = fmaxf(v, dpp_f<DPP_XOR2>(v));
    v = fmaxf(v, dpp_f<DPP_HALF_MIRROR>(v));
    v = fmaxf(v, dpp_f<DPP_MIRROR>(v));
    return fmaxf(fmaxf(lane_f(v, 0), lane_f(v, 16)), fmaxf(lane_f(v, 32), lane_f(v, 48)));
}
DEVI int wave_sum_i(int v) {
    v = v + dpp_i<DPP_XOR1>(v);
    v = v + dpp_i<DPP_XOR2>(v);
    v = v + dpp_i<DPP_HALF_MIRROR>(v);
    v = v + dpp_i<DPP_MIRROR>(v);
    return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
           (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}
// (value, index) maximum over the wave: largest value, lowest index on ties
// (a total order, so the grouping of the comparisons does not matter)
DEVI void argmax_step(int& bv, int& bi, int ov, int oi) {
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
}
DEVI void wave_argmax_i(int& bv, int& bi) {
    argmax_step(bv, bi, dpp_i<DPP_XOR1>(bv), dpp_i<DPP_XOR1>(bi));
    argmax_step(bv, bi, dpp_i<DPP_XOR2>(bv), dpp_i<DPP_XOR2>(bi));
    argmax_step(bv, bi, dpp_i<DPP_HALF_MIRROR>(bv), dpp_i<DPP_HALF_MIRROR>(bi));
    argmax_step(bv, bi, dpp_i<DPP_MIRROR>(bv), dpp_i<DPP_MIRROR>(bi));
    int v = __builtin_amdgcn_readlane(bv, 0), i = __builtin_amdgcn_readlane(bi, 0);
    argmax_step(v, i, __builtin_amdgcn_readlane(bv, 16), __builtin_amdgcn_readlane(bi, 16));
    argmax_step(v, i, __builtin_amdgcn_readlane(bv, 32), __builtin_amdgcn_readlane(bi, 32));
    argmax_step(v, i, __builtin_amdgcn_readlane(bv, 48), __builtin_amdgcn_readlane(bi, 48));
    bv = v;
    bi = i;
}
// inclusive prefix sum over the 64 lanes (integers: exact, so the grouping
// does not matter): Hillis-Steele within each row of 16 lanes by DPP row
// shifts 1, 2, 4, 8 (lanes shifted in from outside the row add 0), then the
// row totals by row_bcast:15 (lane 15 of rows 0, 2 into rows 1, 3) and
// row_bcast:31 (lane 31 into rows 2, 3); no LDS permutes
template <int CTRL, int ROWS>
DEVI int dpp_add_src(int v) { return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false); }
DEVI int wave_incl_scan_i(int v, int) {
    v += dpp_add_src<0x111, 0xF>(v);
    v += dpp_add_src<0x112, 0xF>(v);
    v += dpp_add_src<0x114, 0xF>(v);
    v += dpp_add_src<0x118, 0xF>(v);
    v += dpp_add_src<0x142, 0xA>(v);
    v += dpp_add_src<0x143, 0xC>(v);
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
DEVI uint16_t f2bf_bits(float v) {   // bfloat16 bits of v, rounded to nearest even
    __hip_bfloat16 b = __float2bfloat16(v);
    return *reinterpret_cast<uint16_t*>(&b);
}

// MFMA operand and accumulator vectors
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));


}  // namespace boa
