// Per-element pieces of the hot path shared by every kernel that evaluates
// them (encoder kernels, decoder step kernels, fused decoder): the schedule
// lookup, MFMA operand types, the Mamba mixer pieces, the histogram / CDF of a
// row and the range coder.  Keeping one definition is what makes encoder and
// decoder build identical integer histograms.
#pragma once
#include "boa_internal.h"
#include "device_common.h"

#include <hip/hip_ext.h>

namespace boa {

// Kernel timing: while a bracket is open on this thread (prof_open), launches
// go through hipExtLaunchKernelGGL, which records the start event when the
// first kernel of the bracket begins and the stop event when the last one
// ends (GPU timestamps, no host gaps).
extern thread_local hipEvent_t t_prof_start, t_prof_stop;
extern thread_local bool t_prof_first;
#define BOA_LAUNCH(kern, grid, block, shmem, stream, ...)                                                   \
    do {                                                                                                  \
        if (t_prof_stop) {                                                                                \
            hipExtLaunchKernelGGL(kern, grid, block, shmem, stream, t_prof_first ? t_prof_start : nullptr,  \
                                  t_prof_stop, 0, __VA_ARGS__);                                            \
            t_prof_first = false;                                                                         \
        } else {                                                                                          \
            hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);                            \
        }                                                                                                 \
    } while (0)

// Row (lane, t) of a time tile runs global step step0 + t of that lane.  The
// lane's entries (chunk, first step) are sorted by first step; the chunk
// occupies chunk_steps = len - 1 steps.  pos = -1 marks an idle row.
DEVI void locate(const Plan& p, int lane, long long s, int& chunk, int& pos) {
    int lo = p.lane_first[lane], n = p.lane_cnt[lane];
    int best = -1;
    int a = 0, b = n - 1;
    while (a <= b) {                       // last entry with start <= s
        int mid = (a + b) >> 1;
        if (p.ent_start[lo + mid] <= s) { best = mid; a = mid + 1; } else b = mid - 1;
    }
    chunk = -1;
    pos = -1;
    if (best < 0) return;
    int c = p.ent_chunk[lo + best];
    long long q = s - p.ent_start[lo + best];
    if (q < p.chunk_steps[c]) { chunk = c; pos = (int)q; }
}



// GELU of the feed-forward sub-layer: u Phi(u) with the standard normal CDF
// Phi(u) = (1 + erf(u / sqrt 2)) / 2, the device library's erff; one fixed
// formula for every kernel that applies it.
DEVI float gelu_f(float u) { return 0.5f * u * (1.0f + erff(u * 0.7071067811865476f)); }


// ---------------------------------------------------------------- FP8 (E4M3) projections
// A tensor (weights) or a row (activations) with largest magnitude amax is
// scaled by 2^-e, e the smallest integer with amax * 2^-e <= 448 (the largest
// finite E4M3 value; 0 when amax is 0), and rounded to E4M3 to nearest even.
// Power-of-two scales make scaling and the final rescale of the FP32
// accumulator exact.
DEVI int fp8_exp(float amax) {
    if (!(amax > 0.0f)) return 0;
    int E;
    const float f = frexpf(amax, &E);          // amax = f * 2^E, f in [0.5, 1)
    return E - 9 + (2.0f * f > 1.75f ? 1 : 0);
}
// eight values (already multiplied by 2^-e) -> eight E4M3 bytes, element j in
// bits 8j .. 8j + 7
DEVI uint64_t fp8_pack8(const float* v) {
    uint32_t lo = 0, hi = 0;
    lo = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], (int)lo, false);
    lo = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], (int)lo, true);
    hi = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[4], v[5], (int)hi, false);
    hi = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[6], v[7], (int)hi, true);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
DEVI uint8_t fp8_byte(float v) { return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false) & 0xFF); }

// ---------------------------------------------------------------- elementwise functions
// Built on the hardware's base-2 transcendentals (v_exp_f32, v_log_f32,
// v_rcp_f32, each about 1 ulp), a few instructions each instead of the
// library's correctly rounded forms (the library log1pf runs in double):
//   exp(x)      = 2^(x log2 e)                  relative error about |x| 2^-24
//   SiLU(v)     = v * (1 / (1 + exp(-v)))
//   softplus(v) = v for v > 20, else log1p(e), e = exp(v), with log1p(e) =
//                 log(u) * (e / (u - 1)) for u = 1 + e != 1 and e for u == 1
//                 (Goldberg's rearrangement: the rounding of u cancels, so the
//                 result keeps the log's few-ulp accuracy for every e > 0).
// Every kernel evaluates these same sequences, which is what the encoder and
// decoder tables depend on; the oracle evaluates the exact functions.
DEVI float exp_hp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
DEVI float rcp_hp(float x) { return __builtin_amdgcn_rcpf(x); }
DEVI float silu_hp(float v) { return v * rcp_hp(1.0f + exp_hp(-v)); }
DEVI float softplus_hp(float v) {
    if (v > 20.0f) return v;
    const float e = exp_hp(v);
    const float u = 1.0f + e;
    if (u == 1.0f) return e;
    return (__builtin_amdgcn_logf(u) * 0.693147180559945309f) * (e * rcp_hp(u - 1.0f));
}

// ---------------------------------------------------------------- mixer pieces
// causal depthwise conv over [x_{t-3}, x_{t-2}, x_{t-1}, x_t] plus bias, then SiLU
DEVI float conv_silu(const float* cw, float cb, float w0, float w1, float w2, float x) {
    float acc = cb;
    acc = fmaf(cw[0], w0, acc);
    acc = fmaf(cw[1], w1, acc);
    acc = fmaf(cw[2], w2, acc);
    acc = fmaf(cw[3], x, acc);
    return silu_hp(acc);
}
// x_proj on the matrix cores, the sequence of every kernel that computes it:
// column fragment f (outputs 16 f .. 16 f + 15) of A [16][Di] . W^T for the
// rows of A (LDS, row stride as; rows from `rows` on read as zero, and each
// output row depends on its own A row only).  Per output, four MFMA f32
// 16x16x4 chains from zero, chain c over the k-groups q = c, c + 4, ...
// (group q: steps j = 0..3 with k = 16 q + 4 j + lane / 16), then
// (c0 + c1) + (c2 + c3): four independent chains keep the matrix core busy
// where one chain would wait on each result.  B comes from the
// fragment-ordered copy (xwF / xwF_r) through a ring of R loads (RD at most, a
// multiple of 4; the depth changes no result).  acc[rr] = output (row
// 4 (lane / 16) + rr, column 16 f + lane % 16).
template <int Di, int RD = 8>
DEVI void xproj_fragment(const float* A, int as, int rows, const float* Wf, int f, int wl, v4f& acc) {
    constexpr int SQ = Di / 16, R = SQ < RD ? SQ : RD;
    static_assert(R % 4 == 0 && SQ % R == 0, "whole rings of whole chain rounds");
    typedef float f4v __attribute__((ext_vector_type(4)));
    const int li = wl & 15, lk = wl >> 4;
    const bool live = li < rows;
    const __attribute__((address_space(1))) f4v* B =
        (const __attribute__((address_space(1))) f4v*)Wf + ((long long)f * SQ * 64 + wl);
    f4v ring[R];
#pragma unroll
    for (int u = 0; u < R; ++u) ring[u] = B[u * 64];
    v4f c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int q0 = 0; q0 < SQ; q0 += R) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int q = q0 + u;
            const f4v b = ring[u];
            if (q + R < SQ) ring[u] = B[(q + R) * 64];
            const float* a = A + (live ? li : 0) * as + 16 * q + lk;
            v4f& cc = c[u & 3];
            cc = __builtin_amdgcn_mfma_f32_16x16x4f32(live ? a[0] : 0.0f, b.x, cc, 0, 0, 0);
            cc = __builtin_amdgcn_mfma_f32_16x16x4f32(live ? a[4] : 0.0f, b.y, cc, 0, 0, 0);
            cc = __builtin_amdgcn_mfma_f32_16x16x4f32(live ? a[8] : 0.0f, b.z, cc, 0, 0, 0);
            cc = __builtin_amdgcn_mfma_f32_16x16x4f32(live ? a[12] : 0.0f, b.w, cc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[rr] = (c[0][rr] + c[1][rr]) + (c[2][rr] + c[3][rr]);
}
// Delta = softplus(dt_proj . delta + b)
template <int RR>
DEVI float dt_of(const float* delta, const float* dtw, float dtb) {
    float v = 0.0f;
#pragma unroll
    for (int r = 0; r < RR; ++r) v = fmaf(delta[r], dtw[r], v);
    return softplus_hp(v + dtb);
}
// h <- exp(Delta A) h + (Delta x) B ; y = C.h + D x ; returns y * SiLU(z)
DEVI float scan_update(float* h, float dt, float xs, const float* Bv, const float* Cv, const float* A2,
                       float Dk, float z) {
    float dx = dt * xs;
#pragma unroll
    for (int n = 0; n < NSTATE; ++n) {
        float dA = exp2_hw(dt * A2[n]);
        h[n] = fmaf(dA, h[n], dx * Bv[n]);
    }
    float y = 0.0f;
#pragma unroll
    for (int n = 0; n < NSTATE; ++n) y = fmaf(h[n], Cv[n], y);
    y = fmaf(Dk, xs, y);
    return y * silu_hp(z);
}


// ---------------------------------------------------------------- histogram / CDF
// One wave per row; wave lane i owns symbols 4i..4i+3.  Produces f[4] (the
// strictly positive histogram summing to 2^16) and cx[4] = C(a) for its
// symbols (paper, Range coding: probabilities and integer CDF).
struct QRow {
    int f[4];
    int cx[4];
    float p[4];
    DEVI int fsel(int i) const { return i == 0 ? f[0] : i == 1 ? f[1] : i == 2 ? f[2] : f[3]; }
    DEVI int csel(int i) const { return i == 0 ? cx[0] : i == 1 ? cx[1] : i == 2 ? cx[2] : cx[3]; }
};
DEVI QRow quant_row(const float* __restrict__ lg, int lane) {
    QRow q;
    float4 l4 = *reinterpret_cast<const float4*>(lg + 4 * lane);
    float l[4] = {l4.x, l4.y, l4.z, l4.w};
    float m = fmaxf(fmaxf(l[0], l[1]), fmaxf(l[2], l[3]));
    m = wave_max(m);
    float e[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = exp_hp(l[i] - m);
    float zs = ((e[0] + e[1]) + e[2]) + e[3];
    zs = wave_sum(zs);
    const float rz = rcp_hp(zs);
    int tot = 0;
    int best_v = -1, best_i = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        q.p[i] = e[i] * rz;
        int gi = (int)(q.p[i] * 65536.0f);
        q.f[i] = gi < 1 ? 1 : gi;
        tot += q.f[i];
        if (q.f[i] > best_v) { best_v = q.f[i]; best_i = 4 * lane + i; }
    }
    tot = wave_sum_i(tot);
    // argmax over lanes: largest value, lowest index on ties
    wave_argmax_i(best_v, best_i);
    int dlt = 65536 - tot;
    // remainder to the winning bin; written as selects so f stays in registers
    const bool mine = (best_i >> 2) == lane;
    const int wi = best_i & 3;
#pragma unroll
    for (int i = 0; i < 4; ++i) q.f[i] += (mine && wi == i) ? dlt : 0;
    int loc = ((q.f[0] + q.f[1]) + q.f[2]) + q.f[3];
    int incl = wave_incl_scan_i(loc, lane);
    int c = incl - loc;
#pragma unroll
    for (int i = 0; i < 4; ++i) { q.cx[i] = c; c += q.f[i]; }
    return q;
}


// ---------------------------------------------------------------- range coder
struct Enc {
    uint64_t L, R;
    uint32_t cur;
};
DEVI void enc_reset(Enc& e) { e.L = 0; e.R = 1ULL << 32; e.cur = 0; }
DEVI void enc_emit(Enc& e, uint8_t* out, uint32_t cap, uint32_t b) {
    if (e.cur < cap) out[e.cur] = (uint8_t)b;
    e.cur++;
}
DEVI void enc_put(Enc& e, uint32_t cl, uint32_t f, uint8_t* out, uint32_t cap) {
    uint64_t L = e.L + ((e.R * cl) >> 16);
    uint64_t R = (e.R * f) >> 16;
    for (;;) {
        if ((L >> 24) == ((L + R - 1) >> 24)) {
            enc_emit(e, out, cap, (uint32_t)(L >> 24));
            L = (L << 8) & 0xFFFFFFFFULL;
            R <<= 8;
        } else if (R < 65536ULL) {
            R = 65536ULL - (L & 0xFFFFULL);
        } else {
            break;
        }
    }
    e.L = L;
    e.R = R;
}
DEVI void enc_flush(Enc& e, uint8_t* out, uint32_t cap) {
    for (int k = 0; k < 3; ++k) {
        int sh = 32 - 8 * k;
        uint64_t V = ((e.L + (1ULL << sh) - 1) >> sh) << sh;
        if (V <= e.L + e.R - 1) {
            for (int i = 0; i < k; ++i) enc_emit(e, out, cap, (uint32_t)((V >> (24 - 8 * i)) & 0xFF));
            return;
        }
    }
}

struct Dec {
    uint64_t L, R, X;
    uint32_t cur;
};
DEVI uint32_t dec_byte(const uint8_t* in, uint32_t len, uint32_t i) { return i < len ? in[i] : 0u; }
DEVI void dec_reset(Dec& d, const uint8_t* in, uint32_t len) {
    d.L = 0;
    d.R = 1ULL << 32;
    d.X = 0;
    for (uint32_t i = 0; i < 4; ++i) d.X = (d.X << 8) | dec_byte(in, len, i);
    d.cur = 4;
}
// floor(v / r) for v < 2^53 and 1 <= r <= 2^32: the correctly rounded double
// quotient is within 2^-5 of v / r, so its truncation is the floor or one
// above it, which the integer check corrects (no 64-bit integer division)
DEVI uint64_t udiv_small(uint64_t v, uint64_t r) {
    uint64_t q = (uint64_t)((double)v / (double)r);
    if (q * r > v) --q;
    return q;
}
DEVI uint32_t dec_target(const Dec& d) {   // x = floor(((X - L + 1) M - 1) / R)
    uint64_t v = ((d.X - d.L + 1) << 16) - 1;
    uint64_t x = udiv_small(v, d.R);
    return x > 65535ULL ? 65535u : (uint32_t)x;   // clamp only matters for corrupt input
}
// pf: the next 8 payload bytes from d.cur, read ahead of time, byte i in bits
// 8i..8i+7 (has_pf = false: read each byte when needed)
DEVI void dec_update(Dec& d, uint32_t cl, uint32_t f, const uint8_t* in, uint32_t len,
                     uint64_t pf = 0, bool has_pf = false) {
    uint64_t L = d.L + ((d.R * cl) >> 16);
    uint64_t R = (d.R * f) >> 16;
    uint64_t X = d.X;
    uint32_t used = 0;
    for (;;) {
        if ((L >> 24) == ((L + R - 1) >> 24)) {
            L = (L << 8) & 0xFFFFFFFFULL;
            R <<= 8;
            uint32_t b = (has_pf && used < 8) ? (uint32_t)((pf >> (8 * used)) & 0xFF) : dec_byte(in, len, d.cur);
            X = ((X << 8) & 0xFFFFFFFFULL) | b;
            d.cur++;
            used++;
        } else if (R < 65536ULL) {
            R = 65536ULL - (L & 0xFFFFULL);
        } else {
            break;
        }
    }
    d.L = L;
    d.R = R;
    d.X = X;
}


}  // namespace boa
