// On-device training of the byte-level Mamba predictor: cross-entropy of the
// next byte (paper, Theoretical Framework: the per-step loss whose sum is the
// code length), forward over whole sequences with the activations the
// backward needs, a hand-written reverse pass for every stage and AdamW.
//
// The in-time dependence sits in the causal conv and the selective scan
// (Appendix A: with input-dependent Delta, B, C the recurrence is evaluated by
// a scan during training).  The scan forward keeps h only at chunk starts;
// the backward recomputes h inside each chunk and runs the reverse
// recurrence  gh_t = C_t gy_t + exp(Delta_{t+1} A) gh_{t+1}.
//
// Every projection and its input and weight gradients run on this file's
// MFMA GEMM (k_tg): FP32 operands on v_mfma_f32_16x16x4_f32, or BF16
// operands (activations, gradients and the weights rounded to bf16 as they
// are staged) on v_mfma_f32_16x16x32_bf16, both accumulating in FP32; the
// master weights, the optimiser and every elementwise step stay FP32.
//
// Training is deterministic: no reduction uses atomics.  Sums over rows
// (weight gradients, bias and LayerNorm gradients, the embedding gradient,
// the conv weights) are taken per fixed slice of rows into a partial buffer
// and the slices are then added in increasing order; sums over channel blocks
// or sequences (the scan's dB, dC, dA, dD) are kept per block and added in
// block order; the loss and the gradient norm are summed by fixed trees.
// Two runs from the same weights and data give identical bits.
#include "boa_internal.h"
#include "device_common.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

namespace boa {
namespace {

// ============================================================ GEMM
// C (+)= A . B with A(m, k) = A[m sam + k sak] and B(k, n) = B[k sbk + n sbn]
// (row-major operands used as they are or transposed, by their strides).
// A workgroup of 4 waves owns a 64 x 64 tile of C; each wave a 32 x 32 block
// of 2 x 2 MFMA tiles.  The reduction runs over k in tiles of 32 staged in
// LDS (k-contiguous rows, the MFMA operand order), with the next tile's
// global loads in registers while the current one is multiplied.  AK (BK_)
// selects the thread-to-element map of the global loads: along k when the
// operand is contiguous in k, else along m (n), so that loads coalesce either
// way.  Split reductions (gridDim.z > 1) cover k in [z kspan, (z+1) kspan)
// and write their own partial C + z cstride; the partials are added in z
// order by k_sum_slices.  Within a split the accumulation order over k is
// fixed: increasing, in steps of 4 (FP32) or 32 (BF16).
constexpr int TG_BM = 64, TG_BN = 64, TG_BK = 32;

template <int DT, bool AK, bool BK_>
__global__ __launch_bounds__(256) void k_tg(const float* __restrict__ A, long long sam, long long sak,
                                            const float* __restrict__ B, long long sbk, long long sbn, int M, int N,
                                            long long K, long long kspan, float* __restrict__ C, long long ldc,
                                            long long cstride, int accumulate) {
    using ET = typename std::conditional<DT == 0, float, uint16_t>::type;
    constexpr int RS = DT == 0 ? TG_BK + 4 : TG_BK + 8;      // LDS row stride (elements)
    __shared__ __align__(16) ET As[TG_BM * RS];
    __shared__ __align__(16) ET Bs[TG_BN * RS];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv >> 1, wn = wv & 1;
    const int m0 = blockIdx.y * TG_BM, n0 = blockIdx.x * TG_BN;
    const long long kb = (long long)blockIdx.z * kspan;
    const long long ke = K < kb + kspan ? K : kb + kspan;
    // element map of one thread: 8 elements of a 64 x 32 tile
    const int ar = AK ? tid >> 2 : (tid & 7) * 8, ak = AK ? (tid & 3) * 8 : tid >> 3;
    const int br = BK_ ? tid >> 2 : (tid & 7) * 8, bk = BK_ ? (tid & 3) * 8 : tid >> 3;
    float ra[8], rb[8];
    auto load = [&](long long k0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int m = m0 + ar + (AK ? 0 : j);
            const long long k = k0 + ak + (AK ? j : 0);
            ra[j] = (m < M && k < ke) ? A[(long long)m * sam + k * sak] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int n = n0 + br + (BK_ ? 0 : j);
            const long long k = k0 + bk + (BK_ ? j : 0);
            rb[j] = (n < N && k < ke) ? B[k * sbk + (long long)n * sbn] : 0.0f;
        }
    };
    auto put = [&](ET* S, int r, int k, const float (&v)[8], bool along_k) {
        if (DT == 0) {
            float* F = reinterpret_cast<float*>(S);
            if (along_k) {
                *reinterpret_cast<float4*>(F + r * RS + k) = make_float4(v[0], v[1], v[2], v[3]);
                *reinterpret_cast<float4*>(F + r * RS + k + 4) = make_float4(v[4], v[5], v[6], v[7]);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) F[(r + j) * RS + k] = v[j];
            }
        } else {
            uint16_t* H = reinterpret_cast<uint16_t*>(S);
            if (along_k) {
                uint4 u;
                u.x = (uint32_t)f2bf_bits(v[0]) | ((uint32_t)f2bf_bits(v[1]) << 16);
                u.y = (uint32_t)f2bf_bits(v[2]) | ((uint32_t)f2bf_bits(v[3]) << 16);
                u.z = (uint32_t)f2bf_bits(v[4]) | ((uint32_t)f2bf_bits(v[5]) << 16);
                u.w = (uint32_t)f2bf_bits(v[6]) | ((uint32_t)f2bf_bits(v[7]) << 16);
                *reinterpret_cast<uint4*>(H + r * RS + k) = u;
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) H[(r + j) * RS + k] = f2bf_bits(v[j]);
            }
        }
    };
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    const int li = lane & 15, lk = lane >> 4;
    if (kb < ke) load(kb);
    for (long long k0 = kb; k0 < ke; k0 += TG_BK) {
        put(As, ar, ak, ra, AK);
        put(Bs, br, bk, rb, BK_);
        __syncthreads();
        if (k0 + TG_BK < ke) load(k0 + TG_BK);
        if (DT == 0) {
            const float* Af = reinterpret_cast<const float*>(As);
            const float* Bf = reinterpret_cast<const float*>(Bs);
#pragma unroll
            for (int ks = 0; ks < TG_BK; ks += 4) {
                float af[2], bf[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) af[i] = Af[(wm * 32 + i * 16 + li) * RS + ks + lk];
#pragma unroll
                for (int j = 0; j < 2; ++j) bf[j] = Bf[(wn * 32 + j * 16 + li) * RS + ks + lk];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
            }
        } else {
            const uint16_t* Ah = reinterpret_cast<const uint16_t*>(As);
            const uint16_t* Bh = reinterpret_cast<const uint16_t*>(Bs);
            v8bf af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = *reinterpret_cast<const v8bf*>(Ah + (wm * 32 + i * 16 + li) * RS + 8 * lk);
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = *reinterpret_cast<const v8bf*>(Bh + (wn * 32 + j * 16 + li) * RS + 8 * lk);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // lane holds rows 4 lk + r, column li of each 16 x 16 tile
    float* Cz = C + (long long)blockIdx.z * cstride;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * 32 + i * 16 + 4 * lk + r;
                const int n = n0 + wn * 32 + j * 16 + li;
                if (m < M && n < N) {
                    float* d = Cz + (long long)m * ldc + n;
                    const float v = acc[i][j][r];
                    *d = accumulate ? *d + v : v;
                }
            }
}

// ============================================================ fixed-order sums
// out[i] (+)= part[i] + part[stride + i] + ... (S slices, increasing)
__global__ void k_sum_slices(const float* __restrict__ part, int S, long long n, long long stride,
                             float* __restrict__ out, int accumulate) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    float v = part[i];
    for (int s = 1; s < S; ++s) v += part[(long long)s * stride + i];
    out[i] = accumulate ? out[i] + v : v;
}

// the same for the split partials [S][M][N] of a GEMM, into C[m ldc + n]
__global__ void k_sum_slices_2d(const float* __restrict__ part, int S, int M, int N, float* __restrict__ C,
                                long long ldc, int accumulate) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    const long long n_all = (long long)M * N;
    if (i >= n_all) return;
    float v = part[i];
    for (int s = 1; s < S; ++s) v += part[(long long)s * n_all + i];
    float* d = C + (i / N) * ldc + i % N;
    *d = accumulate ? *d + v : v;
}

// part[s * N + n] = sum over the rows of slice s (increasing) of X[r ld + off + n]
__global__ void k_colsum_part(const float* __restrict__ X, long long rows, int ld, int off, int N, long long per,
                              float* __restrict__ part) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const long long r0 = blockIdx.y * per, r1 = r0 + per < rows ? r0 + per : rows;
    float acc = 0.f;
    for (long long r = r0; r < r1; ++r) acc += X[r * ld + off + n];
    part[(long long)blockIdx.y * N + n] = acc;
}

// One workgroup: *out = sum of in[0 .. n) in double; thread t sums t, t + 256,
// ... in order, then a fixed halving tree.  scale multiplies the result.
template <typename TI>
__global__ __launch_bounds__(256) void k_sum_all(const TI* __restrict__ in, long long n, double scale,
                                                 double* __restrict__ out_d, float* __restrict__ out_f) {
    __shared__ double buf[256];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (long long i = t; i < n; i += 256) acc += (double)in[i];
    buf[t] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) buf[t] += buf[t + h];
        __syncthreads();
    }
    if (t == 0) {
        if (out_d) *out_d = buf[0] * scale;
        if (out_f) *out_f = (float)(buf[0] * scale);
    }
}

// ============================================================ elementwise and per-row kernels
__global__ void k_tr_embed(const uint8_t* __restrict__ tok, int B, int T, const float* __restrict__ E, int D,
                           float* __restrict__ r) {
    const int Tn = T - 1;
    long long row = blockIdx.x * 4LL + threadIdx.y;
    if (row >= (long long)B * Tn) return;
    int b = (int)(row / Tn), t = (int)(row % Tn);
    int y = tok[(long long)b * T + t];
    for (int k = threadIdx.x; k < D; k += 64) r[row * D + k] = E[(long long)y * D + k];
}

// Embedding gradient of one slice of rows and 64 columns: one wave adds the
// rows of its slice in order into a [256][64] LDS table (lane = column, so
// no two lanes touch one address); the table is the slice's partial
// part[s][256][D].
__global__ __launch_bounds__(64) void k_tr_embed_bwd_part(const uint8_t* __restrict__ tok, int B, int T,
                                                          const float* __restrict__ dr, int D, long long per,
                                                          float* __restrict__ part) {
    __shared__ float acc[VOCAB][64];
    const int lane = threadIdx.x, c = blockIdx.x * 64 + lane;
    const int Tn = T - 1;
    const long long rows = (long long)B * Tn;
    for (int y = 0; y < VOCAB; ++y) acc[y][lane] = 0.f;
    const long long r0 = blockIdx.y * per, r1 = r0 + per < rows ? r0 + per : rows;
    for (long long r = r0; r < r1; r += 8) {
        int ys[8];
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const long long rr = r + j;
            ys[j] = -1;
            v[j] = 0.f;
            if (rr < r1) {
                const int b = (int)(rr / Tn), t = (int)(rr % Tn);
                ys[j] = tok[(long long)b * T + t];
                v[j] = dr[rr * D + c];
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (ys[j] >= 0) acc[ys[j]][lane] += v[j];
    }
    float* dst = part + (long long)blockIdx.y * VOCAB * D + c;
    for (int y = 0; y < VOCAB; ++y) dst[(long long)y * D] = acc[y][lane];
}

// LayerNorm forward, one wave per row; keeps (mean, rstd)
__global__ void k_tr_ln_fwd(const float* __restrict__ x, long long rows, int D, const float* __restrict__ w,
                            const float* __restrict__ b, float* __restrict__ out, float* __restrict__ st) {
    long long row = blockIdx.x * 4LL + threadIdx.y;
    if (row >= rows) return;
    int lane = threadIdx.x;
    const float* xr = x + row * D;
    float mu, rs;
    ln_stats(xr, D, lane, mu, rs);
    for (int k = lane; k < D; k += 64) out[row * D + k] = ln_apply(xr[k], mu, rs, w[k], b[k]);
    if (lane == 0) { st[2 * row] = mu; st[2 * row + 1] = rs; }
}

// LayerNorm backward: dx (+)= rstd (dxh - mean(dxh) - xh mean(dxh xh)), dxh = dy w;
// tmp = dy * xh for the weight gradient (column sums taken separately)
__global__ void k_tr_ln_bwd(const float* __restrict__ dy, const float* __restrict__ x, const float* __restrict__ st,
                            long long rows, int D, const float* __restrict__ w, float* __restrict__ dx, int accumulate,
                            float* __restrict__ tmp) {
    long long row = blockIdx.x * 4LL + threadIdx.y;
    if (row >= rows) return;
    int lane = threadIdx.x;
    const float mu = st[2 * row], rs = st[2 * row + 1];
    float s1 = 0.f, s2 = 0.f;
    for (int k = lane; k < D; k += 64) {
        float xh = (x[row * D + k] - mu) * rs;
        float g = dy[row * D + k];
        float dxh = g * w[k];
        s1 += dxh;
        s2 += dxh * xh;
        tmp[row * D + k] = g * xh;
    }
    s1 = wave_sum(s1) / (float)D;
    s2 = wave_sum(s2) / (float)D;
    for (int k = lane; k < D; k += 64) {
        float xh = (x[row * D + k] - mu) * rs;
        float v = rs * (dy[row * D + k] * w[k] - s1 - xh * s2);
        if (accumulate) dx[row * D + k] += v; else dx[row * D + k] = v;
    }
}

// causal depthwise conv + SiLU over each sequence (zero before t = 0)
__global__ void k_tr_conv_fwd(const float* __restrict__ xz, long long rows, int Tn, int Di,
                              const float* __restrict__ cw, const float* __restrict__ cb, float* __restrict__ xc,
                              float* __restrict__ xs) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= rows * Di) return;
    long long row = i / Di;
    int d = (int)(i % Di), t = (int)(row % Tn);
    float acc = cb[d];
    for (int k = 0; k < KCONV; ++k) {
        int back = KCONV - 1 - k;
        if (t - back >= 0) acc = fmaf(cw[d * KCONV + k], xz[(row - back) * 2 * Di + d], acc);
    }
    xc[i] = acc;
    xs[i] = silu_f(acc);
}

DEVI float dsilu_f(float v) {
    float s = 1.0f / (1.0f + expf(-v));
    return s * (1.0f + v * (1.0f - s));
}

// dxc = dxs * silu'(xc); dx[t] = sum_k dxc[t + back_k] w[k] written into dxz[:, :Di]
__global__ void k_tr_conv_bwd_x(const float* __restrict__ dxs, const float* __restrict__ xc, long long rows, int Tn,
                                int Di, const float* __restrict__ cw, float* __restrict__ dxc,
                                float* __restrict__ dxz) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= rows * Di) return;
    long long row = i / Di;
    int d = (int)(i % Di), t = (int)(row % Tn);
    // dxc of rows t..t+3 (same sequence) are needed: recompute them locally
    float acc = 0.f;
    for (int k = 0; k < KCONV; ++k) {
        int fwd = KCONV - 1 - k;               // output row t + fwd used input t through weight k
        if (t + fwd < Tn) {
            long long j = (row + fwd) * Di + d;
            acc += dxs[j] * dsilu_f(xc[j]) * cw[d * KCONV + k];
        }
    }
    dxc[i] = dxs[i] * dsilu_f(xc[i]);
    dxz[row * 2 * Di + d] = acc;
}

// conv weight and bias gradients of one slice of rows, in row order:
// part[s][d * K + k] = sum dxc[t] x[t - back_k], part[s][Di K + d] = sum dxc[t]
__global__ void k_tr_conv_bwd_w_part(const float* __restrict__ dxc, const float* __restrict__ xz, long long rows,
                                     int Tn, int Di, long long per, float* __restrict__ part) {
    int d = blockIdx.x * 256 + threadIdx.x;
    if (d >= Di) return;
    const long long r0 = blockIdx.y * per, r1 = r0 + per < rows ? r0 + per : rows;
    float aw[KCONV] = {0.f, 0.f, 0.f, 0.f}, ab = 0.f;
    for (long long r = r0; r < r1; ++r) {
        int t = (int)(r % Tn);
        float g = dxc[r * Di + d];
        ab += g;
        for (int k = 0; k < KCONV; ++k) {
            int back = KCONV - 1 - k;
            if (t - back >= 0) aw[k] += g * xz[(r - back) * 2 * Di + d];
        }
    }
    float* dst = part + (long long)blockIdx.y * Di * (KCONV + 1);
    for (int k = 0; k < KCONV; ++k) dst[d * KCONV + k] = aw[k];
    dst[Di * KCONV + d] = ab;
}

// feed-forward sub-layer: u += b1 (in place), gu = GELU(u) (exact erf form)
DEVI float gelu_tr(float u) { return 0.5f * u * (1.0f + erff(u * 0.7071067811865476f)); }
DEVI float dgelu_tr(float u) {        // Phi(u) + u phi(u)
    return 0.5f * (1.0f + erff(u * 0.7071067811865476f)) + u * expf(-0.5f * u * u) * 0.3989422804014327f;
}
__global__ void k_tr_bias_gelu(float* __restrict__ u, long long rows, int H, const float* __restrict__ b,
                               float* __restrict__ gu) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= rows * H) return;
    const float v = u[i] + b[i % H];
    u[i] = v;
    gu[i] = gelu_tr(v);
}
// x += b per row (bias of the second feed-forward product)
__global__ void k_tr_add_bias(float* __restrict__ x, long long rows, int N, const float* __restrict__ b) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i < rows * N) x[i] += b[i % N];
}
// du = dgu * GELU'(u), in place in dgu
__global__ void k_tr_gelu_bwd(float* __restrict__ dgu, const float* __restrict__ u, long long n) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i < n) dgu[i] *= dgelu_tr(u[i]);
}

// dtr += bias; dt = softplus(dtr)
__global__ void k_tr_bias_softplus(float* __restrict__ dtr, long long rows, int Di, const float* __restrict__ b,
                                   float* __restrict__ dt) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= rows * Di) return;
    float v = dtr[i] + b[i % Di];
    dtr[i] = v;
    dt[i] = softplus_f(v);
}
__global__ void k_tr_softplus_bwd(const float* __restrict__ ddt, const float* __restrict__ dtr, long long n,
                                  float* __restrict__ ddtr) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    float v = dtr[i];
    ddtr[i] = v > 20.0f ? ddt[i] : ddt[i] / (1.0f + expf(-v));
}

// selective scan forward, one thread per (sequence, channel), one wave per
// (sequence, 64 channels); h saved every Tc steps.  B and C (the same for
// every channel of a row) are staged in LDS for SCAN_SB rows at a time, and
// the next step's dt and x are loaded while the current step is computed.
// exp(dt A) = exp2(dt (A log2 e)) on the hardware exp2.
constexpr int SCAN_CH = 64, SCAN_SB = 64;
constexpr float LOG2E_F = 1.4426950408889634f;

// rows [r0, r1) of B and C (columns R .. R + 31 of dbc, row stride NO) into bc_s
DEVI void stage_bc(float* bc_s, const float* __restrict__ dbc, long long row_base, int r0, int r1, int NO, int R,
                   int lane) {
    __syncthreads();                     // the previous block's reads are done
    for (int i = lane; i < (r1 - r0) * 2 * NSTATE; i += SCAN_CH)
        bc_s[i] = dbc[(row_base + r0 + i / (2 * NSTATE)) * NO + R + i % (2 * NSTATE)];
    __syncthreads();
}

__global__ __launch_bounds__(SCAN_CH) void k_tr_scan_fwd(const float* __restrict__ xs, const float* __restrict__ dt,
                                                         const float* __restrict__ dbc, int NO, int R,
                                                         const float* __restrict__ A_log,
                                                         const float* __restrict__ Dsk, const float* __restrict__ xz,
                                                         int B, int Tn, int Di, int Tc, float* __restrict__ y,
                                                         float* __restrict__ g, float* __restrict__ hsave) {
    __shared__ float bc_s[SCAN_SB * 2 * NSTATE];
    const int b = blockIdx.y, lane = threadIdx.x, d = blockIdx.x * SCAN_CH + lane;
    const bool on = d < Di;
    const int nch = (Tn + Tc - 1) / Tc;
    float A2[NSTATE], h[NSTATE];
    for (int n = 0; n < NSTATE; ++n) { A2[n] = on ? -expf(A_log[d * NSTATE + n]) * LOG2E_F : 0.f; h[n] = 0.f; }
    const float Dv = on ? Dsk[d] : 0.f;
    const long long row0 = (long long)b * Tn;
    float dtn = 0.f, xn = 0.f;
    if (on && Tn > 0) { dtn = dt[row0 * Di + d]; xn = xs[row0 * Di + d]; }
    for (int s0 = 0; s0 < Tn; s0 += SCAN_SB) {
        const int s1 = s0 + SCAN_SB < Tn ? s0 + SCAN_SB : Tn;
        stage_bc(bc_s, dbc, row0, s0, s1, NO, R, lane);
        for (int t = s0; t < s1; ++t) {
            const long long row = row0 + t;
            if (t % Tc == 0 && on) {
                float* hs = hsave + (((long long)b * nch + t / Tc) * NSTATE) * Di + d;
                for (int n = 0; n < NSTATE; ++n) hs[(long long)n * Di] = h[n];
            }
            const float dtv = dtn, x = xn;
            if (on && t + 1 < Tn) { dtn = dt[(row + 1) * Di + d]; xn = xs[(row + 1) * Di + d]; }
            const float* bc = bc_s + (t - s0) * 2 * NSTATE;
            float yv = 0.f;
#pragma unroll
            for (int n = 0; n < NSTATE; ++n) {
                h[n] = exp2_hw(dtv * A2[n]) * h[n] + dtv * x * bc[n];
                yv += h[n] * bc[NSTATE + n];
            }
            yv += Dv * x;
            if (on) {
                y[row * Di + d] = yv;
                if (g) g[row * Di + d] = yv * silu_f(xz[row * 2 * Di + Di + d]);
            }
        }
    }
}

// gate backward: dy = dg silu(z); dz = dg y silu'(z) (into dxz[:, Di:])
__global__ void k_tr_gate_bwd(const float* __restrict__ dg, const float* __restrict__ y, const float* __restrict__ xz,
                              long long rows, int Di, float* __restrict__ dy, float* __restrict__ dxz) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= rows * Di) return;
    long long row = i / Di;
    int d = (int)(i % Di);
    float z = xz[row * 2 * Di + Di + d];
    float gv = dg[i];
    dy[i] = gv * silu_f(z);
    dxz[row * 2 * Di + Di + d] = gv * y[i] * dsilu_f(z);
}

// Sums of 32 values over the 64 lanes of a wave by a transposing tree: at
// partner distance m = 32, 16, 8, 4, 2 every lane keeps the half of its
// values selected by its own bit m and adds the partner's copy of that half
// (2 x 16, ..., 2 x 1 values exchanged); lane l then holds index l >> 1 summed
// over the 32 lanes with its bit 0, and distance 1 completes the sum.  Fixed
// order: identical bits on every call.
template <int C>
DEVI void transpose_level(float (&v)[2 * NSTATE], int lane) {
    const bool hi = (lane & (2 * C)) != 0;
#pragma unroll
    for (int j = 0; j < C; ++j) {
        const float keep = hi ? v[C + j] : v[j];
        const float send = hi ? v[j] : v[C + j];
        v[j] = keep + __shfl_xor(send, 2 * C, 64);
    }
}
DEVI float wave_sum32_transposed(float (&v)[2 * NSTATE], int lane) {
    transpose_level<16>(v, lane);
    transpose_level<8>(v, lane);
    transpose_level<4>(v, lane);
    transpose_level<2>(v, lane);
    transpose_level<1>(v, lane);
    return v[0] + __shfl_xor(v[0], 1, 64);
}

// selective scan backward: one wave per (sequence, 64 channels).  Inside
// each chunk h_{t-1} is recomputed from the saved chunk start into hbuf, then
// the reverse recurrence runs; both passes read B and C from LDS (staged
// SCAN_SB rows at a time) and load the next step's per-channel inputs while
// the current step is computed.  dB and dC (sums over channels) are reduced
// within the wave (wave_sum32_transposed) and written as the block's partial
// pbc[blockIdx.x][row][32]; dA_log and dD (sums over time) are written per
// sequence as pA[b][d][n], pD[b][d].
__global__ __launch_bounds__(SCAN_CH) void k_tr_scan_bwd(
    const float* __restrict__ xs, const float* __restrict__ dt, const float* __restrict__ dbc, int NO, int R,
    const float* __restrict__ A_log, const float* __restrict__ Dsk, const float* __restrict__ dy, int B, int Tn,
    int Di, int Tc, const float* __restrict__ hsave, float* __restrict__ hbuf, float* __restrict__ dxs,
    float* __restrict__ ddt, float* __restrict__ pbc, float* __restrict__ pA, float* __restrict__ pD) {
    __shared__ float bc_s[SCAN_SB * 2 * NSTATE];
    const int b = blockIdx.y, lane = threadIdx.x, d = blockIdx.x * SCAN_CH + lane;
    const bool on = d < Di;
    const int nch = (Tn + Tc - 1) / Tc;
    const long long rows = (long long)B * Tn, row0 = (long long)b * Tn;
    float* hb = hbuf + ((long long)(b * gridDim.x + blockIdx.x) * Tc * NSTATE) * SCAN_CH;
    float A[NSTATE], A2[NSTATE], gh[NSTATE], gA[NSTATE];
    for (int n = 0; n < NSTATE; ++n) {
        A[n] = on ? -expf(A_log[d * NSTATE + n]) : 0.f;
        A2[n] = A[n] * LOG2E_F;
        gh[n] = 0.f;
        gA[n] = 0.f;
    }
    const float Dv = on ? Dsk[d] : 0.f;
    float gD = 0.f;
    for (int c = nch - 1; c >= 0; --c) {
        const int t0 = c * Tc, t1 = t0 + Tc < Tn ? t0 + Tc : Tn;
        // recompute h_{t-1} for t in [t0, t1) from the saved chunk start
        float h[NSTATE];
        const float* hs = hsave + (((long long)b * nch + c) * NSTATE) * Di + (on ? d : 0);
        for (int n = 0; n < NSTATE; ++n) h[n] = on ? hs[(long long)n * Di] : 0.f;
        float dtn = 0.f, xn = 0.f;
        if (on) { dtn = dt[(row0 + t0) * Di + d]; xn = xs[(row0 + t0) * Di + d]; }
        for (int s0 = t0; s0 < t1; s0 += SCAN_SB) {
            const int s1 = s0 + SCAN_SB < t1 ? s0 + SCAN_SB : t1;
            stage_bc(bc_s, dbc, row0, s0, s1, NO, R, lane);
            for (int t = s0; t < s1; ++t) {
                float* dst = hb + (long long)(t - t0) * NSTATE * SCAN_CH + lane;
#pragma unroll
                for (int n = 0; n < NSTATE; ++n) dst[n * SCAN_CH] = h[n];
                const float dtv = dtn, x = xn;
                if (on && t + 1 < t1) { dtn = dt[(row0 + t + 1) * Di + d]; xn = xs[(row0 + t + 1) * Di + d]; }
                const float* bc = bc_s + (t - s0) * 2 * NSTATE;
#pragma unroll
                for (int n = 0; n < NSTATE; ++n) h[n] = exp2_hw(dtv * A2[n]) * h[n] + dtv * x * bc[n];
            }
        }
        // reverse recurrence over the chunk, later blocks of rows first
        float gn = 0.f, hpn[NSTATE];
        auto fetch = [&](int t, float& dv, float& xv, float& gv, float (&hp)[NSTATE]) {
            const long long row = row0 + t;
            if (on) { dv = dt[row * Di + d]; xv = xs[row * Di + d]; gv = dy[row * Di + d]; }
            const float* src = hb + (long long)(t - t0) * NSTATE * SCAN_CH + lane;
#pragma unroll
            for (int n = 0; n < NSTATE; ++n) hp[n] = src[n * SCAN_CH];
        };
        if (t1 > t0) fetch(t1 - 1, dtn, xn, gn, hpn);
        for (int s1 = t1; s1 > t0; s1 -= SCAN_SB) {
            const int s0 = s1 - SCAN_SB > t0 ? s1 - SCAN_SB : t0;
            stage_bc(bc_s, dbc, row0, s0, s1, NO, R, lane);
            for (int t = s1 - 1; t >= s0; --t) {
                const long long row = row0 + t;
                const float dtv = dtn, x = xn, g = gn;
                float hp[NSTATE];
#pragma unroll
                for (int n = 0; n < NSTATE; ++n) hp[n] = hpn[n];
                if (t > t0) fetch(t - 1, dtn, xn, gn, hpn);
                const float* bc = bc_s + (t - s0) * 2 * NSTATE;
                float pv[2 * NSTATE];
                float ddt_v = 0.f, dx_v = 0.f;
#pragma unroll
                for (int n = 0; n < NSTATE; ++n) {
                    float Bn = bc[n], Cn = bc[NSTATE + n];
                    float a = on ? exp2_hw(dtv * A2[n]) : 0.f;
                    float ht = a * hp[n] + dtv * x * Bn;
                    gh[n] += Cn * g;
                    pv[NSTATE + n] = on ? g * ht : 0.f;
                    float ga = gh[n] * hp[n];
                    ddt_v += ga * a * A[n] + gh[n] * x * Bn;
                    gA[n] += ga * a * dtv;
                    dx_v += gh[n] * dtv * Bn;
                    pv[n] = on ? gh[n] * dtv * x : 0.f;
                    gh[n] *= a;
                }
                dx_v += Dv * g;
                gD += g * x;
                if (on) { ddt[row * Di + d] = ddt_v; dxs[row * Di + d] = dx_v; }
                // dB (index n) and dC (index 16 + n) of this row over the wave's 64 channels
                const float v = wave_sum32_transposed(pv, lane);
                if ((lane & 1) == 0) pbc[((long long)blockIdx.x * rows + row) * 2 * NSTATE + (lane >> 1)] = v;
            }
        }
    }
    if (on) {
        for (int n = 0; n < NSTATE; ++n) pA[((long long)b * Di + d) * NSTATE + n] = gA[n] * A[n];
        pD[(long long)b * Di + d] = gD;
    }
}

// dB, dC of every row: the channel blocks' partials added in block order,
// written into columns R .. R + 31 of ddbc (row stride NO)
__global__ void k_tr_dbc_reduce(const float* __restrict__ pbc, int nblk, long long rows, float* __restrict__ ddbc,
                                int NO, int R) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= rows * 2 * NSTATE) return;
    const long long row = i / (2 * NSTATE);
    const int c = (int)(i % (2 * NSTATE));
    float v = pbc[i];
    for (int k = 1; k < nblk; ++k) v += pbc[(long long)k * rows * 2 * NSTATE + i];
    ddbc[row * NO + R + c] = v;
}

// softmax cross-entropy: rowloss[row] = -log p(target); dlogits = (p - onehot) / ntok
__global__ void k_tr_ce(float* __restrict__ logits, const float* __restrict__ bias, const uint8_t* __restrict__ tok,
                        int B, int T, float* __restrict__ rowloss, float inv_ntok) {
    const int Tn = T - 1;
    long long row = blockIdx.x * 4LL + threadIdx.y;
    if (row >= (long long)B * Tn) return;
    int lane = threadIdx.x;
    int b = (int)(row / Tn), t = (int)(row % Tn);
    int tgt = tok[(long long)b * T + t + 1];
    float* lr = logits + row * 256;
    float l[4];
    for (int i = 0; i < 4; ++i) l[i] = lr[4 * lane + i] + bias[4 * lane + i];
    float m = wave_max(fmaxf(fmaxf(l[0], l[1]), fmaxf(l[2], l[3])));
    float e[4], zs = 0.f;
    for (int i = 0; i < 4; ++i) { e[i] = expf(l[i] - m); zs += e[i]; }
    zs = wave_sum(zs);
    float lse = m + logf(zs);
    for (int i = 0; i < 4; ++i) {
        int a = 4 * lane + i;
        float p = e[i] / zs;
        lr[a] = (p - (a == tgt ? 1.0f : 0.0f)) * inv_ntok;
        if (a == tgt) rowloss[row] = lse - l[i];
    }
}

// per-block partial sums of g^2 over a fixed element range (thread-strided,
// then the wave tree, then the 4 waves in order)
__global__ __launch_bounds__(256) void k_sqsum_part(const float* __restrict__ g, long long n, long long per,
                                                    float* __restrict__ part) {
    __shared__ float w4[4];
    const long long i0 = blockIdx.x * per, i1 = i0 + per < n ? i0 + per : n;
    float acc = 0.f;
    for (long long i = i0 + threadIdx.x; i < i1; i += 256) acc += g[i] * g[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) w4[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((w4[0] + w4[1]) + w4[2]) + w4[3];
}

// AdamW with decoupled weight decay and global-norm clipping (norm^2 in *sq)
__global__ void k_adamw(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float wd,
                        float bc1, float bc2, float clip, const float* __restrict__ sq) {
    long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    float nrm = sqrtf(*sq);
    float sc = clip > 0.f && nrm > clip ? clip / (nrm + 1e-6f) : 1.0f;
    float gi = g[i] * sc;
    float wi = w[i] * (1.0f - lr * wd);
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] = wi - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ============================================================ host side
inline unsigned blocks(long long n, int per = 256) { return (unsigned)((n + per - 1) / per); }

struct Buf {
    void* p = nullptr;
    size_t n = 0;
    Buf() = default;
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    Buf(Buf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    ~Buf() { if (p) (void)hipFree(p); }
    hipError_t alloc(size_t b) {
        if (p) { (void)hipFree(p); p = nullptr; }
        n = b;
        return hipMalloc(&p, b ? b : 4);
    }
    // grow only: keeps the allocation when it is large enough
    hipError_t ensure(size_t b) { return (p && n >= b) ? hipSuccess : alloc(b); }
    float* f() const { return static_cast<float*>(p); }
};

// Number of row slices of a fixed-order row reduction (a function of the
// row count only, so the summation order never depends on anything else).
long long row_slices(long long rows, long long max_slices = 256, long long min_rows = 64) {
    long long s = (rows + min_rows - 1) / min_rows;
    return std::max(1LL, std::min(s, max_slices));
}

// GEMM splits: the reduction (K) is split when the output has too few tiles
// to fill the GPU; the split count depends on the shape only.
int gemm_splits(int M, int N, long long K) {
    const long long tiles = (long long)((M + TG_BM - 1) / TG_BM) * ((N + TG_BN - 1) / TG_BN);
    if (tiles >= 1024 || K <= 4 * TG_BK) return 1;
    long long s = (2048 + tiles - 1) / tiles;
    s = std::min(s, (K + 255) / 256);
    return (int)std::max(1LL, s);
}

size_t gemm_ws_floats(int M, int N, long long K) {
    const int S = gemm_splits(M, N, K);
    return S > 1 ? (size_t)S * M * N : 0;
}

}  // namespace

// Training context kept on the model: optimizer moments, step count, the
// activation and gradient buffers of the last (B, T) shape, and scratch.
struct TrainCtx {
    Buf m, v, grad, sqpart, sq;
    long long step = 0;
    // activations (per layer) and backward temporaries, sized for rows x widths
    int B = 0, T = 0, Tc = 0;
    std::vector<Buf> rin, a, st, xz, xc, xs, dbc, dtr, dt, y, g, hs;
    std::vector<Buf> fr, fu, fg, ff, fst;   // feed-forward: input r, W1 r + b1, GELU of it, W2 . + b2, LN stats
    Buf fdu;                                // feed-forward backward: gradient of the hidden row
    Buf rcur, rfin, rf, stf, logits, rowloss;
    Buf dr, tmp, t2, dg, dyb, dxz, ddbc, ddt, ddtr, dxs, dxc, hbuf, pbc, pA, pD, part, gws;
};

void train_ctx_free(void* p) { delete static_cast<TrainCtx*>(p); }

#define TCHK(expr) do { hipError_t e_ = (expr); if (e_ != hipSuccess) { err = std::string(#expr) + ": " + hipGetErrorString(e_); return BOA_E_DEVICE; } } while (0)

namespace {
// C[M, N] (+)= A . B on k_tg (see above); ws holds split partials
hipError_t gemm(int dt, const float* A, long long sam, long long sak, const float* B, long long sbk, long long sbn,
                int M, int N, long long K, float* C, long long ldc, int accumulate, float* ws, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int S = gemm_splits(M, N, K);
    long long kspan = (K + S - 1) / S;
    kspan = (kspan + TG_BK - 1) / TG_BK * TG_BK;
    dim3 grid((N + TG_BN - 1) / TG_BN, (M + TG_BM - 1) / TG_BM, S);
    float* out = S > 1 ? ws : C;
    const long long ld = S > 1 ? N : ldc;
    const int acc = S > 1 ? 0 : accumulate;
    const bool ak = sak == 1, bk = sbk == 1;
#define TG_LAUNCH(DT, AKV, BKV)                                                                                 \
    hipLaunchKernelGGL((k_tg<DT, AKV, BKV>), grid, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, M, N, K, kspan, \
                       out, ld, (long long)M * N, acc)
    if (dt == 0) {
        if (ak && bk) TG_LAUNCH(0, true, true);
        else if (ak) TG_LAUNCH(0, true, false);
        else if (bk) TG_LAUNCH(0, false, true);
        else TG_LAUNCH(0, false, false);
    } else {
        if (ak && bk) TG_LAUNCH(1, true, true);
        else if (ak) TG_LAUNCH(1, true, false);
        else if (bk) TG_LAUNCH(1, false, true);
        else TG_LAUNCH(1, false, false);
    }
#undef TG_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || S == 1) return e;
    hipLaunchKernelGGL(k_sum_slices_2d, dim3(blocks((long long)M * N)), dim3(256), 0, s, ws, S, M, N, C, ldc,
                       accumulate);
    return hipGetLastError();
}

// Row-major linear maps of X [rows, K] (row stride lx) with W [N, K]:
hipError_t lin_fwd(int dt, const float* X, int lx, const float* W, int N, int K, float* Y, int ly, long long rows,
                   int accumulate, float* ws, hipStream_t s) {          // Y (+)= X W^T
    return gemm(dt, X, lx, 1, W, 1, K, (int)rows, N, K, Y, ly, accumulate, ws, s);
}
hipError_t lin_bwd_x(int dt, const float* dY, int ldy, const float* W, int N, int K, float* dX, int ldx,
                     long long rows, int accumulate, float* ws, hipStream_t s) {   // dX (+)= dY W
    return gemm(dt, dY, ldy, 1, W, K, 1, (int)rows, K, N, dX, ldx, accumulate, ws, s);
}
hipError_t lin_bwd_w(int dt, const float* dY, int ldy, const float* X, int lx, int N, int K, float* dW,
                     long long rows, float* ws, hipStream_t s) {         // dW = dY^T X
    return gemm(dt, dY, 1, ldy, X, lx, 1, N, K, rows, dW, K, 0, ws, s);
}

// out[n] = column sums over rows of X[:, off + n], n < N (fixed row slices)
hipError_t colsum(const float* X, long long rows, int ld, int off, int N, float* part, float* out, hipStream_t s) {
    const long long S = row_slices(rows);
    const long long per = (rows + S - 1) / S;
    hipLaunchKernelGGL(k_colsum_part, dim3(blocks(N), (unsigned)S), dim3(256), 0, s, X, rows, ld, off, N, per, part);
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks(N)), dim3(256), 0, s, part, (int)S, (long long)N, (long long)N,
                       out, 0);
    return hipGetLastError();
}

// scratch floats the fixed-order row reductions need
size_t part_floats(long long rows, int D, int Di, int H) {
    const long long S = row_slices(rows);
    return (size_t)S * std::max<size_t>({(size_t)VOCAB * D, (size_t)Di * (KCONV + 1), (size_t)2 * Di, 256,
                                         (size_t)H});
}
}  // namespace

// Sizes the context's buffers for B sequences of T bytes and chunk length Tc.
int train_ensure_buffers(boa_model* m, int B, int T, int Tc, std::string& err) {
    TrainCtx* c = static_cast<TrainCtx*>(m->train);
    if (c->B == B && c->T == T && c->Tc == Tc) return BOA_OK;
    const Layout& L = m->lay;
    const int D = L.D, Di = L.Di, NO = L.R + 2 * NSTATE, Tn = T - 1;
    const size_t rows = (size_t)B * Tn, F = sizeof(float);
    const int nch = (Tn + Tc - 1) / Tc, dblk = (Di + SCAN_CH - 1) / SCAN_CH;
    c->B = c->T = c->Tc = 0;
    c->rin.resize(L.L); c->a.resize(L.L); c->st.resize(L.L); c->xz.resize(L.L); c->xc.resize(L.L);
    c->xs.resize(L.L); c->dbc.resize(L.L); c->dtr.resize(L.L); c->dt.resize(L.L); c->y.resize(L.L);
    c->g.resize(L.L); c->hs.resize(L.L);
    if (L.H) {
        c->fr.resize(L.L); c->fu.resize(L.L); c->fg.resize(L.L); c->ff.resize(L.L); c->fst.resize(L.L);
        for (int l = 0; l < L.L; ++l) {
            TCHK(c->fr[l].ensure(rows * D * F)); TCHK(c->fu[l].ensure(rows * L.H * F));
            TCHK(c->fg[l].ensure(rows * L.H * F)); TCHK(c->ff[l].ensure(rows * D * F));
            TCHK(c->fst[l].ensure(rows * 2 * F));
        }
        TCHK(c->fdu.ensure(rows * L.H * F));
    }
    for (int l = 0; l < L.L; ++l) {
        TCHK(c->rin[l].ensure(rows * D * F)); TCHK(c->a[l].ensure(rows * D * F)); TCHK(c->st[l].ensure(rows * 2 * F));
        TCHK(c->xz[l].ensure(rows * 2 * Di * F)); TCHK(c->xc[l].ensure(rows * Di * F));
        TCHK(c->xs[l].ensure(rows * Di * F)); TCHK(c->dbc[l].ensure(rows * NO * F));
        TCHK(c->dtr[l].ensure(rows * Di * F)); TCHK(c->dt[l].ensure(rows * Di * F));
        TCHK(c->y[l].ensure(rows * Di * F)); TCHK(c->g[l].ensure(rows * Di * F));
        TCHK(c->hs[l].ensure((size_t)B * nch * NSTATE * Di * F));
    }
    TCHK(c->rcur.ensure(rows * D * F)); TCHK(c->rfin.ensure(rows * D * F));
    TCHK(c->rf.ensure(rows * D * F)); TCHK(c->stf.ensure(rows * 2 * F)); TCHK(c->logits.ensure(rows * 256 * F));
    TCHK(c->rowloss.ensure(rows * F));
    TCHK(c->dr.ensure(rows * D * F)); TCHK(c->tmp.ensure(rows * D * F)); TCHK(c->t2.ensure(rows * D * F));
    TCHK(c->dg.ensure(rows * Di * F)); TCHK(c->dyb.ensure(rows * Di * F)); TCHK(c->dxz.ensure(rows * 2 * Di * F));
    TCHK(c->ddbc.ensure(rows * NO * F)); TCHK(c->ddt.ensure(rows * Di * F)); TCHK(c->ddtr.ensure(rows * Di * F));
    TCHK(c->dxs.ensure(rows * Di * F)); TCHK(c->dxc.ensure(rows * Di * F));
    TCHK(c->hbuf.ensure((size_t)B * dblk * Tc * NSTATE * SCAN_CH * F));
    TCHK(c->pbc.ensure((size_t)dblk * rows * 2 * NSTATE * F));
    TCHK(c->pA.ensure((size_t)B * Di * NSTATE * F)); TCHK(c->pD.ensure((size_t)B * Di * F));
    TCHK(c->part.ensure(part_floats((long long)rows, D, Di, L.H) * F));
    // split partials of the weight-gradient GEMMs (the largest of the shapes used)
    size_t ws = 0;
    const long long R = (long long)rows;
    const int Hs = L.H ? L.H : D;
    for (int N : {2 * Di, NO, Di, D, 256, Hs})        // weight gradients [N, K] over the rows
        for (int K : {D, Di, L.R, Hs}) ws = std::max(ws, gemm_ws_floats(N, K, R));
    for (int N : {2 * Di, NO, Di, D, 256, L.R, Hs})   // forward and input gradients of few rows
        for (int K : {D, Di, L.R, 2 * Di, NO, 256, Hs}) ws = std::max(ws, gemm_ws_floats((int)R, N, K));
    TCHK(c->gws.ensure(std::max<size_t>(ws, 1) * F));
    c->B = B; c->T = T; c->Tc = Tc;
    return BOA_OK;
}

// Standalone selective scan (autograd binding): B and C packed as [rows][32].
int scan_fwd(const float* x, const float* dt, const float* A_log, const float* bc, const float* Dsk, int B, int T,
             int Di, int Tc, float* y, float* hsave, hipStream_t s, std::string& err) {
    hipLaunchKernelGGL(k_tr_scan_fwd, dim3((Di + SCAN_CH - 1) / SCAN_CH, B), dim3(SCAN_CH), 0, s, x, dt, bc, 2 * NSTATE,
                       0, A_log, Dsk, (const float*)nullptr, B, T, Di, Tc, y, (float*)nullptr, hsave);
    TCHK(hipGetLastError());
    TCHK(hipStreamSynchronize(s));
    return BOA_OK;
}
int scan_bwd(const float* x, const float* dt, const float* A_log, const float* bc, const float* Dsk, const float* dy,
             int B, int T, int Di, int Tc, const float* hsave, float* dx, float* ddt, float* dbc, float* dA_log,
             float* dD, hipStream_t s, std::string& err) {
    const int dblk = (Di + SCAN_CH - 1) / SCAN_CH;
    const long long rows = (long long)B * T;
    Buf hbuf, pbc, pA, pD;
    TCHK(hbuf.alloc((size_t)B * dblk * Tc * NSTATE * SCAN_CH * sizeof(float)));
    TCHK(pbc.alloc((size_t)dblk * rows * 2 * NSTATE * sizeof(float)));
    TCHK(pA.alloc((size_t)B * Di * NSTATE * sizeof(float)));
    TCHK(pD.alloc((size_t)B * Di * sizeof(float)));
    hipLaunchKernelGGL(k_tr_scan_bwd, dim3(dblk, B), dim3(SCAN_CH), 0, s, x, dt, bc, 2 * NSTATE, 0, A_log, Dsk, dy, B,
                       T, Di, Tc, hsave, hbuf.f(), dx, ddt, pbc.f(), pA.f(), pD.f());
    hipLaunchKernelGGL(k_tr_dbc_reduce, dim3(blocks(rows * 2 * NSTATE)), dim3(256), 0, s, pbc.f(), dblk, rows, dbc,
                       2 * NSTATE, 0);
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks((long long)Di * NSTATE)), dim3(256), 0, s, pA.f(), B,
                       (long long)Di * NSTATE, (long long)Di * NSTATE, dA_log, 1);
    hipLaunchKernelGGL(k_sum_slices, dim3(blocks(Di)), dim3(256), 0, s, pD.f(), B, (long long)Di, (long long)Di, dD, 1);
    TCHK(hipGetLastError());
    TCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

// Forward + backward over B sequences of T bytes (device uint8 [B][T]) with
// projections in dtype dt (BOA_DTYPE_F32 or BOA_DTYPE_BF16).  Writes the mean
// loss (nats) to *d_loss and the gradient (flat layout) to grad.
int loss_grad(boa_model* m, const uint8_t* tok, int B, int T, int Tc, int dt_, double* d_loss, float* grad,
              hipStream_t s, std::string& err) {
    const Layout& L = m->lay;
    const int D = L.D, Di = L.Di, R = L.R, NO = R + 2 * NSTATE, Tn = T - 1;
    const long long rows = (long long)B * Tn;
    if (Tc <= 0) Tc = 256;
    const int dt = dt_ == BOA_DTYPE_BF16 ? 1 : 0;
    int rc = train_ensure_buffers(m, B, T, Tc, err);
    if (rc) return rc;
    TrainCtx* c = static_cast<TrainCtx*>(m->train);
    const float* Wt = m->d_w;
    const size_t F = sizeof(float);
    float* ws = c->gws.f();
    float* part = c->part.f();
    // ---------------- forward
    hipLaunchKernelGGL(k_tr_embed, dim3(blocks(rows, 4)), dim3(64, 4), 0, s, tok, B, T, Wt + L.embed, D, c->rcur.f());
    for (int l = 0; l < L.L; ++l) {
        const LayerOff& o = L.layer[l];
        TCHK(hipMemcpyAsync(c->rin[l].p, c->rcur.p, rows * D * F, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_tr_ln_fwd, dim3(blocks(rows, 4)), dim3(64, 4), 0, s, c->rin[l].f(), rows, D,
                           Wt + o.norm_w, Wt + o.norm_b, c->a[l].f(), c->st[l].f());
        TCHK(lin_fwd(dt, c->a[l].f(), D, Wt + o.in_w, 2 * Di, D, c->xz[l].f(), 2 * Di, rows, 0, ws, s));
        hipLaunchKernelGGL(k_tr_conv_fwd, dim3(blocks(rows * Di)), dim3(256), 0, s, c->xz[l].f(), rows, Tn, Di,
                           Wt + o.conv_w, Wt + o.conv_b, c->xc[l].f(), c->xs[l].f());
        TCHK(lin_fwd(dt, c->xs[l].f(), Di, Wt + o.xw, NO, Di, c->dbc[l].f(), NO, rows, 0, ws, s));
        TCHK(lin_fwd(dt, c->dbc[l].f(), NO, Wt + o.dtw, Di, R, c->dtr[l].f(), Di, rows, 0, ws, s));
        hipLaunchKernelGGL(k_tr_bias_softplus, dim3(blocks(rows * Di)), dim3(256), 0, s, c->dtr[l].f(), rows, Di,
                           Wt + o.dtb, c->dt[l].f());
        hipLaunchKernelGGL(k_tr_scan_fwd, dim3((Di + SCAN_CH - 1) / SCAN_CH, B), dim3(SCAN_CH), 0, s, c->xs[l].f(),
                           c->dt[l].f(),
                           c->dbc[l].f(), NO, R, Wt + o.A_log, Wt + o.Dsk, c->xz[l].f(), B, Tn, Di, Tc, c->y[l].f(),
                           c->g[l].f(), c->hs[l].f());
        TCHK(lin_fwd(dt, c->g[l].f(), Di, Wt + o.out_w, D, Di, c->rcur.f(), D, rows, 1, ws, s));
        if (L.H) {            // r <- LayerNorm(W2 GELU(W1 r + b1) + b2)
            const int H = L.H;
            TCHK(hipMemcpyAsync(c->fr[l].p, c->rcur.p, rows * D * F, hipMemcpyDeviceToDevice, s));
            TCHK(lin_fwd(dt, c->fr[l].f(), D, Wt + o.ffn_w1, H, D, c->fu[l].f(), H, rows, 0, ws, s));
            hipLaunchKernelGGL(k_tr_bias_gelu, dim3(blocks(rows * H)), dim3(256), 0, s, c->fu[l].f(), rows, H,
                               Wt + o.ffn_b1, c->fg[l].f());
            TCHK(lin_fwd(dt, c->fg[l].f(), H, Wt + o.ffn_w2, D, H, c->ff[l].f(), D, rows, 0, ws, s));
            hipLaunchKernelGGL(k_tr_add_bias, dim3(blocks(rows * D)), dim3(256), 0, s, c->ff[l].f(), rows, D,
                               Wt + o.ffn_b2);
            hipLaunchKernelGGL(k_tr_ln_fwd, dim3(blocks(rows, 4)), dim3(64, 4), 0, s, c->ff[l].f(), rows, D,
                               Wt + o.ffn_nw, Wt + o.ffn_nb, c->rcur.f(), c->fst[l].f());
        }
    }
    TCHK(hipMemcpyAsync(c->rfin.p, c->rcur.p, rows * D * F, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_tr_ln_fwd, dim3(blocks(rows, 4)), dim3(64, 4), 0, s, c->rfin.f(), rows, D, Wt + L.norm_f_w,
                       Wt + L.norm_f_b, c->rf.f(), c->stf.f());
    TCHK(lin_fwd(dt, c->rf.f(), D, Wt + L.head_w, 256, D, c->logits.f(), 256, rows, 0, ws, s));
    hipLaunchKernelGGL(k_tr_ce, dim3(blocks(rows, 4)), dim3(64, 4), 0, s, c->logits.f(), Wt + L.head_b, tok, B, T,
                       c->rowloss.f(), 1.0f / (float)rows);
    hipLaunchKernelGGL((k_sum_all<float>), dim3(1), dim3(256), 0, s, (const float*)c->rowloss.f(), rows,
                       1.0 / (double)rows, d_loss, (float*)nullptr);
    // ---------------- backward (every gradient region is written exactly once)
    float* G = grad;
    float* dr = c->dr.f();
    float* tmp = c->tmp.f();
    float* t2 = c->t2.f();
    const int dblk = (Di + SCAN_CH - 1) / SCAN_CH;
    TCHK(lin_bwd_w(dt, c->logits.f(), 256, c->rf.f(), D, 256, D, G + L.head_w, rows, ws, s));
    TCHK(colsum(c->logits.f(), rows, 256, 0, 256, part, G + L.head_b, s));
    TCHK(lin_bwd_x(dt, c->logits.f(), 256, Wt + L.head_w, 256, D, tmp, D, rows, 0, ws, s));   // d rf
    hipLaunchKernelGGL(k_tr_ln_bwd, dim3(blocks(rows, 4)), dim3(64, 4), 0, s, tmp, c->rfin.f(), c->stf.f(), rows, D,
                       Wt + L.norm_f_w, dr, 0, t2);
    TCHK(colsum(t2, rows, D, 0, D, part, G + L.norm_f_w, s));
    TCHK(colsum(tmp, rows, D, 0, D, part, G + L.norm_f_b, s));
    for (int l = L.L - 1; l >= 0; --l) {
        const LayerOff& o = L.layer[l];
        if (L.H) {            // through LayerNorm(FFN(r)); no residual around it
            const int H = L.H;
            hipLaunchKernelGGL(k_tr_ln_bwd, dim3(blocks(rows, 4)), dim3(64, 4), 0, s, dr, c->ff[l].f(),
                               c->fst[l].f(), rows, D, Wt + o.ffn_nw, tmp, 0, t2);          // tmp = d f
            TCHK(colsum(t2, rows, D, 0, D, part, G + o.ffn_nw, s));
            TCHK(colsum(dr, rows, D, 0, D, part, G + o.ffn_nb, s));
            TCHK(lin_bwd_w(dt, tmp, D, c->fg[l].f(), H, D, H, G + o.ffn_w2, rows, ws, s));
            TCHK(colsum(tmp, rows, D, 0, D, part, G + o.ffn_b2, s));
            TCHK(lin_bwd_x(dt, tmp, D, Wt + o.ffn_w2, D, H, c->fdu.f(), H, rows, 0, ws, s));   // d GELU
            hipLaunchKernelGGL(k_tr_gelu_bwd, dim3(blocks(rows * H)), dim3(256), 0, s, c->fdu.f(), c->fu[l].f(),
                               rows * H);
            TCHK(lin_bwd_w(dt, c->fdu.f(), H, c->fr[l].f(), D, H, D, G + o.ffn_w1, rows, ws, s));
            TCHK(colsum(c->fdu.f(), rows, H, 0, H, part, G + o.ffn_b1, s));
            TCHK(lin_bwd_x(dt, c->fdu.f(), H, Wt + o.ffn_w1, H, D, dr, D, rows, 0, ws, s));    // d r
        }
        TCHK(lin_bwd_w(dt, dr, D, c->g[l].f(), Di, D, Di, G + o.out_w, rows, ws, s));
        TCHK(lin_bwd_x(dt, dr, D, Wt + o.out_w, D, Di, c->dg.f(), Di, rows, 0, ws, s));
        hipLaunchKernelGGL(k_tr_gate_bwd, dim3(blocks(rows * Di)), dim3(256), 0, s, c->dg.f(), c->y[l].f(),
                           c->xz[l].f(), rows, Di, c->dyb.f(), c->dxz.f());
        hipLaunchKernelGGL(k_tr_scan_bwd, dim3(dblk, B), dim3(SCAN_CH), 0, s, c->xs[l].f(), c->dt[l].f(), c->dbc[l].f(),
                           NO, R, Wt + o.A_log, Wt + o.Dsk, c->dyb.f(), B, Tn, Di, Tc, c->hs[l].f(), c->hbuf.f(),
                           c->dxs.f(), c->ddt.f(), c->pbc.f(), c->pA.f(), c->pD.f());
        hipLaunchKernelGGL(k_tr_dbc_reduce, dim3(blocks(rows * 2 * NSTATE)), dim3(256), 0, s, c->pbc.f(), dblk, rows,
                           c->ddbc.f(), NO, R);
        hipLaunchKernelGGL(k_sum_slices, dim3(blocks((long long)Di * NSTATE)), dim3(256), 0, s, c->pA.f(), B,
                           (long long)Di * NSTATE, (long long)Di * NSTATE, G + o.A_log, 0);
        hipLaunchKernelGGL(k_sum_slices, dim3(blocks(Di)), dim3(256), 0, s, c->pD.f(), B, (long long)Di, (long long)Di,
                           G + o.Dsk, 0);
        hipLaunchKernelGGL(k_tr_softplus_bwd, dim3(blocks(rows * Di)), dim3(256), 0, s, c->ddt.f(), c->dtr[l].f(),
                           rows * Di, c->ddtr.f());
        TCHK(lin_bwd_w(dt, c->ddtr.f(), Di, c->dbc[l].f(), NO, Di, R, G + o.dtw, rows, ws, s));
        TCHK(colsum(c->ddtr.f(), rows, Di, 0, Di, part, G + o.dtb, s));
        TCHK(lin_bwd_x(dt, c->ddtr.f(), Di, Wt + o.dtw, Di, R, c->ddbc.f(), NO, rows, 0, ws, s));   // d delta
        TCHK(lin_bwd_w(dt, c->ddbc.f(), NO, c->xs[l].f(), Di, NO, Di, G + o.xw, rows, ws, s));
        TCHK(lin_bwd_x(dt, c->ddbc.f(), NO, Wt + o.xw, NO, Di, c->dxs.f(), Di, rows, 1, ws, s));  // dxs += ddbc W_x
        hipLaunchKernelGGL(k_tr_conv_bwd_x, dim3(blocks(rows * Di)), dim3(256), 0, s, c->dxs.f(), c->xc[l].f(), rows,
                           Tn, Di, Wt + o.conv_w, c->dxc.f(), c->dxz.f());
        {
            const long long S = row_slices(rows);
            const long long per = (rows + S - 1) / S;
            const long long stride = (long long)Di * (KCONV + 1);
            hipLaunchKernelGGL(k_tr_conv_bwd_w_part, dim3(blocks(Di), (unsigned)S), dim3(256), 0, s, c->dxc.f(),
                               c->xz[l].f(), rows, Tn, Di, per, part);
            hipLaunchKernelGGL(k_sum_slices, dim3(blocks((long long)Di * KCONV)), dim3(256), 0, s, part, (int)S,
                               (long long)Di * KCONV, stride, G + o.conv_w, 0);
            hipLaunchKernelGGL(k_sum_slices, dim3(blocks(Di)), dim3(256), 0, s, part + (long long)Di * KCONV, (int)S,
                               (long long)Di, stride, G + o.conv_b, 0);
        }
        TCHK(lin_bwd_w(dt, c->dxz.f(), 2 * Di, c->a[l].f(), D, 2 * Di, D, G + o.in_w, rows, ws, s));
        TCHK(lin_bwd_x(dt, c->dxz.f(), 2 * Di, Wt + o.in_w, 2 * Di, D, tmp, D, rows, 0, ws, s));   // d a
        hipLaunchKernelGGL(k_tr_ln_bwd, dim3(blocks(rows, 4)), dim3(64, 4), 0, s, tmp, c->rin[l].f(), c->st[l].f(),
                           rows, D, Wt + o.norm_w, dr, 1, t2);
        TCHK(colsum(t2, rows, D, 0, D, part, G + o.norm_w, s));
        TCHK(colsum(tmp, rows, D, 0, D, part, G + o.norm_b, s));
    }
    {
        const long long S = row_slices(rows);
        const long long per = (rows + S - 1) / S;
        hipLaunchKernelGGL(k_tr_embed_bwd_part, dim3(D / 64, (unsigned)S), dim3(64), 0, s, tok, B, T, dr, D, per,
                           part);
        hipLaunchKernelGGL(k_sum_slices, dim3(blocks((long long)VOCAB * D)), dim3(256), 0, s, part, (int)S,
                           (long long)VOCAB * D, (long long)VOCAB * D, G + L.embed, 0);
    }
    TCHK(hipGetLastError());
    TCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

int train_ctx_ensure(boa_model* m, std::string& err) {
    if (m->train) return BOA_OK;
    TrainCtx* c = new TrainCtx;
    const size_t n = m->lay.total * sizeof(float);
    if (c->m.alloc(n) != hipSuccess || c->v.alloc(n) != hipSuccess || c->grad.alloc(n) != hipSuccess ||
        c->sqpart.alloc(1024 * sizeof(float)) != hipSuccess || c->sq.alloc(sizeof(float)) != hipSuccess) {
        delete c;
        err = "optimizer state";
        return BOA_E_OOM;
    }
    if (hipMemset(c->m.p, 0, n) != hipSuccess || hipMemset(c->v.p, 0, n) != hipSuccess) {
        delete c;
        err = "optimizer state";
        return BOA_E_DEVICE;
    }
    m->train = c;
    return BOA_OK;
}

// One AdamW step from the gradient in g (device, flat layout): global norm by
// a fixed tree, clipping, decoupled weight decay, bias-corrected moments.
int optimizer_step(boa_model* m, const float* g, const boa_train_opts& o, float lr, hipStream_t s, std::string& err) {
    int rc = train_ctx_ensure(m, err);
    if (rc) return rc;
    TrainCtx* c = static_cast<TrainCtx*>(m->train);
    const long long n = (long long)m->lay.total;
    const long long per = (n + 1023) / 1024;
    hipLaunchKernelGGL(k_sqsum_part, dim3(1024), dim3(256), 0, s, g, n, per, c->sqpart.f());
    hipLaunchKernelGGL((k_sum_all<float>), dim3(1), dim3(256), 0, s, (const float*)c->sqpart.f(), 1024LL, 1.0,
                       (double*)nullptr, c->sq.f());
    c->step += 1;
    const float bc1 = 1.0f - std::pow(o.beta1, (float)c->step), bc2 = 1.0f - std::pow(o.beta2, (float)c->step);
    hipLaunchKernelGGL(k_adamw, dim3(blocks(n)), dim3(256), 0, s, m->d_w, g, c->m.f(), c->v.f(), n, lr, o.beta1,
                       o.beta2, o.eps, o.weight_decay, bc1, bc2, o.grad_clip, c->sq.f());
    TCHK(hipGetLastError());
    TCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

// One optimisation step on device tokens; *loss gets the mean loss (nats).
int train_step(boa_model* m, const uint8_t* tok, int B, int T, const boa_train_opts& o, float lr, double* d_loss,
               hipStream_t s, std::string& err) {
    int rc = train_ctx_ensure(m, err);
    if (rc) return rc;
    TrainCtx* c = static_cast<TrainCtx*>(m->train);
    rc = loss_grad(m, tok, B, T, (int)o.chunk_t, (int)o.dtype, d_loss, c->grad.f(), s, err);
    if (rc) return rc;
    return optimizer_step(m, c->grad.f(), o, lr, s, err);
}

// ============================================================ C ABI
namespace {
boa_train_opts with_defaults(const boa_train_opts* in) {
    boa_train_opts o{};
    if (in) o = *in;
    if (o.lr <= 0.f) o.lr = 1e-3f;
    if (o.beta1 <= 0.f) o.beta1 = 0.9f;
    if (o.beta2 <= 0.f) o.beta2 = 0.999f;
    if (o.eps <= 0.f) o.eps = 1e-8f;
    if (o.weight_decay < 0.f) o.weight_decay = 0.f;
    if (in == nullptr || (in->weight_decay == 0.f && in->lr == 0.f)) o.weight_decay = 0.01f;
    if (in == nullptr || in->grad_clip == 0.f) o.grad_clip = 1.0f;
    if (o.warmup == 0 && (in == nullptr || in->lr == 0.f)) o.warmup = 100;
    if (o.batch == 0) o.batch = 32;
    if (o.seq_len == 0) o.seq_len = 8192;
    if (o.chunk_t == 0) o.chunk_t = 256;
    return o;
}
float lr_at(const boa_train_opts& o, long long step) {   // step counts from 1
    if (o.warmup == 0 || step >= (long long)o.warmup) return o.lr;
    return o.lr * (float)step / (float)o.warmup;
}
uint64_t splitmix64(uint64_t& x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
bool train_dtype_ok(uint32_t d) { return d == BOA_DTYPE_F32 || d == BOA_DTYPE_BF16; }
uint64_t fnv1a64(const void* data, size_t n, uint64_t h) {
    const uint8_t* p = static_cast<const uint8_t*>(data);
    for (size_t i = 0; i < n; ++i) { h ^= p[i]; h *= 1099511628211ULL; }
    return h;
}
int refresh_after_update(boa_model* m, hipStream_t s) {
    // derived copies (transposed small weights, bf16 and fragment-ordered projections) follow the master weights
    if (launch_prep(m, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return set_error(BOA_E_DEVICE, "refreshing derived weights");
    m->fp_stale = true;
    return BOA_OK;
}
}  // namespace
}  // namespace boa

using namespace boa;

extern "C" int boa_loss_grad_dev(boa_model* m, const uint8_t* d_tokens, uint32_t B, uint32_t T, uint32_t chunk_t,
                                 uint32_t dtype, double* d_loss, float* d_grad, void* stream) {
    if (!m || !d_tokens || !d_loss || !d_grad || B == 0 || T < 2) return set_error(BOA_E_ARG, "bad argument");
    if (!train_dtype_ok(dtype)) return set_error(BOA_E_UNSUPPORTED, "training runs in f32 or bf16");
    std::string err;
    (void)hipSetDevice(m->device);
    int rc = train_ctx_ensure(m, err);
    if (!rc) rc = loss_grad(m, d_tokens, (int)B, (int)T, (int)chunk_t, (int)dtype, d_loss, d_grad, (hipStream_t)stream,
                            err);
    return rc ? set_error(rc, err) : BOA_OK;
}

extern "C" int boa_optimizer_step_dev(boa_model* m, const float* d_grad, const boa_train_opts* opts, void* stream) {
    if (!m || !d_grad) return set_error(BOA_E_ARG, "bad argument");
    std::string err;
    (void)hipSetDevice(m->device);
    boa_train_opts o = with_defaults(opts);
    int rc = train_ctx_ensure(m, err);
    if (rc) return set_error(rc, err);
    TrainCtx* c = static_cast<TrainCtx*>(m->train);
    rc = optimizer_step(m, d_grad, o, lr_at(o, c->step + 1), (hipStream_t)stream, err);
    if (rc) return set_error(rc, err);
    return refresh_after_update(m, (hipStream_t)stream);
}

extern "C" int boa_train_step_dev(boa_model* m, const uint8_t* d_tokens, uint32_t B, uint32_t T,
                                  const boa_train_opts* opts, double* d_loss, void* stream) {
    if (!m || !d_tokens || !d_loss || B == 0 || T < 2) return set_error(BOA_E_ARG, "bad argument");
    boa_train_opts o = with_defaults(opts);
    if (!train_dtype_ok(o.dtype)) return set_error(BOA_E_UNSUPPORTED, "training runs in f32 or bf16");
    std::string err;
    (void)hipSetDevice(m->device);
    int rc = train_ctx_ensure(m, err);
    if (rc) return set_error(rc, err);
    TrainCtx* c = static_cast<TrainCtx*>(m->train);
    rc = train_step(m, d_tokens, (int)B, (int)T, o, lr_at(o, c->step + 1), d_loss, (hipStream_t)stream, err);
    if (rc) return set_error(rc, err);
    return refresh_after_update(m, (hipStream_t)stream);
}

extern "C" int boa_train(boa_model* m, const uint8_t* h_bytes, uint64_t n, const boa_train_opts* opts,
                         float* h_losses, uint64_t n_losses) {
    if (!m || (!h_bytes && n)) return set_error(BOA_E_ARG, "bad argument");
    boa_train_opts o = with_defaults(opts);
    if (!train_dtype_ok(o.dtype)) return set_error(BOA_E_UNSUPPORTED, "training runs in f32 or bf16");
    const uint64_t W = o.seq_len, nwin = W ? n / W : 0;
    if (nwin == 0) return set_error(BOA_E_ARG, "input shorter than one training window");
    const uint32_t B = (uint32_t)std::min<uint64_t>(o.batch, nwin);
    (void)hipSetDevice(m->device);
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return set_error(BOA_E_DEVICE, "stream");
    Buf d_all, d_tok, d_loss;
    if (d_all.alloc(nwin * W) != hipSuccess || d_tok.alloc((size_t)B * W) != hipSuccess ||
        d_loss.alloc(sizeof(double)) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return set_error(BOA_E_OOM, "training buffers");
    }
    if (hipMemcpy(d_all.p, h_bytes, nwin * W, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return set_error(BOA_E_DEVICE, "copying the training bytes");
    }
    std::vector<uint64_t> order(nwin);
    uint64_t rng = o.seed ? o.seed : 1;
    uint64_t pos = nwin;   // forces a shuffle at the first step
    auto next_window = [&]() {
        if (pos >= nwin) {          // new epoch: Fisher-Yates with splitmix64
            for (uint64_t i = 0; i < nwin; ++i) order[i] = i;
            for (uint64_t i = nwin - 1; i > 0; --i) std::swap(order[i], order[splitmix64(rng) % (i + 1)]);
            pos = 0;
        }
        return order[pos++];
    };
    // a model that has already taken steps (a resumed checkpoint) continues
    // the window sequence where those steps left it
    const long long done = m->train ? static_cast<TrainCtx*>(m->train)->step : 0;
    for (long long k = 0; k < done * (long long)B; ++k) (void)next_window();
    int rc = BOA_OK;
    for (uint32_t step = 0; step < o.steps && rc == BOA_OK; ++step) {
        for (uint32_t b = 0; b < B; ++b) {
            const uint64_t w = next_window();
            (void)hipMemcpyAsync(static_cast<uint8_t*>(d_tok.p) + (size_t)b * W,
                                 static_cast<uint8_t*>(d_all.p) + w * W, W, hipMemcpyDeviceToDevice, s);
        }
        rc = boa_train_step_dev(m, static_cast<uint8_t*>(d_tok.p), B, (uint32_t)W, &o,
                                static_cast<double*>(d_loss.p), s);
        if (rc == BOA_OK && h_losses && step < n_losses) {
            double l = 0;
            (void)hipMemcpy(&l, d_loss.p, sizeof(double), hipMemcpyDeviceToHost);
            h_losses[step] = (float)l;
        }
    }
    (void)hipStreamDestroy(s);
    return rc;
}

// Training checkpoint: "BOAT", version 1, config, step count, then the
// float32 master weights, first and second AdamW moments (n each), then an
// FNV-1a hash of everything before it.
extern "C" int boa_train_state_save(const boa_model* m, const char* path) {
    if (!m || !path) return set_error(BOA_E_ARG, "null argument");
    const uint64_t n = m->lay.total;
    std::vector<float> w(n), mo(n, 0.f), vo(n, 0.f);
    int64_t step = 0;
    (void)hipSetDevice(m->device);
    if (hipMemcpy(w.data(), m->d_w, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return set_error(BOA_E_DEVICE, "reading the weights");
    if (m->train) {
        const TrainCtx* c = static_cast<const TrainCtx*>(m->train);
        step = c->step;
        if (hipMemcpy(mo.data(), c->m.p, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(vo.data(), c->v.p, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
            return set_error(BOA_E_DEVICE, "reading the optimiser moments");
    }
    const uint32_t ver = 1;
    uint64_t h = 1469598103934665603ULL;
    h = fnv1a64("BOAT", 4, h);
    h = fnv1a64(&ver, 4, h);
    h = fnv1a64(&m->cfg, sizeof(boa_config), h);
    h = fnv1a64(&step, 8, h);
    h = fnv1a64(w.data(), n * 4, h);
    h = fnv1a64(mo.data(), n * 4, h);
    h = fnv1a64(vo.data(), n * 4, h);
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(BOA_E_ARG, std::string("cannot open ") + path);
    bool ok = std::fwrite("BOAT", 1, 4, f) == 4 && std::fwrite(&ver, 4, 1, f) == 1 &&
              std::fwrite(&m->cfg, sizeof(boa_config), 1, f) == 1 && std::fwrite(&step, 8, 1, f) == 1 &&
              std::fwrite(w.data(), 4, n, f) == n && std::fwrite(mo.data(), 4, n, f) == n &&
              std::fwrite(vo.data(), 4, n, f) == n && std::fwrite(&h, 8, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? BOA_OK : set_error(BOA_E_ARG, "short write");
}

extern "C" int boa_train_state_load(boa_model* m, const char* path) {
    if (!m || !path) return set_error(BOA_E_ARG, "null argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(BOA_E_ARG, std::string("cannot open ") + path);
    const uint64_t n = m->lay.total;
    char mg[4];
    uint32_t ver = 0;
    boa_config cfg{};
    int64_t step = 0;
    std::vector<float> w(n), mo(n), vo(n);
    uint64_t hs = 0;
    bool ok = std::fread(mg, 1, 4, f) == 4 && std::memcmp(mg, "BOAT", 4) == 0 && std::fread(&ver, 4, 1, f) == 1 &&
              ver == 1 && std::fread(&cfg, sizeof(cfg), 1, f) == 1;
    if (!ok) { std::fclose(f); return set_error(BOA_E_FORMAT, "not a BOAT v1 training checkpoint"); }
    if (std::memcmp(&cfg, &m->cfg, sizeof(cfg)) != 0) {
        std::fclose(f);
        return set_error(BOA_E_MODEL, "checkpoint config differs from the model's");
    }
    ok = std::fread(&step, 8, 1, f) == 1 && std::fread(w.data(), 4, n, f) == n && std::fread(mo.data(), 4, n, f) == n &&
         std::fread(vo.data(), 4, n, f) == n && std::fread(&hs, 8, 1, f) == 1;
    std::fclose(f);
    if (!ok || step < 0) return set_error(BOA_E_FORMAT, "truncated training checkpoint");
    uint64_t h = 1469598103934665603ULL;
    h = fnv1a64("BOAT", 4, h);
    h = fnv1a64(&ver, 4, h);
    h = fnv1a64(&cfg, sizeof(cfg), h);
    h = fnv1a64(&step, 8, h);
    h = fnv1a64(w.data(), n * 4, h);
    h = fnv1a64(mo.data(), n * 4, h);
    h = fnv1a64(vo.data(), n * 4, h);
    if (h != hs) return set_error(BOA_E_CORRUPT, "training checkpoint hash mismatch");
    int rc = boa_model_set_weights(m, w.data(), n);
    if (rc) return rc;
    std::string err;
    rc = train_ctx_ensure(m, err);
    if (rc) return set_error(rc, err);
    TrainCtx* c = static_cast<TrainCtx*>(m->train);
    if (hipMemcpy(c->m.p, mo.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->v.p, vo.data(), n * 4, hipMemcpyHostToDevice) != hipSuccess)
        return set_error(BOA_E_DEVICE, "writing the optimiser moments");
    c->step = step;
    return BOA_OK;
}

extern "C" int boa_train_steps_done(const boa_model* m, uint64_t* steps) {
    if (!m || !steps) return set_error(BOA_E_ARG, "null argument");
    *steps = m->train ? (uint64_t)static_cast<const TrainCtx*>(m->train)->step : 0;
    return BOA_OK;
}

extern "C" int boa_scan_fwd_dev(const float* d_x, const float* d_dt, const float* d_A_log, const float* d_bc,
                                const float* d_Dskip, uint32_t B, uint32_t T, uint32_t Di, uint32_t chunk_t,
                                float* d_y, float* d_hsave, void* stream) {
    if (!d_x || !d_dt || !d_A_log || !d_bc || !d_Dskip || !d_y || !d_hsave || B == 0 || T == 0 || Di == 0)
        return set_error(BOA_E_ARG, "bad argument");
    std::string err;
    int rc = scan_fwd(d_x, d_dt, d_A_log, d_bc, d_Dskip, (int)B, (int)T, (int)Di, chunk_t ? (int)chunk_t : 256, d_y,
                      d_hsave, (hipStream_t)stream, err);
    return rc ? set_error(rc, err) : BOA_OK;
}

extern "C" int boa_scan_bwd_dev(const float* d_x, const float* d_dt, const float* d_A_log, const float* d_bc,
                                const float* d_Dskip, const float* d_dy, uint32_t B, uint32_t T, uint32_t Di,
                                uint32_t chunk_t, const float* d_hsave, float* d_dx, float* d_ddt, float* d_dbc,
                                float* d_dA_log, float* d_dDskip, void* stream) {
    if (!d_x || !d_dt || !d_A_log || !d_bc || !d_Dskip || !d_dy || !d_hsave || !d_dx || !d_ddt || !d_dbc ||
        !d_dA_log || !d_dDskip || B == 0 || T == 0 || Di == 0)
        return set_error(BOA_E_ARG, "bad argument");
    std::string err;
    int rc = scan_bwd(d_x, d_dt, d_A_log, d_bc, d_Dskip, d_dy, (int)B, (int)T, (int)Di, chunk_t ? (int)chunk_t : 256,
                      d_hsave, d_dx, d_ddt, d_dbc, d_dA_log, d_dDskip, (hipStream_t)stream, err);
    return rc ? set_error(rc, err) : BOA_OK;
}
