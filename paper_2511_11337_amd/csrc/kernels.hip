// gfx950 kernels of the BOA Constrictor hot path: the byte-level Mamba step
// over many independent streams, the probability -> integer CDF stage and the
// range coder (one integer lane per stream).
//
// Numerics contract (shared by encoder and decoder, so that both build the
// same integer histograms; paper, Range coding: determinism and
// synchronisation).  Every per-element result below depends only on that
// element's inputs, never on the lane count, the lane's slot, the time-tile
// length or the launch shape:
//  * projections (in_proj, out_proj, head, feed-forward): MFMA accumulation
//    over k in increasing steps from zero with the dtype's instruction, then
//    the epilogue (+bias or residual add);
//  * x_proj: f32 MFMA, four chains per output over the k-groups of 16 taken
//    round robin, then (c0 + c1) + (c2 + c3) (xproj_fragment);
//  * LayerNorm statistics and the softmax normaliser: each wave lane sums its
//    strided elements in order, then a fixed xor-butterfly over 64 lanes;
//  * exp(Delta A) = exp2(Delta * (A log2 e)) with the hardware exp2; exp,
//    SiLU and softplus as the hardware-transcendental sequences exp_hp,
//    silu_hp, softplus_hp;
//  * histogram: e_a = exp_hp(l_a - max), p_a = e_a * rcp(Z), then
//    floor(p_a * 2^16), floor at 1, remainder to the lowest-index largest
//    bin; then integer prefix sums (exact).
// The whole library is compiled with -ffp-contract=off, so no implicit
// contraction changes these sequences.
#include "boa_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>

#include "hotpath_common.h"

namespace boa {

// ============================================================== kernel timing
// When a timing bracket is open on this thread, launches go through
// hipExtLaunchKernelGGL, which records the start event when the first kernel
// of the bracket begins and the stop event when the last one ends (GPU
// timestamps, no host gaps).
thread_local hipEvent_t t_prof_start = nullptr, t_prof_stop = nullptr;
thread_local bool t_prof_first = false;
void prof_open(hipEvent_t a, hipEvent_t b) { t_prof_start = a; t_prof_stop = b; t_prof_first = true; }
void prof_close() { t_prof_start = t_prof_stop = nullptr; }

// ============================================================== prep
// Derived tensors: conv weight and dt_proj transposed to [.., Di], and
// A2 = -exp(A_log) * log2(e) transposed to [N, Di]; bf16 copies of the big
// projections.
__global__ void k_prep_layer(const float* __restrict__ conv_w, const float* __restrict__ dtw,
                             const float* __restrict__ A_log, int Di, int R, float* __restrict__ convT,
                             float* __restrict__ dtwT, float* __restrict__ A2T) {
    int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= Di) return;
    for (int k = 0; k < KCONV; ++k) convT[k * Di + d] = conv_w[d * KCONV + k];
    for (int r = 0; r < R; ++r) dtwT[r * Di + d] = dtw[d * R + r];
    for (int n = 0; n < NSTATE; ++n)
        A2T[n * Di + d] = -expf(A_log[d * NSTATE + n]) * 1.4426950408889634f;
}
// BF16-mode copies of a float tensor: the values rounded to bf16 (nearest
// even) as floats (rf, may be null) and as bf16 bits (h, may be null)
__global__ void k_round_bf16(const float* __restrict__ src, long long n, float* __restrict__ rf,
                             uint16_t* __restrict__ h) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint16_t b = f2bf_bits(src[i]);
    if (rf) rf[i] = bf16_bits_to_f(b);
    if (h) h[i] = b;
}
__global__ void k_to_bf16(const float* __restrict__ src, long long n, uint16_t* __restrict__ dst) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        __hip_bfloat16 b = __float2bfloat16(src[i]);
        dst[i] = *reinterpret_cast<uint16_t*>(&b);
    }
}

hipError_t launch_prep(const boa_model* m, hipStream_t s) {
    const Layout& L = m->lay;
    for (int l = 0; l < L.L; ++l) {
        const LayerOff& o = L.layer[l];
        const LayerDev& w = m->ld[l];
        hipLaunchKernelGGL(k_prep_layer, dim3((L.Di + 255) / 256), dim3(256), 0, s, m->d_w + o.conv_w,
                           m->d_w + o.dtw, m->d_w + o.A_log, L.Di, L.R, const_cast<float*>(w.convT),
                           const_cast<float*>(w.dtwT), const_cast<float*>(w.A2T));
        const int NO = L.R + 2 * L.N;
        {
            const long long nx = (long long)NO * L.Di, nd = (long long)L.R * L.Di;
            const dim3 bx((unsigned)((nx + 255) / 256)), bd((unsigned)((nd + 255) / 256));
            hipLaunchKernelGGL(k_round_bf16, bx, dim3(256), 0, s, m->d_w + o.xw, nx, const_cast<float*>(w.xw_r),
                               (uint16_t*)nullptr);
            hipLaunchKernelGGL(k_round_bf16, bd, dim3(256), 0, s, w.dtwT, nd, const_cast<float*>(w.dtwT_r),
                               (uint16_t*)nullptr);
            hipLaunchKernelGGL(k_round_bf16, bd, dim3(256), 0, s, m->d_w + o.dtw, nd, (float*)nullptr,
                               const_cast<uint16_t*>(w.dtw16));
            const int NOP = (NO + 15) / 16 * 16;
            hipError_t ef = launch_frag_pad(m->d_w + o.xw, NO, NOP, L.Di, const_cast<float*>(w.xwF), s);
            if (ef == hipSuccess) ef = launch_frag_pad(w.xw_r, NO, NOP, L.Di, const_cast<float*>(w.xwF_r), s);
            if (ef != hipSuccess) return ef;
        }
        long long n1 = 2LL * L.Di * L.D, n2 = (long long)L.D * L.Di;
        hipLaunchKernelGGL(k_to_bf16, dim3((n1 + 255) / 256), dim3(256), 0, s, m->d_w + o.in_w, n1,
                           const_cast<uint16_t*>(w.in_w16));
        hipLaunchKernelGGL(k_to_bf16, dim3((n2 + 255) / 256), dim3(256), 0, s, m->d_w + o.out_w, n2,
                           const_cast<uint16_t*>(w.out_w16));
        const int mpl = L.H ? 4 : 2;            // projection matrices per layer
        hipError_t e = launch_frag(m->d_w + o.in_w, 2 * L.Di, L.D, const_cast<float*>(w.in_f32f),
                                   const_cast<uint16_t*>(w.in_b16f), const_cast<uint8_t*>(w.in_f8f),
                                   m->d_amax + mpl * l, const_cast<int*>(w.in_ew), s);
        if (e != hipSuccess) return e;
        e = launch_frag(m->d_w + o.out_w, L.D, L.Di, const_cast<float*>(w.out_f32f),
                        const_cast<uint16_t*>(w.out_b16f), const_cast<uint8_t*>(w.out_f8f), m->d_amax + mpl * l + 1,
                        const_cast<int*>(w.out_ew), s);
        if (e != hipSuccess) return e;
        if (L.H) {                              // feed-forward W1 [H, D] and W2 [D, H]
            const long long nh = (long long)L.H * L.D;
            hipLaunchKernelGGL(k_to_bf16, dim3((nh + 255) / 256), dim3(256), 0, s, w.w1, nh,
                               const_cast<uint16_t*>(w.w1_16));
            hipLaunchKernelGGL(k_to_bf16, dim3((nh + 255) / 256), dim3(256), 0, s, w.w2, nh,
                               const_cast<uint16_t*>(w.w2_16));
            e = launch_frag(w.w1, L.H, L.D, const_cast<float*>(w.w1_f32f), const_cast<uint16_t*>(w.w1_b16f),
                            const_cast<uint8_t*>(w.w1_f8f), m->d_amax + mpl * l + 2, const_cast<int*>(w.w1_ew), s);
            if (e != hipSuccess) return e;
            e = launch_frag(w.w2, L.D, L.H, const_cast<float*>(w.w2_f32f), const_cast<uint16_t*>(w.w2_b16f),
                            const_cast<uint8_t*>(w.w2_f8f), m->d_amax + mpl * l + 3, const_cast<int*>(w.w2_ew), s);
            if (e != hipSuccess) return e;
        }
    }
    {
        hipError_t e = launch_frag(m->d_w + L.head_w, 256, L.D, const_cast<float*>(m->head_f32f),
                                   const_cast<uint16_t*>(m->head_b16f), const_cast<uint8_t*>(m->head_f8f),
                                   m->d_amax + (L.H ? 4 : 2) * L.L, const_cast<int*>(m->head_ew), s);
        if (e != hipSuccess) return e;
    }
    long long nh = 256LL * L.D;
    hipLaunchKernelGGL(k_to_bf16, dim3((nh + 255) / 256), dim3(256), 0, s, m->d_w + L.head_w, nh,
                       const_cast<uint16_t*>(m->head_w16));
    return hipGetLastError();
}

// ============================================================== schedule
// Row (lane, t) of a time tile runs global step step0 + t of that lane.  The
// lane's entries (chunk, first step) are sorted by first step; the chunk
// occupies chunk_steps = len - 1 steps.  pos = -1 marks an idle row.
__global__ void k_rowinfo(Plan p, int lanes, int T, long long step0, const long long* __restrict__ d_step,
                          int* __restrict__ row_chunk, int* __restrict__ row_pos) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= lanes * T) return;
    int lane = i / T, t = i % T;
    long long s = step0 + t + (d_step ? *d_step : 0LL);
    int c, pos;
    locate(p, lane, s, c, pos);
    row_chunk[i] = c;
    row_pos[i] = pos;
}
hipError_t launch_rowinfo(const Plan& p, int lanes, int T, long long step0, const long long* d_step,
                          int* row_chunk, int* row_pos, hipStream_t s) {
    int n = lanes * T;
    hipLaunchKernelGGL(k_rowinfo, dim3((n + 255) / 256), dim3(256), 0, s, p, lanes, T, step0, d_step,
                       row_chunk, row_pos);
    return hipGetLastError();
}

// ============================================================== embedding
// Locate each row's (chunk, pos) in the lane schedule and gather r = E[y_t]
// (Models: embedding layer); one wave per row, 16 bytes per lane (an idle row
// is zero).  D is a multiple of 4.
__global__ void k_embed(const float* __restrict__ E, const uint8_t* __restrict__ bytes, Plan p, int lanes, int T,
                        long long step0, const long long* __restrict__ d_step, int D,
                        int* __restrict__ row_chunk, int* __restrict__ row_pos, float* __restrict__ r) {
    int row = blockIdx.x * 4 + threadIdx.y;
    if (row >= lanes * T) return;
    int lane = row / T, t = row % T;
    long long step = step0 + t + (d_step ? *d_step : 0LL);
    int c, pos;
    locate(p, lane, step, c, pos);
    if (threadIdx.x == 0) { row_chunk[row] = c; row_pos[row] = pos; }
    float4* dst = reinterpret_cast<float4*>(r + (long long)row * D);
    if (pos < 0) {
        for (int k = threadIdx.x; k < D / 4; k += 64) dst[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    int y = bytes[p.chunk_off[c] + pos];
    const float4* src = reinterpret_cast<const float4*>(E + (long long)y * D);
    for (int k = threadIdx.x; k < D / 4; k += 64) dst[k] = src[k];
}
hipError_t launch_embed(const float* E, const uint8_t* bytes, const Plan& p, int lanes, int T, long long step0,
                        const long long* d_step, int D, int* row_chunk, int* row_pos, float* r, hipStream_t s) {
    if (D % 4) return hipErrorInvalidValue;
    int M = lanes * T;
    BOA_LAUNCH(k_embed, dim3((M + 3) / 4), dim3(64, 4), 0, s, E, bytes, p, lanes, T, step0, d_step, D,
                       row_chunk, row_pos, r);
    return hipGetLastError();
}

// ============================================================== MFMA GEMM
// C[M,N] = epi(A'[M,K] . W[N,K]^T) on the matrix cores.  With LNA, A' =
// LayerNorm(A): the workgroup stages its BM full rows of A in LDS, takes the
// row statistics with ln_stats (fixed reduction order), normalises and rounds
// them to the compute dtype in place; otherwise A is streamed with W.  Every
// output element is the same MFMA accumulation sequence over k whatever the
// tile shape, M, or the row's slot in the tile:
//   f32 : v_mfma_f32_16x16x4_f32, k in steps of 4, increasing;
//   bf16: v_mfma_f32_16x16x32_bf16, k in steps of 32, increasing;
// starting from zero; then the epilogue: 0 store, 1 + bias[n], 2 C += result.
template <int DT, int EPI, bool LNA, int BM, int BN, int WM, int WN, int KT>
__global__ __launch_bounds__(256) void k_mgemm(const float* __restrict__ A, int M, int Kr,
                                               const float* __restrict__ W32,
                                               const uint16_t* __restrict__ W16, int N,
                                               float* __restrict__ C, const float* __restrict__ ln_w,
                                               const float* __restrict__ ln_b,
                                               const float* __restrict__ bias) {
    // KT > 0: K = KT, and the whole K extent is one tile (every global load of
    // the workgroup is issued in one batch: the small-M decoder shapes);
    // KT == 0: runtime K streamed in tiles of 32 with one tile of prefetch.
    constexpr int NT = 256;
    constexpr int BK = KT > 0 ? KT : 32;
    const int K = KT > 0 ? KT : Kr;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    static_assert(FM * 16 * WM == BM && FN * 16 * WN == BN && WM * WN <= 4, "tile");
    constexpr int ES = DT == 0 ? 4 : 2;                 // element size in LDS
    constexpr int RS = DT == 0 ? BK + 4 : BK + 8;       // streamed-tile row stride (elements)
    extern __shared__ __align__(16) unsigned char smem[];
    // LNA: normalised A resident in f32 as [BM][K + 4] (rounded to the dtype
    // when MFMA fragments are built); else A streamed with W as [BM][RS]
    const size_t a_bytes = LNA ? (size_t)BM * (K + 4) * 4 : (size_t)BM * RS * ES;
    unsigned char* As = smem;
    unsigned char* Ws = smem + a_bytes;
    __shared__ float mu_s[BM], rs_s[BM];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const bool computes = wv < WM * WN;
    const int wm = wv / WN, wn = wv % WN;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;

    constexpr int AV = LNA ? 0 : (BM * BK / 4 + NT - 1) / NT;   // float4 per thread for streamed A
    constexpr int WVV = DT == 0 ? (BN * BK / 4 + NT - 1) / NT : (BN * BK / 8 + NT - 1) / NT;
    float4 ra[AV > 0 ? AV : 1];
    uint4 rw[WVV];
    auto load_tile = [&](int k0) {
#pragma unroll
        for (int i = 0; i < AV; ++i) {
            int it = tid + i * NT;
            int r = it / (BK / 4), k = (it % (BK / 4)) * 4;
            int row = m0 + r;
            ra[i] = (it < BM * BK / 4 && row < M)
                        ? *reinterpret_cast<const float4*>(A + (long long)row * K + k0 + k)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int i = 0; i < WVV; ++i) {
            int it = tid + i * NT;
            if (DT == 0) {
                int r = it / (BK / 4), k = (it % (BK / 4)) * 4;
                int n = n0 + r;
                rw[i] = (it < BN * BK / 4 && n < N)
                            ? *reinterpret_cast<const uint4*>(W32 + (long long)n * K + k0 + k)
                            : make_uint4(0, 0, 0, 0);
            } else {
                int r = it / (BK / 8), k = (it % (BK / 8)) * 8;
                int n = n0 + r;
                rw[i] = (it < BN * BK / 8 && n < N)
                            ? *reinterpret_cast<const uint4*>(W16 + (long long)n * K + k0 + k)
                            : make_uint4(0, 0, 0, 0);
            }
        }
    };
    auto store_tile = [&]() {
#pragma unroll
        for (int i = 0; i < AV; ++i) {
            int it = tid + i * NT;
            if (it >= BM * BK / 4) break;
            int r = it / (BK / 4), k = (it % (BK / 4)) * 4;
            if (DT == 0) {
                *reinterpret_cast<float4*>(As + (r * RS + k) * 4) = ra[i];
            } else {
                uint2 u;
                u.x = (uint32_t)f2bf_bits(ra[i].x) | ((uint32_t)f2bf_bits(ra[i].y) << 16);
                u.y = (uint32_t)f2bf_bits(ra[i].z) | ((uint32_t)f2bf_bits(ra[i].w) << 16);
                *reinterpret_cast<uint2*>(As + (r * RS + k) * 2) = u;
            }
        }
#pragma unroll
        for (int i = 0; i < WVV; ++i) {
            int it = tid + i * NT;
            if (DT == 0) {
                if (it >= BN * BK / 4) break;
                int r = it / (BK / 4), k = (it % (BK / 4)) * 4;
                *reinterpret_cast<uint4*>(Ws + (r * RS + k) * 4) = rw[i];
            } else {
                if (it >= BN * BK / 8) break;
                int r = it / (BK / 8), k = (it % (BK / 8)) * 8;
                *reinterpret_cast<uint4*>(Ws + (r * RS + k) * 2) = rw[i];
            }
        }
    };

    load_tile(0);                // W (and streamed A) of the first tile in flight during the LayerNorm phase
    if (LNA) {
        // stage BM rows (f32), statistics, normalise in place
        float* Af = reinterpret_cast<float*>(As);
        if (KT > 0) {
            constexpr int NV = (BM * (KT > 0 ? KT : 4) / 4 + NT - 1) / NT;
            float4 v[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                int it = tid + i * NT;
                int r = it / (K / 4), k = (it % (K / 4)) * 4;
                int row = m0 + r;
                v[i] = (it < BM * K / 4 && row < M) ? *reinterpret_cast<const float4*>(A + (long long)row * K + k)
                                                    : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                int it = tid + i * NT;
                if (it < BM * K / 4) {
                    int r = it / (K / 4), k = (it % (K / 4)) * 4;
                    *reinterpret_cast<float4*>(Af + r * (K + 4) + k) = v[i];
                }
            }
        } else {
            const int K4 = K / 4;
            for (int it = tid; it < BM * K4; it += NT) {
                int r = it / K4, k = (it % K4) * 4;
                int row = m0 + r;
                float4 v = row < M ? *reinterpret_cast<const float4*>(A + (long long)row * K + k)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
                *reinterpret_cast<float4*>(Af + r * (K + 4) + k) = v;
            }
        }
        __syncthreads();
        for (int rr = wv; rr < BM; rr += NT / 64) {
            float mu, rs;
            ln_stats(Af + rr * (K + 4), K, lane, mu, rs);
            if (lane == 0) { mu_s[rr] = mu; rs_s[rr] = rs; }
        }
        __syncthreads();
        if (K >= NT) {                       // each thread owns columns tid, tid + NT, ...
            for (int k = tid; k < K; k += NT) {
                const float gw = ln_w[k], gb = ln_b[k];
                for (int r = 0; r < BM; ++r) {
                    float a = ln_apply(Af[r * (K + 4) + k], mu_s[r], rs_s[r], gw, gb);
                    Af[r * (K + 4) + k] = (m0 + r < M) ? a : 0.0f;
                }
            }
        } else {                             // column tid % K, rows tid / K + j * (NT / K)
            const int k = tid % K;
            const float gw = ln_w[k], gb = ln_b[k];
            for (int r = tid / K; r < BM; r += NT / K) {
                float a = ln_apply(Af[r * (K + 4) + k], mu_s[r], rs_s[r], gw, gb);
                Af[r * (K + 4) + k] = (m0 + r < M) ? a : 0.0f;
            }
        }
        __syncthreads();
    }

    v4f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    const int li = lane & 15, lk = lane >> 4;
    const int ars = LNA ? K + 4 : RS;                           // A row stride, elements
    for (int k0 = 0; k0 < K; k0 += BK) {
        store_tile();
        __syncthreads();
        if (k0 + BK < K) load_tile(k0 + BK);
        const int ak = LNA ? k0 : 0;                                 // column offset of this tile in A
        if (computes) {
            if (DT == 0) {
                const float* Af = reinterpret_cast<const float*>(As);
                const float* Wf = reinterpret_cast<const float*>(Ws);
#pragma unroll 8
                for (int ks = 0; ks < BK; ks += 4) {
                    float af[FM], bf[FN];
#pragma unroll
                    for (int i = 0; i < FM; ++i) af[i] = Af[(wm * TM + i * 16 + li) * ars + ak + ks + lk];
#pragma unroll
                    for (int j = 0; j < FN; ++j) bf[j] = Wf[(wn * TN + j * 16 + li) * RS + ks + lk];
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
                }
            } else {
                const uint16_t* Ah = reinterpret_cast<const uint16_t*>(As);
                const uint16_t* Wh = reinterpret_cast<const uint16_t*>(Ws);
#pragma unroll 4
                for (int ks = 0; ks < BK; ks += 32) {
                    v8bf af[FM], bfr[FN];
#pragma unroll
                    for (int i = 0; i < FM; ++i) {
                        if (LNA) {
                            const float* src = reinterpret_cast<const float*>(As) +
                                               (wm * TM + i * 16 + li) * ars + ak + ks + 8 * lk;
                            float4 x0 = *reinterpret_cast<const float4*>(src);
                            float4 x1 = *reinterpret_cast<const float4*>(src + 4);
                            uint4 u;
                            u.x = (uint32_t)f2bf_bits(x0.x) | ((uint32_t)f2bf_bits(x0.y) << 16);
                            u.y = (uint32_t)f2bf_bits(x0.z) | ((uint32_t)f2bf_bits(x0.w) << 16);
                            u.z = (uint32_t)f2bf_bits(x1.x) | ((uint32_t)f2bf_bits(x1.y) << 16);
                            u.w = (uint32_t)f2bf_bits(x1.z) | ((uint32_t)f2bf_bits(x1.w) << 16);
                            af[i] = *reinterpret_cast<const v8bf*>(&u);
                        } else {
                            af[i] = *reinterpret_cast<const v8bf*>(Ah + (wm * TM + i * 16 + li) * ars + ks + 8 * lk);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        bfr[j] = *reinterpret_cast<const v8bf*>(Wh + (wn * TN + j * 16 + li) * RS + ks + 8 * lk);
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    if (!computes) return;

    // epilogue; lane holds rows 4*lk + r of each 16x16 tile, column li
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = m0 + wm * TM + i * 16 + 4 * lk + r;
                int n = n0 + wn * TN + j * 16 + li;
                if (row < M && n < N) {
                    float* dst = C + (long long)row * N + n;
                    float v = acc[i][j][r];
                    if (EPI == 1) v = v + bias[n];
                    if (EPI == 2) v = *dst + v;
                    if (EPI == 3) v = gelu_f(v + bias[n]);
                    *dst = v;
                }
            }
}

template <int DT, int EPI, bool LNA, int BM, int BN, int WM, int WN, int KT>
hipError_t mgemm_launch(const float* A, int M, int K, const float* W32, const uint16_t* W16, int N, float* C,
                        const float* ln_w, const float* ln_b, const float* bias, hipStream_t s) {
    constexpr int ES = DT == 0 ? 4 : 2;
    constexpr int BK = KT > 0 ? KT : 32;
    constexpr int RS = DT == 0 ? BK + 4 : BK + 8;
    size_t a_bytes = LNA ? (size_t)BM * (K + 4) * 4 : (size_t)BM * RS * ES;
    size_t lds = a_bytes + (size_t)BN * RS * ES;
    auto kern = k_mgemm<DT, EPI, LNA, BM, BN, WM, WN, KT>;
    if (lds > 65536) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
    BOA_LAUNCH(kern, grid, dim3(256), lds, s, A, M, K, W32, W16, N, C, ln_w, ln_b, bias);
    return hipGetLastError();
}

// Row-block GEMM for many rows (the encoder's tiles): a workgroup owns BM
// rows and every output column.  Its A rows are staged in LDS once --
// LayerNorm'd when LNA (ln_stats on the row, ln_apply per element) and rounded
// to the compute dtype -- and the B operand streams from the fragment-ordered
// weight copy straight into registers, one KiB per wave per load, with one
// k step of prefetch.  Wave w computes the column groups w, w + 4, ... of
// FN = 4 fragments for all BM rows.  Per output element the MFMA sequence,
// the A rounding and the epilogue are those of k_mgemm.
// DT 2 (fp8): each staged row is scaled by its own power of two 2^-ea (ea from
// the row's largest magnitude, fp8_exp) and rounded to E4M3; B is the fp8
// fragment copy with per-tensor exponent *ew; the accumulator is rescaled
// exactly by 2^(ea + ew) before the epilogue.  MFMA 16x16x32 fp8 in k steps of
// 32 from zero.
template <int DT, int EPI, bool LNA, int K, int BM, bool A16 = false>
__global__ __launch_bounds__(256) void k_rowgemm(const float* __restrict__ A, int M, const void* __restrict__ Wf,
                                                 int N, float* __restrict__ C, const float* __restrict__ ln_w,
                                                 const float* __restrict__ ln_b, const float* __restrict__ bias,
                                                 const int* __restrict__ ew) {
    constexpr int FM = BM / 16, FN = 4;
    constexpr int AS = DT == 0 ? K + 4 : (DT == 1 ? K + 8 : K + 16);   // LDS row stride (elements)
    extern __shared__ __align__(16) unsigned char smem[];
    float* Af = reinterpret_cast<float*>(smem);
    uint16_t* Ah = reinterpret_cast<uint16_t*>(smem);
    uint8_t* A8 = reinterpret_cast<uint8_t*>(smem);
    __shared__ int ea_s[DT == 2 ? BM : 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m0 = blockIdx.x * BM;

    constexpr int RPW = BM / 4, NV = K / 64;
    if constexpr (A16) {
        // A is already bf16 bits (the gated rows as the mixer wrote them):
        // the rows are copied into LDS 16 bytes per lane
        static_assert(DT == 1 && !LNA, "bf16 rows: BF16 products without LayerNorm");
        const uint16_t* A16p = reinterpret_cast<const uint16_t*>(A);
        uint4 q[RPW][(K / 8 + 63) / 64];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int row = m0 + wv + 4 * i;
#pragma unroll
            for (int c = 0; c < (K / 8 + 63) / 64; ++c) {
                const int cc = lane + 64 * c;
                q[i][c] = make_uint4(0u, 0u, 0u, 0u);
                if (row < M && cc < K / 8) q[i][c] = *reinterpret_cast<const uint4*>(A16p + (long long)row * K + 8 * cc);
            }
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = wv + 4 * i;
#pragma unroll
            for (int c = 0; c < (K / 8 + 63) / 64; ++c) {
                const int cc = lane + 64 * c;
                if (cc < K / 8) *reinterpret_cast<uint4*>(Ah + r * AS + 8 * cc) = q[i][c];
            }
        }
    } else {
    // wave wv stages rows wv, wv + 4, ...: all of them are fetched first (one
    // memory latency), then normalised from registers
    float v[RPW][NV];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int row = m0 + wv + 4 * i;
#pragma unroll
        for (int j = 0; j < NV; ++j) v[i][j] = row < M ? A[(long long)row * K + lane + 64 * j] : 0.0f;
    }
    float gw[NV], gb[NV];
    if (LNA) {
#pragma unroll
        for (int j = 0; j < NV; ++j) { gw[j] = ln_w[lane + 64 * j]; gb[j] = ln_b[lane + 64 * j]; }
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int r = wv + 4 * i;
        const bool ok = m0 + r < M;
        float mu = 0.0f, rs = 1.0f;
        if (LNA) ln_stats_v<NV>(v[i], K, mu, rs);
        float x[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            x[j] = v[i][j];
            if (LNA) x[j] = ok ? ln_apply(x[j], mu, rs, gw[j], gb[j]) : 0.0f;
        }
        if (DT == 2) {
            float am = 0.0f;
#pragma unroll
            for (int j = 0; j < NV; ++j) am = fmaxf(am, fabsf(x[j]));
            const int ea = fp8_exp(wave_max(am));
            if (lane == 0) ea_s[r] = ea;
#pragma unroll
            for (int j = 0; j < NV; ++j) A8[r * AS + lane + 64 * j] = fp8_byte(ldexpf(x[j], -ea));
        } else {
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const int k = lane + 64 * j;
                if (DT == 0) Af[r * AS + k] = x[j];
                else Ah[r * AS + k] = f2bf_bits(x[j]);
            }
        }
    }
    }
    __syncthreads();

    const int li = lane & 15, lk = lane >> 4;
    const int NF = N / 16;
    const int ew0 = DT == 2 ? *ew : 0;
    for (int nf0 = wv * FN; nf0 < NF; nf0 += 4 * FN) {
        v4f acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
        if (DT == 0) {
            constexpr int Q = K / 16;
            const float4* W4 = reinterpret_cast<const float4*>(Wf) + (long long)nf0 * Q * 64 + lane;
            float4 bc[FN], bn[FN];
#pragma unroll
            for (int j = 0; j < FN; ++j) bc[j] = W4[(long long)j * Q * 64];
#pragma unroll 1
            for (int q = 0; q < Q; ++q) {
                if (q + 1 < Q) {
#pragma unroll
                    for (int j = 0; j < FN; ++j) bn[j] = W4[((long long)j * Q + q + 1) * 64];
                }
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    float af[FM];
#pragma unroll
                    for (int i = 0; i < FM; ++i) af[i] = Af[(i * 16 + li) * AS + 16 * q + 4 * jj + lk];
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        const float b = jj == 0 ? bc[j].x : jj == 1 ? bc[j].y : jj == 2 ? bc[j].z : bc[j].w;
#pragma unroll
                        for (int i = 0; i < FM; ++i)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], b, acc[i][j], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) bc[j] = bn[j];
            }
        } else if (DT == 2) {
            constexpr int SP = K / 64;                   // pairs of k steps (one uint4 per lane)
            const uint4* W8 = reinterpret_cast<const uint4*>(Wf) + (long long)nf0 * SP * 64 + lane;
            uint4 bc[FN], bn[FN];
#pragma unroll
            for (int j = 0; j < FN; ++j) bc[j] = W8[(long long)j * SP * 64];
#pragma unroll 1
            for (int p = 0; p < SP; ++p) {
                if (p + 1 < SP) {
#pragma unroll
                    for (int j = 0; j < FN; ++j) bn[j] = W8[((long long)j * SP + p + 1) * 64];
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    long af[FM];
#pragma unroll
                    for (int i = 0; i < FM; ++i)
                        af[i] = *reinterpret_cast<const long*>(A8 + (i * 16 + li) * AS + 32 * (2 * p + h) + 8 * lk);
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        const long b = h == 0 ? (long)((uint64_t)bc[j].x | ((uint64_t)bc[j].y << 32))
                                              : (long)((uint64_t)bc[j].z | ((uint64_t)bc[j].w << 32));
#pragma unroll
                        for (int i = 0; i < FM; ++i)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(af[i], b, acc[i][j], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) bc[j] = bn[j];
            }
        } else {
            constexpr int S = K / 32;
            const uint4* W8 = reinterpret_cast<const uint4*>(Wf) + (long long)nf0 * S * 64 + lane;
            uint4 bc[FN], bn[FN];
#pragma unroll
            for (int j = 0; j < FN; ++j) bc[j] = W8[(long long)j * S * 64];
#pragma unroll 1
            for (int s = 0; s < S; ++s) {
                if (s + 1 < S) {
#pragma unroll
                    for (int j = 0; j < FN; ++j) bn[j] = W8[((long long)j * S + s + 1) * 64];
                }
                v8bf af[FM];
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    af[i] = *reinterpret_cast<const v8bf*>(Ah + (i * 16 + li) * AS + 32 * s + 8 * lk);
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            af[i], *reinterpret_cast<const v8bf*>(&bc[j]), acc[i][j], 0, 0, 0);
#pragma unroll
                for (int j = 0; j < FN; ++j) bc[j] = bn[j];
            }
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int row = m0 + i * 16 + 4 * lk + rr;
                    const int n = (nf0 + j) * 16 + li;
                    if (row < M) {
                        float* dst = C + (long long)row * N + n;
                        float v = acc[i][j][rr];
                        if (DT == 2) v = ldexpf(v, ea_s[i * 16 + 4 * lk + rr] + ew0);
                        if (EPI == 1) v = v + bias[n];
                        if (EPI == 2) v = *dst + v;
                        if (EPI == 3) v = gelu_f(v + bias[n]);
                        *dst = v;
                    }
                }
    }
}

template <int DT, int EPI, bool LNA, int K, bool A16 = false>
hipError_t rowgemm_launch(const float* A, int M, const void* Wf, int N, float* C, const float* ln_w,
                          const float* ln_b, const float* bias, const int* ew, hipStream_t s) {
    // rows per workgroup: the LDS tile and the staging registers bound the
    // workgroups per CU, which this memory-bound kernel needs more than the
    // weight reuse of taller tiles (BF16 at K = 512 from f32 rows: 16 rows
    // measured 11 % faster than 32, and 64 rows 60 % slower; from bf16 rows,
    // whose staging needs half the registers, 32 rows 20 % faster than 16 and
    // than 64; the BF16 head, 256 columns: 32 rows 21 % faster than 64, where
    // the in_proj's 1024 columns want 64)
    constexpr bool HEAD16 = DT == 1 && EPI == 1 && LNA && K <= 256;
    constexpr int BM = A16 ? 32 : K <= 256 ? (HEAD16 ? 32 : 64) : (K == 512 ? (DT == 1 ? 16 : 32) : 16);
    constexpr int AS = DT == 0 ? K + 4 : (DT == 1 ? K + 8 : K + 16);
    const size_t lds = (size_t)BM * AS * (DT == 0 ? 4 : (DT == 1 ? 2 : 1));
    auto kern = k_rowgemm<DT, EPI, LNA, K, BM, A16>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    BOA_LAUNCH(kern, dim3((M + BM - 1) / BM), dim3(256), lds, s, A, M, Wf, N, C, ln_w, ln_b, bias, ew);
    return hipGetLastError();
}

hipError_t launch_rowgemm(int dtype, int kind, const float* A, int M, int K, const void* Wf, int N, float* C,
                          const float* ln_w, const float* ln_b, const float* bias, const int* ew, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    if (N % 64) return hipErrorInvalidValue;
    if (dtype == BOA_DTYPE_FP8 && !ew) return hipErrorInvalidValue;
#define RG(DTV, EPIV, LNV, KV) \
    if (K == KV) return rowgemm_launch<DTV, EPIV, LNV, KV>(A, M, Wf, N, C, ln_w, ln_b, bias, ew, s);
#define RG_K(DTV, EPIV, LNV) RG(DTV, EPIV, LNV, 64) RG(DTV, EPIV, LNV, 128) RG(DTV, EPIV, LNV, 256) \
    RG(DTV, EPIV, LNV, 512) RG(DTV, EPIV, LNV, 1024)
    if (dtype == BOA_DTYPE_FP8) {
        if (kind == 0) { RG_K(2, 0, true) }
        if (kind == 1) { RG_K(2, 1, true) }
        if (kind == 2) { RG_K(2, 2, false) }
        if (kind == 3) { RG_K(2, 3, false) }
        if (kind == 4) { RG_K(2, 1, false) }
    } else if (dtype == BOA_DTYPE_BF16) {
        if (kind == 0) { RG_K(1, 0, true) }
        if (kind == 1) { RG_K(1, 1, true) }
        if (kind == 2) { RG_K(1, 2, false) }
        if (kind == 3) { RG_K(1, 3, false) }
        if (kind == 4) { RG_K(1, 1, false) }
        if (kind == 5) {
            if (K == 512) return rowgemm_launch<1, 2, false, 512, true>(A, M, Wf, N, C, ln_w, ln_b, bias, ew, s);
            if (K == 256) return rowgemm_launch<1, 2, false, 256, true>(A, M, Wf, N, C, ln_w, ln_b, bias, ew, s);
            if (K == 128) return rowgemm_launch<1, 2, false, 128, true>(A, M, Wf, N, C, ln_w, ln_b, bias, ew, s);
        }
    } else {
        if (kind == 0) { RG_K(0, 0, true) }
        if (kind == 1) { RG_K(0, 1, true) }
        if (kind == 2) { RG_K(0, 2, false) }
        if (kind == 3) { RG_K(0, 3, false) }
        if (kind == 4) { RG_K(0, 1, false) }
    }
#undef RG_K
#undef RG
    return hipErrorInvalidValue;
}

// kind: 0 = in_proj (LN, store), 1 = head (LN, + bias), 2 = out_proj (residual add),
// 3 = feed-forward W1 (+ bias, GELU), 4 = feed-forward W2 (+ bias)
hipError_t launch_mgemm(int dtype, int kind, const float* A, int M, int K, const float* W32, const uint16_t* W16,
                        int N, float* C, const float* ln_w, const float* ln_b, const float* bias, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    if (K % 32 || N % 64 || K > 1024) return hipErrorInvalidValue;
    const bool small = M <= 2048;
#define MG(DTV, EPIV, LNV, BMV, BNV, WMV, WNV, KTV) \
    return mgemm_launch<DTV, EPIV, LNV, BMV, BNV, WMV, WNV, KTV>(A, M, K, W32, W16, N, C, ln_w, ln_b, bias, s)
#define BY_DT(EPIV, LNV, BMV, BNV, WMV, WNV, KTV) \
    { if (dtype == BOA_DTYPE_BF16) MG(1, EPIV, LNV, BMV, BNV, WMV, WNV, KTV); else MG(0, EPIV, LNV, BMV, BNV, WMV, WNV, KTV); }
    if (small) {
        // whole-K single tile; BN chosen so the staged W fits LDS and registers
        if (kind == 0 || kind == 1) {
#define LN_SMALL(KV, BNV, WNV) \
            if (K == KV) { if (kind == 0) BY_DT(0, true, 16, BNV, 1, WNV, KV) else BY_DT(1, true, 16, BNV, 1, WNV, KV) }
            LN_SMALL(64, 64, 4) LN_SMALL(128, 64, 4) LN_SMALL(256, 64, 4) LN_SMALL(512, 32, 2)
#undef LN_SMALL
        } else if (kind == 2) {
            if (K == 128) BY_DT(2, false, 16, 64, 1, 4, 128)
            if (K == 256) BY_DT(2, false, 16, 64, 1, 4, 256)
            if (K == 512) BY_DT(2, false, 16, 32, 1, 2, 512)
            if (K == 1024) BY_DT(2, false, 16, 16, 1, 1, 1024)
        } else if (kind == 3) {
            if (K == 64) BY_DT(3, false, 16, 64, 1, 4, 64)
            if (K == 128) BY_DT(3, false, 16, 64, 1, 4, 128)
            if (K == 256) BY_DT(3, false, 16, 64, 1, 4, 256)
            if (K == 512) BY_DT(3, false, 16, 32, 1, 2, 512)
        } else if (kind == 4) {
            if (K == 64) BY_DT(1, false, 16, 64, 1, 4, 64)
            if (K == 128) BY_DT(1, false, 16, 64, 1, 4, 128)
            if (K == 256) BY_DT(1, false, 16, 64, 1, 4, 256)
            if (K == 512) BY_DT(1, false, 16, 32, 1, 2, 512)
            if (K == 1024) BY_DT(1, false, 16, 16, 1, 1, 1024)
        }
        return hipErrorInvalidValue;
    }
    if (kind == 0) BY_DT(0, true, 64, 64, 2, 2, 0)
    if (kind == 1) BY_DT(1, true, 64, 64, 2, 2, 0)
    if (kind == 2) BY_DT(2, false, 64, 64, 2, 2, 0)
    if (kind == 3) BY_DT(3, false, 64, 64, 2, 2, 0)
    if (kind == 4) BY_DT(1, false, 64, 64, 2, 2, 0)
#undef BY_DT
#undef MG
    return hipErrorInvalidValue;
}

// LayerNorm of whole rows (the feed-forward sub-layer's output norm): one wave
// per row, ln_stats then ln_apply, out may alias x.
__global__ void k_ln_rows(const float* __restrict__ x, int M, int D, const float* __restrict__ w,
                          const float* __restrict__ b, float* __restrict__ out) {
    const long long row = blockIdx.x * 4LL + threadIdx.y;
    if (row >= M) return;
    const int lane = threadIdx.x;
    float mu, rs;
    ln_stats(x + row * D, D, lane, mu, rs);
    for (int k = lane; k < D; k += 64) out[row * D + k] = ln_apply(x[row * D + k], mu, rs, w[k], b[k]);
}
hipError_t launch_ln_rows(const float* x, int M, int D, const float* w, const float* b, float* out, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ln_rows, dim3((M + 3) / 4), dim3(64, 4), 0, s, x, M, D, w, b, out);
    return hipGetLastError();
}

// ============================================================== mixer middle
// Per-element pieces of the Mamba mixer between in_proj and out_proj
// (Appendix A: selection mechanism and discrete recurrence).  Both the
// encoder kernels (k_convx + k_scan) and the decoder step kernel (k_mid) call
// exactly these functions with the same operands in the same order.

// ---------------------------------------------------------------- decoder step
// One workgroup per lane (or a few lanes): conv, x_proj, dt, scan and gate for
// one row per lane, with the conv window and h kept in registers.
template <int NT, int CPT, int RR>
__global__ __launch_bounds__(NT) void k_mid(LayerDev w, const float* __restrict__ xz,
                                            float* __restrict__ g, int lanes, int T, int lanes_per_wg,
                                            const int* __restrict__ row_pos,
                                            float* __restrict__ conv_state,
                                            float* __restrict__ hstate) {
    constexpr int Di = NT * CPT;
    constexpr int NO = RR + 2 * NSTATE;          // x_proj outputs
    constexpr int NF = (NO + 15) / 16;           // x_proj column fragments
    __shared__ __align__(16) float xs_s[Di];
    __shared__ float dbc_s[NO];
    const int tid = threadIdx.x;

    float cw[CPT][KCONV], cb[CPT], dtw[CPT][RR], dtb[CPT], A2[CPT][NSTATE], Dk[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        int d = tid + j * NT;
#pragma unroll
        for (int k = 0; k < KCONV; ++k) cw[j][k] = w.convT[k * Di + d];
        cb[j] = w.conv_b[d];
#pragma unroll
        for (int r = 0; r < RR; ++r) dtw[j][r] = w.dtwT[r * Di + d];
        dtb[j] = w.dtb[d];
#pragma unroll
        for (int n = 0; n < NSTATE; ++n) A2[j][n] = w.A2T[n * Di + d];
        Dk[j] = w.Dsk[d];
    }

    for (int li = 0; li < lanes_per_wg; ++li) {
        const int lane = blockIdx.x * lanes_per_wg + li;
        if (lane >= lanes) break;
        float win[CPT][KCONV - 1], h[CPT][NSTATE];
        float* cst = conv_state + (long long)lane * (KCONV - 1) * Di;
        float* hst = hstate + (long long)lane * NSTATE * Di;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            int d = tid + j * NT;
#pragma unroll
            for (int k = 0; k < KCONV - 1; ++k) win[j][k] = cst[k * Di + d];
#pragma unroll
            for (int n = 0; n < NSTATE; ++n) h[j][n] = hst[n * Di + d];
        }
        bool touched = false;
        for (int t = 0; t < T; ++t) {
            const long long row = (long long)lane * T + t;
            const float* xzr = xz + row * (2 * Di);
            float xv[CPT], zv[CPT];
#pragma unroll
            for (int j = 0; j < CPT; ++j) {          // issued before the row check (valid memory either way)
                xv[j] = xzr[tid + j * NT];
                zv[j] = xzr[Di + tid + j * NT];
            }
            const int pos = row_pos[row];
            if (pos < 0) continue;                 // uniform across the block
            touched = true;
            if (pos == 0) {
#pragma unroll
                for (int j = 0; j < CPT; ++j) {
#pragma unroll
                    for (int k = 0; k < KCONV - 1; ++k) win[j][k] = 0.0f;
#pragma unroll
                    for (int n = 0; n < NSTATE; ++n) h[j][n] = 0.0f;
                }
            }
            float xs[CPT];
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                int d = tid + j * NT;
                float x = xv[j];
                xs[j] = conv_silu(cw[j], cb[j], win[j][0], win[j][1], win[j][2], x);
                win[j][0] = win[j][1];
                win[j][1] = win[j][2];
                win[j][2] = x;
                xs_s[d] = xs[j];
            }
            __syncthreads();
            // x_proj of the row (the one live row of the MFMA tile)
            for (int f = tid >> 6; f < NF; f += NT / 64) {
                v4f acc;
                xproj_fragment<Di, CPT == 1 ? 8 : 4>(xs_s, 0, 1, w.xwF, f, tid & 63, acc);
                const int col = 16 * f + (tid & 15);
                if ((tid & 63) < 16 && col < NO) dbc_s[col] = acc[0];
            }
            __syncthreads();
            float* gr = g + row * Di;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                int d = tid + j * NT;
                float dt = dt_of<RR>(dbc_s, dtw[j], dtb[j]);
                gr[d] = scan_update(h[j], dt, xs[j], dbc_s + RR, dbc_s + RR + NSTATE, A2[j], Dk[j], zv[j]);
            }
        }
        if (touched) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                int d = tid + j * NT;
#pragma unroll
                for (int k = 0; k < KCONV - 1; ++k) cst[k * Di + d] = win[j][k];
#pragma unroll
                for (int n = 0; n < NSTATE; ++n) hst[n * Di + d] = h[j][n];
            }
        }
        __syncthreads();
    }
}

static size_t g_max_lds = 65536;
void set_max_lds(size_t b) { g_max_lds = b; }
size_t get_max_lds() { return g_max_lds; }

hipError_t launch_mid(const LayerDev& w, int Di, int R, const float* xz, float* g, int lanes, int T,
                      int lanes_per_wg, const int* row_pos, float* conv_state, float* hstate,
                      hipStream_t s) {
    if (lanes_per_wg < 1) lanes_per_wg = 1;
    dim3 grid((lanes + lanes_per_wg - 1) / lanes_per_wg);
#define MID_CASE(DI, RV, NTV, CPTV) \
    if (Di == DI && R == RV) { \
        BOA_LAUNCH((k_mid<NTV, CPTV, RV>), grid, dim3(NTV), 0, s, w, xz, g, lanes, T, lanes_per_wg, \
                           row_pos, conv_state, hstate); \
        return hipGetLastError(); }
    MID_CASE(128, 4, 128, 1)
    MID_CASE(256, 8, 256, 1)
    MID_CASE(512, 16, 512, 1)
    MID_CASE(1024, 32, 512, 2)
#undef MID_CASE
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- encoder
// k_convx: RB consecutive rows of one lane per workgroup.  Conv + SiLU for
// every channel (window from earlier rows of the tile, the lane's carried
// conv state, or zero before the chunk start), then x_proj on the matrix
// cores: wave f computes column fragments f, f + 4, ... (xproj_fragment).
template <int Di, int RR>
__global__ __launch_bounds__(256) void k_convx(LayerDev w, const float* __restrict__ xz, int lanes, int T,
                                               const int* __restrict__ row_pos,
                                               const float* __restrict__ conv_state,
                                               float* __restrict__ xs_out, float* __restrict__ dbc_out) {
    constexpr int RB = 16;
    constexpr int NO = RR + 2 * NSTATE, NF = (NO + 15) / 16;
    constexpr int XSR = Di + 4;                  // row stride in LDS: rows 4 banks apart
    __shared__ __align__(16) float xs_s[RB * XSR];
    const int tid = threadIdx.x;
    const int lane = blockIdx.y;
    const int r0 = blockIdx.x * RB;
    const long long base = (long long)lane * T;
    const float* cst = conv_state + (long long)lane * (KCONV - 1) * Di;

    // phase 1: conv + SiLU
    for (int it = tid; it < RB * Di; it += 256) {
        int r = it / Di, d = it % Di;
        int tr = r0 + r;
        float v = 0.0f;
        if (tr < T) {
            int pos = row_pos[base + tr];
            if (pos >= 0) {
                float wv[KCONV];
#pragma unroll
                for (int j = 0; j < KCONV; ++j) {       // wv[j] = x at offset j - 3
                    int back = KCONV - 1 - j;
                    float x = 0.0f;
                    if (pos - back >= 0) {
                        int idx = tr - back;
                        x = idx >= 0 ? xz[(base + idx) * (2 * Di) + d] : cst[(KCONV - 1 + idx) * Di + d];
                    }
                    wv[j] = x;
                }
                float cw[KCONV];
#pragma unroll
                for (int k = 0; k < KCONV; ++k) cw[k] = w.convT[k * Di + d];
                v = conv_silu(cw, w.conv_b[d], wv[0], wv[1], wv[2], wv[3]);
                xs_out[(base + tr) * Di + d] = v;
            }
        }
        xs_s[r * XSR + d] = v;
    }
    __syncthreads();
    // phase 2: x_proj
    const int wv = tid >> 6, wl = tid & 63;
    for (int f = wv; f < NF; f += 4) {
        v4f acc;
        xproj_fragment<Di>(xs_s, XSR, RB, w.xwF, f, wl, acc);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int row = 4 * (wl >> 4) + rr, col = 16 * f + (wl & 15);
            if (r0 + row < T && col < NO) dbc_out[(base + r0 + row) * NO + col] = acc[rr];
        }
    }
}

// k_scan: one thread per (lane, channel) walks the tile's rows in order:
// dt_proj + softplus, the scan update and the gate.  h stays in registers;
// the lane's conv state is advanced to the last three inputs of the tile.
template <int RR>
__global__ __launch_bounds__(256) void k_scan(LayerDev w, const float* __restrict__ xz,
                                              const float* __restrict__ xs, const float* __restrict__ dbc,
                                              int lanes, int T, int Di, const int* __restrict__ row_pos,
                                              float* __restrict__ conv_state, float* __restrict__ hstate,
                                              float* __restrict__ g) {
    constexpr int NO = RR + 2 * NSTATE;
    const int lane = blockIdx.y;
    const int d = blockIdx.x * 256 + threadIdx.x;
    if (d >= Di) return;
    const long long base = (long long)lane * T;
    float A2[NSTATE], h[NSTATE], dtw[RR];
    float* hst = hstate + (long long)lane * NSTATE * Di;
#pragma unroll
    for (int n = 0; n < NSTATE; ++n) { A2[n] = w.A2T[n * Di + d]; h[n] = hst[n * Di + d]; }
#pragma unroll
    for (int k = 0; k < RR; ++k) dtw[k] = w.dtwT[k * Di + d];
    const float Dk = w.Dsk[d], dtb = w.dtb[d];
    bool touched = false;
    for (int t = 0; t < T; ++t) {
        const long long row = base + t;
        const int pos = row_pos[row];
        if (pos < 0) continue;
        touched = true;
        if (pos == 0) {
#pragma unroll
            for (int n = 0; n < NSTATE; ++n) h[n] = 0.0f;
        }
        const float* dr = dbc + row * NO;
        float dl[NO];
#pragma unroll
        for (int k = 0; k < NO; ++k) dl[k] = dr[k];
        const float dt = dt_of<RR>(dl, dtw, dtb);
        g[row * Di + d] = scan_update(h, dt, xs[row * Di + d], dl + RR, dl + RR + NSTATE, A2, Dk,
                                      xz[row * (2 * Di) + Di + d]);
    }
    if (touched) {
#pragma unroll
        for (int n = 0; n < NSTATE; ++n) hst[n * Di + d] = h[n];
    }
    // conv state <- inputs at offsets T-3, T-2, T-1 of this tile
    float* cst = conv_state + (long long)lane * (KCONV - 1) * Di;
    float old[KCONV - 1];
#pragma unroll
    for (int k = 0; k < KCONV - 1; ++k) old[k] = cst[k * Di + d];
#pragma unroll
    for (int k = 0; k < KCONV - 1; ++k) {
        int idx = T - (KCONV - 1) + k;
        cst[k * Di + d] = idx >= 0 ? xz[(base + idx) * (2 * Di) + d] : old[T + k];
    }
}

// Encoder mixer in one pass (d_inner <= 512): one workgroup per lane runs the
// tile's rows of that lane in blocks of 16 -- conv + SiLU, x_proj, dt_proj +
// softplus, scan and gate -- with everything between the phases in LDS.
// Thread d owns channel d: its conv window, scan state h and conv / dt / scan
// weights stay in registers for the whole tile.  x_proj runs on the matrix
// cores: wave f < NF computes column fragment f of the block's 16 rows
// (xproj_fragment).  Same per-element functions, operands and orders as
// the decoder kernels; the window restarts at a chunk start (pos 0) exactly
// like the zero padding before a chunk.
template <int Di, int RR, bool G16>
__global__ __launch_bounds__(512) void k_mixer_enc(LayerDev w, const float* __restrict__ xz, int lanes, int T,
                                                   const int* __restrict__ row_pos, float* __restrict__ conv_state,
                                                   float* __restrict__ hstate, float* __restrict__ g) {
    constexpr int NT = 512, RB = 16;
    constexpr int NO = RR + 2 * NSTATE, XSR = Di + 4;     // row stride of xs in LDS: rows 4 banks apart
    constexpr int NF = (NO + 15) / 16;                    // x_proj column fragments
    static_assert(Di <= NT && NF <= NT / 64 && Di % 16 == 0, "one channel per thread, one fragment per wave");
    __shared__ __align__(16) float xs_s[RB * XSR];
    __shared__ float dbc_s[RB * NO];
    __shared__ int pos_s[RB], start_s;
    const int tid = threadIdx.x;
    const int lane = blockIdx.x;
    if (lane >= lanes) return;
    const long long base = (long long)lane * T;
    const bool ch = tid < Di;
    const int d = tid;
    float* cst = conv_state + (long long)lane * (KCONV - 1) * Di;
    float* hst = hstate + (long long)lane * NSTATE * Di;

    float cw[KCONV], cb = 0.0f, dtw[RR], dtb = 0.0f, A2[NSTATE], Dk = 0.0f, h[NSTATE], win[KCONV - 1];
    if (ch) {
#pragma unroll
        for (int k = 0; k < KCONV; ++k) cw[k] = w.convT[k * Di + d];
        cb = w.conv_b[d];
#pragma unroll
        for (int k = 0; k < RR; ++k) dtw[k] = w.dtwT[k * Di + d];
        dtb = w.dtb[d];
#pragma unroll
        for (int n = 0; n < NSTATE; ++n) { A2[n] = w.A2T[n * Di + d]; h[n] = hst[n * Di + d]; }
        Dk = w.Dsk[d];
#pragma unroll
        for (int k = 0; k < KCONV - 1; ++k) win[k] = cst[k * Di + d];
    }
    const int wv = tid >> 6, wl = tid & 63, li = wl & 15, lk = wl >> 4;

    for (int t0 = 0; t0 < T; t0 += RB) {
        const int nb = T - t0 < RB ? T - t0 : RB;
        float xv[RB], zv[RB];
        if (ch) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                if (r < nb) {
                    const float* row = xz + (base + t0 + r) * (2 * Di);
                    xv[r] = row[d];
                    zv[r] = row[Di + d];
                }
            }
        }
        __syncthreads();                       // the previous block's readers are done
        if (tid < 64) {                        // wave 0: the rows' positions, and whether a chunk starts here
            const int p = tid < nb && tid < RB ? row_pos[base + t0 + tid] : -1;
            if (tid < RB) pos_s[tid] = p;
            const bool any0 = __ballot(p == 0) != 0;
            if (tid == 0) start_s = any0 ? 1 : 0;
        }
        __syncthreads();
        const int starts = start_s;
        // conv + SiLU
        if (ch) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int pos = pos_s[r];
                if (pos < 0) continue;
                if (starts && pos == 0) { win[0] = 0.0f; win[1] = 0.0f; win[2] = 0.0f; }
                const float x = xv[r];
                xs_s[r * XSR + d] = conv_silu(cw, cb, win[0], win[1], win[2], x);
                win[0] = win[1];
                win[1] = win[2];
                win[2] = x;
            }
        }
        __syncthreads();
        // x_proj (rows of idle slots compute stale values and are not used)
        if (wv < NF) {
            v4f acc;
            xproj_fragment<Di>(xs_s, XSR, RB, w.xwF, wv, wl, acc);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int row = 4 * lk + rr, col = 16 * wv + li;
                if (row < nb && col < NO) dbc_s[row * NO + col] = acc[rr];
            }
        }
        __syncthreads();
        // dt_proj + softplus, scan, gate.  A block without a chunk start (the
        // common case) runs a copy of the loop without the state reset, which
        // the compiler would otherwise turn into per-row selects.
        auto scan_rows = [&](auto reset) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int pos = pos_s[r];
                if (pos < 0) continue;
                if (decltype(reset)::value && pos == 0) {
#pragma unroll
                    for (int n = 0; n < NSTATE; ++n) h[n] = 0.0f;
                }
                const float* db = dbc_s + r * NO;
                const float dt = dt_of<RR>(db, dtw, dtb);
                const float xs = xs_s[r * XSR + d];
                const float gv = scan_update(h, dt, xs, db + RR, db + RR + NSTATE, A2, Dk, zv[r]);
                if (G16) reinterpret_cast<uint16_t*>(g)[(base + t0 + r) * Di + d] = f2bf_bits(gv);
                else g[(base + t0 + r) * Di + d] = gv;
            }
        };
        if (ch) {
            if (__builtin_amdgcn_readfirstlane(starts)) scan_rows(std::true_type{});
            else scan_rows(std::false_type{});
        }
    }
    if (ch) {
#pragma unroll
        for (int n = 0; n < NSTATE; ++n) hst[n * Di + d] = h[n];
#pragma unroll
        for (int k = 0; k < KCONV - 1; ++k) cst[k * Di + d] = win[k];
    }
}

hipError_t launch_mid_tiled(const LayerDev& w, int Di, int R, const float* xz, float* xs, float* dbc, float* dt,
                            float* g, int lanes, int T, const int* row_pos, float* conv_state, float* hstate,
                            bool g_bf16, hipStream_t s) {
    (void)dt;
    dim3 g1((T + 15) / 16, lanes), g2((Di + 255) / 256, lanes);
#define CX_CASE(DI, RV) \
    if (Di == DI && R == RV) { \
        if (g_bf16) return hipErrorInvalidValue; \
        BOA_LAUNCH((k_convx<DI, RV>), g1, dim3(256), 0, s, w, xz, lanes, T, row_pos, conv_state, xs, dbc); \
        hipError_t e = hipGetLastError(); \
        if (e != hipSuccess) return e; \
        BOA_LAUNCH((k_scan<RV>), g2, dim3(256), 0, s, w, xz, xs, dbc, lanes, T, Di, row_pos, conv_state, \
                           hstate, g); \
        return hipGetLastError(); }
#define MX_CASE(DI, RV) \
    if (Di == DI && R == RV) { \
        if (g_bf16) \
            BOA_LAUNCH((k_mixer_enc<DI, RV, true>), dim3(lanes), dim3(512), 0, s, w, xz, lanes, T, row_pos, \
                       conv_state, hstate, g); \
        else \
            BOA_LAUNCH((k_mixer_enc<DI, RV, false>), dim3(lanes), dim3(512), 0, s, w, xz, lanes, T, row_pos, \
                       conv_state, hstate, g); \
        return hipGetLastError(); }
    MX_CASE(128, 4) MX_CASE(256, 8) MX_CASE(512, 16)
    CX_CASE(1024, 32)
#undef MX_CASE
#undef CX_CASE
    return hipErrorInvalidValue;
}

// ============================================================== histogram / CDF
// One wave per row; wave lane i owns symbols 4i..4i+3.  Produces f[4] (the
// strictly positive histogram summing to 2^16) and cx[4] = C(a) for its
// symbols (paper, Range coding: probabilities and integer CDF).
// Encoder side: (C(s), f(s)) of the true next byte s per row; optional dumps.
__global__ void k_quant_sym(const float* __restrict__ logits, int M, const uint8_t* __restrict__ data,
                            Plan p, const int* __restrict__ row_chunk, const int* __restrict__ row_pos,
                            uint32_t* __restrict__ cf, float* __restrict__ probs,
                            uint16_t* __restrict__ tables) {
    int row = blockIdx.x * 4 + threadIdx.y;
    int lane = threadIdx.x;
    if (row >= M) return;
    int pos = row_pos[row];
    if (pos < 0) return;
    QRow q = quant_row(logits + (long long)row * 256, lane);
    if (probs) {
        float4 v = make_float4(q.p[0], q.p[1], q.p[2], q.p[3]);
        *reinterpret_cast<float4*>(probs + (long long)row * 256 + 4 * lane) = v;
    }
    if (tables) {
        uint2 v;
        v.x = (uint32_t)q.f[0] | ((uint32_t)q.f[1] << 16);
        v.y = (uint32_t)q.f[2] | ((uint32_t)q.f[3] << 16);
        *reinterpret_cast<uint2*>(tables + (long long)row * 256 + 4 * lane) = v;
    }
    if (cf) {
        int s = data[p.chunk_off[row_chunk[row]] + pos + 1];
        if ((s >> 2) == lane) {
            cf[2 * row] = (uint32_t)q.csel(s & 3);
            cf[2 * row + 1] = (uint32_t)q.fsel(s & 3);
        }
    }
}
hipError_t launch_quant_sym(const float* logits, int M, const uint8_t* data, const Plan& p,
                            const int* row_chunk, const int* row_pos, uint32_t* cf,
                            float* probs, uint16_t* tables, hipStream_t s) {
    BOA_LAUNCH(k_quant_sym, dim3((M + 3) / 4), dim3(64, 4), 0, s, logits, M, data, p, row_chunk,
                       row_pos, cf, probs, tables);
    return hipGetLastError();
}

// ============================================================== predictor diagnostics
// One wave per row, from the probabilities the coder quantises (quant_row):
// pred = argmax p (lowest index on ties), conf = p[pred], rank of the true
// byte y = #{a : p[a] > p[y]} + #{a < y : p[a] == p[y]}; accumulates the
// confusion count [y][pred], the rank histogram and the reliability bin of
// conf (count, correct, conf * 2^32 -- exact for conf >= 2^-9).  Integer
// atomics only, so the totals do not depend on the order of the rows.
// (Paper, Results: confusion matrices, Top-k curves, reliability and ECE.)
__global__ void k_diag(const float* __restrict__ logits, int M, const uint8_t* __restrict__ data, Plan p,
                       const int* __restrict__ row_chunk, const int* __restrict__ row_pos, int n_bins,
                       uint32_t* __restrict__ confusion, uint32_t* __restrict__ rank_hist,
                       unsigned long long* __restrict__ calib) {
    const int row = blockIdx.x * 4 + threadIdx.y;
    const int lane = threadIdx.x;
    if (row >= M) return;
    const int pos = row_pos[row];
    if (pos < 0) return;
    const QRow q = quant_row(logits + (long long)row * 256, lane);
    const int y = __builtin_amdgcn_readfirstlane((int)data[p.chunk_off[row_chunk[row]] + pos + 1]);
    // non-negative floats order like their bit patterns
    int bv = -1, bi = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int v = __float_as_int(q.p[i]);
        if (v > bv) { bv = v; bi = 4 * lane + i; }
    }
    wave_argmax_i(bv, bi);
    const int pred = bi;
    const float conf = __int_as_float(bv);
    const int yi = y & 3;
    const float mine = yi == 0 ? q.p[0] : yi == 1 ? q.p[1] : yi == 2 ? q.p[2] : q.p[3];
    const float py = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine), y >> 2));
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int a = 4 * lane + i;
        cnt += (q.p[i] > py || (q.p[i] == py && a < y)) ? 1 : 0;
    }
    const int rank = wave_sum_i(cnt);
    if (lane == 0) {
        atomicAdd(&confusion[y * 256 + pred], 1u);
        atomicAdd(&rank_hist[rank], 1u);
        int b = (int)(conf * (float)n_bins);
        if (b > n_bins - 1) b = n_bins - 1;
        atomicAdd(&calib[3 * b], 1ull);
        atomicAdd(&calib[3 * b + 1], pred == y ? 1ull : 0ull);
        atomicAdd(&calib[3 * b + 2], (unsigned long long)(conf * 4294967296.0f));
    }
}
hipError_t launch_diag(const float* logits, int M, const uint8_t* data, const Plan& p, const int* row_chunk,
                       const int* row_pos, int n_bins, uint32_t* confusion, uint32_t* rank_hist,
                       unsigned long long* calib, hipStream_t s) {
    BOA_LAUNCH(k_diag, dim3((M + 3) / 4), dim3(64, 4), 0, s, logits, M, data, p, row_chunk, row_pos, n_bins,
               confusion, rank_hist, calib);
    return hipGetLastError();
}

// ============================================================== range coder
// State per lane: L (32-bit base), R (width in [1, 2^32], kept in 64 bits),
// byte cursor.  Paper, Range coding: encoder update, renormalisation while the
// top byte of L and E = L + R - 1 agree; readings: R is not reduced mod 2^32,
// straddle fix R <- 2^16 - (L mod 2^16), flush with at most 2 bytes.
// Encoder lanes: one thread per lane walks its rows of the tile in order.
// cst per lane: [L, R_lo, R_hi, cur] (uint32).
__global__ void k_encode(const uint32_t* __restrict__ cf, int lanes, int T, const int* __restrict__ row_chunk,
                         const int* __restrict__ row_pos, Plan p, uint32_t* __restrict__ cst,
                         uint8_t* __restrict__ payload, const long long* __restrict__ pay_off,
                         const long long* __restrict__ pay_cap, uint32_t* __restrict__ pay_len,
                         double* __restrict__ ideal) {
    constexpr int RB = 16;                       // rows fetched per batch (independent loads, one latency)
    int lane = blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= lanes) return;
    Enc e;
    e.L = cst[4 * lane];
    e.R = (uint64_t)cst[4 * lane + 1] | ((uint64_t)cst[4 * lane + 2] << 32);
    e.cur = cst[4 * lane + 3];
    double ib = 0.0;
    int cur_chunk = -1;
    uint8_t* out = nullptr;
    uint32_t cap = 0;
    long long last = -1;                         // last position of the current chunk
    for (int t0 = 0; t0 < T; t0 += RB) {
        int pos_b[RB], chk_b[RB];
        uint32_t cl_b[RB], f_b[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const long long row = (long long)lane * T + t0 + r;
            const bool in = t0 + r < T;
            pos_b[r] = in ? row_pos[row] : -1;
            chk_b[r] = in ? row_chunk[row] : -1;
            cl_b[r] = in ? cf[2 * row] : 0u;
            f_b[r] = in ? cf[2 * row + 1] : 0u;
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int pos = pos_b[r];
            if (pos < 0) continue;
            const int c = chk_b[r];
            if (c != cur_chunk) {
                if (cur_chunk >= 0 && ideal) ideal[cur_chunk] = ib;
                out = payload + pay_off[c];
                cap = (uint32_t)pay_cap[c];
                last = p.chunk_steps[c] - 1;
                ib = (pos > 0 && ideal) ? ideal[c] : 0.0;
                cur_chunk = c;
            }
            if (pos == 0) { enc_reset(e); ib = 0.0; }
            const uint32_t f = f_b[r];
            // ideal cost -log2(f / 2^16) = 16 - log2 f: hardware log2 in FP32
            // (about 1 ulp), summed in FP64
            if (ideal) ib += (double)(16.0f - __builtin_amdgcn_logf((float)f));
            enc_put(e, cl_b[r], f, out, cap);
            if (pos == last) {
                enc_flush(e, out, cap);
                pay_len[c] = e.cur <= cap ? e.cur : 0xFFFFFFFFu;
            }
        }
    }
    if (cur_chunk >= 0 && ideal) ideal[cur_chunk] = ib;
    cst[4 * lane] = (uint32_t)e.L;
    cst[4 * lane + 1] = (uint32_t)(e.R & 0xFFFFFFFFULL);
    cst[4 * lane + 2] = (uint32_t)(e.R >> 32);
    cst[4 * lane + 3] = e.cur;
}
hipError_t launch_encode(const uint32_t* cf, int lanes, int T, const int* row_chunk, const int* row_pos,
                         const Plan& p, uint32_t* cst, uint8_t* payload, const long long* pay_off,
                         const long long* pay_cap, uint32_t* pay_len, double* ideal, hipStream_t s) {
    BOA_LAUNCH(k_encode, dim3((lanes + 63) / 64), dim3(64), 0, s, cf, lanes, T, row_chunk, row_pos, p,
                       cst, payload, pay_off, pay_cap, pay_len, ideal);
    return hipGetLastError();
}

// Decoder lanes: one wave per lane builds the histogram of its row, finds the
// symbol whose CDF interval holds the target, updates the coder, writes the
// byte, and prepares the lane's next step: its (chunk, pos) and the embedding
// row r = E[next input byte] (the decoded byte, or the stored first byte of
// the lane's next chunk).  dst per lane: [L, R_lo, R_hi, X, cur, step_lo, step_hi, 0].
__global__ void k_decode(const float* __restrict__ logits, int lanes, int* __restrict__ row_chunk,
                         int* __restrict__ row_pos, Plan p, uint32_t* __restrict__ dst,
                         const uint8_t* __restrict__ payload, const long long* __restrict__ pay_off,
                         const long long* __restrict__ pay_len, uint8_t* __restrict__ out,
                         const float* __restrict__ E, int D, float* __restrict__ r) {
    int lane_id = blockIdx.x * 4 + threadIdx.y;
    int wl = threadIdx.x;
    if (lane_id >= lanes) return;
    const int pos = row_pos[lane_id];
    if (pos < 0) return;
    const int c = row_chunk[lane_id];
    uint32_t* st = dst + 8 * lane_id;
    const uint32_t s0 = st[0], s1 = st[1], s2 = st[2], s3 = st[3], s4 = st[4], s5 = st[5], s6 = st[6];
    const long long poff = pay_off[c];
    const uint32_t len = (uint32_t)pay_len[c];
    const uint8_t* in = payload + poff;
    QRow q = quant_row(logits + (long long)lane_id * 256, wl);
    Dec d;
    if (pos == 0) {
        dec_reset(d, in, len);
    } else {
        d.L = s0;
        d.R = (uint64_t)s1 | ((uint64_t)s2 << 32);
        d.X = s3;
        d.cur = s4;
    }
    uint64_t pf = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) pf |= (uint64_t)dec_byte(in, len, d.cur + i) << (8 * i);
    uint32_t x = dec_target(d);
    int hit = -1;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if ((uint32_t)q.cx[i] <= x && x < (uint32_t)(q.cx[i] + q.f[i])) hit = 4 * wl + i;
    unsigned long long bal = __ballot(hit >= 0);
    int src = bal ? (__ffsll((long long)bal) - 1) : 0;
    int sym = __builtin_amdgcn_readlane(hit, src);   // wave-uniform lane indices
    if (sym < 0) sym = 0;                      // unreachable for a valid stream
    int cl = __builtin_amdgcn_readlane(q.csel(sym & 3), sym >> 2);
    int fs = __builtin_amdgcn_readlane(q.fsel(sym & 3), sym >> 2);
    const long long lstep = (long long)((uint64_t)s5 | ((uint64_t)s6 << 32));
    // next step of this lane
    int nc, npos, ny;
    if (pos + 1 < p.chunk_steps[c]) {
        nc = c; npos = pos + 1; ny = sym;
    } else {
        locate(p, lane_id, lstep + 1, nc, npos);
        ny = npos >= 0 ? out[p.chunk_off[nc] + npos] : -1;
    }
    float* rr = r + (long long)lane_id * D;
    if (ny >= 0) {
        const float* er = E + (long long)ny * D;
        for (int k = wl; k < D; k += 64) rr[k] = er[k];
    } else {
        for (int k = wl; k < D; k += 64) rr[k] = 0.0f;
    }
    if (wl == 0) {
        dec_update(d, (uint32_t)cl, (uint32_t)fs, in, len, pf, true);
        st[0] = (uint32_t)d.L;
        st[1] = (uint32_t)(d.R & 0xFFFFFFFFULL);
        st[2] = (uint32_t)(d.R >> 32);
        st[3] = (uint32_t)d.X;
        st[4] = d.cur;
        st[5] = (uint32_t)((uint64_t)(lstep + 1) & 0xFFFFFFFFULL);
        st[6] = (uint32_t)((uint64_t)(lstep + 1) >> 32);
        out[p.chunk_off[c] + pos + 1] = (uint8_t)sym;
        row_chunk[lane_id] = nc;
        row_pos[lane_id] = npos;
    }
}
hipError_t launch_decode(const float* logits, int lanes, int* row_chunk, int* row_pos, const Plan& p, uint32_t* dst,
                         const uint8_t* payload, const long long* pay_off, const long long* pay_len, uint8_t* out,
                         const float* E, int D, float* r, hipStream_t s) {
    BOA_LAUNCH(k_decode, dim3((lanes + 3) / 4), dim3(64, 4), 0, s, logits, lanes, row_chunk, row_pos, p, dst,
                       payload, pay_off, pay_len, out, E, D, r);
    return hipGetLastError();
}

__global__ void k_prefill(const uint8_t* __restrict__ first, const long long* __restrict__ off,
                          const long long* __restrict__ len, int n, uint8_t* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && len[i] > 0) out[off[i]] = first[i];
}
hipError_t launch_prefill(const uint8_t* first, const long long* off, const long long* len, int n,
                          uint8_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_prefill, dim3((n + 255) / 256), dim3(256), 0, s, first, off, len, n, out);
    return hipGetLastError();
}

// rows (lane, t) of a tile -> dst[(lane * Tout + t0 + t) * width]
template <typename TT>
__global__ void k_scatter_rows(const TT* __restrict__ src, int lanes, int T, int width, long long t0,
                               long long Tout, TT* __restrict__ dst) {
    long long row = blockIdx.x;
    int lane = (int)(row / T), t = (int)(row % T);
    if (t0 + t >= Tout) return;
    const TT* a = src + row * width;
    TT* b = dst + ((long long)lane * Tout + t0 + t) * width;
    for (int k = threadIdx.x; k < width; k += blockDim.x) b[k] = a[k];
}
hipError_t launch_scatter_rows(const float* src, int lanes, int T, int width, long long t0, long long Tout,
                               float* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_rows<float>, dim3(lanes * T), dim3(256), 0, s, src, lanes, T, width, t0, Tout, dst);
    return hipGetLastError();
}
hipError_t launch_scatter_rows_u16(const uint16_t* src, int lanes, int T, int width, long long t0,
                                   long long Tout, uint16_t* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_rows<uint16_t>, dim3(lanes * T), dim3(256), 0, s, src, lanes, T, width, t0,
                       Tout, dst);
    return hipGetLastError();
}

// ============================================================== explicit-table coder (parity)
__global__ void k_code_tables(const uint8_t* __restrict__ sym, const uint16_t* __restrict__ freq,
                              const long long* __restrict__ sym_off, const long long* __restrict__ nsym,
                              int lanes, uint8_t* __restrict__ payload, const long long* __restrict__ pay_off,
                              const long long* __restrict__ pay_cap, uint32_t* __restrict__ pay_len) {
    int lane_id = blockIdx.x * 4 + threadIdx.y;
    int wl = threadIdx.x;
    if (lane_id >= lanes) return;
    Enc e;
    enc_reset(e);
    uint8_t* out = payload + pay_off[lane_id];
    uint32_t cap = (uint32_t)pay_cap[lane_id];
    long long base = sym_off[lane_id];
    for (long long j = 0; j < nsym[lane_id]; ++j) {
        const uint16_t* f = freq + (base + j) * 256;
        int s = sym[base + j];
        int loc = ((f[4 * wl] + f[4 * wl + 1]) + f[4 * wl + 2]) + f[4 * wl + 3];
        int incl = wave_incl_scan_i(loc, wl);
        int cl = incl - loc;
        for (int i = 0; i < (s & 3); ++i) cl += f[4 * wl + i];
        cl = __shfl(cl, s >> 2, 64);
        if (wl == 0) enc_put(e, (uint32_t)cl, f[s], out, cap);
    }
    if (wl == 0) {
        enc_flush(e, out, cap);
        pay_len[lane_id] = e.cur <= cap ? e.cur : 0xFFFFFFFFu;
    }
}
hipError_t launch_code_tables(const uint8_t* sym, const uint16_t* freq, const long long* sym_off,
                              const long long* nsym, int lanes, uint8_t* payload, const long long* pay_off,
                              const long long* pay_cap, uint32_t* pay_len, hipStream_t s) {
    hipLaunchKernelGGL(k_code_tables, dim3((lanes + 3) / 4), dim3(64, 4), 0, s, sym, freq, sym_off, nsym, lanes,
                       payload, pay_off, pay_cap, pay_len);
    return hipGetLastError();
}

__global__ void k_decode_tables(const uint8_t* __restrict__ payload, const long long* __restrict__ pay_off,
                                const long long* __restrict__ pay_len, const uint16_t* __restrict__ freq,
                                const long long* __restrict__ sym_off, const long long* __restrict__ nsym,
                                int lanes, uint8_t* __restrict__ sym) {
    int lane_id = blockIdx.x * 4 + threadIdx.y;
    int wl = threadIdx.x;
    if (lane_id >= lanes) return;
    const uint8_t* in = payload + pay_off[lane_id];
    uint32_t len = (uint32_t)pay_len[lane_id];
    Dec d;
    dec_reset(d, in, len);
    long long base = sym_off[lane_id];
    for (long long j = 0; j < nsym[lane_id]; ++j) {
        const uint16_t* f = freq + (base + j) * 256;
        int fl[4] = {f[4 * wl], f[4 * wl + 1], f[4 * wl + 2], f[4 * wl + 3]};
        int loc = ((fl[0] + fl[1]) + fl[2]) + fl[3];
        int incl = wave_incl_scan_i(loc, wl);
        int c = incl - loc;
        uint32_t x = dec_target(d);
        int hit = -1, hc = 0, hf = 0;
        for (int i = 0; i < 4; ++i) {
            if ((uint32_t)c <= x && x < (uint32_t)(c + fl[i])) { hit = 4 * wl + i; hc = c; hf = fl[i]; }
            c += fl[i];
        }
        unsigned long long bal = __ballot(hit >= 0);
        int src = bal ? (__ffsll((long long)bal) - 1) : 0;
        int s = __shfl(hit, src, 64);
        hc = __shfl(hc, src, 64);
        hf = __shfl(hf, src, 64);
        if (s < 0) { s = 0; hc = 0; hf = f[0]; }
        if (wl == 0) {
            dec_update(d, (uint32_t)hc, (uint32_t)hf, in, len);
            sym[base + j] = (uint8_t)s;
        }
        // broadcast the updated state from wave lane 0
        d.L = __shfl(d.L, 0, 64);
        d.R = __shfl(d.R, 0, 64);
        d.X = __shfl(d.X, 0, 64);
        d.cur = __shfl(d.cur, 0, 64);
    }
}
hipError_t launch_decode_tables(const uint8_t* payload, const long long* pay_off, const long long* pay_len,
                                const uint16_t* freq, const long long* sym_off, const long long* nsym, int lanes,
                                uint8_t* sym, hipStream_t s) {
    hipLaunchKernelGGL(k_decode_tables, dim3((lanes + 3) / 4), dim3(64, 4), 0, s, payload, pay_off, pay_len, freq,
                       sym_off, nsym, lanes, sym);
    return hipGetLastError();
}

// ============================================================== CRC32 per chunk
// Reflected CRC-32 (polynomial 0xEDB88320), bitwise, one thread per chunk.
__global__ void k_crc32(const uint8_t* __restrict__ data, const long long* __restrict__ off,
                        const long long* __restrict__ len, int n, uint32_t* __restrict__ crc) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c = 0xFFFFFFFFu;
    const uint8_t* p = data + off[i];
    for (long long j = 0; j < len[i]; ++j) {
        c ^= p[j];
#pragma unroll
        for (int b = 0; b < 8; ++b) c = (c >> 1) ^ (0xEDB88320u & (0u - (c & 1u)));
    }
    crc[i] = ~c;
}
hipError_t launch_crc32(const uint8_t* data, const long long* off, const long long* len, int n, uint32_t* crc,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_crc32, dim3((n + 63) / 64), dim3(64), 0, s, data, off, len, n, crc);
    return hipGetLastError();
}

// ============================================================== order-2 context model
// One wave per chunk.  counts: [chunks][65536 contexts][256] uint16, zeroed by
// the caller.  KT estimate f(a) = max(1, floor(M (2 n(a) + 1) / (2 T + 256)))
// with the remainder rule of the neural histogram; halve a context's counts
// (ceil) when its total reaches 2^16.
DEVI void o2_table(const uint16_t* row, int wl, int f[4], int cx[4], int& total) {
    int n[4];
    uint2 u = *reinterpret_cast<const uint2*>(row + 4 * wl);
    n[0] = u.x & 0xFFFF; n[1] = u.x >> 16; n[2] = u.y & 0xFFFF; n[3] = u.y >> 16;
    int T = wave_sum_i(((n[0] + n[1]) + n[2]) + n[3]);
    total = T;
    uint64_t den = 2ULL * (uint64_t)T + 256ULL;
    int tot = 0, best_v = -1, best_i = 0;
    for (int i = 0; i < 4; ++i) {
        uint64_t v = (65536ULL * (2ULL * (uint64_t)n[i] + 1ULL)) / den;
        f[i] = v < 1 ? 1 : (int)v;
        tot += f[i];
        if (f[i] > best_v) { best_v = f[i]; best_i = 4 * wl + i; }
    }
    tot = wave_sum_i(tot);
    wave_argmax_i(best_v, best_i);
    {
        const bool mine = (best_i >> 2) == wl;
#pragma unroll
        for (int i = 0; i < 4; ++i) f[i] += (mine && (best_i & 3) == i) ? 65536 - tot : 0;
    }
    int loc = ((f[0] + f[1]) + f[2]) + f[3];
    int c = wave_incl_scan_i(loc, wl) - loc;
    for (int i = 0; i < 4; ++i) { cx[i] = c; c += f[i]; }
}
DEVI void o2_update(uint16_t* row, int wl, int s, int total) {
    if ((s >> 2) == wl) row[s] = (uint16_t)(row[s] + 1);
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
    if (total + 1 >= 65536) {
        for (int i = 0; i < 4; ++i) {
            int v = row[4 * wl + i];
            row[4 * wl + i] = (uint16_t)((v + 1) >> 1);
        }
    }
    __threadfence_block();
}

__global__ void k_order2_encode(const uint8_t* __restrict__ data, const long long* __restrict__ off,
                                const long long* __restrict__ len, int n, uint16_t* __restrict__ counts,
                                uint8_t* __restrict__ payload, const long long* __restrict__ pay_off,
                                const long long* __restrict__ pay_cap, uint32_t* __restrict__ pay_len,
                                double* __restrict__ ideal) {
    int ch = blockIdx.x;
    int wl = threadIdx.x;
    if (ch >= n) return;
    long long ln = len[ch];
    if (ln <= 1) { if (wl == 0) { pay_len[ch] = 0; if (ideal) ideal[ch] = 0.0; } return; }
    const uint8_t* x = data + off[ch];
    uint16_t* cnt = counts + (long long)blockIdx.x * 65536LL * 256LL;
    uint8_t* out = payload + pay_off[ch];
    uint32_t cap = (uint32_t)pay_cap[ch];
    Enc e;
    enc_reset(e);
    double ib = 0.0;
    for (long long t = 1; t < ln; ++t) {
        int c2 = t >= 2 ? x[t - 2] : 0, c1 = x[t - 1];
        uint16_t* row = cnt + ((long long)(c2 * 256 + c1)) * 256;
        int f[4], cx[4], total;
        o2_table(row, wl, f, cx, total);
        int s = x[t];
        int cl = __shfl(cx[s & 3], s >> 2, 64), fs = __shfl(f[s & 3], s >> 2, 64);
        if (wl == 0) {
            enc_put(e, (uint32_t)cl, (uint32_t)fs, out, cap);
            ib += -log2((double)fs / 65536.0);
        }
        o2_update(row, wl, s, total);
    }
    if (wl == 0) {
        enc_flush(e, out, cap);
        pay_len[ch] = e.cur <= cap ? e.cur : 0xFFFFFFFFu;
        if (ideal) ideal[ch] = ib;
    }
}
hipError_t launch_order2_encode(const uint8_t* data, const long long* off, const long long* len, int n,
                                uint16_t* counts, uint8_t* payload, const long long* pay_off,
                                const long long* pay_cap, uint32_t* pay_len, double* ideal, hipStream_t s) {
    hipLaunchKernelGGL(k_order2_encode, dim3(n), dim3(64), 0, s, data, off, len, n, counts, payload, pay_off,
                       pay_cap, pay_len, ideal);
    return hipGetLastError();
}

__global__ void k_order2_decode(const uint8_t* __restrict__ payload, const long long* __restrict__ pay_off,
                                const long long* __restrict__ pay_len, const long long* __restrict__ off,
                                const long long* __restrict__ len, int n, uint16_t* __restrict__ counts,
                                uint8_t* __restrict__ outb) {
    int ch = blockIdx.x;
    int wl = threadIdx.x;
    if (ch >= n) return;
    long long ln = len[ch];
    if (ln <= 1) return;
    uint8_t* x = outb + off[ch];               // x[0] prefilled by the caller
    uint16_t* cnt = counts + (long long)blockIdx.x * 65536LL * 256LL;
    const uint8_t* in = payload + pay_off[ch];
    uint32_t plen = (uint32_t)pay_len[ch];
    Dec d;
    dec_reset(d, in, plen);
    int p1 = x[0], p2 = 0;
    for (long long t = 1; t < ln; ++t) {
        uint16_t* row = cnt + ((long long)(p2 * 256 + p1)) * 256;
        int f[4], cx[4], total;
        o2_table(row, wl, f, cx, total);
        uint32_t xt = dec_target(d);
        int hit = -1;
        for (int i = 0; i < 4; ++i)
            if ((uint32_t)cx[i] <= xt && xt < (uint32_t)(cx[i] + f[i])) hit = 4 * wl + i;
        unsigned long long bal = __ballot(hit >= 0);
        int src = bal ? (__ffsll((long long)bal) - 1) : 0;
        int s = __shfl(hit, src, 64);
        if (s < 0) s = 0;
        int cl = __shfl(cx[s & 3], s >> 2, 64), fs = __shfl(f[s & 3], s >> 2, 64);
        if (wl == 0) {
            dec_update(d, (uint32_t)cl, (uint32_t)fs, in, plen);
            x[t] = (uint8_t)s;
        }
        d.L = __shfl(d.L, 0, 64);
        d.R = __shfl(d.R, 0, 64);
        d.X = __shfl(d.X, 0, 64);
        d.cur = __shfl(d.cur, 0, 64);
        o2_update(row, wl, s, total);
        p2 = p1;
        p1 = s;
    }
}
hipError_t launch_order2_decode(const uint8_t* payload, const long long* pay_off, const long long* pay_len,
                                const long long* off, const long long* len, int n, uint16_t* counts,
                                uint8_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_order2_decode, dim3(n), dim3(64), 0, s, payload, pay_off, pay_len, off, len, n, counts,
                       out);
    return hipGetLastError();
}

}  // namespace boa
