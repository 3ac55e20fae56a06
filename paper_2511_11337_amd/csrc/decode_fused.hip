// Fused persistent decoder: one workgroup runs every decoding step of G
// lanes (streams) in a single launch -- embedding, all Mamba blocks, final
// LayerNorm, head, histogram / CDF and range decoding -- with the lanes'
// activations in LDS, the range-decoder state in registers, and the conv and
// scan state of each lane in LDS (one lane per workgroup) or in its own slice
// of device memory.  Decoding is
// inherently sequential per stream (each step needs the byte the previous
// step decoded; paper, Coders & Parallelisation); the per-step kernel chain
// of the step-graph decoder pays a launch and a cold start per kernel, this
// kernel pays them once per call.
//
// Every output element is produced by the same per-element operation
// sequence as in the encoder kernels, so the integer frequency tables (and
// hence the decoded bytes) are identical:
//   LayerNorm      the statistics of ln_stats (each wave takes them for its
//                  row) + ln_apply per element;
//   projections    the same MFMA instruction and k order as the encoder
//                  (f32: 16x16x4 in k steps of 4; bf16: 16x16x32 in k steps of
//                  32; fp8: 16x16x32 fp8 with the same per-row and per-tensor
//                  scales; from zero), the lane's row placed in a 16-row tile
//                  whose other rows are zero (MFMA rows are independent);
//   conv, x_proj, dt, scan, gate, histogram, coder: the shared device
//                  functions with the same operands in the same order.
//
// Projection weights are read in a fragment-ordered copy made at model load,
// so each MFMA operand load of a wave is 1 KiB of contiguous memory.
#include "boa_internal.h"

#include <hip/hip_bf16.h>

#include <type_traits>

#include "hotpath_common.h"

namespace boa {

// ============================================================== fragment-ordered weights
// f32 : element (nf, q, lane, j) = W[16 nf + (lane & 15)][16 q + 4 j + (lane >> 4)]
//       (one float4 per lane per q covers the MFMA k steps 4q .. 4q + 3)
// bf16: element (nf, s, lane, j) = bf16(W[16 nf + (lane & 15)][32 s + 8 (lane >> 4) + j])
__global__ void k_frag_f32(const float* __restrict__ W, int N, int K, float* __restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)N * K) return;
    const int j = (int)(i & 3);
    long long t = i >> 2;
    const int lane = (int)(t & 63);
    t >>= 6;
    const int q = (int)(t % (K / 16));
    const int nf = (int)(t / (K / 16));
    out[i] = W[(long long)(16 * nf + (lane & 15)) * K + 16 * q + 4 * j + (lane >> 4)];
}
__global__ void k_frag_f32_pad(const float* __restrict__ W, int N, int NP, int K, float* __restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)NP * K) return;
    const int j = (int)(i & 3);
    long long t = i >> 2;
    const int lane = (int)(t & 63);
    t >>= 6;
    const int q = (int)(t % (K / 16));
    const int nf = (int)(t / (K / 16));
    const int row = 16 * nf + (lane & 15);
    out[i] = row < N ? W[(long long)row * K + 16 * q + 4 * j + (lane >> 4)] : 0.0f;
}
hipError_t launch_frag_pad(const float* W, int N, int NP, int K, float* out, hipStream_t s) {
    if (NP % 16 || NP < N || K % 16) return hipErrorInvalidValue;
    const long long n = (long long)NP * K;
    hipLaunchKernelGGL(k_frag_f32_pad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, N, NP, K, out);
    return hipGetLastError();
}
__global__ void k_frag_bf16(const float* __restrict__ W, int N, int K, uint16_t* __restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)N * K) return;
    const int j = (int)(i & 7);
    long long t = i >> 3;
    const int lane = (int)(t & 63);
    t >>= 6;
    const int s = (int)(t % (K / 32));
    const int nf = (int)(t / (K / 32));
    out[i] = f2bf_bits(W[(long long)(16 * nf + (lane & 15)) * K + 32 * s + 8 * (lane >> 4) + j]);
}
// Largest |w| of a tensor as float bits (non-negative floats order like their
// unsigned bit patterns, so an integer maximum is exact and order-free).
__global__ void k_amax(const float* __restrict__ W, long long n, unsigned* __restrict__ amax_bits) {
    float m = 0.0f;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(W[i]));
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) atomicMax(amax_bits, __float_as_uint(m));
}
// fp8: element (nf, p, lane, h, j) = e4m3(W[16 nf + lane % 16][32 (2p + h) + 8 (lane / 16) + j] * 2^-e)
// (16 bytes per lane cover MFMA k steps 2p and 2p + 1); e = fp8_exp(amax),
// written to *ew by element 0.
__global__ void k_frag_fp8(const float* __restrict__ W, int N, int K, const unsigned* __restrict__ amax_bits,
                           int* __restrict__ ew, uint8_t* __restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)N * K) return;
    const int e = fp8_exp(__uint_as_float(*amax_bits));
    if (i == 0) *ew = e;
    const int j = (int)(i & 7), h = (int)((i >> 3) & 1), lane = (int)((i >> 4) & 63);
    const long long t = i >> 10;
    const int SP = K / 64;
    const int p = (int)(t % SP), nf = (int)(t / SP);
    const float w = W[(long long)(16 * nf + (lane & 15)) * K + 32 * (2 * p + h) + 8 * (lane >> 4) + j];
    out[i] = fp8_byte(ldexpf(w, -e));
}
hipError_t launch_frag(const float* W, int N, int K, float* f32, uint16_t* b16, uint8_t* f8, unsigned* amax,
                       int* ew, hipStream_t s) {
    if (N % 16 || K % 64) return hipErrorInvalidValue;
    const long long n = (long long)N * K;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_frag_f32, dim3(nb), dim3(256), 0, s, W, N, K, f32);
    hipLaunchKernelGGL(k_frag_bf16, dim3(nb), dim3(256), 0, s, W, N, K, b16);
    hipError_t e = hipMemsetAsync(amax, 0, sizeof(unsigned), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_amax, dim3(256), dim3(256), 0, s, W, n, amax);
    hipLaunchKernelGGL(k_frag_fp8, dim3(nb), dim3(256), 0, s, W, N, K, amax, ew, f8);
    return hipGetLastError();
}

// ============================================================== fused decoder
namespace {
// Weight pointers reach the kernel through a device array, so the compiler
// cannot prove they address global memory and would emit FLAT loads, which
// share the LDS wait counter and serialise every LDS access behind every
// outstanding weight load.  Casting them to the global address space keeps
// the weight stream asynchronous.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
DEVI float gld(const float* p) { return *(const __attribute__((address_space(1))) float*)p; }
DEVI float4 gld(const float4* p) {
    const f32x4 v = *(const __attribute__((address_space(1))) f32x4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
DEVI uint4 gld(const uint4* p) {
    const u32x4 v = *(const __attribute__((address_space(1))) u32x4*)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
DEVI uint2 gld(const uint2* p) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 v = *(const __attribute__((address_space(1))) u32x2*)p;
    return make_uint2(v.x, v.y);
}
// The lanes' conv and scan state is read once and written once per step, a
// stream far larger than the L2: non-temporal accesses keep it from evicting
// the weights, which every workgroup reads every step.
DEVI float gld_nt(const float* p) { return __builtin_nontemporal_load((const __attribute__((address_space(1))) float*)p); }
DEVI float4 gld_nt(const float4* p) {
    const f32x4 v = __builtin_nontemporal_load((const __attribute__((address_space(1))) f32x4*)p);
    return make_float4(v.x, v.y, v.z, v.w);
}
DEVI void gst_nt(float* p, float v) { __builtin_nontemporal_store(v, (__attribute__((address_space(1))) float*)p); }
DEVI void gst_nt(float4* p, float4 v) {
    const f32x4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, (__attribute__((address_space(1))) f32x4*)p);
}
// four bf16 (element j in bits 16 j .. 16 j + 15) as exact floats
DEVI float4 bf4(uint2 v) {
    return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xFFFF0000u), __uint_as_float(v.y << 16),
                       __uint_as_float(v.y & 0xFFFF0000u));
}
DEVI float4 xq_f(float4 v) { return v; }
DEVI float4 xq_f(uint2 v) { return bf4(v); }
// dt_proj weights of channel d: float [R][Di] copy, or in BF16 mode the bf16
// parameter [Di][R] (R / 4 loads of four)
template <int DT, int RR>
struct DtW {
    static constexpr int NQ = DT == 1 ? RR / 4 : 1;
    float f[DT == 1 ? 1 : RR];
    uint2 q[NQ];
    DEVI void load(const FusedLayer& w, int Di, int d) {
        if (DT == 1) {
            const uint2* src = reinterpret_cast<const uint2*>(w.dtw16 + (long long)d * RR);
#pragma unroll
            for (int i = 0; i < NQ; ++i) q[i] = gld(src + i);
        } else {
#pragma unroll
            for (int k = 0; k < RR; ++k) f[k] = gld(w.dtwT + k * Di + d);
        }
    }
    DEVI void get(float (&o)[RR]) const {
        if (DT == 1) {
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                const float4 v = bf4(q[i]);
                o[4 * i] = v.x; o[4 * i + 1] = v.y; o[4 * i + 2] = v.z; o[4 * i + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < RR; ++k) o[k] = f[DT == 1 ? 0 : k];
        }
    }
};
static_assert(sizeof(uint16_t) == 2, "bf16 bits");

// base + an unsigned 32-bit byte offset: a scalar base and a per-lane offset
// map onto the scalar-base addressing mode of the global loads
template <typename T>
DEVI T gld_off(const T* base, uint32_t byte_off) {
    return gld(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off));
}

constexpr int FNT = 512;              // threads per workgroup
constexpr int FNW = FNT / 64;         // waves

template <int D, int Di, int RR, int G>
struct FusedLds {
    static constexpr int NO = RR + 2 * NSTATE;
    static constexpr int DS = D + 4;          // padded row strides (floats)
    static constexpr int GS = Di + 4;
    static constexpr int XSR = Di + 4;        // row stride of xs (rows 4 banks apart)
    static constexpr int ZS = Di > VOCAB ? Di : VOCAB;     // row stride of the z half / logits
    static constexpr int r = 0;                            // [G][D]    residual stream
    static constexpr int a = r + G * D;                    // [G][DS]   LayerNorm output
    static constexpr int xz = a + G * DS;                  // [G][ZS]   z half of in_proj / logits [G][256]
    static constexpr int g = xz + G * ZS;                  // [G][GS]   gated mixer output
    static constexpr int xs = g + G * GS;                  // [G][XSR]  conv + SiLU output
    static constexpr int dbc = xs + G * XSR;               // [G][NO]   (delta, B, C)
    static constexpr int g8 = dbc + G * NO;                // [G][Di] bytes: fp8 gated rows
    static constexpr int total = g8 + G * Di / 4;          // floats
};

// One projection of the G rows of A: C[row][n] = A[row][:] . W[n][:].  The B
// operand is read in load steps (f32: one float4 = 4 MFMA k steps; bf16: one
// uint4 = one k step; fp8: one uint4 = two k steps) through a register ring
// that keeps about 16 loads per wave in flight.
template <int DT> struct BLoad;
template <> struct BLoad<0> { using T = float4; static constexpr int KPL = 16; };
template <> struct BLoad<1> { using T = uint4; static constexpr int KPL = 32; };
template <> struct BLoad<2> { using T = uint4; static constexpr int KPL = 64; };   // fp8: two k steps of 32

// The NF fragments of W are dealt to the waves (wave w owns w, w + 8, ...),
// at most 8 per pass.  issue() requests the first ring of B loads of the
// wave's first pass; it can be called a phase early so the loads arrive while
// other work runs.  run() completes the product and hands each pass's
// accumulators to the caller's epilogue, epi(acc, f0): lane l holds rows
// 4 (l >> 4) + rr (rr < 4) of column l & 15 of fragments f0 + 8 j (fp8:
// already rescaled by the row and weight scales).
// A8 (fp8 only): the A rows are already E4M3 bytes (row stride 4 * as bytes,
// scaled by 2^-ea of their row) instead of floats quantised here per k step.
template <int DT, int G, int K, int NF, bool A8 = false>
struct FGemm {
    using BT = typename BLoad<DT>::T;
    static constexpr int FALL = (NF + FNW - 1) / FNW;      // fragments per wave
    static constexpr int FPW = FALL < 8 ? FALL : 8;        // per pass
    static constexpr int SK = K / BLoad<DT>::KPL;          // load steps per fragment
    static constexpr int PW = 16 / FPW > 0 ? 16 / FPW : 1;
    static constexpr int P = PW < SK ? PW : SK;            // load steps in flight (power of 2, divides SK)
    static_assert(SK % P == 0, "ring period");
    using Acc = v4f[FPW];
    BT ring[P][FPW];

    // Weight loads are raw buffer loads: the fragment offset (wave-uniform,
    // f0 comes from a scalar) goes in a scalar register, the lane offset is
    // the one vector register, so a load costs no address arithmetic;
    // fragments past the matrix (nf >= NF) lie outside the buffer's range and
    // read as zero.
    static constexpr int ES = DT == 0 ? 4 : (DT == 1 ? 2 : 1);   // bytes per weight
    DEVI static __amdgpu_buffer_rsrc_t rsrc(const void* Wf) {
        // base, stride 0, range = the whole fragment-ordered matrix (16 NF x K)
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(Wf), (short)0, 16 * NF * K * ES, 0x00020000);
    }
    DEVI static BT ld(__amdgpu_buffer_rsrc_t r, int f0, int st, int j, int wl) {
        const int nf = f0 + FNW * j;
        typedef unsigned int u4v __attribute__((ext_vector_type(4)));
        const u4v v = __builtin_amdgcn_raw_buffer_load_b128(r, wl * (int)sizeof(BT), (nf * SK + st) * 64 * (int)sizeof(BT), 0);
        BT o;
        __builtin_memcpy(&o, &v, sizeof(BT));
        return o;
    }
    DEVI void issue(const void* Wf, int f0, int wl) {
        const __amdgpu_buffer_rsrc_t r = rsrc(Wf);
#pragma unroll
        for (int u = 0; u < P; ++u)
#pragma unroll
            for (int j = 0; j < FPW; ++j) ring[u][j] = ld(r, f0, u, j, wl);
    }
    // the pass over fragments f0, f0 + 8, ... whose first ring is in flight
    template <class Epi>
    DEVI void pass(const float* __restrict__ A, int as, const void* __restrict__ Wf, const unsigned* amax_rows,
                   int ew, int wl, int f0, Epi& epi) {
        const int li = wl & 15, lk = wl >> 4;
        const bool arow = li < G;
        const __amdgpu_buffer_rsrc_t rs = rsrc(Wf);
        // fp8: this lane's A row scale 2^-ea (rows >= G are zero)
        const int ea = (DT == 2 && !A8 && arow) ? fp8_exp(__uint_as_float(amax_rows[li])) : 0;
        v4f acc[FPW];
#pragma unroll
        for (int j = 0; j < FPW; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s0 = 0; s0 < SK; s0 += P) {
#pragma unroll
            for (int u = 0; u < P; ++u) {
                const int st = s0 + u;
                BT cur[FPW];
#pragma unroll
                for (int j = 0; j < FPW; ++j) cur[j] = ring[u][j];
                if (st + P < SK) {
#pragma unroll
                    for (int j = 0; j < FPW; ++j) ring[u][j] = ld(rs, f0, st + P, j, wl);
                }
                if (DT == 0) {
                    float av[4];
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) av[jj] = arow ? A[li * as + 16 * st + 4 * jj + lk] : 0.0f;
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                        for (int j = 0; j < FPW; ++j) {
                            const float4 c4 = *reinterpret_cast<const float4*>(&cur[j]);
                            const float b = jj == 0 ? c4.x : jj == 1 ? c4.y : jj == 2 ? c4.z : c4.w;
                            acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[jj], b, acc[j], 0, 0, 0);
                        }
                } else if (DT == 2) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        uint64_t a8 = 0;
                        if (arow && A8) {
                            a8 = *reinterpret_cast<const uint64_t*>(reinterpret_cast<const uint8_t*>(A) + li * 4 * as +
                                                                    32 * (2 * st + h) + 8 * lk);
                        } else if (arow) {
                            const float* src = A + li * as + 32 * (2 * st + h) + 8 * lk;
                            const float4 x0 = *reinterpret_cast<const float4*>(src);
                            const float4 x1 = *reinterpret_cast<const float4*>(src + 4);
                            const float xv[8] = {ldexpf(x0.x, -ea), ldexpf(x0.y, -ea), ldexpf(x0.z, -ea),
                                                 ldexpf(x0.w, -ea), ldexpf(x1.x, -ea), ldexpf(x1.y, -ea),
                                                 ldexpf(x1.z, -ea), ldexpf(x1.w, -ea)};
                            a8 = fp8_pack8(xv);
                        }
#pragma unroll
                        for (int j = 0; j < FPW; ++j) {
                            const uint4 c4 = *reinterpret_cast<const uint4*>(&cur[j]);
                            const uint64_t b8 = h == 0 ? ((uint64_t)c4.x | ((uint64_t)c4.y << 32))
                                                       : ((uint64_t)c4.z | ((uint64_t)c4.w << 32));
                            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8((long)a8, (long)b8, acc[j], 0, 0, 0);
                        }
                    }
                } else {
                    // bf16: the A rows were rounded to bf16 when written (row
                    // stride 2 * as halves in the same buffer)
                    uint4 uu = make_uint4(0, 0, 0, 0);
                    if (arow)
                        uu = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint16_t*>(A) + li * 2 * as +
                                                             32 * st + 8 * lk);
                    const v8bf av = *reinterpret_cast<const v8bf*>(&uu);
#pragma unroll
                    for (int j = 0; j < FPW; ++j)
                        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            av, *reinterpret_cast<const v8bf*>(&cur[j]), acc[j], 0, 0, 0);
                }
            }
        }
        if (DT == 2) {
#pragma unroll
            for (int j = 0; j < FPW; ++j)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int row = 4 * lk + rr;
                    if (row < G) acc[j][rr] = ldexpf(acc[j][rr], fp8_exp(__uint_as_float(amax_rows[row])) + ew);
                }
        }
        epi(acc, f0);
    }
    // every pass of wave wv; the first pass's ring must have been issued
    // (fp8: amax_rows are the A rows' largest magnitudes as float bits, ew
    // W's scale exponent)
    template <class Epi>
    DEVI void run(const float* __restrict__ A, int as, const void* __restrict__ Wf, int wl, int wv,
                  const unsigned* amax_rows, const int* ewp, Epi&& epi) {
        const int ew = DT == 2 ? *ewp : 0;
        pass(A, as, Wf, amax_rows, ew, wl, wv, epi);
#pragma unroll 1
        for (int f = FPW; f < FALL; f += FPW) {
            issue(Wf, wv + FNW * f, wl);
            pass(A, as, Wf, amax_rows, ew, wl, wv + FNW * f, epi);
        }
    }
};

// f(j, rr, row, n, v) for every output of a pass that this lane holds
template <int FPW, int G, int NF, class F>
DEVI void for_outputs(const v4f (&acc)[FPW], int f0, int wl, F&& f) {
    const int li = wl & 15, lk = wl >> 4;
#pragma unroll
    for (int j = 0; j < FPW; ++j) {
        const int nf = f0 + FNW * j;
        if (nf >= NF) continue;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int row = 4 * lk + rr;
            if (row < G) f(j, rr, row, 16 * nf + li, acc[j][rr]);
        }
    }
}

// LayerNorm of the G residual rows into a_s.  Element i = tid + 512 m is
// normalised by its thread; the 64 elements of a wave lie in one row (D is a
// multiple of 64), and the wave takes that row's statistics itself
// (ln_stats_v: every wave that reads a row gets the same values), so no
// barrier separates statistics from normalisation.  With G * D <= 512 the
// caller loads each thread's LayerNorm weight and bias early (LnPre).
template <int D, int G>
struct LnPre {
    static constexpr bool ONE = G * D <= FNT;
    float w = 0.0f, b = 0.0f;
    DEVI void load(const float* lw, const float* lb, int tid) {
        if (ONE && tid < G * D) { w = gld(lw + tid % D); b = gld(lb + tid % D); }
    }
};
// With amax_s (fp8), the first wave of each row also takes the row's largest
// normalised magnitude (the same ln_apply values as the normalisation).
// B16: the normalised rows are stored rounded to bf16 (the GEMM's A operand
// in bf16 mode), row stride 2 * ds halves.
// F8: every wave takes the row's largest normalised magnitude itself and
// stores its elements as E4M3 bytes scaled by 2^-ea (row stride 4 * ds bytes),
// the A operand of the fp8 GEMM.
template <int D, int G, bool B16 = false, bool F8 = false>
DEVI void fused_ln(const float* __restrict__ r_s, float* __restrict__ a_s, int ds, const float* __restrict__ lw,
                   const float* __restrict__ lb, const LnPre<D, G>& pre, int wl, int wv, unsigned* amax_s = nullptr) {
    constexpr int NV = D / 64;
    static_assert(D % 64 == 0, "rows of whole waves");
#pragma unroll 1
    for (int i0 = 64 * wv; i0 < G * D; i0 += FNT) {      // wave-uniform
        const int row = i0 / D, kw = i0 % D;
        float v[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = r_s[row * D + wl + 64 * j];
        float mu, rs;
        ln_stats_v<NV>(v, D, mu, rs);
        float am = 0.0f;
        if (amax_s && (F8 || kw == 0)) {
#pragma unroll
            for (int j = 0; j < NV; ++j)
                am = fmaxf(am, fabsf(ln_apply(v[j], mu, rs, gld(lw + wl + 64 * j), gld(lb + wl + 64 * j))));
            am = wave_max(am);
            if (kw == 0 && wl == 0) amax_s[row] = __float_as_uint(am);
        }
        const int k = kw + wl;
        float x = 0.0f;
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (64 * j == kw) x = v[j];
        const float g = LnPre<D, G>::ONE ? pre.w : gld(lw + k);
        const float bb = LnPre<D, G>::ONE ? pre.b : gld(lb + k);
        const float y = ln_apply(x, mu, rs, g, bb);
        if (F8) reinterpret_cast<uint8_t*>(a_s)[row * 4 * ds + k] = fp8_byte(ldexpf(y, -fp8_exp(am)));
        else if (B16) reinterpret_cast<uint16_t*>(a_s)[row * 2 * ds + k] = f2bf_bits(y);
        else a_s[row * ds + k] = y;
    }
    __syncthreads();
}
}  // namespace

// SL: the lanes' conv and scan state live in LDS after the activations
// ([n_layers][G][K-1][Di] then [n_layers][G][N][Di]) instead of device memory.
// Without SL the state lives in device memory, one record per (layer, lane):
// conv window [K-1][Di] (taps t-3, t-2, t-1) and h [N/4][Di] float4, so the
// accesses of a wave are contiguous.
//
// Decoding waves: wave w decodes lanes w, w + 8, ... of the workgroup (one
// lane per wave up to G = 8, two at G = 16).
template <int DT, int D, int Di, int RR, int G, bool SL>
__global__ __launch_bounds__(FNT) void k_dec_fused(FusedArgs a) {
    using S = FusedLds<D, Di, RR, G>;
    constexpr int NO = S::NO, ZS = S::ZS;
    constexpr int LPW = (G + FNW - 1) / FNW;      // lanes decoded per wave
    static_assert(G >= 1 && G <= 16, "at most 16 lanes (one MFMA tile of rows) per workgroup");
    static_assert(!SL || G == 1, "state in LDS with one lane per workgroup only");
    extern __shared__ __align__(16) float sm[];
    float* r_s = sm + S::r;
    float* a_s = sm + S::a;
    float* xz_s = sm + S::xz;
    float* g_s = sm + S::g;
    float* xs_s = sm + S::xs;
    float* dbc_s = sm + S::dbc;
    uint8_t* g8_s = reinterpret_cast<uint8_t*>(sm + S::g8);
    float* cst_s = sm + S::total;                                  // SL only
    float* hst_s = cst_s + (size_t)a.n_layers * G * (KCONV - 1) * Di;
    __shared__ int pos_s[G], chunk_s[G];
    __shared__ float hb_s[VOCAB];                 // head bias, read every step
    __shared__ unsigned am_ln[G], am_g[G];        // fp8: row maxima of the LayerNorm output and of g
    unsigned* am_ln_p = DT == 2 ? am_ln : nullptr;
    // wave index as a wave-uniform (scalar) value: weight addresses that depend
    // only on it are formed in scalar registers
    const int tid = threadIdx.x, wl = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane0 = blockIdx.x * G;

    for (int i = tid; i < S::total; i += FNT) sm[i] = 0.0f;
    for (int i = tid; i < VOCAB; i += FNT) hb_s[i] = a.head_b[i];
    // Per decoded lane of this wave: its schedule position, range decoder and
    // the current chunk's payload, output offset and step count (read once
    // per chunk instead of every step).  Decoded bytes gather in the decoding
    // wave's lanes, lane i holding the byte at offset i of the current
    // 64-byte output block; they leave in one store when the block or the
    // chunk ends.
    struct LaneDec {
        int c, pos;
        long long lstep;
        Dec dc;
        const uint8_t* pin;
        uint32_t plen;
        long long obase;
        int csteps;
        uint32_t obyte, pbyte;
    };
    LaneDec ld[LPW];
    auto enter_chunk = [&](LaneDec& q, int ch) {
        q.pin = a.payload + a.pay_off[ch];
        q.plen = (uint32_t)a.pay_len[ch];
        q.obase = a.p.chunk_off[ch];
        q.csteps = a.p.chunk_steps[ch];
    };
#pragma unroll
    for (int k = 0; k < LPW; ++k) {
        LaneDec& q = ld[k];
        q.c = -1; q.pos = -1; q.lstep = 0; q.dc = Dec{}; q.pin = nullptr; q.plen = 0; q.obase = 0; q.csteps = 0;
        q.obyte = 0; q.pbyte = 0;
        const int gl = wv + FNW * k;
        if (gl < G && lane0 + gl < a.lanes) locate(a.p, lane0 + gl, 0, q.c, q.pos);
        if (gl < G && q.pos >= 0) enter_chunk(q, q.c);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < LPW; ++k) {
        const LaneDec& q = ld[k];
        const int gl = wv + FNW * k;
        if (gl < G) {
            if (q.pos >= 0) {
                const int y = a.out[q.obase + q.pos];
                const float* er = a.E + (long long)y * D;
                for (int kk = wl; kk < D; kk += 64) r_s[gl * D + kk] = er[kk];
            }
            if (wl == 0) { pos_s[gl] = q.pos; chunk_s[gl] = q.c; }
        }
    }
    __syncthreads();

    // The LayerNorm weights of the next LayerNorm (layer l, or the final one
    // for l == n_layers) are requested one phase ahead; with one lane per
    // workgroup, the conv weights of the in_proj epilogue before its LayerNorm
    using GIn = FGemm<DT, G, D, 2 * Di / 16, DT == 2>;
    constexpr int XF = GIn::FALL / 2 < GIn::FPW ? GIn::FALL / 2 : GIn::FPW;   // x-half fragments per wave
    constexpr bool CWP = XF <= 4 && G == 1 && DT != 2;
    LnPre<D, G> lnp;
    float pcw[CWP ? XF : 1][KCONV], pcb[CWP ? XF : 1];
    auto pre_layer = [&](int l) {
        if (l == a.n_layers) lnp.load(a.norm_f_w, a.norm_f_b, tid);
        else lnp.load(a.layers[l].norm_w, a.layers[l].norm_b, tid);
    };
    auto pre_conv = [&](const FusedLayer& w) {
        if (CWP) {
#pragma unroll
            for (int j = 0; j < XF; ++j) {
                const int n = 16 * (wv + FNW * j) + (wl & 15);
#pragma unroll
                for (int k = 0; k < KCONV; ++k) pcw[j][k] = gld(w.convT + k * Di + n);
                pcb[j] = gld(w.conv_b + n);
            }
        }
    };
    pre_layer(0);
    for (long long it = 0; it < a.max_steps; ++it) {
        bool any = false;
#pragma unroll
        for (int g = 0; g < G; ++g) any = any || pos_s[g] >= 0;
        if (!any) break;                                 // uniform: read after a barrier
        // the decoding wave requests its next 8 payload bytes now, one per
        // lane (lane i: byte cur + i, zero past the payload); nothing waits
        // for them until the decoding after the model pass
#pragma unroll
        for (int k = 0; k < LPW; ++k) {
            LaneDec& q = ld[k];
            q.pbyte = 0;
            if (wv + FNW * k < G && q.pos >= 0) {
                if (q.pos == 0) dec_reset(q.dc, q.pin, q.plen);
                if (wl < 8 && q.dc.cur + (uint32_t)wl < q.plen)
                    q.pbyte = *(const __attribute__((address_space(1))) uint8_t*)(q.pin + q.dc.cur + wl);
            }
        }

        for (int l = 0; l < a.n_layers; ++l) {
            const FusedLayer& w = a.layers[l];
            // Weights are requested ahead of their phase where that hides a
            // latency without delaying other loads: the LayerNorm weights
            // during the previous out_proj (pre_layer), the conv weights
            // before the LayerNorm, the dt / scan weights before the barrier
            // that precedes x_proj, the out_proj ring at the
            // end of the scan (issued before it, the ring's registers pushed
            // the scan's state loads into spills).
            pre_conv(w);
            // the in_proj ring goes out before the LayerNorm (fp8: after it;
            // there the early ring cost more than it hid)
            GIn gin;
            if (DT != 2) gin.issue(w.in_frag, wv, wl);
            fused_ln<D, G, DT == 1, DT == 2>(r_s, a_s, S::DS, w.norm_w, w.norm_b, lnp, wl, wv, am_ln_p);
            {
                // epilogue: the x half goes through the causal conv + SiLU
                // right here (channels are independent), advancing the conv
                // state; the z half is stored for the gate
                auto epi_in = [&](const typename GIn::Acc& acc, int f0) {
                    const int li = wl & 15, lk = wl >> 4;
                    // conv window of (row, channel n): [K-1][Di] in LDS (SL) or
                    // in the row's device record
                    auto cst_lds = [&](int row) { return cst_s + (l * G + row) * (KCONV - 1) * Di; };
                    auto cst_dev = [&](int row) {
                        return a.conv_state + ((long long)l * a.lanes + lane0 + row) * (KCONV - 1) * Di;
                    };
                    // every weight and state load of the pass first, then the arithmetic
                    float cw[XF][KCONV], cb[XF], st[XF][4][KCONV - 1];
#pragma unroll
                    for (int j = 0; j < XF; ++j) {
                        const int nf = f0 + FNW * j;
                        if (nf >= Di / 16) continue;             // later passes hold z only
                        const int n = 16 * nf + li;
                        if (CWP) {
#pragma unroll
                            for (int k = 0; k < KCONV; ++k) cw[j][k] = pcw[CWP ? j : 0][k];
                            cb[j] = pcb[CWP ? j : 0];
                        } else {
#pragma unroll
                            for (int k = 0; k < KCONV; ++k) cw[j][k] = gld(w.convT + k * Di + n);
                            cb[j] = gld(w.conv_b + n);
                        }
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr) {
                            const int row = 4 * lk + rr;
                            const bool live = row < G && pos_s[row] > 0;
                            if (SL) {
                                const float* cs = cst_lds(0);
#pragma unroll
                                for (int k = 0; k < KCONV - 1; ++k) st[j][rr][k] = live ? cs[k * Di + n] : 0.0f;
                            } else {
                                const float* cs = cst_dev(live ? row : 0);
#pragma unroll
                                for (int k = 0; k < KCONV - 1; ++k) st[j][rr][k] = live ? gld_nt(cs + k * Di + n) : 0.0f;
                            }
                        }
                    }
                    for_outputs<GIn::FPW, G, 2 * Di / 16>(acc, f0, wl, [&](int j, int rr, int row, int n, float v) {
                        if (n < Di) {
                            const int jx = j < XF ? j : 0;           // x fragments are j < XF
                            if (pos_s[row] < 0) return;
                            xs_s[row * S::XSR + n] =
                                conv_silu(cw[jx], cb[jx], st[jx][rr][0], st[jx][rr][1], st[jx][rr][2], v);
                            if (SL) {
                                float* cs = cst_lds(row);
                                cs[n] = st[jx][rr][1];
                                cs[Di + n] = st[jx][rr][2];
                                cs[2 * Di + n] = v;
                            } else {
                                float* cs = cst_dev(row);
                                gst_nt(cs + n, st[jx][rr][1]);
                                gst_nt(cs + Di + n, st[jx][rr][2]);
                                gst_nt(cs + 2 * Di + n, v);
                            }
                        } else {
                            xz_s[row * ZS + (n - Di)] = v;
                        }
                    });
                };
                if (DT == 2) gin.issue(w.in_frag, wv, wl);
                gin.run(a_s, S::DS, w.in_frag, wl, wv, am_ln, w.in_ew, epi_in);
            }
            constexpr bool ONE = Di <= FNT;                    // one channel per thread in the scan
            DtW<DT, RR> pdtw;
            float pA2[NSTATE], pdtb = 0.0f, pDk = 0.0f;
            if (ONE && tid < Di) {
                pdtw.load(w, Di, tid);
#pragma unroll
                for (int n = 0; n < NSTATE; ++n) pA2[n] = gld(w.A2T + n * Di + tid);
                pdtb = gld(w.dtb + tid);
                pDk = gld(w.Dsk + tid);
            }
            constexpr int NFX = (NO + 15) / 16;
            __syncthreads();
            // x_proj on the matrix cores: wave f computes column fragment f
            // of the lanes' rows (xproj_fragment, a ring of 4 weight loads)
            if (wv < NFX) {
                v4f acc;
                xproj_fragment<Di, 4>(xs_s, S::XSR, G, w.xw_frag, wv, wl, acc);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int row = 4 * (wl >> 4) + rr, col = 16 * wv + (wl & 15);
                    if (row < G && col < NO) dbc_s[row * NO + col] = acc[rr];
                }
            }
            if (DT == 2 && tid < G) am_g[tid] = 0u;
            using GOut = FGemm<DT, G, Di, D / 16, DT == 2>;
            GOut gout;
            __syncthreads();
            // dt_proj + softplus, selective scan, gate
            for (int d = tid; d < Di; d += FNT) {
                float dtw[RR], A2[NSTATE], dtb, Dk;
                if (ONE) {
                    pdtw.get(dtw);
#pragma unroll
                    for (int n = 0; n < NSTATE; ++n) A2[n] = pA2[n];
                    dtb = pdtb;
                    Dk = pDk;
                } else {
                    {
                        DtW<DT, RR> t;
                        t.load(w, Di, d);
                        t.get(dtw);
                    }
#pragma unroll
                    for (int n = 0; n < NSTATE; ++n) A2[n] = gld(w.A2T + n * Di + d);
                    dtb = gld(w.dtb + d);
                    Dk = gld(w.Dsk + d);
                }
                // The scan state goes in parts of SQ states for a group of up to
                // 8 lane slots at once, so the loads of a part are all in
                // flight together (one slot after another would wait G times
                // per layer).  h of slot g: LDS [N][Di] (SL) or the slot's
                // device record [N/4][Di] float4 (a wave's access is 1 KiB
                // contiguous).  Each state is updated and folded into y in
                // increasing n, the sequence of scan_update.
                constexpr int GB = G < 8 ? G : 8;                  // slots per group
                constexpr int SQ = GB <= 4 ? NSTATE : 8;           // states per part
                constexpr int NP = NSTATE / SQ;
                static_assert(SQ % 4 == 0 && NSTATE % SQ == 0 && G % GB == 0, "parts of whole float4s");
                auto hrec = [&](int g) {
                    return reinterpret_cast<float4*>(a.h_state) +
                           ((long long)l * a.lanes + lane0 + g) * (NSTATE / 4) * Di + d;
                };
#pragma unroll 1
                for (int g0 = 0; g0 < G; g0 += GB) {
                    float hp[GB][SQ];
                    auto load_part = [&](int p) {
#pragma unroll
                        for (int b = 0; b < GB; ++b) {
                            const int g = g0 + b;
                            const bool live = pos_s[g] > 0;
                            if (SL) {
                                const float* hst = hst_s + (l * G + g) * NSTATE * Di;
#pragma unroll
                                for (int s = 0; s < SQ; ++s) hp[b][s] = live ? hst[(p * SQ + s) * Di + d] : 0.0f;
                            } else {
#pragma unroll
                                for (int q = 0; q < SQ / 4; ++q) {
                                    float4 v4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                                    if (live) v4 = gld_nt(hrec(g) + (long long)(p * SQ / 4 + q) * Di);
                                    hp[b][4 * q] = v4.x; hp[b][4 * q + 1] = v4.y;
                                    hp[b][4 * q + 2] = v4.z; hp[b][4 * q + 3] = v4.w;
                                }
                            }
                        }
                    };
                    load_part(0);
                    float dtv[GB], xsv[GB], yv[GB];
#pragma unroll
                    for (int b = 0; b < GB; ++b) {
                        const int g = g0 + b;
                        dtv[b] = 0.0f; xsv[b] = 0.0f; yv[b] = 0.0f;
                        if (pos_s[g] < 0) continue;
                        dtv[b] = dt_of<RR>(dbc_s + g * NO, dtw, dtb);
                        xsv[b] = xs_s[g * S::XSR + d];
                    }
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        if (p > 0) load_part(p);
#pragma unroll
                        for (int b = 0; b < GB; ++b) {
                            const int g = g0 + b;
                            if (pos_s[g] < 0) continue;
                            const float* Bv = dbc_s + g * NO + RR + p * SQ;
                            const float* Cv = Bv + NSTATE;
                            const float dx = dtv[b] * xsv[b];
#pragma unroll
                            for (int s = 0; s < SQ; ++s) {
                                const float dA = exp2_hw(dtv[b] * A2[p * SQ + s]);
                                hp[b][s] = fmaf(dA, hp[b][s], dx * Bv[s]);
                            }
                            float y = yv[b];
#pragma unroll
                            for (int s = 0; s < SQ; ++s) y = fmaf(hp[b][s], Cv[s], y);
                            yv[b] = y;
                            if (SL) {
                                float* hst = hst_s + (l * G + g) * NSTATE * Di;
#pragma unroll
                                for (int s = 0; s < SQ; ++s) hst[(p * SQ + s) * Di + d] = hp[b][s];
                            } else {
#pragma unroll
                                for (int q = 0; q < SQ / 4; ++q)
                                    gst_nt(hrec(g) + (long long)(p * SQ / 4 + q) * Di,
                                        make_float4(hp[b][4 * q], hp[b][4 * q + 1], hp[b][4 * q + 2], hp[b][4 * q + 3]));
                            }
                        }
                    }
#pragma unroll
                    for (int b = 0; b < GB; ++b) {
                        const int g = g0 + b;
                        if (pos_s[g] < 0) continue;
                        const float gv = fmaf(Dk, xsv[b], yv[b]) * silu_hp(xz_s[g * ZS + d]);
                        if (DT == 1) reinterpret_cast<uint16_t*>(g_s)[g * 2 * S::GS + d] = f2bf_bits(gv);
                        else g_s[g * S::GS + d] = gv;
                        if (DT == 2) {            // row maximum: per wave first, then one LDS atomic per wave
                            const float wm = wave_max(fabsf(gv));
                            if (wl == 0) atomicMax(&am_g[g], __float_as_uint(wm));
                        }
                    }
                }
            }
            gout.issue(w.out_frag, wv, wl);
            __syncthreads();
            pre_layer(l + 1);
            if (DT == 2) {
                // the gated rows as E4M3 bytes scaled by 2^-ea of their row (the
                // row maxima are complete)
                for (int d = tid; d < Di; d += FNT) {
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        if (pos_s[g] >= 0)
                            g8_s[g * Di + d] = fp8_byte(ldexpf(g_s[g * S::GS + d], -fp8_exp(__uint_as_float(am_g[g]))));
                }
                __syncthreads();
            }
            // out_proj, added into the residual stream
            gout.run(DT == 2 ? reinterpret_cast<float*>(g8_s) : g_s, DT == 2 ? Di / 4 : S::GS, w.out_frag, wl, wv, am_g, w.out_ew, [&](const typename GOut::Acc& acc, int f0) {
                for_outputs<GOut::FPW, G, D / 16>(acc, f0, wl, [&](int, int, int row, int n, float v) {
                    r_s[row * D + n] = r_s[row * D + n] + v;
                });
            });
            __syncthreads();
        }
        using GH = FGemm<DT, G, D, VOCAB / 16, DT == 2>;
        GH ghead;
        if (DT != 2) ghead.issue(a.head_frag, wv, wl);   // the head ring goes out before the final LayerNorm
        fused_ln<D, G, DT == 1, DT == 2>(r_s, a_s, S::DS, a.norm_f_w, a.norm_f_b, lnp, wl, wv, am_ln_p);
        float* lg_s = xz_s;
        {
            if (DT == 2) ghead.issue(a.head_frag, wv, wl);
            ghead.run(a_s, S::DS, a.head_frag, wl, wv, am_ln, a.head_ew, [&](const typename GH::Acc& acc, int f0) {
                for_outputs<GH::FPW, G, VOCAB / 16>(acc, f0, wl, [&](int, int, int row, int n, float v) {
                    lg_s[row * VOCAB + n] = v + hb_s[n];
                });
            });
        }
        pre_layer(0);                                    // the next step's first LayerNorm
        __syncthreads();

        // histogram, range decoding and the lane's next input row
#pragma unroll
        for (int k = 0; k < LPW; ++k) {
            LaneDec& q = ld[k];
            const int gl = wv + FNW * k;
            if (gl >= G || q.pos < 0) continue;
            const int lane = lane0 + gl;
            QRow qr = quant_row(lg_s + gl * VOCAB, wl);
            const uint32_t x = dec_target(q.dc);
            int hit = -1;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if ((uint32_t)qr.cx[i] <= x && x < (uint32_t)(qr.cx[i] + qr.f[i])) hit = 4 * wl + i;
            const unsigned long long bal = __ballot(hit >= 0);
            const int src = bal ? (__ffsll((long long)bal) - 1) : 0;
            int sym = __builtin_amdgcn_readlane(hit, src);  // wave-uniform lane indices: lane reads
            if (sym < 0) sym = 0;                          // unreachable for a valid stream
            const int cl = __builtin_amdgcn_readlane(qr.csel(sym & 3), sym >> 2);
            const int fs = __builtin_amdgcn_readlane(qr.fsel(sym & 3), sym >> 2);
            uint64_t pf = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) pf |= (uint64_t)(__builtin_amdgcn_readlane(q.pbyte, i) & 0xFF) << (8 * i);
            dec_update(q.dc, (uint32_t)cl, (uint32_t)fs, q.pin, q.plen, pf, true);   // every lane, same values
            const long long ob = q.obase;
            const long long oa = ob + q.pos + 1;         // this byte's output index
            const int oi = (int)(oa & 63);
            if (wl == oi) q.obyte = (uint32_t)sym;
            if (oi == 63 || q.pos + 1 >= q.csteps) {     // block full or chunk done
                // the block's bytes from the chunk's first decoded byte on
                const long long ob0 = oa - oi;
                const int lo = ob + 1 > ob0 ? (int)(ob + 1 - ob0) : 0;
                if (wl >= lo && wl <= oi) a.out[ob0 + wl] = (uint8_t)q.obyte;
            }
            int nc, npos, ny;
            if (q.pos + 1 < q.csteps) {
                nc = q.c; npos = q.pos + 1; ny = sym;
            } else {
                locate(a.p, lane, q.lstep + 1, nc, npos);
                if (npos >= 0) enter_chunk(q, nc);
                ny = npos >= 0 ? a.out[q.obase + npos] : -1;
            }
            if (ny >= 0) {
                const float* er = a.E + (long long)ny * D;
                for (int kk = wl; kk < D; kk += 64) r_s[gl * D + kk] = er[kk];
            }
            if (wl == 0) {
                pos_s[gl] = npos;
                chunk_s[gl] = nc;
            }
            q.c = nc;
            q.pos = npos;
            ++q.lstep;
        }
        __syncthreads();
    }
}

size_t fused_lds_bytes(int D, int G, int n_layers, bool state_in_lds) {
    const int Di = 2 * D, RR = (D + 15) / 16, NO = RR + 2 * NSTATE;
    const int ZS = Di > VOCAB ? Di : VOCAB;
    size_t f = (size_t)G * ((size_t)D + (D + 4) + ZS + (Di + 4) + (Di + 4) + NO + Di / 4);
    if (state_in_lds) f += (size_t)n_layers * G * (KCONV - 1 + NSTATE) * Di;
    return f * sizeof(float);
}

template <int DT, int D, int G, bool SL>
hipError_t fused_launch(const FusedArgs& a, int blocks, hipStream_t s) {
    if constexpr (G * D > 16 * 256) {
        return hipErrorInvalidValue;           // beyond the LDS of one CU
    } else {
    constexpr int Di = 2 * D, RR = (D + 15) / 16;
    auto kern = k_dec_fused<DT, D, Di, RR, G, SL>;
    const size_t lds = fused_lds_bytes(D, G, a.n_layers, SL);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    BOA_LAUNCH(kern, dim3(blocks), dim3(FNT), lds, s, a);
    return hipGetLastError();
    }
}

hipError_t launch_dec_fused(int dtype, int D, int G, bool state_in_lds, const FusedArgs& a, hipStream_t s) {
    if (a.lanes <= 0) return hipSuccess;
    const int blocks = (a.lanes + G - 1) / G;
    if (state_in_lds && G != 1) return hipErrorInvalidValue;
#define FD_G(DTV, DV)                                                                      \
    switch (G) {                                                                           \
        case 1: return state_in_lds ? fused_launch<DTV, DV, 1, true>(a, blocks, s)         \
                                    : fused_launch<DTV, DV, 1, false>(a, blocks, s);       \
        case 2: return fused_launch<DTV, DV, 2, false>(a, blocks, s);                      \
        case 4: return fused_launch<DTV, DV, 4, false>(a, blocks, s);                      \
        case 8: return fused_launch<DTV, DV, 8, false>(a, blocks, s);                      \
        case 16: return fused_launch<DTV, DV, 16, false>(a, blocks, s);                    \
        default: return hipErrorInvalidValue;                                              \
    }
#define FD_D(DTV)                          \
    switch (D) {                           \
        case 64: FD_G(DTV, 64)             \
        case 128: FD_G(DTV, 128)           \
        case 256: FD_G(DTV, 256)           \
        case 512: FD_G(DTV, 512)           \
        default: return hipErrorInvalidValue; \
    }
    if (dtype == BOA_DTYPE_FP8) { FD_D(2) } else if (dtype == BOA_DTYPE_BF16) { FD_D(1) } else { FD_D(0) }
#undef FD_D
#undef FD_G
}

}  // namespace boa
