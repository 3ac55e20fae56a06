// Internal declarations shared by the gfx950 kernels (kernels.hip) and the
// host runtime (runtime.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/boa.h"

namespace boa {

constexpr int VOCAB = 256;
constexpr int NSTATE = 16;     // d_state
constexpr int KCONV = 4;       // d_conv
constexpr uint32_t KERNEL_VERSION = 4;       // 4: x_proj on the f32 MFMA
// largest chunk (its positions index int counters) and largest total input
constexpr uint64_t MAX_CHUNK = (1ull << 31) - 1;
constexpr uint64_t MAX_TOTAL = 1ull << 48;

// Offsets (in floats) of every tensor inside the flat float32 weight vector.
struct LayerOff {
    uint64_t norm_w, norm_b, in_w, conv_w, conv_b, xw, dtw, dtb, A_log, Dsk, out_w;
    uint64_t ffn_w1 = 0, ffn_b1 = 0, ffn_w2 = 0, ffn_b2 = 0, ffn_nw = 0, ffn_nb = 0;   // with H > 0
};
struct Layout {
    int D = 0, Di = 0, N = 0, K = 0, R = 0, L = 0;
    int H = 0;                 // feed-forward hidden width (0: no feed-forward sub-layer)
    uint64_t embed = 0, norm_f_w = 0, norm_f_b = 0, head_w = 0, head_b = 0, total = 0;
    std::vector<LayerOff> layer;
};
bool make_layout(const boa_config& c, Layout* out);

// Derived per-layer tensors the kernels read (device).
struct LayerDev {
    const float* norm_w; const float* norm_b;
    const float* in_w;       // [2Di, D]
    const float* convT;      // [K, Di]
    const float* conv_b;     // [Di]
    const float* xw;         // [R+2N, Di]
    const float* dtwT;       // [R, Di]
    const float* dtb;        // [Di]
    const float* A2T;        // [N, Di]  = -exp(A_log) * log2(e)
    // BF16 mode: x_proj and dt_proj weights rounded to bf16, as exact float
    // copies (the kernels that read floats) and as bf16 (the fused decoder)
    const float* xw_r;       // [R+2N, Di]
    const float* dtwT_r;     // [R, Di]
    const uint16_t* dtw16;   // [Di, R] (the parameter's own layout)
    // x_proj fragment-ordered for the f32 MFMA (rows padded to 16 with zeros):
    // element (nf, q, lane, j) = xw[16 nf + lane % 16][16 q + 4 j + lane / 16];
    // xwF from the weights, xwF_r from their bf16-rounded values (BF16 mode)
    const float* xwF;
    const float* xwF_r;
    const float* Dsk;        // [Di]
    const float* out_w;      // [D, Di]
    const uint16_t* in_w16;  // bf16 copies
    const uint16_t* out_w16;
    const float* in_f32f;    // fragment-ordered copies (row-block GEMM, fused decoder)
    const uint16_t* in_b16f;
    const float* out_f32f;
    const uint16_t* out_b16f;
    const uint8_t* in_f8f;   // fp8 (E4M3) fragment copies, per-tensor scale 2^in_ew[0]
    const uint8_t* out_f8f;
    const int* in_ew;        // device int: scale exponent of in_proj
    const int* out_ew;
    // feed-forward sub-layer (H > 0): master weights, bf16 row-major copies,
    // fragment-ordered f32 / bf16 / fp8 copies and fp8 scale exponents
    const float* w1; const float* b1; const float* w2; const float* b2; const float* fnw; const float* fnb;
    const uint16_t* w1_16; const uint16_t* w2_16;
    const float* w1_f32f; const uint16_t* w1_b16f; const uint8_t* w1_f8f; const int* w1_ew;
    const float* w2_f32f; const uint16_t* w2_b16f; const uint8_t* w2_f8f; const int* w2_ew;
};

// Per-layer weight pointers of the fused decoder (device array).
struct FusedLayer {
    const float* norm_w; const float* norm_b;
    const void* in_frag;                 // fragment-ordered in_proj (dtype of the launch)
    const float* convT; const float* conv_b; const float* xw; const float* dtwT; const float* dtb;
    const float* A2T; const float* Dsk;
    const uint16_t* dtw16;               // BF16 mode: bf16 dt_proj [Di, R]
    const float* xw_frag;                // fragment-ordered f32 x_proj of the launch's numerics (xwF / xwF_r)
    const void* out_frag;                // fragment-ordered out_proj
    const int* in_ew; const int* out_ew; // fp8: scale exponents of in_proj / out_proj (device)
};

}  // namespace boa

struct boa_model {
    boa_config cfg{};
    boa::Layout lay;
    int device = 0;
    float* d_w = nullptr;         // master float32 weights (flat layout)
    float* d_derived = nullptr;   // per layer: convT, dtwT, A2T
    uint16_t* d_w16 = nullptr;    // bf16 copies of in_w, out_w per layer, then head_w
    std::vector<boa::LayerDev> ld;
    const uint16_t* head_w16 = nullptr;
    float* d_frag32 = nullptr;    // fragment-ordered in_w, out_w per layer, then head_w (float32)
    uint16_t* d_frag16 = nullptr; // the same in bf16
    const float* head_f32f = nullptr;
    const uint16_t* head_b16f = nullptr;
    uint8_t* d_frag8 = nullptr;   // the same in fp8 (E4M3)
    int* d_ew = nullptr;          // per matrix scale exponents: in, out per layer, then head
    unsigned* d_amax = nullptr;   // per matrix |w| maximum (prep scratch)
    const uint8_t* head_f8f = nullptr;
    const int* head_ew = nullptr;
    uint64_t fingerprint = 0;
    void* train = nullptr;        // optimiser state, created by the first training step
    bool fp_stale = false;        // weights changed on device since the fingerprint was taken
};

namespace boa {

// ----------------------------------------------------------------- workspace
struct Plan {              // device arrays describing the static lane schedule
    const int* lane_first;   // [lanes] first entry of each lane
    const int* lane_cnt;     // [lanes]
    const int* ent_chunk;    // [entries]
    const long long* ent_start;  // [entries] first global step of the entry
    const long long* chunk_off;  // [chunks] byte offset of the chunk
    const long long* chunk_steps;// [chunks] len - 1
};

constexpr int MAX_LAYERS = 16;
struct FusedArgs {
    FusedLayer layers[MAX_LAYERS];   // in the kernel arguments: read through the scalar cache
    int n_layers, lanes;
    long long max_steps;         // longest lane schedule (loop bound)
    const float* E; const float* norm_f_w; const float* norm_f_b; const void* head_frag; const float* head_b;
    const int* head_ew;                  // fp8: head scale exponent (device)
    Plan p;
    const uint8_t* payload; const long long* pay_off; const long long* pay_len;
    uint8_t* out;                // decoded bytes; first byte of every chunk already in place
    float* conv_state;           // [n_layers][lanes][K-1][Di]: taps t-3, t-2, t-1
    float* h_state;              // [n_layers][lanes][N/4][Di] float4
};

// ----------------------------------------------------------------- launches
// fragment-ordered float32 and bf16 copies of W[N, K] for the fused decoder
// and the fp8 (E4M3) copy with its per-tensor power-of-two scale exponent
// (*ew; *amax is scratch for the largest |w|)
hipError_t launch_frag(const float* W, int N, int K, float* f32, uint16_t* b16, uint8_t* f8, unsigned* amax,
                       int* ew, hipStream_t s);
// LDS bytes of the fused decoder for d_model D and G lanes per workgroup,
// with the lanes' conv and scan state in LDS when state_in_lds
size_t fused_lds_bytes(int D, int G, int n_layers, bool state_in_lds);
// Fused persistent decoder: ceil(lanes / G) workgroups of 512 threads,
// G in {1, 2, 4, 8}; state_in_lds only with G = 1 (then the state buffers of
// FusedArgs are not touched).
hipError_t launch_dec_fused(int dtype, int D, int G, bool state_in_lds, const FusedArgs& a, hipStream_t s);
hipError_t launch_prep(const boa_model* m, hipStream_t s);
// time the launches issued on this thread until prof_close() with GPU timestamps
void prof_open(hipEvent_t start, hipEvent_t stop);
void prof_close();
void set_max_lds(size_t bytes);
size_t get_max_lds();
hipError_t launch_rowinfo(const Plan& p, int lanes, int T, long long step0, const long long* d_step,
                          int* row_chunk, int* row_pos, hipStream_t s);
hipError_t launch_embed(const float* E, const uint8_t* bytes, const Plan& p, int lanes, int T, long long step0,
                        const long long* d_step, int D, int* row_chunk, int* row_pos, float* r, hipStream_t s);
// C[M,N] = epi( A'[M,K] . W[N,K]^T ) on MFMA.  kind 0: in_proj (A' = LN(A));
// 1: head (LN, + bias); 2: out_proj (C += result); 3: feed-forward W1
// (+ bias, GELU); 4: feed-forward W2 (+ bias).
hipError_t launch_mgemm(int dtype, int kind, const float* A, int M, int K, const float* W32, const uint16_t* W16,
                        int N, float* C, const float* ln_w, const float* ln_b, const float* bias, hipStream_t s);
// The same products for many rows: a workgroup owns a block of rows and every
// column; Wf is the fragment-ordered copy of W in the launch's dtype (fp8:
// ew is the device pointer to W's scale exponent).  Kind 5 (BF16 only) is the
// out_proj of kind 2 with A already bf16 bits [M, K] (the mixer's gated rows).
// f32 fragment order of W [N, K] with the rows padded to NP (a multiple of 16)
// by zeros, for the f32 MFMA: element (nf, q, lane, j) = W[16 nf + lane % 16]
// [16 q + 4 j + lane / 16]; K a multiple of 16.
hipError_t launch_frag_pad(const float* W, int N, int NP, int K, float* out, hipStream_t s);
hipError_t launch_rowgemm(int dtype, int kind, const float* A, int M, int K, const void* Wf, int N, float* C,
                          const float* ln_w, const float* ln_b, const float* bias, const int* ew, hipStream_t s);
// rows of x [M, D] LayerNorm'd into out (may alias x)
hipError_t launch_ln_rows(const float* x, int M, int D, const float* w, const float* b, float* out, hipStream_t s);
hipError_t launch_mid(const LayerDev& w, int Di, int R, const float* xz, float* g, int lanes, int T,
                      int lanes_per_wg, const int* row_pos, float* conv_state, float* hstate,
                      hipStream_t s);
// g_bf16: the gated rows are written as bf16 bits (d_inner <= 512 only)
hipError_t launch_mid_tiled(const LayerDev& w, int Di, int R, const float* xz, float* xs, float* dbc, float* dt,
                            float* g, int lanes, int T, const int* row_pos, float* conv_state, float* hstate,
                            bool g_bf16, hipStream_t s);
hipError_t launch_quant_sym(const float* logits, int M, const uint8_t* data, const Plan& p,
                            const int* row_chunk, const int* row_pos, uint32_t* cf,
                            float* probs, uint16_t* tables, hipStream_t s);
// sets this thread's boa_last_error() text and returns code
int report_error(int code, const std::string& msg);
hipError_t launch_diag(const float* logits, int M, const uint8_t* data, const Plan& p, const int* row_chunk,
                       const int* row_pos, int n_bins, uint32_t* confusion, uint32_t* rank_hist,
                       unsigned long long* calib, hipStream_t s);
hipError_t launch_encode(const uint32_t* cf, int lanes, int T, const int* row_chunk,
                         const int* row_pos, const Plan& p, uint32_t* cst, uint8_t* payload,
                         const long long* pay_off, const long long* pay_cap, uint32_t* pay_len,
                         double* ideal, hipStream_t s);
// Decoder step: decode one byte per active lane and prepare the lane's next
// row (row_chunk / row_pos) and embedding row r.  dst: 8 uint32 per lane.
hipError_t launch_decode(const float* logits, int lanes, int* row_chunk, int* row_pos, const Plan& p,
                         uint32_t* dst, const uint8_t* payload, const long long* pay_off,
                         const long long* pay_len, uint8_t* out, const float* E, int D, float* r,
                         hipStream_t s);
hipError_t launch_prefill(const uint8_t* first, const long long* chunk_off, const long long* chunk_len,
                          int n, uint8_t* out, hipStream_t s);
hipError_t launch_scatter_rows(const float* src, int lanes, int T, int width, long long t0,
                               long long Tout, float* dst, hipStream_t s);
hipError_t launch_scatter_rows_u16(const uint16_t* src, int lanes, int T, int width, long long t0,
                                   long long Tout, uint16_t* dst, hipStream_t s);
hipError_t launch_code_tables(const uint8_t* sym, const uint16_t* freq, const long long* sym_off,
                              const long long* nsym, int lanes, uint8_t* payload,
                              const long long* pay_off, const long long* pay_cap,
                              uint32_t* pay_len, hipStream_t s);
hipError_t launch_decode_tables(const uint8_t* payload, const long long* pay_off,
                                const long long* pay_len, const uint16_t* freq,
                                const long long* sym_off, const long long* nsym, int lanes,
                                uint8_t* sym, hipStream_t s);
hipError_t launch_crc32(const uint8_t* data, const long long* off, const long long* len, int n,
                        uint32_t* crc, hipStream_t s);
hipError_t launch_order2_encode(const uint8_t* data, const long long* off, const long long* len, int n,
                                uint16_t* counts, uint8_t* payload, const long long* pay_off,
                                const long long* pay_cap, uint32_t* pay_len, double* ideal,
                                hipStream_t s);
hipError_t launch_order2_decode(const uint8_t* payload, const long long* pay_off,
                                const long long* pay_len, const long long* off,
                                const long long* len, int n, uint16_t* counts, uint8_t* out,
                                hipStream_t s);

// The fused decoder with every device buffer carved from region (region_bytes);
// never allocates (BOA_E_ARG when the region is too small).
int decode_into_region(const boa_model* m, const uint8_t* d_payload, const uint64_t* h_pay_off,
                       const uint64_t* h_pay_len, const uint8_t* h_first, const uint64_t* h_chunk_off,
                       const uint64_t* h_chunk_len, uint64_t n_chunks, const boa_run_opts* opts, uint8_t* d_out,
                       void* region, size_t region_bytes, void* stream);

void train_ctx_free(void* p);
// fingerprint of the current weights (recomputed after on-device training)
uint64_t model_fingerprint(const boa_model* m);
// records a failure message for boa_last_error() and returns code
int set_error(int code, const std::string& msg);
}  // namespace boa
