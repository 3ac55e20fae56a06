/*
 * boa.h -- C ABI of libboa, an MI355X (gfx950) implementation of the hot path
 * of the BOA Constrictor lossless compressor (arXiv 2511.11337).
 *
 * The paper's problem statement (Theoretical Framework; Range coding) pairs a
 * next-byte predictor Q exposing a `step` function with an integer range
 * coder C; compression splits the input into independent chunks (streams),
 * computes next-byte probabilities for every active stream per timestep and
 * codes all streams in parallel (Coders & Parallelisation).  This header
 * exposes that as train / compress / decompress over a byte-level Mamba model,
 * plus device-level entry points used by the Python binding and the tests.
 *
 * Conventions (all functions):
 *  - Return 0 (BOA_OK) on success or a negative BOA_E_* code; never abort,
 *    never throw across the ABI.  boa_last_error() gives a thread-local
 *    message for the last failure on the calling thread.
 *  - "h_" pointers are host memory, "d_" pointers are device memory on the
 *    model's device.  The caller owns every buffer it passes in; the library
 *    never frees caller buffers.  Buffers the library returns through
 *    uint8_t** out parameters are allocated with malloc and released with
 *    boa_free().
 *  - `stream` is a hipStream_t passed as void* (0 = the default stream).
 *    Device-level calls enqueue work on it and synchronise it before
 *    returning unless stated otherwise.
 *  - A model is read-only during compress/decompress; several host threads
 *    may use one model concurrently.  boa_train mutates it.
 *  - Bit-exact decoding of the float dtypes requires the same library build,
 *    dtype and device architecture as the encoder (the container records a
 *    numerics id and the decoder refuses a mismatch with BOA_E_MODEL).
 *    BOA_DTYPE_INT8 containers come from the integer-only pipeline (see
 *    boa_qmodel_create) and decode on any device.
 */
#ifndef BOA_H
#define BOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define BOA_OK              0
#define BOA_E_ARG          -1   /* bad argument (null pointer, size, config) */
#define BOA_E_OOM          -2   /* host or device allocation failed */
#define BOA_E_DEVICE       -3   /* HIP runtime error; message has the HIP string */
#define BOA_E_FORMAT       -4   /* bad container / model-file magic or version */
#define BOA_E_CRC          -5   /* container index CRC mismatch */
#define BOA_E_MODEL        -6   /* model fingerprint or numerics id mismatch */
#define BOA_E_CORRUPT      -7   /* truncated payload or per-chunk CRC mismatch */
#define BOA_E_UNSUPPORTED  -8   /* e.g. no gfx950 device, unsupported shape */

/* projection precision for in_proj / out_proj / head */
#define BOA_DTYPE_F32   0
#define BOA_DTYPE_BF16  1
#define BOA_DTYPE_FP8   2
/* compress / decompress only: the integer-only pipeline of boa_qmodel_create,
 * whose tables, and so whose containers, do not depend on the device */
#define BOA_DTYPE_INT8  3

/* coder ids recorded per chunk in the container index */
#define BOA_CODER_MAMBA   0
#define BOA_CODER_ORDER2  1
#define BOA_CODER_RAW     2

/*
 * Model shape (Models section: model dimension d_m and layer count n_l; the
 * Mamba block's state size, conv width and expansion follow the cited Mamba
 * design).  dt_rank = ceil(d_model / 16), d_inner = expand * d_model.
 * Supported: d_model in {64, 128, 256, 512}, d_state = 16, d_conv = 4,
 * expand = 2, 1 <= n_layers <= 16.
 * ffn_mult > 0 adds Algorithm 1's sub-layer after every Mamba block,
 * r <- LayerNorm(FFN(r)) with FFN(r) = W2 GELU(W1 r + b1) + b2 (exact GELU,
 * hidden width ffn_mult * d_model, no residual around it); supported when
 * ffn_mult * d_model <= 1024.  0 = no feed-forward sub-layer.
 */
typedef struct {
    uint32_t d_model;
    uint32_t n_layers;
    uint32_t d_state;
    uint32_t d_conv;
    uint32_t expand;
    uint32_t ffn_mult;
} boa_config;

typedef struct boa_model boa_model;   /* opaque; owned by the library */

/* Run options for compress / decompress.  Zero-initialise for defaults. */
typedef struct {
    uint32_t dtype;       /* BOA_DTYPE_*; default F32 */
    uint32_t max_lanes;   /* concurrent streams; 0 = chosen by the library (boa_plan_lanes) */
    uint32_t tile_t;      /* encoder time tile; 0 = auto */
    uint32_t use_graph;   /* decoder: 1 = replay a captured hipGraph per step (default), 2 = plain launches */
    uint32_t fallback;    /* encoder: 1 = per chunk keep the smaller of Mamba / order-2 / raw */
    uint32_t decode_groups; /* decoder: lanes split into this many independent groups, each with its own
                               stream and step graph (0 = 1); does not change the output */
    uint32_t decode_kernel; /* decoder: 0 = auto, 1 = fused persistent kernel (every step of a lane in one
                               launch), 2 = per-step kernel chain (step graph or plain launches per
                               use_graph); does not change the output */
    uint32_t fused_lanes;   /* fused decoder: lanes per workgroup, 1, 2, 4, 8 or 16; 0 = auto */
} boa_run_opts;

/* ------------------------------------------------------------------ model */

/* Number of float32 parameters of `cfg` in the flat layout:
 * embed[256,D]; per layer: norm_w[D], norm_b[D], in_proj_w[2Di,D],
 * conv_w[Di,K], conv_b[Di], x_proj_w[R+2N,Di], dt_proj_w[Di,R],
 * dt_proj_b[Di], A_log[Di,N], D[Di], out_proj_w[D,Di], and with ffn_mult > 0
 * (H = ffn_mult * D) ffn_w1[H,D], ffn_b1[H], ffn_w2[D,H], ffn_b2[D],
 * ffn_norm_w[D], ffn_norm_b[D]; then norm_f_w[D], norm_f_b[D], head_w[256,D],
 * head_b[256].  Row-major, Linear weights as [out, in].  Returns 0 for an
 * unsupported config. */
uint64_t boa_param_count(const boa_config* cfg);

/* Create a model on HIP device `device` from `n` float32 weights (host
 * memory, copied).  *out is owned by the library; release with
 * boa_model_free. */
int boa_model_create(const boa_config* cfg, const float* h_weights, uint64_t n,
                     int device, boa_model** out);
void boa_model_free(boa_model* m);

/* Copy the current float32 master weights to host memory (n = param count). */
int boa_model_get_weights(const boa_model* m, float* h_out, uint64_t n);
/* Overwrite the master weights from host memory and refresh derived copies. */
int boa_model_set_weights(boa_model* m, const float* h_weights, uint64_t n);
int boa_model_config(const boa_model* m, boa_config* out);
/* 64-bit fingerprint of config + weight bytes (FNV-1a), stored in containers
 * (Coders & Parallelisation: compact model fingerprint). */
int boa_model_fingerprint(const boa_model* m, uint64_t* out);
/* Model file: "BOAM" magic, version 2, config (6 x uint32), float32 weights,
 * fingerprint.  Version 1 files (5-field config, no feed-forward sub-layer)
 * load too. */
int boa_model_save(const boa_model* m, const char* path);
int boa_model_load(const char* path, int device, boa_model** out);

/* ------------------------------------------------------------------ compress / decompress */

/*
 * compress(model, bytes) -> .boa container.
 * h_data holds n_chunks consecutive chunks of lengths h_chunk_len[i]
 * (their sum is the input length).  The first byte of every chunk is stored
 * raw in the index; bytes 2..len are range coded from the model's
 * probabilities (Coders & Parallelisation).  *out is malloc'd; free with
 * boa_free.
 */
int boa_compress(const boa_model* m, const uint8_t* h_data, const uint64_t* h_chunk_len,
                 uint64_t n_chunks, const boa_run_opts* opts, uint8_t** out, uint64_t* out_len);

/* decompress(model, container) -> bytes.  Verifies magic, index CRC, model
 * fingerprint, numerics id and per-chunk CRC32.  *out is malloc'd (may be
 * NULL when the original length is 0). */
int boa_decompress(const boa_model* m, const uint8_t* h_container, uint64_t len,
                   const boa_run_opts* opts, uint8_t** out, uint64_t* out_len);

/* ------------------------------------------------------------------ streaming compress */

/*
 * Streaming compressor (paper, Streaming: a distributor cuts the incoming
 * bytes into fixed-size chunks; each full group of lanes is compressed into a
 * shard while the next group is buffered).  boa_stream_push appends host
 * bytes; every time lanes x chunk_len bytes are buffered that group becomes
 * a shard, compressed by one of `workers` host threads (1..8), each with its
 * own HIP stream, exactly as boa_compress(group, chunks of chunk_len) would
 * (same container bytes).  At most `workers` full groups wait for a worker;
 * push blocks beyond that.  boa_stream_finish submits the last, partial group
 * (its last chunk may be short).  boa_stream_next_shard hands out the shards
 * in input order: *out (malloc'd, free with boa_free) and *out_len, or *out =
 * NULL when none is ready (wait = 0) or none is in flight; with wait != 0 it
 * blocks until the next shard in flight is done.  A shard that failed returns
 * its error code.  boa_stream_close drops groups no worker has started, waits
 * for the running ones and frees the stream (the model must outlive it).
 * Push after finish is BOA_E_ARG.  The calls of one stream must not overlap.
 */
typedef struct boa_stream boa_stream;
int boa_stream_open(const boa_model* m, uint64_t chunk_len, uint32_t lanes, uint32_t workers,
                    const boa_run_opts* opts, boa_stream** out);
int boa_stream_push(boa_stream* st, const uint8_t* h_data, uint64_t n);
int boa_stream_finish(boa_stream* st);
int boa_stream_next_shard(boa_stream* st, int wait, uint8_t** out, uint64_t* out_len);
void boa_stream_close(boa_stream* st);

/* Parse a container header/index without decoding: n_chunks, total length. */
int boa_container_info(const uint8_t* h_container, uint64_t len, uint64_t* n_chunks,
                       uint64_t* total_len, uint64_t* fingerprint, uint32_t* numerics_id);

/* Per-chunk statistics of the last boa_compress on this thread:
 * coded payload bytes and coder id per chunk (n entries). */
int boa_last_chunk_stats(uint64_t* h_payload_bytes, uint32_t* h_coder, uint64_t n);

void boa_free(void* p);
const char* boa_last_error(void);
/* Numerics id of this library for `dtype` (kernel version, dtype, reduction
 * orders); compress writes it, decompress requires equality.  For
 * BOA_DTYPE_INT8 it is the integer pipeline's version alone. */
uint32_t boa_numerics_id(uint32_t dtype);

/* ------------------------------------------------------------------ device-level */

/* ------------------------------------------------------------------ device-level workspace */
#define BOA_WS_ENCODE 0
#define BOA_WS_DECODE 1

/*
 * Device workspace (bytes) that boa_encode_dev (mode BOA_WS_ENCODE) or
 * boa_decode_dev (BOA_WS_DECODE) needs for these chunk lengths and options:
 * the lane schedule, per-chunk arrays, activation tiles, coder inputs and,
 * for the fused decoder with several lanes per workgroup, every lane's conv
 * and scan state.  A caller that passes a workspace of at least this size
 * makes those calls allocate no device memory.  0 when there is nothing to
 * code, and for the per-step decoder (decode_kernel = 2), which allocates its
 * own buffers.  Host-only computation (no device work).
 */
int boa_workspace_size(const boa_model* m, const uint64_t* h_chunk_len, uint64_t n_chunks, const boa_run_opts* opts,
                       uint32_t mode, uint64_t* bytes);

/* Lane count of a call's schedule (Coders & Parallelisation: chunks are
 * independent streams run side by side; a lane runs its chunks back to back,
 * longest first onto the least-loaded lane).  max_lanes > 0: min(coded
 * chunks, max_lanes).  max_lanes = 0, the default of every call: the most
 * lanes (at most 8192; candidates min(chunks, 8192) halved down to 256 and
 * ceil(chunks / k) for k = 2 .. 16) whose schedule keeps the idle rows (a lane
 * out of chunks while others run) within 5 % of the rows the lanes occupy,
 * else the candidate with the fewest idle rows.  Chunks of 0 or 1
 * byte are not scheduled.  *lanes receives the count (0 for no coded chunk).
 * Host-only; BOA_E_ARG for null pointers or lengths beyond the limits. */
int boa_plan_lanes(const uint64_t* h_chunk_len, uint64_t n_chunks, uint32_t max_lanes, uint32_t* lanes);

/* Fixed-length chunking (Coders & Parallelisation: the input is split into
 * chunks of a nominal length, the final chunk shorter): *n_chunks =
 * ceil(n / chunk_len); when h_lens is not NULL it receives the lengths
 * (cap entries at least, else BOA_E_ARG). */
int boa_split_fixed(uint64_t n, uint64_t chunk_len, uint64_t* h_lens, uint64_t cap, uint64_t* n_chunks);

/* Offsets of concatenated chunks and the payload regions boa_encode_dev
 * writes: h_chunk_off[i] = sum of earlier lengths, h_pay_cap[i] = 2 len + 64
 * (the range coder's worst case with margin), h_pay_off[i] = sum of earlier
 * capacities, *total_cap = sum of all capacities.  Host arrays of n entries. */
int boa_payload_layout(const uint64_t* h_chunk_len, uint64_t n, uint64_t* h_chunk_off, uint64_t* h_pay_off,
                       uint64_t* h_pay_cap, uint64_t* total_cap);

/*
 * Encode on device.  d_data: concatenated chunks (device); h_chunk_off /
 * h_chunk_len: host arrays (n_chunks).  Payload of chunk i is written at
 * d_payload + h_pay_off[i] with capacity h_pay_cap[i] bytes; its length goes
 * to d_pay_len[i] (device, uint32), or 0xFFFFFFFF if it would exceed the
 * capacity (the caller then stores that chunk raw).  Chunks of length <= 1
 * get length 0.  Optional d_ideal_bits (device, float64, n_chunks) receives
 * sum -log2(f(s)/M) over each chunk's coded symbols; pass NULL to skip.
 * d_ws (device, ws_bytes >= boa_workspace_size(..., BOA_WS_ENCODE), owned by
 * the caller, contents need not be initialised) holds every buffer of the
 * call; with d_ws NULL the library allocates them for the call.  The range
 * coder runs on a second stream the call creates, ordered after `stream`.
 */
int boa_encode_dev(const boa_model* m, const uint8_t* d_data, const uint64_t* h_chunk_off,
                   const uint64_t* h_chunk_len, uint64_t n_chunks, const boa_run_opts* opts,
                   uint8_t* d_payload, const uint64_t* h_pay_off, const uint64_t* h_pay_cap,
                   uint32_t* d_pay_len, double* d_ideal_bits, void* d_ws, uint64_t ws_bytes, void* stream);

/*
 * Decode on device into d_out (concatenated chunks at h_chunk_off).  The first
 * byte of each chunk is taken from h_first[i]; payload i is d_payload +
 * h_pay_off[i] with h_pay_len[i] bytes (bytes past the end read as 0).
 * d_ws / ws_bytes as for boa_encode_dev (mode BOA_WS_DECODE); the per-step
 * decoder (decode_kernel = 2) ignores d_ws and allocates.
 */
int boa_decode_dev(const boa_model* m, const uint8_t* d_payload, const uint64_t* h_pay_off,
                   const uint64_t* h_pay_len, const uint8_t* h_first, const uint64_t* h_chunk_off,
                   const uint64_t* h_chunk_len, uint64_t n_chunks, const boa_run_opts* opts,
                   uint8_t* d_out, void* d_ws, uint64_t ws_bytes, void* stream);

/*
 * boa_decode_dev without any device allocation, for callers that cannot
 * allocate device memory (code under stream capture, serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and output as
 * boa_decode_dev with the fused decoder; every buffer of the call comes from
 * a fixed 2 MiB scratch array the library holds on each device until the
 * process ends (roughly 70 bytes per chunk, plus the lanes' scan state when
 * several lanes share a workgroup).  A call that needs more than 2 MiB, or
 * asks for the per-step decoder (decode_kernel = 2), fails with BOA_E_ARG and
 * does nothing.  Calls on one GPU share the array: calls that overlap on one
 * GPU race and must be serialised by the caller.
 */
int boa_decode_noalloc_dev(const boa_model* m, const uint8_t* d_payload, const uint64_t* h_pay_off,
                           const uint64_t* h_pay_len, const uint8_t* h_first, const uint64_t* h_chunk_off,
                           const uint64_t* h_chunk_len, uint64_t n_chunks, const boa_run_opts* opts,
                           uint8_t* d_out, void* stream);

/*
 * Teacher-forced logits (parity checks).  For n_lanes equal-length sequences
 * d_seqs[lane * T + t] (device, uint8), writes d_logits[(lane*(T-1)+t)*256 + a]
 * (float32) = logit of byte a at position t+1 given bytes <= t, computed by
 * the same kernels as compress/decompress in the given dtype.  If d_probs is
 * not NULL it receives the float32 probabilities and d_tables (uint16 [.,256],
 * may be NULL) the integer histograms the coder uses.
 */
int boa_logits_dev(const boa_model* m, const uint8_t* d_seqs, uint32_t n_lanes, uint32_t T,
                   uint32_t dtype, uint32_t tile_t, float* d_logits, float* d_probs,
                   uint16_t* d_tables, void* stream);

/*
 * Predictor diagnostics (paper, Results: confusion matrices, Top-k curves,
 * reliability diagrams and ECE), from the probabilities the coder quantises.
 * For n_lanes equal-length sequences d_seqs[lane * T + t] (device, uint8) and
 * every position t+1 (t < T - 1) with true byte y and probabilities p of the
 * given dtype's numerics (the same kernels as compress):
 *   pred = argmax p (lowest index on ties), conf = p[pred],
 *   rank = #{a : p[a] > p[y]} + #{a < y : p[a] == p[y]}   (0 = Top-1 hit).
 * The call zeroes and then fills (device arrays owned by the caller):
 *   d_confusion  uint32 [256 * 256]: [y * 256 + pred] position counts;
 *   d_rank_hist  uint32 [256]: positions per rank (Top-k = ranks < k);
 *   d_calib      uint64 [3 * n_bins]: per reliability bin
 *                b = min(floor(conf * n_bins), n_bins - 1) (float32 product):
 *                count, correct count (pred == y), sum of conf * 2^32 (exact).
 * n_bins in [1, 1024] (else BOA_E_ARG).  n_lanes == 0 or T < 2 leaves the
 * zeroed arrays.  Synchronises the stream before returning.
 */
int boa_diagnostics_dev(const boa_model* m, const uint8_t* d_seqs, uint32_t n_lanes, uint32_t T,
                        uint32_t dtype, uint32_t tile_t, uint32_t n_bins, uint32_t* d_confusion,
                        uint32_t* d_rank_hist, uint64_t* d_calib, void* stream);

/* Summary of boa_diagnostics_dev's counts (host arrays): *positions = sum of
 * the rank histogram; h_topk[k] (256 entries) = fraction of positions whose
 * true byte has rank <= k, i.e. Top-(k+1) accuracy; *ece = sum over bins of
 * (n_b / N) |acc_b - conf_b| with N = sum of the bin counts, acc_b =
 * correct_b / n_b and conf_b = (sum of conf 2^32) / 2^32 / n_b (empty bins
 * add nothing). */
int boa_diagnostics_summary(const uint32_t* h_rank_hist, const uint64_t* h_calib, uint32_t n_bins, double* h_topk,
                            double* ece, uint64_t* positions);

/*
 * Range-code explicit integer tables (coder parity).  Lane i codes
 * h_nsym[i] symbols d_sym[lane_off_i + j] with histograms
 * d_freq[(lane_off_i + j) * 256 .. +256] (uint16, each summing to 65536;
 * lane_off_i = sum of earlier h_nsym).  Payload i goes to d_payload +
 * h_pay_off[i], capacity h_pay_cap[i]; length to d_pay_len[i].
 */
int boa_code_tables_dev(const uint8_t* d_sym, const uint16_t* d_freq, const uint64_t* h_nsym,
                        uint64_t n_lanes, uint8_t* d_payload, const uint64_t* h_pay_off,
                        const uint64_t* h_pay_cap, uint32_t* d_pay_len, void* stream);
/* Inverse of boa_code_tables_dev: decode h_nsym[i] symbols per lane into d_sym. */
int boa_decode_tables_dev(const uint8_t* d_payload, const uint64_t* h_pay_off,
                          const uint64_t* h_pay_len, const uint16_t* d_freq, const uint64_t* h_nsym,
                          uint64_t n_lanes, uint8_t* d_sym, void* stream);

/* ------------------------------------------------------------------ order-2 fallback */

/* Adaptive order-2 context-count model (KT estimate, same quantiser and coder)
 * run on device, one lane per chunk.  Same buffer conventions as
 * boa_encode_dev / boa_decode_dev. */
int boa_order2_encode_dev(const uint8_t* d_data, const uint64_t* h_chunk_off,
                          const uint64_t* h_chunk_len, uint64_t n_chunks, uint8_t* d_payload,
                          const uint64_t* h_pay_off, const uint64_t* h_pay_cap, uint32_t* d_pay_len,
                          double* d_ideal_bits, void* stream);
int boa_order2_decode_dev(const uint8_t* d_payload, const uint64_t* h_pay_off,
                          const uint64_t* h_pay_len, const uint8_t* h_first,
                          const uint64_t* h_chunk_off, const uint64_t* h_chunk_len,
                          uint64_t n_chunks, uint8_t* d_out, void* stream);

/* ------------------------------------------------------------------ kernel timing */

/* Kernel classes of the model pass that can be timed with HIP events. */
#define BOA_K_EMBED    0   /* row location + embedding gather */
#define BOA_K_INPROJ   1   /* LayerNorm + in_proj (MFMA) */
#define BOA_K_MIXER    2   /* conv, x_proj, dt_proj, selective scan, gate */
#define BOA_K_OUTPROJ  3   /* out_proj + residual (MFMA) */
#define BOA_K_HEAD     4   /* final LayerNorm + head (MFMA) */
#define BOA_K_DECODE   5   /* decoder: histogram, CDF search, range decoding */
#define BOA_K_QUANT    6   /* encoder: histogram and CDF of the coded byte */
#define BOA_K_ENCODE   7   /* encoder: range coder lanes */
#define BOA_K_DEC_FUSED 8  /* fused persistent decoder (all steps of a call) */
#define BOA_K_FFN      9   /* feed-forward sub-layer: W1 + GELU, W2, LayerNorm (MFMA) */
#define BOA_K_COUNT    10

/* Record a HIP event pair around every launch of the classes in `mask`
 * (bit k = class k) on the stream the launch is enqueued on, for launches
 * that are not part of a captured graph; 0 disables.  Process-wide. */
int boa_prof_enable(uint32_t mask);
/* Per class: total milliseconds and number of timed launches since the last
 * reset (arrays of BOA_K_COUNT entries; either may be NULL).  Waits for the
 * recorded events. */
int boa_prof_read(double* h_total_ms, uint64_t* h_launches, int reset);

/* ------------------------------------------------------------------ training */

/* Optimiser and schedule (paper, Models: cross-entropy training; sequence
 * length, batch and learning rate are its tunable hyper-parameters).
 * AdamW with decoupled weight decay, global-norm gradient clipping
 * (grad_clip <= 0 disables), linear warm-up over `warmup` steps then constant
 * learning rate.  Zero-initialise, then set; zeros mean: lr 1e-3, betas
 * (0.9, 0.999), eps 1e-8, weight decay 0.01, clip 1.0, warmup 100, batch 32,
 * seq_len 8192, chunk_t 256. */
typedef struct {
    float lr, beta1, beta2, eps, weight_decay, grad_clip;
    uint32_t warmup, steps, batch, seq_len, chunk_t;
    uint32_t dtype;       /* projections: BOA_DTYPE_F32 or BOA_DTYPE_BF16 (FP32 master weights either way) */
    uint64_t seed;
} boa_train_opts;

/*
 * Mean next-byte cross-entropy (nats) of B device sequences d_tokens[b*T + t]
 * (uint8, T >= 2; position t predicts t+1) and its gradient with respect to
 * the float32 master weights, in the flat weight layout (d_grad: device
 * float32, boa_param_count entries).  The selective scan keeps its state only
 * every chunk_t steps and recomputes it in the backward pass (Appendix A:
 * the scan evaluated over the sequence during training).  dtype selects the
 * projections' operands: BOA_DTYPE_F32, or BOA_DTYPE_BF16 (activations,
 * gradients and weights rounded to bf16 as they enter the matrix cores, FP32
 * accumulation); everything else is FP32.  Every reduction has a fixed order
 * (no atomics), so equal inputs give bit-identical results.  *d_loss is a
 * device double.  The activation buffers of the last (B, T, chunk_t) stay
 * allocated with the model.  Synchronises `stream`.  BOA_E_UNSUPPORTED for
 * other dtypes.
 */
int boa_loss_grad_dev(boa_model* m, const uint8_t* d_tokens, uint32_t B, uint32_t T, uint32_t chunk_t,
                      uint32_t dtype, double* d_loss, float* d_grad, void* stream);

/* One AdamW step from a caller-supplied gradient (device float32, flat
 * layout, boa_param_count entries; not modified): global-norm clipping at
 * opts->grad_clip, decoupled weight decay, bias-corrected moments, learning
 * rate from the warm-up schedule at the model's step count + 1.  The moments
 * and the step count live with the model.  Synchronises `stream`. */
int boa_optimizer_step_dev(boa_model* m, const float* d_grad, const boa_train_opts* opts, void* stream);

/* One training step on B device sequences of T bytes: boa_loss_grad_dev in
 * opts->dtype, then boa_optimizer_step_dev.  *d_loss (device double) gets the
 * step's mean loss. */
int boa_train_step_dev(boa_model* m, const uint8_t* d_tokens, uint32_t B, uint32_t T, const boa_train_opts* opts,
                       double* d_loss, void* stream);

/* Training checkpoint for an exact resume: "BOAT" magic, version 1, config,
 * step count, float32 master weights, both AdamW moments, FNV-1a hash.  Load
 * requires a model of the same config (BOA_E_MODEL otherwise), verifies the
 * hash (BOA_E_CORRUPT) and replaces the weights, moments and step count. */
int boa_train_state_save(const boa_model* m, const char* path);
/* Optimiser steps the model has taken (0 before the first). */
int boa_train_steps_done(const boa_model* m, uint64_t* steps);
int boa_train_state_load(boa_model* m, const char* path);

/* train(model, bytes): opts->steps AdamW steps over non-overlapping windows
 * of seq_len bytes of h_bytes (shuffled every epoch with opts->seed), batch
 * windows per step.  A model that has already taken k steps (a resumed
 * checkpoint, or an earlier call) continues the window sequence after its
 * first k x batch windows, so a run split into several calls equals one
 * call.  h_losses (may be NULL) receives up to n_losses per-step mean losses
 * in nats. */
int boa_train(boa_model* m, const uint8_t* h_bytes, uint64_t n, const boa_train_opts* opts, float* h_losses,
              uint64_t n_losses);

/*
 * Selective scan alone (Appendix A: h_t = exp(Delta_t A) h_{t-1} + Delta_t
 * x_t B_t, y_t = C_t . h_t + D x_t, A = -exp(A_log)), for the autograd
 * binding.  Device float32 tensors: x, dt [B][T][Di]; A_log [Di][16];
 * bc [B][T][32] (B_t then C_t); Dskip [Di].  Forward writes y [B][T][Di]
 * and the states at chunk starts hsave [B][ceil(T/chunk_t)][16][Di].
 * Backward takes dy and hsave and writes dx, ddt [B][T][Di], dbc
 * [B][T][32], and adds into dA_log [Di][16], dDskip [Di] (caller zeroes them).
 */
int boa_scan_fwd_dev(const float* d_x, const float* d_dt, const float* d_A_log, const float* d_bc,
                     const float* d_Dskip, uint32_t B, uint32_t T, uint32_t Di, uint32_t chunk_t, float* d_y,
                     float* d_hsave, void* stream);
int boa_scan_bwd_dev(const float* d_x, const float* d_dt, const float* d_A_log, const float* d_bc,
                     const float* d_Dskip, const float* d_dy, uint32_t B, uint32_t T, uint32_t Di, uint32_t chunk_t,
                     const float* d_hsave, float* d_dx, float* d_ddt, float* d_dbc, float* d_dA_log,
                     float* d_dDskip, void* stream);

/* ------------------------------------------------------------------ integer-only pipeline */

/*
 * Integer-only predictor for decoding on another device (Results &
 * Discussion, portability and limitations: the paper proposes INT8 or
 * fixed-point state-space and affine maps with explicit rounding and
 * saturation, and deterministic integer LayerNorm and softmax).  After the
 * weight conversion every quantity is an integer:
 *  - projections INT8 x INT8 with exact INT32 sums; the weights carry one
 *    power-of-two scale per output row, and the activations one per vector,
 *    chosen from the vector's maximum;
 *  - activations Q12, Delta Q20, the scan state Q16, exponentials Q30;
 *  - exp, SiLU, softplus and the softmax have integer forms.
 * Integer sums do not depend on their order, so the frequency tables, and
 * with them the coded bytes, are the same on any device that follows the
 * rules.  The range coder is the one of boa_encode_dev.
 *
 * boa_qmodel_create converts the model's current float32 weights (host,
 * float64, one rounding per value) and uploads the integer model to the
 * model's device.  The float model may then change or be freed.  Supported:
 * d_state 16, d_conv 4, d_model <= 512, no feed-forward sub-layer
 * (BOA_E_UNSUPPORTED otherwise).  Release with boa_qmodel_free.
 */
typedef struct boa_qmodel boa_qmodel;
int boa_qmodel_create(const boa_model* m, boa_qmodel** out);
void boa_qmodel_free(boa_qmodel* q);

/* Integer tables for `batch` device sequences of seq_len bytes (d_seqs
 * [batch][seq_len]) from the zero state: d_tables (uint16) and d_logits
 * (int32, Q12), both [batch][seq_len - 1][256], row t predicting byte t + 1.
 * Every row sums to 65536 with every entry >= 1.  Synchronises `stream`. */
int boa_int_tables_dev(const boa_qmodel* q, const uint8_t* d_seqs, uint32_t batch, uint32_t seq_len,
                       uint16_t* d_tables, int32_t* d_logits, void* stream);

/* Encode chunks with the integer pipeline (Coders & Parallelisation: chunks
 * are independent streams, the first byte of each stored by the caller).
 * Chunk i is h_chunk_len[i] bytes at d_data + h_chunk_off[i]; its payload
 * goes to d_payload + h_pay_off[i], at most h_pay_cap[i] bytes, and
 * d_pay_len[i] gets the bytes written (0xFFFFFFFF: the payload exceeded its
 * capacity).  One workgroup per chunk; the call allocates its per-chunk
 * state (19 x d_inner x n_layers int32 per chunk) and synchronises `stream`.
 */
int boa_int_encode_dev(const boa_qmodel* q, const uint8_t* d_data, const uint64_t* h_chunk_off,
                       const uint64_t* h_chunk_len, uint64_t n_chunks, uint8_t* d_payload,
                       const uint64_t* h_pay_off, const uint64_t* h_pay_cap, uint32_t* d_pay_len, void* stream);

/* Decode what boa_int_encode_dev wrote, on any device: chunk i (first byte
 * h_first[i], payload h_pay_len[i] bytes at d_payload + h_pay_off[i]) is
 * written to d_out + h_chunk_off[i] (h_chunk_len[i] bytes).  Allocates its
 * per-chunk state and synchronises `stream`. */
int boa_int_decode_dev(const boa_qmodel* q, const uint8_t* d_payload, const uint64_t* h_pay_off,
                       const uint64_t* h_pay_len, const uint8_t* h_first, const uint64_t* h_chunk_off,
                       const uint64_t* h_chunk_len, uint64_t n_chunks, uint8_t* d_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* BOA_H */
