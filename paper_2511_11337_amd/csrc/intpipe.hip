// Integer-only predictor and coder: the deterministic pipeline the paper
// proposes for decoding on another device (Results & Discussion, portability
// and limitations).  Every projection is INT8 x INT8 with an exact INT32
// accumulation, every other quantity is a fixed-point integer with a stated
// rounding and saturation, and LayerNorm, the exponential, SiLU, softplus and
// the softmax-to-histogram step have integer forms.  Integer sums do not
// depend on their order, so the frequency tables -- and with them the coded
// bytes -- are the same on any device that follows these rules.
//
// The rules (Q formats, rounding shifts, the exponential's table and Taylor
// polynomial, the logarithm's series) are written out at the functions below.
// Weight conversion (boa_qmodel_create) runs on the host in float64 with one
// rounding per value; the kernel then sees only integers.
//
// Kernel shape: one workgroup of 256 threads per chunk walks the chunk's steps
// in order (the state is a recurrence); the conv window and scan state of the
// chunk live in a device buffer, every other vector in LDS.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hotpath_common.h"

namespace {

using ll = long long;
constexpr int NT = 256;
constexpr ll SAT23 = (1LL << 23) - 1;
constexpr ll SAT31 = (1LL << 31) - 1;
constexpr ll EPS_Q24 = 168;                       // rint(1e-5 * 2^24)
constexpr int QN = 16;                            // d_state

// 2^(k/16) in Q30
__constant__ ll kT16[16] = {1073741824LL, 1121280436LL, 1170923762LL, 1222764986LL, 1276901417LL, 1333434672LL,
                            1392470869LL, 1454120821LL, 1518500250LL, 1585730000LL, 1655936265LL, 1729250827LL,
                            1805811301LL, 1885761398LL, 1969251188LL, 2056437387LL};
// ln(1 + k/16) in Q30
__constant__ ll kLNC[17] = {0LL, 65095192LL, 126468572LL, 184522808LL, 239598564LL, 291986604LL,
                            341937090LL, 389666807LL, 435364845LL, 479197128LL, 521310048LL, 561833416LL,
                            600882877LL, 638561895LL, 674963409LL, 710171213LL, 744261118LL};
const ll hT16[16] = {1073741824LL, 1121280436LL, 1170923762LL, 1222764986LL, 1276901417LL, 1333434672LL,
                     1392470869LL, 1454120821LL, 1518500250LL, 1585730000LL, 1655936265LL, 1729250827LL,
                     1805811301LL, 1885761398LL, 1969251188LL, 2056437387LL};
// (ln 2)^k / k! in Q30, log2(e) in Q30, 1/5 and 1/3 in Q30
constexpr ll C1 = 744261118LL, C2 = 257941248LL, C3 = 59597083LL, C4 = 10327387LL;
constexpr ll LOG2E = 1549082005LL;
constexpr ll H5 = 214748365LL, H3 = 357913941LL;

// round(x / 2^s), half up (arithmetic shifts are floors); x 2^-s for s < 0
__host__ __device__ inline ll rsh(ll x, int s) {
    if (s > 0) return (x + (1LL << (s - 1))) >> s;
    if (s < 0) return (ll)((unsigned long long)x << (-s));
    return x;
}
__host__ __device__ inline ll clampll(ll x, ll lo, ll hi) { return x < lo ? lo : (x > hi ? hi : x); }
// exact products of operands known to fit in 32 bits (one 32 x 32 -> 64 multiply
// instead of the 64 x 64 sequence)
__host__ __device__ inline ll mul32(ll a, ll b) { return (ll)(int)a * (ll)(int)b; }
__host__ __device__ inline ll mulu32(ll a, ll b) { return (ll)((unsigned long long)(unsigned)a * (unsigned)b); }
// floor(a / b) for b > 0, |a| < 2^62, b < 2^53: the double quotient is within
// 2^-4 of a / b for every use here (numerators exact in double, or the one
// sum of squares whose rounding moves the quotient by under 1/4), so its
// floor is the answer or one off, and the integer checks settle it exactly
__device__ inline ll fdiv(ll a, ll b) {
    ll q = (ll)floor((double)a / (double)b);
    while (q * b > a) --q;
    while ((q + 1) * b <= a) ++q;
    return q;
}
// 2^30 2^(g / 2^30) for 0 <= g < 2^30: 2^(k/16) from the table times a
// degree-4 Taylor polynomial of 2^u on [0, 1/16), Horner in Q30
__host__ __device__ inline ll exp2_frac(ll g, ll tk) {
    const ll u = g & ((1LL << 26) - 1);
    ll q = C4;                                    // 0 < q <= 2^31, 0 <= u < 2^26, tk < 2^31
    q = C3 + rsh(mulu32(q, u), 30);
    q = C2 + rsh(mulu32(q, u), 30);
    q = C1 + rsh(mulu32(q, u), 30);
    q = (1LL << 30) + rsh(mulu32(q, u), 30);
    return rsh(mulu32(tk, q), 30);
}
// exp(x / 2^24) in Q30 for x <= 0 (0 below 2^-46)
__device__ inline ll exp_neg(ll x, const ll* T16) {
    if (x < -(64LL << 24)) x = -(64LL << 24);     // -2^30 <= x <= 0
    const ll y = rsh(mul32(x, LOG2E), 24);
    const ll n = y >> 30;
    const ll g = y - (n << 30);
    const ll p = exp2_frac(g, T16[g >> 26]);
    const ll sh = -n;                             // >= 0: a right shift, rounded half up, without branches
    return sh >= 62 ? 0 : (p + ((1LL << sh) >> 1)) >> sh;
}
__device__ inline ll sigmoid_q30(ll u, const ll* T16) {          // u Q12
    const ll e = exp_neg(-(u < 0 ? -u : u) << 12, T16);
    return u >= 0 ? fdiv(1LL << 60, (1LL << 30) + e) : fdiv(e << 30, (1LL << 30) + e);
}
__device__ inline ll silu_q12(ll u, const ll* T16) {
    return clampll(rsh(mul32(u, sigmoid_q30(u, T16)), 30), -SAT23, SAT23);
}
// ln(1 + w / 2^30) in Q30 for 0 <= w <= 2^30: ln(1 + k/16) from the table plus
// the series of ln(1 + r), r = (1 + w) / (1 + k/16) - 1 < 1/17, to r^5
__device__ inline ll log1p_q30(ll w, const ll* LNC) {
    const ll k = w >> 26;
    const ll c = (1LL << 30) + (k << 26);
    const ll r = fdiv(((1LL << 30) + w - c) << 30, c);
    ll h = H5;                                    // 0 < h <= 2^30, 0 <= r < 2^26
    h = (1LL << 28) - rsh(mulu32(h, r), 30);
    h = H3 - rsh(mulu32(h, r), 30);
    h = (1LL << 29) - rsh(mulu32(h, r), 30);
    h = (1LL << 30) - rsh(mulu32(h, r), 30);
    return LNC[k] + rsh(mulu32(h, r), 30);
}
__device__ inline ll softplus_q20(ll v, const ll* T16, const ll* LNC) {         // v Q12 -> Delta Q20
    const ll w = exp_neg(-(v < 0 ? -v : v) << 12, T16);
    return clampll(((v > 0 ? v : 0) << 8) + rsh(log1p_q30(w, LNC), 10), 0, 1LL << 30);
}
__device__ inline ll isqrt64(ll v) {              // floor(sqrt(v)), v >= 0
    ll r = (ll)sqrt((double)v);
    while (r > 0 && r * r > v) --r;
    while ((r + 1) * (r + 1) <= v) ++r;
    return r;
}
__device__ inline int bitlen(unsigned m) { return m ? 32 - __clz(m) : 0; }

// ---------------------------------------------------------------- model
struct QLayer {
    const int* ln_g; const int* ln_b;
    const int* in_w; const int* in_p;           // words [D/4][2Di]: byte b of (k4, o) = w8[o][4 k4 + b]; [2Di]
    const int* cw; const int* cb;               // [4][Di] Q14; [Di] Q12
    const int* x_w; const int* x_p;             // words [NO][Di/4]; [NO]
    const int* dt_w; const int* dt_p; const int* dtb;   // words [R/4][Di]; [Di]; [Di]
    const int* A; const int* Dq;                // [N][Di] Q12; [Di] Q12
    const int* out_w; const int* out_p;         // words [Di/4][D]; [D]
};
constexpr int QMAX_LAYERS = 16;
struct QArgs {
    QLayer L[QMAX_LAYERS];
    int n_layers, D, Di, R;
    const int* embed;                            // [256][D] Q12
    const int* nf_g; const int* nf_b;
    const int* head_w; const int* head_p; const int* head_b;   // words [D/4][256]; [256]; [256]
};

constexpr int MODE_TABLES = 0, MODE_ENCODE = 1, MODE_DECODE = 2;
struct QJob {
    const uint8_t* in;          // tables: seqs [B][T]; encode: the data; decode: the payloads
    const ll* chunk_off;        // byte offset of each chunk in the data (tables, encode) or output (decode)
    const ll* chunk_len;
    const ll* pay_off;          // encode / decode
    const ll* pay_n;            // encode: capacity; decode: payload length
    const uint8_t* first;       // decode: first byte of each chunk
    uint8_t* out;               // encode: payloads; decode: decoded bytes
    uint32_t* pay_len;          // encode: bytes written (0xFFFFFFFF: over capacity)
    uint16_t* tables;           // tables: [B][T-1][256]
    int* logits;                // tables: [B][T-1][256] Q12
    int* state;                 // per chunk: conv window [L][3][Di], then h [L][N][Di]
    ll state_words;
};

// ---------------------------------------------------------------- block helpers
__device__ inline ll blk_sum(ll v, ll* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}
__device__ inline ll blk_max(ll v, ll* red) {
    for (int o = 32; o > 0; o >>= 1) { ll w = __shfl_xor(v, o); v = w > v ? w : v; }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    ll m = red[0];
    for (int i = 1; i < 4; ++i) m = red[i] > m ? red[i] : m;
    return m;
}
// the largest value, lowest index among ties
__device__ inline int blk_argmax(ll v, int idx, ll* red, int* redi) {
    for (int o = 32; o > 0; o >>= 1) {
        ll w = __shfl_xor(v, o);
        int wi = __shfl_xor(idx, o);
        if (w > v || (w == v && wi < idx)) { v = w; idx = wi; }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6] = v; redi[threadIdx.x >> 6] = idx; }
    __syncthreads();
    ll bv = red[0];
    int bi = redi[0];
    for (int i = 1; i < 4; ++i)
        if (red[i] > bv || (red[i] == bv && redi[i] < bi)) { bv = red[i]; bi = redi[i]; }
    return bi;
}

// LayerNorm of D Q12 values (src) into dst
__device__ void int_ln(const int* src, int* dst, const int* g, const int* b, int D, ll* red) {
    const int t = threadIdx.x;
    ll s = 0;
    for (int d = t; d < D; d += NT) s += src[d];
    s = blk_sum(s, red);
    const ll mu = fdiv(s, D);
    ll v = 0;
    for (int d = t; d < D; d += NT) { ll dd = src[d] - mu; v += mul32(dd, dd); }   // |dd| < 2^24
    v = blk_sum(v, red);
    const ll sd = isqrt64(fdiv(v, D) + EPS_Q24);
    for (int d = t; d < D; d += NT) {
        const ll dd = src[d] - mu;
        const ll nn = fdiv(2 * (dd << 12) + sd, 2 * sd);
        dst[d] = (int)clampll(rsh(nn * g[d], 12) + b[d], -SAT23, SAT23);
    }
    __syncthreads();
}
// dynamic INT8 input of a projection: packs n values of src (n % 4 == 0) into
// words and returns the shift e
__device__ int int_q8(const int* src, int n, int* words, ll* red) {
    const int t = threadIdx.x;
    ll m = 0;
    for (int i = t; i < n; i += NT) { ll a = src[i] < 0 ? -(ll)src[i] : src[i]; m = a > m ? a : m; }
    m = blk_max(m, red);
    const int bl = bitlen((unsigned)m);
    const int e = bl > 7 ? bl - 7 : 0;
    for (int w = t; w < n / 4; w += NT) {
        unsigned pk = 0;
        for (int b = 0; b < 4; ++b) {
            ll q = clampll(rsh(src[4 * w + b], e), -127, 127);
            pk |= ((unsigned)q & 0xFFu) << (8 * b);
        }
        words[w] = (int)pk;
    }
    __syncthreads();
    return e;
}

struct QShared {
    int r[512], nrm[512];
    int a8[256];
    int xz[2048];
    int xs[1024];
    int gate[1024];
    int dbc[64];
    int f[256], cx[256];
    ll red[4];
    int redi[4];
    int sym, x;
    ll t16[16], lnc[17];         // the exponential's and logarithm's tables, read with divergent indexes
};

// DM = d_model: every loop bound below is a compile-time constant
template <int DM>
__global__ __launch_bounds__(NT) void k_int_chunk(QArgs a, QJob j, int mode) {
    __shared__ QShared sh;
    const int t = threadIdx.x;
    const ll c = blockIdx.x;
    const ll len = j.chunk_len[c];
    constexpr int D = DM, Di = 2 * DM, R = DM / 16, NO = R + 2 * QN;
    if (len <= 0) {
        if (mode == MODE_ENCODE && t == 0) j.pay_len[c] = 0;
        return;
    }
    int* st = j.state + c * j.state_words;
    for (ll i = t; i < j.state_words; i += NT) st[i] = 0;
    if (t < 16) sh.t16[t] = kT16[t];
    if (t < 17) sh.lnc[t] = kLNC[t];
    const ll off = j.chunk_off[c];
    int y = mode == MODE_DECODE ? j.first[c] : j.in[off];
    if (mode == MODE_DECODE && t == 0) j.out[off] = (uint8_t)y;
    boa::Enc enc;
    boa::Dec dec;
    uint8_t* pay_out = nullptr;
    const uint8_t* pay_in = nullptr;
    uint32_t cap = 0, plen = 0;
    if (mode == MODE_ENCODE) {
        boa::enc_reset(enc);
        pay_out = j.out + j.pay_off[c];
        cap = (uint32_t)j.pay_n[c];
    } else if (mode == MODE_DECODE) {
        pay_in = j.in + j.pay_off[c];
        plen = (uint32_t)j.pay_n[c];
        boa::dec_reset(dec, pay_in, plen);
    }
    __syncthreads();

    for (ll s = 0; s + 1 < len; ++s) {
        for (int d = t; d < D; d += NT) sh.r[d] = a.embed[y * D + d];
        __syncthreads();
        for (int l = 0; l < a.n_layers; ++l) {
            const QLayer& L = a.L[l];
            int* win = st + (ll)l * 3 * Di;
            int* hst = st + (ll)a.n_layers * 3 * Di + (ll)l * QN * Di;
            // LayerNorm, in_proj
            int_ln(sh.r, sh.nrm, L.ln_g, L.ln_b, D, sh.red);
            int e = int_q8(sh.nrm, D, sh.a8, sh.red);
            for (int o = t; o < 2 * Di; o += NT) {
                int acc = 0;
#pragma unroll 16
                for (int k = 0; k < D / 4; ++k) acc = __builtin_amdgcn_sdot4(sh.a8[k], L.in_w[k * 2 * Di + o], acc, false);
                sh.xz[o] = (int)clampll(rsh(acc, L.in_p[o] - e), -SAT23, SAT23);
            }
            __syncthreads();
            // causal conv over x_{t-3} .. x_t, SiLU
            for (int d = t; d < Di; d += NT) {
                const ll x = sh.xz[d];
                const ll w0 = win[d], w1 = win[Di + d], w2 = win[2 * Di + d];
                const ll u = clampll(rsh((ll)L.cw[d] * w0 + (ll)L.cw[Di + d] * w1 + (ll)L.cw[2 * Di + d] * w2 +
                                             (ll)L.cw[3 * Di + d] * x, 14) + L.cb[d], -SAT23, SAT23);
                win[d] = (int)w1;
                win[Di + d] = (int)w2;
                win[2 * Di + d] = (int)x;
                sh.xs[d] = (int)silu_q12(u, sh.t16);
            }
            __syncthreads();
            // x_proj: one wave per output, the lanes split the inputs
            e = int_q8(sh.xs, Di, sh.a8, sh.red);
            {
                const int wv = t >> 6, ln = t & 63;
                for (int o = wv; o < NO; o += NT / 64) {
                    int acc = 0;
                    for (int k = ln; k < Di / 4; k += 64) acc = __builtin_amdgcn_sdot4(sh.a8[k], L.x_w[o * (Di / 4) + k], acc, false);
                    for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
                    if (ln == 0) sh.dbc[o] = (int)clampll(rsh(acc, L.x_p[o] - e), -SAT23, SAT23);
                }
            }
            __syncthreads();
            // dt_proj (its R inputs quantised by every thread alike), softplus,
            // the scan and the gate, one channel per thread
            {
                ll m = 0;
                for (int k = 0; k < R; ++k) { ll v = sh.dbc[k] < 0 ? -(ll)sh.dbc[k] : sh.dbc[k]; m = v > m ? v : m; }
                const int bl = bitlen((unsigned)m);
                const int e3 = bl > 7 ? bl - 7 : 0;
                int dq[8];
                for (int k4 = 0; k4 < R / 4; ++k4) {
                    unsigned pk = 0;
                    for (int b = 0; b < 4; ++b)
                        pk |= ((unsigned)clampll(rsh(sh.dbc[4 * k4 + b], e3), -127, 127) & 0xFFu) << (8 * b);
                    dq[k4] = (int)pk;
                }
                for (int d = t; d < Di; d += NT) {
                    int acc = 0;
                    for (int k4 = 0; k4 < R / 4; ++k4) acc = __builtin_amdgcn_sdot4(dq[k4], L.dt_w[k4 * Di + d], acc, false);
                    const ll v = clampll(rsh(acc, L.dt_p[d] - e3) + L.dtb[d], -SAT23, SAT23);
                    const ll dl = softplus_q20(v, sh.t16, sh.lnc);
                    const ll xs = sh.xs[d];
                    const ll dx = rsh(mul32(dl, xs), 20);           // dl <= 2^30, |xs| < 2^23
                    ll ys = 0;
                    // four states at a time: their A and h loads go out together (h is
                    // written back in the same pass, so the compiler would not move the
                    // next loads above those stores by itself)
                    for (int n0 = 0; n0 < QN; n0 += 4) {
                        int Av[4], hv[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            Av[i] = L.A[(n0 + i) * Di + d];
                            hv[i] = hst[(n0 + i) * Di + d];
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int n = n0 + i;
                            // dl <= 2^30, |A| <= 2^24, dA <= 2^30, |h| < 2^31: 32-bit operands
                            const ll dA = exp_neg(rsh(mul32(dl, Av[i]), 8), sh.t16);
                            const ll hn = clampll(rsh(mul32(dA, hv[i]), 30) + rsh(dx * (ll)sh.dbc[R + n], 8), -SAT31, SAT31);
                            hst[n * Di + d] = (int)hn;
                            ys += mul32(sh.dbc[R + QN + n], hn);
                        }
                    }
                    const ll yv = clampll(rsh(ys, 16) + rsh(mul32(L.Dq[d], xs), 12), -SAT23, SAT23);
                    sh.gate[d] = (int)clampll(rsh(mul32(yv, silu_q12(sh.xz[Di + d], sh.t16)), 12), -SAT23, SAT23);
                }
            }
            __syncthreads();
            // out_proj and the residual
            e = int_q8(sh.gate, Di, sh.a8, sh.red);
            for (int o = t; o < D; o += NT) {
                int acc = 0;
#pragma unroll 16
                for (int k = 0; k < Di / 4; ++k) acc = __builtin_amdgcn_sdot4(sh.a8[k], L.out_w[k * D + o], acc, false);
                const ll pr = clampll(rsh(acc, L.out_p[o] - e), -SAT23, SAT23);
                sh.r[o] = (int)clampll(sh.r[o] + pr, -SAT23, SAT23);
            }
            __syncthreads();
        }
        // final LayerNorm, head: thread t owns symbol t
        int_ln(sh.r, sh.nrm, a.nf_g, a.nf_b, D, sh.red);
        const int e = int_q8(sh.nrm, D, sh.a8, sh.red);
        int acc = 0;
#pragma unroll 16
        for (int k = 0; k < D / 4; ++k) acc = __builtin_amdgcn_sdot4(sh.a8[k], a.head_w[k * 256 + t], acc, false);
        const ll lg = clampll(rsh(acc, a.head_p[t] - e) + a.head_b[t], -SAT23, SAT23);
        // integer softmax and histogram
        const ll mx = blk_max(lg, sh.red);
        const ll ex = exp_neg((lg - mx) << 12, sh.t16);
        const ll S = blk_sum(ex, sh.red);
        ll f = fdiv(ex << 16, S);
        f = f < 1 ? 1 : f;
        const ll tot = blk_sum(f, sh.red);
        const int am = blk_argmax(f, t, sh.red, sh.redi);
        if (t == am) f += 65536 - tot;
        // exclusive prefix sum: wave scan, then the waves' totals
        ll inc = f;
        for (int o = 1; o < 64; o <<= 1) {
            ll v = __shfl_up(inc, o);
            if ((t & 63) >= o) inc += v;
        }
        __syncthreads();
        if ((t & 63) == 63) sh.red[t >> 6] = inc;
        __syncthreads();
        ll base = 0;
        for (int w = 0; w < (t >> 6); ++w) base += sh.red[w];
        const ll cx = base + inc - f;
        sh.f[t] = (int)f;
        sh.cx[t] = (int)cx;
        if (mode == MODE_TABLES) {
            const ll row = c * (len - 1) + s;
            j.tables[row * 256 + t] = (uint16_t)f;
            j.logits[row * 256 + t] = (int)lg;
            y = j.in[off + s + 1];
        } else if (mode == MODE_ENCODE) {
            y = j.in[off + s + 1];
            __syncthreads();
            if (t == 0) boa::enc_put(enc, (uint32_t)sh.cx[y], (uint32_t)sh.f[y], pay_out, cap);
        } else {
            if (t == 0) sh.x = (int)boa::dec_target(dec);
            __syncthreads();
            if (cx <= sh.x && sh.x < cx + f) sh.sym = t;
            __syncthreads();
            y = sh.sym;
            if (t == 0) {
                boa::dec_update(dec, (uint32_t)sh.cx[y], (uint32_t)sh.f[y], pay_in, plen);
                j.out[off + s + 1] = (uint8_t)y;
            }
        }
        __syncthreads();
    }
    if (mode == MODE_ENCODE && t == 0) {
        boa::enc_flush(enc, pay_out, cap);
        j.pay_len[c] = enc.cur <= cap ? enc.cur : 0xFFFFFFFFu;
    }
}

// ---------------------------------------------------------------- host conversion
ll fixq(double v, int frac, ll lim) { return clampll((ll)std::nearbyint(std::ldexp(v, frac)), -lim, lim); }

// per-row power-of-two INT8: p = largest integer with max|W_j| 2^p <= 127,
// clamped to [0, 40]; w8 = clamp(rint(W 2^p), -127, 127)
void conv_proj(const float* W, int out, int in, std::vector<int8_t>& w8, std::vector<int>& p) {
    w8.assign((size_t)out * in, 0);
    p.assign(out, 0);
    for (int j = 0; j < out; ++j) {
        double m = 0;
        for (int i = 0; i < in; ++i) m = std::fmax(m, std::fabs((double)W[(size_t)j * in + i]));
        int pj = 0;
        if (m != 0.0) {
            int E = 0;
            const double fr = std::frexp(m, &E);
            pj = fr <= 127.0 / 128.0 ? 7 - E : 6 - E;
            pj = pj < 0 ? 0 : (pj > 40 ? 40 : pj);
        }
        p[j] = pj;
        for (int i = 0; i < in; ++i)
            w8[(size_t)j * in + i] = (int8_t)clampll((ll)std::nearbyint(std::ldexp((double)W[(size_t)j * in + i], pj)), -127, 127);
    }
}
inline int pack4(const int8_t* v) {
    unsigned pk = 0;
    for (int b = 0; b < 4; ++b) pk |= ((unsigned)(uint8_t)v[b]) << (8 * b);
    return (int)pk;
}

}  // namespace

struct boa_qmodel {
    boa_config cfg{};
    int device = 0;
    uint64_t fingerprint = 0;
    int* d_blob = nullptr;
    QArgs args{};
};

#define QCHK(expr)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return boa::set_error(BOA_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" int boa_qmodel_create(const boa_model* m, boa_qmodel** out) {
    if (!m || !out) return boa::set_error(BOA_E_ARG, "null argument");
    *out = nullptr;
    const boa_config& cfg = m->cfg;
    const boa::Layout& lay = m->lay;
    if (cfg.ffn_mult != 0 || cfg.d_state != 16 || cfg.d_conv != 4 || cfg.n_layers > QMAX_LAYERS || cfg.d_model > 512)
        return boa::set_error(BOA_E_UNSUPPORTED, "integer pipeline: d_state 16, d_conv 4, d_model <= 512, no feed-forward sub-layer");
    std::vector<float> w(lay.total);
    int rc = boa_model_get_weights(m, w.data(), w.size());
    if (rc) return rc;
    const int D = lay.D, Di = lay.Di, R = lay.R, N = lay.N, K = lay.K, NL = lay.L, NO = R + 2 * N;
    std::vector<int> blob;
    std::vector<size_t> at;             // offsets of the pieces, in order
    auto put = [&](const std::vector<int>& v) { at.push_back(blob.size()); blob.insert(blob.end(), v.begin(), v.end()); };
    auto fixv = [&](uint64_t o, size_t n, int frac, ll lim) {
        std::vector<int> v(n);
        for (size_t i = 0; i < n; ++i) v[i] = (int)fixq(w[o + i], frac, lim);
        return v;
    };
    std::vector<int8_t> w8;
    std::vector<int> p;
    // rows-as-outputs words [in/4][out]
    auto words_kmajor = [&](int outn, int inn) {
        std::vector<int> v((size_t)(inn / 4) * outn);
        for (int k = 0; k < inn / 4; ++k)
            for (int o = 0; o < outn; ++o) v[(size_t)k * outn + o] = pack4(&w8[(size_t)o * inn + 4 * k]);
        return v;
    };
    put(fixv(lay.embed, (size_t)256 * D, 12, SAT23));
    put(fixv(lay.norm_f_w, D, 12, SAT23));
    put(fixv(lay.norm_f_b, D, 12, SAT23));
    conv_proj(&w[lay.head_w], 256, D, w8, p);
    put(words_kmajor(256, D));
    put(p);
    put(fixv(lay.head_b, 256, 12, SAT23));
    for (int l = 0; l < NL; ++l) {
        const boa::LayerOff& o = lay.layer[l];
        put(fixv(o.norm_w, D, 12, SAT23));
        put(fixv(o.norm_b, D, 12, SAT23));
        conv_proj(&w[o.in_w], 2 * Di, D, w8, p);
        put(words_kmajor(2 * Di, D));
        put(p);
        std::vector<int> cw((size_t)K * Di);
        for (int d = 0; d < Di; ++d)
            for (int k = 0; k < K; ++k) cw[(size_t)k * Di + d] = (int)fixq(w[o.conv_w + (size_t)d * K + k], 14, 1LL << 20);
        put(cw);
        put(fixv(o.conv_b, Di, 12, SAT23));
        conv_proj(&w[o.xw], NO, Di, w8, p);
        {
            std::vector<int> v((size_t)NO * (Di / 4));
            for (int r = 0; r < NO; ++r)
                for (int k = 0; k < Di / 4; ++k) v[(size_t)r * (Di / 4) + k] = pack4(&w8[(size_t)r * Di + 4 * k]);
            put(v);
        }
        put(p);
        conv_proj(&w[o.dtw], Di, R, w8, p);
        put(words_kmajor(Di, R));
        put(p);
        put(fixv(o.dtb, Di, 12, SAT23));
        // A = -exp(A_log): A_log in Q24 clamped to [-16, 9], the integer exp2
        std::vector<int> A((size_t)N * Di);
        for (int d = 0; d < Di; ++d)
            for (int n = 0; n < N; ++n) {
                const ll a24 = clampll(fixq(w[o.A_log + (size_t)d * N + n], 24, 1LL << 40), -(16LL << 24), 9LL << 24);
                const ll y = rsh(a24 * LOG2E, 24);
                const ll nn = y >> 30;
                const ll g = y - (nn << 30);
                const ll mant = exp2_frac(g, hT16[g >> 26]);
                const ll v = rsh(mant, (int)(18 - nn));
                A[(size_t)n * Di + d] = (int)-(v < (1LL << 24) ? v : (1LL << 24));
            }
        put(A);
        put(fixv(o.Dsk, Di, 12, SAT23));
        conv_proj(&w[o.out_w], D, Di, w8, p);
        put(words_kmajor(D, Di));
        put(p);
    }
    boa_qmodel* q = new boa_qmodel();
    q->cfg = cfg;
    q->device = m->device;
    q->fingerprint = boa::model_fingerprint(m);
    hipError_t he = hipSetDevice(m->device);
    if (he == hipSuccess) he = hipMalloc(&q->d_blob, blob.size() * sizeof(int));
    if (he == hipSuccess) he = hipMemcpy(q->d_blob, blob.data(), blob.size() * sizeof(int), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
        if (q->d_blob) (void)hipFree(q->d_blob);
        delete q;
        return boa::set_error(BOA_E_DEVICE, std::string("integer model upload: ") + hipGetErrorString(he));
    }
    const int* b = q->d_blob;
    size_t i = 0;
    QArgs& A = q->args;
    A.n_layers = NL; A.D = D; A.Di = Di; A.R = R;
    A.embed = b + at[i++]; A.nf_g = b + at[i++]; A.nf_b = b + at[i++];
    A.head_w = b + at[i++]; A.head_p = b + at[i++]; A.head_b = b + at[i++];
    for (int l = 0; l < NL; ++l) {
        QLayer& L = A.L[l];
        L.ln_g = b + at[i++]; L.ln_b = b + at[i++];
        L.in_w = b + at[i++]; L.in_p = b + at[i++];
        L.cw = b + at[i++]; L.cb = b + at[i++];
        L.x_w = b + at[i++]; L.x_p = b + at[i++];
        L.dt_w = b + at[i++]; L.dt_p = b + at[i++]; L.dtb = b + at[i++];
        L.A = b + at[i++]; L.Dq = b + at[i++];
        L.out_w = b + at[i++]; L.out_p = b + at[i++];
    }
    *out = q;
    return BOA_OK;
}

extern "C" void boa_qmodel_free(boa_qmodel* q) {
    if (!q) return;
    if (q->d_blob) {
        (void)hipSetDevice(q->device);
        (void)hipFree(q->d_blob);
    }
    delete q;
}

namespace {
// per-chunk arrays and state in one device allocation; runs the kernel and waits
int run_chunks(const boa_qmodel* q, QJob j, int mode, uint64_t n_chunks, const uint64_t* h_off, const uint64_t* h_len,
               const uint64_t* h_poff, const uint64_t* h_pn, const uint8_t* h_first, void* stream) {
    if (n_chunks == 0) return BOA_OK;
    if (n_chunks > (uint64_t)INT32_MAX) return boa::set_error(BOA_E_ARG, "too many chunks");
    QCHK(hipSetDevice(q->device));
    const ll sw = (ll)q->args.n_layers * (3 + QN) * q->args.Di;
    std::vector<ll> hv((size_t)n_chunks * 4);
    for (uint64_t c = 0; c < n_chunks; ++c) {
        if (h_len[c] > (uint64_t)INT64_MAX / 2) return boa::set_error(BOA_E_ARG, "chunk length out of range");
        hv[c] = (ll)h_off[c];
        hv[n_chunks + c] = (ll)h_len[c];
        hv[2 * n_chunks + c] = h_poff ? (ll)h_poff[c] : 0;
        hv[3 * n_chunks + c] = h_pn ? (ll)h_pn[c] : 0;
        if (h_pn && h_pn[c] > 0xFFFFFFFFull) return boa::set_error(BOA_E_ARG, "payload size beyond 32 bits");
    }
    const size_t arr = hv.size() * sizeof(ll);
    const size_t firsts = h_first ? ((n_chunks + 255) / 256) * 256 : 0;
    const size_t state = (size_t)n_chunks * (size_t)sw * sizeof(int);
    char* buf = nullptr;
    QCHK(hipMalloc(&buf, arr + firsts + state));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(buf, hv.data(), arr, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && h_first) e = hipMemcpyAsync(buf + arr, h_first, n_chunks, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        const ll* dv = (const ll*)buf;
        j.chunk_off = dv;
        j.chunk_len = dv + n_chunks;
        j.pay_off = dv + 2 * n_chunks;
        j.pay_n = dv + 3 * n_chunks;
        j.first = h_first ? (const uint8_t*)(buf + arr) : nullptr;
        j.state = (int*)(buf + arr + firsts);
        j.state_words = sw;
        const dim3 grid((unsigned)n_chunks), blk(NT);
        switch (q->args.D) {
            case 64: hipLaunchKernelGGL(k_int_chunk<64>, grid, blk, 0, s, q->args, j, mode); break;
            case 128: hipLaunchKernelGGL(k_int_chunk<128>, grid, blk, 0, s, q->args, j, mode); break;
            case 256: hipLaunchKernelGGL(k_int_chunk<256>, grid, blk, 0, s, q->args, j, mode); break;
            default: hipLaunchKernelGGL(k_int_chunk<512>, grid, blk, 0, s, q->args, j, mode); break;
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipError_t ef = hipFree(buf);
    if (e != hipSuccess) return boa::set_error(BOA_E_DEVICE, std::string("integer pipeline: ") + hipGetErrorString(e));
    if (ef != hipSuccess) return boa::set_error(BOA_E_DEVICE, std::string("hipFree: ") + hipGetErrorString(ef));
    return BOA_OK;
}
}  // namespace

extern "C" int boa_int_tables_dev(const boa_qmodel* q, const uint8_t* d_seqs, uint32_t batch, uint32_t seq_len,
                                  uint16_t* d_tables, int32_t* d_logits, void* stream) {
    if (!q || (batch && (!d_seqs || (seq_len > 1 && (!d_tables || !d_logits)))))
        return boa::set_error(BOA_E_ARG, "null argument");
    std::vector<uint64_t> off(batch), len(batch, seq_len);
    for (uint32_t b = 0; b < batch; ++b) off[b] = (uint64_t)b * seq_len;
    QJob j{};
    j.in = d_seqs;
    j.tables = d_tables;
    j.logits = d_logits;
    return run_chunks(q, j, MODE_TABLES, batch, off.data(), len.data(), nullptr, nullptr, nullptr, stream);
}

extern "C" int boa_int_encode_dev(const boa_qmodel* q, const uint8_t* d_data, const uint64_t* h_chunk_off,
                                  const uint64_t* h_chunk_len, uint64_t n_chunks, uint8_t* d_payload,
                                  const uint64_t* h_pay_off, const uint64_t* h_pay_cap, uint32_t* d_pay_len,
                                  void* stream) {
    if (!q || (n_chunks && (!d_data || !h_chunk_off || !h_chunk_len || !d_payload || !h_pay_off || !h_pay_cap ||
                            !d_pay_len)))
        return boa::set_error(BOA_E_ARG, "null argument");
    QJob j{};
    j.in = d_data;
    j.out = d_payload;
    j.pay_len = d_pay_len;
    return run_chunks(q, j, MODE_ENCODE, n_chunks, h_chunk_off, h_chunk_len, h_pay_off, h_pay_cap, nullptr, stream);
}

extern "C" int boa_int_decode_dev(const boa_qmodel* q, const uint8_t* d_payload, const uint64_t* h_pay_off,
                                  const uint64_t* h_pay_len, const uint8_t* h_first, const uint64_t* h_chunk_off,
                                  const uint64_t* h_chunk_len, uint64_t n_chunks, uint8_t* d_out, void* stream) {
    if (!q || (n_chunks && (!d_payload || !h_pay_off || !h_pay_len || !h_first || !h_chunk_off || !h_chunk_len ||
                            !d_out)))
        return boa::set_error(BOA_E_ARG, "null argument");
    QJob j{};
    j.in = d_payload;
    j.out = d_out;
    return run_chunks(q, j, MODE_DECODE, n_chunks, h_chunk_off, h_chunk_len, h_pay_off, h_pay_len, h_first, stream);
}
