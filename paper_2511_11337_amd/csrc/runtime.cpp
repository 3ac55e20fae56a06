// Host runtime of libboa: model management, the static lane schedule, the
// encoder / decoder drivers (time-tiled encoder, hipGraph-replayed decoder
// step), the .boa container and the C ABI declared in include/boa.h.
#include "boa_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

using namespace boa;

// =================================================================== errors
namespace {
thread_local std::string g_err;
thread_local std::vector<uint64_t> g_last_pay;
thread_local std::vector<uint32_t> g_last_coder;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}
#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(BOA_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

// ----------------------------------------------------------------- device buffers
// Device memory of one call carved from one region -- a workspace the caller
// owns, or one allocation of the measured size.  A measuring arena hands out
// no memory and only adds up the bytes (each piece 256-byte aligned).
struct Arena {
    uint8_t* base = nullptr;
    size_t cap = 0, used = 0;
    bool measuring = true;
    void* take(size_t bytes) {
        used = (used + 255) & ~(size_t)255;
        void* q = measuring ? nullptr : base + used;
        used += bytes ? bytes : 1;
        return q;
    }
};

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    bool own = false;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p && own) (void)hipFree(p);
        p = nullptr;
        own = false;
    }
    hipError_t alloc(size_t bytes) {
        release();
        n = bytes;
        own = true;
        return hipMalloc(&p, bytes ? bytes : 1);
    }
    // a piece of the arena (not freed by this buffer)
    void carve(Arena& a, size_t bytes) {
        release();
        n = bytes;
        p = a.take(bytes);
    }
    template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};
#define ALLOC(buf, bytes) HIPCHK((buf).alloc(bytes))

template <typename T>
hipError_t copy_in(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

template <typename T>
hipError_t upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
    hipError_t e = b.alloc(v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    e = hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);   // host vector may go away after return
}

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ULL) {
    const uint8_t* p = static_cast<const uint8_t*>(data);
    for (size_t i = 0; i < n; ++i) { h ^= p[i]; h *= 1099511628211ULL; }
    return h;
}

uint32_t crc32_host(const uint8_t* p, size_t n, uint32_t c = 0xFFFFFFFFu) {
    static uint32_t table[256];
    static bool init = false;
    if (!init) {
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t v = i;
            for (int b = 0; b < 8; ++b) v = (v >> 1) ^ (0xEDB88320u & (0u - (v & 1u)));
            table[i] = v;
        }
        init = true;
    }
    for (size_t i = 0; i < n; ++i) c = table[(c ^ p[i]) & 0xFF] ^ (c >> 8);
    return c;
}
uint32_t crc32_final(const uint8_t* p, size_t n) { return ~crc32_host(p, n); }

bool config_ok(const boa_config& c) {
    return (c.d_model == 64 || c.d_model == 128 || c.d_model == 256 || c.d_model == 512) &&
           c.d_state == 16 && c.d_conv == 4 && c.expand == 2 && c.n_layers >= 1 && c.n_layers <= 16 &&
           (uint64_t)c.ffn_mult * c.d_model <= 1024;
}
}  // namespace

namespace boa {
int set_error(int code, const std::string& msg) { return fail(code, msg); }

uint64_t model_fingerprint(const boa_model* m) {
    if (m->fp_stale) {
        std::vector<float> w(m->lay.total);
        if (hipMemcpy(w.data(), m->d_w, w.size() * sizeof(float), hipMemcpyDeviceToHost) == hipSuccess) {
            boa_model* mm = const_cast<boa_model*>(m);
            mm->fingerprint = fnv1a(w.data(), w.size() * sizeof(float), fnv1a(&m->cfg, sizeof(boa_config)));
            mm->fp_stale = false;
        }
    }
    return m->fingerprint;
}

bool make_layout(const boa_config& c, Layout* out) {
    if (!config_ok(c)) return false;
    Layout L;
    L.D = (int)c.d_model;
    L.Di = (int)(c.expand * c.d_model);
    L.N = (int)c.d_state;
    L.K = (int)c.d_conv;
    L.R = (int)((c.d_model + 15) / 16);
    L.L = (int)c.n_layers;
    L.H = (int)(c.ffn_mult * c.d_model);
    uint64_t o = 0;
    auto take = [&](uint64_t n) { uint64_t r = o; o += n; return r; };
    const uint64_t D = L.D, Di = L.Di, N = L.N, K = L.K, R = L.R;
    L.embed = take(256 * D);
    for (int l = 0; l < L.L; ++l) {
        LayerOff lo;
        lo.norm_w = take(D); lo.norm_b = take(D);
        lo.in_w = take(2 * Di * D);
        lo.conv_w = take(Di * K); lo.conv_b = take(Di);
        lo.xw = take((R + 2 * N) * Di);
        lo.dtw = take(Di * R); lo.dtb = take(Di);
        lo.A_log = take(Di * N); lo.Dsk = take(Di);
        lo.out_w = take(D * Di);
        if (L.H) {
            const uint64_t H = L.H;
            lo.ffn_w1 = take(H * D); lo.ffn_b1 = take(H);
            lo.ffn_w2 = take(D * H); lo.ffn_b2 = take(D);
            lo.ffn_nw = take(D); lo.ffn_nb = take(D);
        }
        L.layer.push_back(lo);
    }
    L.norm_f_w = take(D); L.norm_f_b = take(D);
    L.head_w = take(256 * D); L.head_b = take(256);
    L.total = o;
    *out = L;
    return true;
}
}  // namespace boa

// =================================================================== model
namespace {
void model_release(boa_model* m) {
    if (!m) return;
    if (m->d_w) (void)hipFree(m->d_w);
    if (m->d_derived) (void)hipFree(m->d_derived);
    if (m->d_w16) (void)hipFree(m->d_w16);
    if (m->d_frag32) (void)hipFree(m->d_frag32);
    if (m->d_frag16) (void)hipFree(m->d_frag16);
    if (m->d_frag8) (void)hipFree(m->d_frag8);
    if (m->d_ew) (void)hipFree(m->d_ew);
    if (m->d_amax) (void)hipFree(m->d_amax);
    if (m->train) train_ctx_free(m->train);
    delete m;
}

int refresh_derived(boa_model* m, const float* h_w) {
    const Layout& L = m->lay;
    m->fingerprint = fnv1a(&m->cfg, sizeof(boa_config));
    m->fingerprint = fnv1a(h_w, L.total * sizeof(float), m->fingerprint);
    HIPCHK(hipSetDevice(m->device));
    HIPCHK(hipMemcpy(m->d_w, h_w, L.total * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(launch_prep(m, nullptr));
    HIPCHK(hipDeviceSynchronize());
    m->fp_stale = false;
    return BOA_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
}  // namespace

extern "C" uint64_t boa_param_count(const boa_config* cfg) {
    Layout L;
    if (!cfg || !make_layout(*cfg, &L)) return 0;
    return L.total;
}

extern "C" int boa_model_create(const boa_config* cfg, const float* h_weights, uint64_t n, int device,
                                boa_model** out) {
    if (!cfg || !h_weights || !out) return fail(BOA_E_ARG, "null argument");
    Layout L;
    if (!make_layout(*cfg, &L)) return fail(BOA_E_ARG, "unsupported model config");
    if (n != L.total) return fail(BOA_E_ARG, "weight count does not match the config");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(BOA_E_UNSUPPORTED, "no HIP device");
    if (device < 0 || device >= ndev) return fail(BOA_E_ARG, "bad device index");
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BOA_E_UNSUPPORTED, std::string("libboa is built for gfx950, device is ") + prop.gcnArchName);
    set_max_lds(prop.sharedMemPerBlock);
    std::unique_ptr<boa_model, void (*)(boa_model*)> m(new boa_model, model_release);
    m->cfg = *cfg;
    m->lay = L;
    m->device = device;
    HIPCHK(hipSetDevice(device));
    if (hipMalloc(&m->d_w, L.total * sizeof(float)) != hipSuccess) return fail(BOA_E_OOM, "weights");
    // convT, dtwT, A2T; BF16 mode: xw_r, dtwT_r (floats) and dtw16 (bf16, two
    // per float slot; R and Di are even); x_proj fragment-ordered for the f32
    // MFMA (xwF, and xwF_r in BF16 mode; rows padded to 16)
    const size_t NOx = (size_t)L.R + 2 * L.N, NOp = (NOx + 15) / 16 * 16;
    const size_t der_base = (size_t)L.Di * (L.K + L.R + L.N) + (size_t)L.Di * (NOx + L.R) + (size_t)L.Di * L.R / 2;
    const size_t per_layer_derived = der_base + 2 * NOp * L.Di;
    if (hipMalloc(&m->d_derived, per_layer_derived * L.L * sizeof(float)) != hipSuccess)
        return fail(BOA_E_OOM, "derived weights");
    // projection matrices per layer: in_proj, out_proj, and with the feed-forward sub-layer W1, W2
    const int mpl = L.H ? 4 : 2;
    const size_t ffn16 = (size_t)2 * L.H * L.D;
    const size_t per_layer16 = (size_t)2 * L.Di * L.D + (size_t)L.D * L.Di + ffn16;
    if (hipMalloc(&m->d_w16, (per_layer16 * L.L + 256 * (size_t)L.D) * sizeof(uint16_t)) != hipSuccess)
        return fail(BOA_E_OOM, "bf16 weights");
    const size_t nfrag = per_layer16 * L.L + 256 * (size_t)L.D;
    if (hipMalloc(&m->d_frag32, nfrag * sizeof(float)) != hipSuccess ||
        hipMalloc(&m->d_frag16, nfrag * sizeof(uint16_t)) != hipSuccess)
        return fail(BOA_E_OOM, "fragment-ordered weights");
    if (hipMalloc(&m->d_frag8, nfrag) != hipSuccess ||
        hipMalloc(&m->d_ew, (mpl * L.L + 1) * sizeof(int)) != hipSuccess ||
        hipMalloc(&m->d_amax, (mpl * L.L + 1) * sizeof(unsigned)) != hipSuccess)
        return fail(BOA_E_OOM, "fp8 weights");
    for (int l = 0; l < L.L; ++l) {
        const LayerOff& o = L.layer[l];
        LayerDev w;
        w.norm_w = m->d_w + o.norm_w; w.norm_b = m->d_w + o.norm_b;
        w.in_w = m->d_w + o.in_w;
        float* der = m->d_derived + per_layer_derived * l;
        w.convT = der; w.dtwT = der + (size_t)L.K * L.Di; w.A2T = der + (size_t)(L.K + L.R) * L.Di;
        w.xw_r = der + (size_t)(L.K + L.R + L.N) * L.Di;
        w.dtwT_r = w.xw_r + NOx * L.Di;
        w.dtw16 = reinterpret_cast<const uint16_t*>(w.dtwT_r + (size_t)L.R * L.Di);
        w.xwF = der + der_base;
        w.xwF_r = w.xwF + NOp * L.Di;
        w.conv_b = m->d_w + o.conv_b; w.xw = m->d_w + o.xw; w.dtb = m->d_w + o.dtb;
        w.Dsk = m->d_w + o.Dsk; w.out_w = m->d_w + o.out_w;
        uint16_t* w16 = m->d_w16 + per_layer16 * l;
        w.in_w16 = w16; w.out_w16 = w16 + (size_t)2 * L.Di * L.D;
        w.in_f32f = m->d_frag32 + per_layer16 * l;
        w.out_f32f = w.in_f32f + (size_t)2 * L.Di * L.D;
        w.in_b16f = m->d_frag16 + per_layer16 * l;
        w.out_b16f = w.in_b16f + (size_t)2 * L.Di * L.D;
        w.in_f8f = m->d_frag8 + per_layer16 * l;
        w.out_f8f = w.in_f8f + (size_t)2 * L.Di * L.D;
        w.in_ew = m->d_ew + mpl * l;
        w.out_ew = m->d_ew + mpl * l + 1;
        w.w1 = w.b1 = w.w2 = w.b2 = w.fnw = w.fnb = nullptr;
        w.w1_16 = w.w2_16 = nullptr;
        w.w1_f32f = w.w2_f32f = nullptr;
        w.w1_b16f = w.w2_b16f = nullptr;
        w.w1_f8f = w.w2_f8f = nullptr;
        w.w1_ew = w.w2_ew = nullptr;
        if (L.H) {
            const size_t base = (size_t)2 * L.Di * L.D + (size_t)L.D * L.Di, hd = (size_t)L.H * L.D;
            w.w1 = m->d_w + o.ffn_w1; w.b1 = m->d_w + o.ffn_b1; w.w2 = m->d_w + o.ffn_w2; w.b2 = m->d_w + o.ffn_b2;
            w.fnw = m->d_w + o.ffn_nw; w.fnb = m->d_w + o.ffn_nb;
            w.w1_16 = w16 + base; w.w2_16 = w16 + base + hd;
            w.w1_f32f = w.in_f32f + base; w.w2_f32f = w.in_f32f + base + hd;
            w.w1_b16f = w.in_b16f + base; w.w2_b16f = w.in_b16f + base + hd;
            w.w1_f8f = w.in_f8f + base; w.w2_f8f = w.in_f8f + base + hd;
            w.w1_ew = m->d_ew + mpl * l + 2; w.w2_ew = m->d_ew + mpl * l + 3;
        }
        m->ld.push_back(w);
    }
    m->head_w16 = m->d_w16 + per_layer16 * L.L;
    m->head_f32f = m->d_frag32 + per_layer16 * L.L;
    m->head_b16f = m->d_frag16 + per_layer16 * L.L;
    m->head_f8f = m->d_frag8 + per_layer16 * L.L;
    m->head_ew = m->d_ew + mpl * L.L;
    int rc = refresh_derived(m.get(), h_weights);
    if (rc) return rc;
    *out = m.release();
    return BOA_OK;
}

extern "C" void boa_model_free(boa_model* m) { model_release(m); }

extern "C" int boa_model_get_weights(const boa_model* m, float* h_out, uint64_t n) {
    if (!m || !h_out || n != m->lay.total) return fail(BOA_E_ARG, "bad argument");
    HIPCHK(hipSetDevice(m->device));
    HIPCHK(hipMemcpy(h_out, m->d_w, n * sizeof(float), hipMemcpyDeviceToHost));
    return BOA_OK;
}

extern "C" int boa_model_set_weights(boa_model* m, const float* h_w, uint64_t n) {
    if (!m || !h_w || n != m->lay.total) return fail(BOA_E_ARG, "bad argument");
    return refresh_derived(m, h_w);
}

extern "C" int boa_model_config(const boa_model* m, boa_config* out) {
    if (!m || !out) return fail(BOA_E_ARG, "null argument");
    *out = m->cfg;
    return BOA_OK;
}

extern "C" int boa_model_fingerprint(const boa_model* m, uint64_t* out) {
    if (!m || !out) return fail(BOA_E_ARG, "null argument");
    *out = model_fingerprint(m);
    return BOA_OK;
}

extern "C" int boa_model_save(const boa_model* m, const char* path) {
    if (!m || !path) return fail(BOA_E_ARG, "null argument");
    std::vector<float> w(m->lay.total);
    int rc = boa_model_get_weights(m, w.data(), w.size());
    if (rc) return rc;
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(BOA_E_ARG, std::string("cannot open ") + path);
    const uint32_t ver = 2;
    uint64_t fp = fnv1a(&m->cfg, sizeof(boa_config));
    fp = fnv1a(w.data(), w.size() * sizeof(float), fp);
    bool ok = std::fwrite("BOAM", 1, 4, f) == 4 && std::fwrite(&ver, 4, 1, f) == 1 &&
              std::fwrite(&m->cfg, sizeof(boa_config), 1, f) == 1 &&
              std::fwrite(w.data(), sizeof(float), w.size(), f) == w.size() &&
              std::fwrite(&fp, 8, 1, f) == 1;
    std::fclose(f);
    return ok ? BOA_OK : fail(BOA_E_ARG, "short write");
}

extern "C" int boa_model_load(const char* path, int device, boa_model** out) {
    if (!path || !out) return fail(BOA_E_ARG, "null argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(BOA_E_ARG, std::string("cannot open ") + path);
    char mg[4];
    uint32_t ver = 0;
    boa_config cfg{};
    // version 1 files carry the first five config fields (no feed-forward sub-layer)
    bool ok = std::fread(mg, 1, 4, f) == 4 && std::memcmp(mg, "BOAM", 4) == 0 && std::fread(&ver, 4, 1, f) == 1 &&
              (ver == 1 || ver == 2) && std::fread(&cfg, ver == 1 ? 20 : sizeof(cfg), 1, f) == 1;
    Layout L;
    if (!ok || !make_layout(cfg, &L)) { std::fclose(f); return fail(BOA_E_FORMAT, "not a BOAM v1/v2 model file"); }
    std::vector<float> w(L.total);
    uint64_t fp = 0;
    ok = std::fread(w.data(), sizeof(float), w.size(), f) == w.size() && std::fread(&fp, 8, 1, f) == 1;
    std::fclose(f);
    if (!ok) return fail(BOA_E_FORMAT, "truncated model file");
    uint64_t chk = fnv1a(w.data(), w.size() * sizeof(float), fnv1a(&cfg, ver == 1 ? 20 : sizeof(cfg)));
    if (chk != fp) return fail(BOA_E_CORRUPT, "model file fingerprint mismatch");
    return boa_model_create(&cfg, w.data(), w.size(), device, out);
}

// the integer pipeline's tables depend only on its own rules, not on the
// device or on the float kernels' version
constexpr uint32_t INT_PIPELINE_VERSION = 0x101;
extern "C" uint32_t boa_numerics_id(uint32_t dtype) {
    return dtype == BOA_DTYPE_INT8 ? (INT_PIPELINE_VERSION << 8) | BOA_DTYPE_INT8 : (KERNEL_VERSION << 8) | (dtype & 0xFF);
}

// the error of a call made on this thread, for host code in other files
namespace boa {
int report_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace boa

extern "C" void boa_free(void* p) { std::free(p); }
extern "C" const char* boa_last_error(void) { return g_err.c_str(); }

// =================================================================== kernel timing
namespace {
struct Prof {
    uint32_t mask = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[BOA_K_COUNT];
    double ms[BOA_K_COUNT] = {};
    uint64_t n[BOA_K_COUNT] = {};
} g_prof;
std::mutex g_prof_mu;

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st == hipStreamCaptureStatusActive;
}
// RAII bracket: records start on construction, stop on destruction
struct ProfScope {
    int k = -1;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(int kind, hipStream_t st) {
        if (!(g_prof.mask & (1u << kind)) || capturing(st)) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
        k = kind;
        s = st;
        prof_open(a, b);
    }
    ~ProfScope() {
        if (k < 0) return;
        prof_close();
        std::lock_guard<std::mutex> g(g_prof_mu);
        g_prof.ev[k].push_back({a, b});
    }
};
}  // namespace

extern "C" int boa_prof_enable(uint32_t mask) {
    g_prof.mask = mask;
    return BOA_OK;
}

extern "C" int boa_prof_read(double* h_total_ms, uint64_t* h_launches, int reset) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (int k = 0; k < BOA_K_COUNT; ++k) {
        for (auto& e : g_prof.ev[k]) {
            float ms = 0.f;
            if (hipEventSynchronize(e.second) == hipSuccess && hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
                g_prof.ms[k] += ms;
                g_prof.n[k] += 1;
            }
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        g_prof.ev[k].clear();
        if (h_total_ms) h_total_ms[k] = g_prof.ms[k];
        if (h_launches) h_launches[k] = g_prof.n[k];
        if (reset) { g_prof.ms[k] = 0; g_prof.n[k] = 0; }
    }
    return BOA_OK;
}

// =================================================================== lane plan
namespace {
struct HostPlan {
    int lanes = 0;
    long long total_steps = 0;
    std::vector<int> lane_first, lane_cnt, ent_chunk;
    std::vector<long long> ent_start;
};

// Longest-processing-time-first assignment of chunks (steps = len - 1) to
// lanes; each lane runs its chunks back to back (Coders & Parallelisation:
// finished streams are masked, free lanes take the next chunk).
HostPlan build_plan(const std::vector<long long>& steps, int max_lanes) {
    HostPlan P;
    std::vector<int> idx;
    for (size_t i = 0; i < steps.size(); ++i)
        if (steps[i] > 0) idx.push_back((int)i);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return steps[a] > steps[b]; });
    int lanes = (int)std::min<size_t>(idx.size(), (size_t)std::max(1, max_lanes));
    P.lanes = lanes;
    if (lanes == 0) return P;
    std::vector<std::vector<std::pair<int, long long>>> per(lanes);
    using Item = std::pair<long long, int>;   // (load, lane)
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> pq;
    for (int l = 0; l < lanes; ++l) pq.push({0, l});
    for (int c : idx) {
        Item it = pq.top();
        pq.pop();
        per[it.second].push_back({c, it.first});
        it.first += steps[c];
        P.total_steps = std::max(P.total_steps, it.first);
        pq.push(it);
    }
    for (int l = 0; l < lanes; ++l) {
        P.lane_first.push_back((int)P.ent_chunk.size());
        P.lane_cnt.push_back((int)per[l].size());
        for (auto& e : per[l]) { P.ent_chunk.push_back(e.first); P.ent_start.push_back(e.second); }
    }
    return P;
}

// Lane count when the caller leaves it open: the most lanes (at most cap)
// whose schedule keeps idle rows within 5 % of the rows the lanes occupy.  A
// row is idle when its lane has run out of chunks while others still run; the
// encoder's row kernels compute every row of a tile, so with one chunk per
// lane and uneven lengths (uniform in [32, 256] KiB) 44 % of the rows were
// idle.  Fewer lanes let the LPT schedule pack several chunks per lane to
// about the same total.  Candidates, largest first: min(chunks, cap) halved
// down to 256, and ceil(chunks / k) for k = 2 .. 16 (equal lengths pack
// exactly there).  Failing 5 %, the candidate with the fewest idle rows.
int auto_lanes(const std::vector<long long>& steps, int cap) {
    long long sum = 0, n = 0;
    for (long long v : steps)
        if (v > 0) { sum += v; ++n; }
    if (n == 0) return 1;
    const int top = (int)std::min<long long>(n, cap);
    std::vector<int> cand;
    for (int L = top;; L /= 2) {
        cand.push_back(L);
        if (L <= 256) break;
    }
    for (long long k = 2; k <= 16; ++k) {
        const long long L = (n + k - 1) / k;
        if (L >= 1 && L < top) cand.push_back((int)L);
    }
    std::sort(cand.begin(), cand.end(), std::greater<int>());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    int best = top;
    double best_idle = 2.0;
    for (int L : cand) {
        const HostPlan P = build_plan(steps, L);
        const double idle = 1.0 - (double)sum / ((double)P.lanes * (double)P.total_steps);
        if (idle <= 0.05) return P.lanes;
        if (idle < best_idle) { best_idle = idle; best = P.lanes; }
    }
    return best;
}
int plan_lanes(const boa_run_opts& o, const std::vector<long long>& steps) {
    return o.max_lanes ? (int)o.max_lanes : auto_lanes(steps, 8192);
}

struct PlanDev {
    DevBuf lane_first, lane_cnt, ent_chunk, ent_start, chunk_off, chunk_steps;
    Plan view() const {
        Plan p;
        p.lane_first = lane_first.as<int>();
        p.lane_cnt = lane_cnt.as<int>();
        p.ent_chunk = ent_chunk.as<int>();
        p.ent_start = ent_start.as<long long>();
        p.chunk_off = chunk_off.as<long long>();
        p.chunk_steps = chunk_steps.as<long long>();
        return p;
    }
};

void carve_plan(Arena& A, const HostPlan& P, size_t n_chunks, PlanDev& D) {
    D.lane_first.carve(A, P.lane_first.size() * sizeof(int));
    D.lane_cnt.carve(A, P.lane_cnt.size() * sizeof(int));
    D.ent_chunk.carve(A, P.ent_chunk.size() * sizeof(int));
    D.ent_start.carve(A, P.ent_start.size() * sizeof(long long));
    D.chunk_off.carve(A, n_chunks * sizeof(long long));
    D.chunk_steps.carve(A, n_chunks * sizeof(long long));
}
// copies into carved buffers; the caller synchronises before the host vectors go away
int fill_plan(const HostPlan& P, const std::vector<long long>& off, const std::vector<long long>& steps, PlanDev& D,
              hipStream_t s) {
    HIPCHK(copy_in(D.lane_first, P.lane_first, s));
    HIPCHK(copy_in(D.lane_cnt, P.lane_cnt, s));
    HIPCHK(copy_in(D.ent_chunk, P.ent_chunk, s));
    HIPCHK(copy_in(D.ent_start, P.ent_start, s));
    HIPCHK(copy_in(D.chunk_off, off, s));
    HIPCHK(copy_in(D.chunk_steps, steps, s));
    return BOA_OK;
}

int upload_plan(const HostPlan& P, const std::vector<long long>& off, const std::vector<long long>& steps,
                PlanDev& D, hipStream_t s) {
    HIPCHK(upload(D.lane_first, P.lane_first, s));
    HIPCHK(upload(D.lane_cnt, P.lane_cnt, s));
    HIPCHK(upload(D.ent_chunk, P.ent_chunk, s));
    HIPCHK(upload(D.ent_start, P.ent_start, s));
    HIPCHK(upload(D.chunk_off, off, s));
    HIPCHK(upload(D.chunk_steps, steps, s));
    return BOA_OK;
}

// Per-call activation and state buffers for `lanes` lanes and tiles of T rows.
struct Work {
    DevBuf r, xz, g, logits, cf, row_chunk, row_pos, conv, h, coder, step, xs, dbc, dt;
    DevBuf fh, ff;     // feed-forward hidden [M, H] and output [M, D]
    int lanes = 0, T = 0;
    Arena own_arena;
    DevBuf own_mem;
    // every buffer as a piece of A
    void carve(Arena& A, const boa_model* m, int lanes_, int T_) {
        lanes = lanes_;
        T = T_;
        const Layout& L = m->lay;
        size_t M = (size_t)lanes * T;
        r.carve(A, M * L.D * 4);
        xz.carve(A, M * 2 * L.Di * 4);
        g.carve(A, M * L.Di * 4);
        if (T > 1 && L.Di > 512) {             // the two-kernel mixer's intermediates
            xs.carve(A, M * L.Di * 4);
            dbc.carve(A, M * (L.R + 2 * L.N) * 4);
        }
        logits.carve(A, M * 256 * 4);
        cf.carve(A, M * 2 * 4);
        row_chunk.carve(A, M * 4);
        row_pos.carve(A, M * 4);
        conv.carve(A, (size_t)L.L * lanes * (L.K - 1) * L.Di * 4);
        h.carve(A, (size_t)L.L * lanes * L.N * L.Di * 4);
        coder.carve(A, (size_t)lanes * 8 * 4);
        step.carve(A, 8);
        if (L.H) {
            fh.carve(A, M * L.H * 4);
            ff.carve(A, M * L.D * 4);
        }
    }
    // every buffer in one allocation owned by this Work
    int alloc(const boa_model* m, int lanes_, int T_) {
        Arena meas;
        carve(meas, m, lanes_, T_);
        ALLOC(own_mem, meas.used);
        own_arena = Arena{own_mem.as<uint8_t>(), meas.used, 0, false};
        carve(own_arena, m, lanes_, T_);
        return BOA_OK;
    }
};

int mid_lanes_per_wg(int lanes, int T) {
    if (T > 1) return 1;
    // decoder step: amortise the per-launch weight loads over a few lanes
    // while keeping at least ~256 workgroups in flight
    int g = lanes / 256;
    return std::max(1, std::min(g, 8));
}

// One model pass over a tile of rows already located by rowinfo.
// Locates the tile's rows (step0 + t, plus *d_step when given) and runs the
// model over them.
int forward_tile(const boa_model* m, Work& W, int dtype, const uint8_t* bytes, const Plan& p, long long step0,
                 const long long* d_step, hipStream_t s, bool embed = true) {
    const Layout& L = m->lay;
    const int M = W.lanes * W.T;
    float* r = W.r.as<float>();
    if (embed) {
        ProfScope ps(BOA_K_EMBED, s);
        HIPCHK(launch_embed(m->d_w + L.embed, bytes, p, W.lanes, W.T, step0, d_step, L.D, W.row_chunk.as<int>(),
                            W.row_pos.as<int>(), r, s));
    }
    const int lpw = mid_lanes_per_wg(W.lanes, W.T);
    // many rows: row-block GEMMs on the fragment-ordered weights; few rows
    // (decoder steps): column-tiled GEMMs with the whole K in one tile
    // (fp8 runs on the row-block GEMM at every row count)
    const bool rows_big = M > 2048 || dtype == BOA_DTYPE_FP8;
    auto frag = [&](const float* f32, const uint16_t* h16, const uint8_t* f8) {
        return dtype == BOA_DTYPE_FP8 ? (const void*)f8 : dtype == BOA_DTYPE_BF16 ? (const void*)h16 : (const void*)f32;
    };
    // BF16 encoder tiles: the one-pass mixer writes the gated rows as the bf16
    // bits the out_proj stages anyway (half the bytes both ways)
    const bool g16 = dtype == BOA_DTYPE_BF16 && rows_big && W.T > 1 && L.Di <= 512;
    for (int l = 0; l < L.L; ++l) {
        const LayerDev& w = m->ld[l];
        // the mixer reads the x_proj / dt_proj weights of the dtype's numerics
        LayerDev wm = w;
        if (dtype == BOA_DTYPE_BF16) { wm.xw = w.xw_r; wm.dtwT = w.dtwT_r; wm.xwF = w.xwF_r; }
        {
            ProfScope ps(BOA_K_INPROJ, s);
            if (rows_big)
                HIPCHK(launch_rowgemm(dtype, 0, r, M, L.D, frag(w.in_f32f, w.in_b16f, w.in_f8f), 2 * L.Di,
                                      W.xz.as<float>(), w.norm_w, w.norm_b, nullptr, w.in_ew, s));
            else
                HIPCHK(launch_mgemm(dtype, 0, r, M, L.D, w.in_w, w.in_w16, 2 * L.Di, W.xz.as<float>(), w.norm_w,
                                    w.norm_b, nullptr, s));
        }
        float* conv = W.conv.as<float>() + (size_t)l * W.lanes * (L.K - 1) * L.Di;
        float* h = W.h.as<float>() + (size_t)l * W.lanes * L.N * L.Di;
        {
            ProfScope ps(BOA_K_MIXER, s);
            if (W.T > 1)
                HIPCHK(launch_mid_tiled(wm, L.Di, L.R, W.xz.as<float>(), W.xs.as<float>(), W.dbc.as<float>(),
                                        W.dt.as<float>(), W.g.as<float>(), W.lanes, W.T, W.row_pos.as<int>(), conv,
                                        h, g16, s));
            else
                HIPCHK(launch_mid(wm, L.Di, L.R, W.xz.as<float>(), W.g.as<float>(), W.lanes, W.T, lpw,
                                  W.row_pos.as<int>(), conv, h, s));
        }
        {
            ProfScope ps(BOA_K_OUTPROJ, s);
            if (rows_big)
                HIPCHK(launch_rowgemm(dtype, g16 ? 5 : 2, W.g.as<float>(), M, L.Di,
                                      frag(w.out_f32f, w.out_b16f, w.out_f8f), L.D, r, nullptr, nullptr, nullptr,
                                      w.out_ew, s));
            else
                HIPCHK(launch_mgemm(dtype, 2, W.g.as<float>(), M, L.Di, w.out_w, w.out_w16, L.D, r, nullptr,
                                    nullptr, nullptr, s));
        }
        if (L.H) {
            // Algorithm 1's sub-layer: r <- LayerNorm(W2 GELU(W1 r + b1) + b2)
            ProfScope ps(BOA_K_FFN, s);
            float* fh = W.fh.as<float>();
            float* ff = W.ff.as<float>();
            if (rows_big) {
                HIPCHK(launch_rowgemm(dtype, 3, r, M, L.D, frag(w.w1_f32f, w.w1_b16f, w.w1_f8f), L.H, fh, nullptr,
                                      nullptr, w.b1, w.w1_ew, s));
                HIPCHK(launch_rowgemm(dtype, 4, fh, M, L.H, frag(w.w2_f32f, w.w2_b16f, w.w2_f8f), L.D, ff, nullptr,
                                      nullptr, w.b2, w.w2_ew, s));
            } else {
                HIPCHK(launch_mgemm(dtype, 3, r, M, L.D, w.w1, w.w1_16, L.H, fh, nullptr, nullptr, w.b1, s));
                HIPCHK(launch_mgemm(dtype, 4, fh, M, L.H, w.w2, w.w2_16, L.D, ff, nullptr, nullptr, w.b2, s));
            }
            HIPCHK(launch_ln_rows(ff, M, L.D, w.fnw, w.fnb, r, s));
        }
    }
    {
        ProfScope ps(BOA_K_HEAD, s);
        if (rows_big)
            HIPCHK(launch_rowgemm(dtype, 1, r, M, L.D, frag(m->head_f32f, m->head_b16f, m->head_f8f), 256,
                                  W.logits.as<float>(), m->d_w + L.norm_f_w, m->d_w + L.norm_f_b, m->d_w + L.head_b,
                                  m->head_ew, s));
        else
            HIPCHK(launch_mgemm(dtype, 1, r, M, L.D, m->d_w + L.head_w, m->head_w16, 256, W.logits.as<float>(),
                                m->d_w + L.norm_f_w, m->d_w + L.norm_f_b, m->d_w + L.head_b, s));
    }
    return BOA_OK;
}

int pick_tile(int lanes, long long total_steps, uint32_t req) {
    long long T = req ? (long long)req : std::max<long long>(1, (1LL << 17) / std::max(1, lanes));
    T = std::min<long long>(T, std::max<long long>(1, total_steps));
    T = std::min<long long>(T, 4096);
    return (int)T;
}

bool dtype_ok(uint32_t d) { return d == BOA_DTYPE_F32 || d == BOA_DTYPE_BF16 || d == BOA_DTYPE_FP8; }

// Chunk lengths index int step counters on the device; total lengths and
// offsets stay far inside int64.
bool lens_ok(const uint64_t* len, uint64_t n) {
    uint64_t tot = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (len[i] > MAX_CHUNK) return false;
        tot += len[i];
        if (tot > MAX_TOTAL) return false;
    }
    return true;
}
}  // namespace

// =================================================================== encode
namespace {
// Device buffers of one encode call (all carved from one arena).
struct EncBufs {
    PlanDev PD;
    DevBuf d_poff, d_pcap;
    Work W;
    DevBuf cfb[2], rcb[2], rpb[2];
    void carve(Arena& A, const boa_model* m, const HostPlan& P, size_t n_chunks, int T) {
        carve_plan(A, P, n_chunks, PD);
        d_poff.carve(A, n_chunks * sizeof(long long));
        d_pcap.carve(A, n_chunks * sizeof(long long));
        W.carve(A, m, P.lanes, T);
        const size_t M = (size_t)P.lanes * T;
        for (int b = 0; b < 2; ++b) {
            cfb[b].carve(A, M * 2 * 4);
            rcb[b].carve(A, M * 4);
            rpb[b].carve(A, M * 4);
        }
    }
};

std::vector<long long> chunk_steps(const uint64_t* h_chunk_len, uint64_t n) {
    std::vector<long long> steps(n);
    for (uint64_t i = 0; i < n; ++i) steps[i] = h_chunk_len[i] > 1 ? (long long)h_chunk_len[i] - 1 : 0;
    return steps;
}

// Workspace bytes of an encode call (0 when no chunk has a coded byte).
size_t encode_ws_bytes(const boa_model* m, const std::vector<long long>& steps, const boa_run_opts& o) {
    HostPlan P = build_plan(steps, plan_lanes(o, steps));
    if (P.lanes == 0) return 0;
    const int T = pick_tile(P.lanes, P.total_steps, o.tile_t);
    Arena meas;
    EncBufs B;
    B.carve(meas, m, P, steps.size(), T);
    return meas.used;
}
}  // namespace

extern "C" int boa_encode_dev(const boa_model* m, const uint8_t* d_data, const uint64_t* h_chunk_off,
                              const uint64_t* h_chunk_len, uint64_t n_chunks, const boa_run_opts* opts,
                              uint8_t* d_payload, const uint64_t* h_pay_off, const uint64_t* h_pay_cap,
                              uint32_t* d_pay_len, double* d_ideal_bits, void* d_ws, uint64_t ws_bytes,
                              void* stream) {
    if (!m || (!d_data && n_chunks) || (n_chunks && (!h_chunk_off || !h_chunk_len || !d_payload || !h_pay_off ||
                                                     !h_pay_cap || !d_pay_len)))
        return fail(BOA_E_ARG, "null argument");
    boa_run_opts o{};
    if (opts) o = *opts;
    if (!dtype_ok(o.dtype)) return fail(BOA_E_UNSUPPORTED, "dtype not supported by this library");
    if (n_chunks == 0) return BOA_OK;
    if (n_chunks > (1u << 30)) return fail(BOA_E_ARG, "too many chunks");
    if (!lens_ok(h_chunk_len, n_chunks)) return fail(BOA_E_ARG, "chunk length beyond 2^31 - 1 bytes or total beyond 2^48");
    hipStream_t s = as_stream(stream);
    HIPCHK(hipSetDevice(m->device));
    std::vector<long long> off(n_chunks), steps = chunk_steps(h_chunk_len, n_chunks), poff(n_chunks),
        pcap(n_chunks);
    for (uint64_t i = 0; i < n_chunks; ++i) {
        off[i] = (long long)h_chunk_off[i];
        poff[i] = (long long)h_pay_off[i];
        pcap[i] = (long long)std::min<uint64_t>(h_pay_cap[i], 0xFFFFFFF0ULL);
    }
    HIPCHK(hipMemsetAsync(d_pay_len, 0, n_chunks * 4, s));
    if (d_ideal_bits) HIPCHK(hipMemsetAsync(d_ideal_bits, 0, n_chunks * 8, s));
    HostPlan P = build_plan(steps, plan_lanes(o, steps));
    if (P.lanes == 0) { HIPCHK(hipStreamSynchronize(s)); return BOA_OK; }
    const int T = pick_tile(P.lanes, P.total_steps, o.tile_t);
    // device memory: the caller's workspace, else one allocation of the measured size
    EncBufs B;
    Arena meas;
    B.carve(meas, m, P, n_chunks, T);
    DevBuf own;
    Arena A;
    if (d_ws) {
        if (ws_bytes < meas.used)
            return fail(BOA_E_ARG, "workspace of " + std::to_string(ws_bytes) + " bytes, this call needs " +
                                       std::to_string(meas.used) + " (boa_workspace_size)");
        A = Arena{static_cast<uint8_t*>(d_ws), (size_t)ws_bytes, 0, false};
    } else {
        ALLOC(own, meas.used);
        A = Arena{own.as<uint8_t>(), meas.used, 0, false};
    }
    B.carve(A, m, P, n_chunks, T);
    int rc = fill_plan(P, off, steps, B.PD, s);
    if (rc) return rc;
    HIPCHK(copy_in(B.d_poff, poff, s));
    HIPCHK(copy_in(B.d_pcap, pcap, s));
    HIPCHK(hipStreamSynchronize(s));          // host vectors of the copies may go away on an error return
    Work& W = B.W;
    const Plan p = B.PD.view();
    const int M = P.lanes * T;
    // The range coder of tile k (one thread per lane, a few waves) runs on a
    // second stream while the model runs tile k + 1; its inputs -- the tile's
    // (C(s), f(s)) pairs and row schedule -- are double-buffered, and tile
    // k + 2 waits for the coder of tile k before reusing its buffers.
    hipStream_t s2;
    HIPCHK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    struct Side {
        hipStream_t s = nullptr;
        hipEvent_t ev[5] = {};
        ~Side() {
            for (hipEvent_t e : ev)
                if (e) (void)hipEventDestroy(e);
            if (s) (void)hipStreamDestroy(s);
        }
    } side;
    side.s = s2;
    for (hipEvent_t& e : side.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipEvent_t* ready = side.ev;          // [2] tile's coder inputs written (on s)
    hipEvent_t* coded = side.ev + 2;      // [2] tile's coder finished (on s2)
    long long k = 0;
    for (long long s0 = 0; s0 < P.total_steps; s0 += T, ++k) {
        const int b = (int)(k & 1);
        rc = forward_tile(m, W, (int)o.dtype, d_data, p, s0, nullptr, s);
        if (rc) return rc;
        if (k >= 2) HIPCHK(hipStreamWaitEvent(s, coded[b], 0));
        {
            ProfScope ps(BOA_K_QUANT, s);
            HIPCHK(launch_quant_sym(W.logits.as<float>(), M, d_data, p, W.row_chunk.as<int>(),
                                    W.row_pos.as<int>(), B.cfb[b].as<uint32_t>(), nullptr, nullptr, s));
        }
        HIPCHK(hipMemcpyAsync(B.rcb[b].p, W.row_chunk.p, (size_t)M * 4, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(B.rpb[b].p, W.row_pos.p, (size_t)M * 4, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipEventRecord(ready[b], s));
        HIPCHK(hipStreamWaitEvent(s2, ready[b], 0));
        {
            ProfScope ps(BOA_K_ENCODE, s2);
            HIPCHK(launch_encode(B.cfb[b].as<uint32_t>(), P.lanes, T, B.rcb[b].as<int>(), B.rpb[b].as<int>(), p,
                                 W.coder.as<uint32_t>(), d_payload, B.d_poff.as<long long>(),
                                 B.d_pcap.as<long long>(), d_pay_len, d_ideal_bits, s2));
        }
        HIPCHK(hipEventRecord(coded[b], s2));
    }
    HIPCHK(hipEventRecord(side.ev[4], s2));
    HIPCHK(hipStreamWaitEvent(s, side.ev[4], 0));
    HIPCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

// =================================================================== decode
namespace {
// Lanes per workgroup of the fused decoder: the largest of 16, 8, 4, 2 that
// fits LDS and still leaves at least 256 workgroups (one per CU), else 1.
int pick_fused_lanes(int D, int lanes, int n_layers) {
    for (int g : {16, 8, 4, 2})
        if (g * D <= 16 * 256 && fused_lds_bytes(D, g, n_layers, false) + 2048 <= get_max_lds() && lanes / g >= 256)
            return g;
    return 1;
}

// Schedule and launch shape of the fused decoder for these chunks.
struct FusedShape {
    HostPlan P;
    int G = 1;
    bool state_lds = false;
};
int fused_shape(const boa_model* m, const boa_run_opts& o, const std::vector<long long>& steps, FusedShape& F) {
    const Layout& L = m->lay;
    if (L.H) return fail(BOA_E_UNSUPPORTED, "the fused decoder has no feed-forward sub-layer: use the per-step decoder");
    F.P = build_plan(steps, plan_lanes(o, steps));
    if (F.P.lanes == 0) return BOA_OK;
    if (L.L > MAX_LAYERS) return fail(BOA_E_UNSUPPORTED, "too many layers for the fused decoder");
    int G = (int)o.fused_lanes;
    if (G == 0) G = pick_fused_lanes(L.D, F.P.lanes, L.L);
    if (G != 1 && G != 2 && G != 4 && G != 8 && G != 16)
        return fail(BOA_E_ARG, "fused_lanes must be 1, 2, 4, 8 or 16");
    if (G * L.D > 16 * 256) return fail(BOA_E_ARG, "fused_lanes x d_model exceeds 16 x 256");
    if (fused_lds_bytes(L.D, G, L.L, false) + 2048 > get_max_lds())
        return fail(BOA_E_ARG, "fused_lanes needs more LDS than the device has");
    F.G = G;
    // one lane per workgroup: keep its conv and scan state in LDS when it fits
    F.state_lds = G == 1 && fused_lds_bytes(L.D, 1, L.L, true) + 2048 <= get_max_lds();
    return BOA_OK;
}

// Device buffers of one fused decode call (all carved from one arena): the
// per-chunk arrays, the lane schedule, and the conv and scan state of every
// lane when it does not stay in LDS.
struct DecBufs {
    DevBuf d_first, d_off, d_len, d_poff, d_plen;
    PlanDev PD;
    DevBuf conv, h;
    void carve(Arena& A, const boa_model* m, const FusedShape& F, size_t n) {
        const Layout& L = m->lay;
        d_first.carve(A, n);
        d_off.carve(A, n * sizeof(long long));
        d_len.carve(A, n * sizeof(long long));
        d_poff.carve(A, n * sizeof(long long));
        d_plen.carve(A, n * sizeof(long long));
        carve_plan(A, F.P, n, PD);
        const size_t sl = F.state_lds ? 0 : (size_t)F.P.lanes;
        // per (layer, lane): conv window [K-1][Di], h [N/4][Di] float4
        conv.carve(A, (size_t)L.L * sl * (L.K - 1) * L.Di * sizeof(float));
        h.carve(A, (size_t)L.L * sl * L.N * L.Di * sizeof(float));
    }
};

// Host copies of a decode call's per-chunk arguments.
struct DecHost {
    std::vector<long long> off, len, steps, poff, plen;
    std::vector<uint8_t> first;
    DecHost(const uint64_t* h_pay_off, const uint64_t* h_pay_len, const uint8_t* h_first, const uint64_t* h_chunk_off,
            const uint64_t* h_chunk_len, uint64_t n)
        : off(n), len(n), steps(n), poff(n), plen(n), first(h_first, h_first + n) {
        for (uint64_t i = 0; i < n; ++i) {
            off[i] = (long long)h_chunk_off[i];
            len[i] = (long long)h_chunk_len[i];
            steps[i] = h_chunk_len[i] > 1 ? (long long)h_chunk_len[i] - 1 : 0;
            poff[i] = (long long)h_pay_off[i];
            plen[i] = (long long)std::min<uint64_t>(h_pay_len[i], 0xFFFFFFF0ULL);
        }
    }
};

size_t decode_ws_bytes(const boa_model* m, const boa_run_opts& o, const std::vector<long long>& steps) {
    FusedShape F;
    if (fused_shape(m, o, steps, F)) return 0;
    Arena meas;
    DecBufs B;
    B.carve(meas, m, F, steps.size());
    return meas.used;
}

// The whole decode in one persistent launch (ceil(lanes / G) workgroups),
// its device memory carved from ws (ws_bytes) or, when ws is null and
// allow_alloc, from one allocation.
int decode_fused(const boa_model* m, const boa_run_opts& o, const DecHost& H, const uint8_t* d_payload,
                 uint8_t* d_out, void* ws, size_t ws_bytes, bool allow_alloc, hipStream_t s) {
    const Layout& L = m->lay;
    const size_t n = H.off.size();
    FusedShape F;
    int rc = fused_shape(m, o, H.steps, F);
    if (rc) return rc;
    DecBufs B;
    Arena meas;
    B.carve(meas, m, F, n);
    DevBuf own;
    Arena A;
    if (ws) {
        if (ws_bytes < meas.used)
            return fail(BOA_E_ARG, "workspace of " + std::to_string(ws_bytes) + " bytes, this call needs " +
                                       std::to_string(meas.used) + " (boa_workspace_size)");
        A = Arena{static_cast<uint8_t*>(ws), ws_bytes, 0, false};
    } else {
        if (!allow_alloc) return fail(BOA_E_ARG, "no workspace");
        ALLOC(own, meas.used);
        A = Arena{own.as<uint8_t>(), meas.used, 0, false};
    }
    B.carve(A, m, F, n);
    HIPCHK(copy_in(B.d_first, H.first, s));
    HIPCHK(copy_in(B.d_off, H.off, s));
    HIPCHK(copy_in(B.d_len, H.len, s));
    HIPCHK(copy_in(B.d_poff, H.poff, s));
    HIPCHK(copy_in(B.d_plen, H.plen, s));
    rc = fill_plan(F.P, H.off, H.steps, B.PD, s);
    if (rc) return rc;
    HIPCHK(launch_prefill(B.d_first.as<uint8_t>(), B.d_off.as<long long>(), B.d_len.as<long long>(), (int)n, d_out,
                          s));
    if (F.P.lanes == 0) { HIPCHK(hipStreamSynchronize(s)); return BOA_OK; }
    const bool b16 = o.dtype == BOA_DTYPE_BF16, f8 = o.dtype == BOA_DTYPE_FP8;
    auto pick = [&](const float* f32p, const uint16_t* b16p, const uint8_t* f8p) {
        return f8 ? (const void*)f8p : b16 ? (const void*)b16p : (const void*)f32p;
    };
    FusedArgs a{};
    for (int l = 0; l < L.L; ++l) {
        const LayerDev& w = m->ld[l];
        FusedLayer& f = a.layers[l];
        f.norm_w = w.norm_w; f.norm_b = w.norm_b;
        f.in_frag = pick(w.in_f32f, w.in_b16f, w.in_f8f);
        f.in_ew = w.in_ew;
        f.out_ew = w.out_ew;
        f.convT = w.convT; f.conv_b = w.conv_b; f.xw = w.xw; f.dtwT = w.dtwT; f.dtb = w.dtb;
        f.A2T = w.A2T; f.Dsk = w.Dsk;
        f.dtw16 = w.dtw16;
        f.xw_frag = o.dtype == BOA_DTYPE_BF16 ? w.xwF_r : w.xwF;
        f.out_frag = pick(w.out_f32f, w.out_b16f, w.out_f8f);
    }
    a.n_layers = L.L;
    a.lanes = F.P.lanes;
    a.max_steps = F.P.total_steps;
    a.E = m->d_w + L.embed;
    a.norm_f_w = m->d_w + L.norm_f_w;
    a.norm_f_b = m->d_w + L.norm_f_b;
    a.head_frag = pick(m->head_f32f, m->head_b16f, m->head_f8f);
    a.head_ew = m->head_ew;
    a.head_b = m->d_w + L.head_b;
    a.p = B.PD.view();
    a.payload = d_payload;
    a.pay_off = B.d_poff.as<long long>();
    a.pay_len = B.d_plen.as<long long>();
    a.out = d_out;
    a.conv_state = B.conv.as<float>();
    a.h_state = B.h.as<float>();
    {
        ProfScope ps(BOA_K_DEC_FUSED, s);
        HIPCHK(launch_dec_fused((int)o.dtype, L.D, F.G, F.state_lds, a, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

// One decoder step: the model over the rows prepared by the previous step
// (or by the initial embedding), then decoding, which prepares the next step.
int enqueue_decode_step(const boa_model* m, Work& W, int dtype, const Plan& p, uint8_t* d_out,
                        const uint8_t* d_payload, const long long* d_poff, const long long* d_plen,
                        hipStream_t s) {
    int rc = forward_tile(m, W, dtype, d_out, p, 0, nullptr, s, false);
    if (rc) return rc;
    ProfScope ps(BOA_K_DECODE, s);
    HIPCHK(launch_decode(W.logits.as<float>(), W.lanes, W.row_chunk.as<int>(), W.row_pos.as<int>(), p,
                         W.coder.as<uint32_t>(), d_payload, d_poff, d_plen, d_out, m->d_w + m->lay.embed,
                         m->lay.D, W.r.as<float>(), s));
    return BOA_OK;
}
}  // namespace

namespace {
int decode_args_ok(const boa_model* m, const uint8_t* d_payload, const uint64_t* h_pay_off, const uint64_t* h_pay_len,
                   const uint8_t* h_first, const uint64_t* h_chunk_off, const uint64_t* h_chunk_len,
                   uint64_t n_chunks, const boa_run_opts& o, const uint8_t* d_out) {
    if (!m || (n_chunks && (!d_payload || !h_pay_off || !h_pay_len || !h_first || !h_chunk_off || !h_chunk_len ||
                            !d_out)))
        return fail(BOA_E_ARG, "null argument");
    if (!dtype_ok(o.dtype)) return fail(BOA_E_UNSUPPORTED, "dtype not supported by this library");
    if (o.decode_kernel > 2) return fail(BOA_E_ARG, "decode_kernel must be 0, 1 or 2");
    if (n_chunks > (1u << 30)) return fail(BOA_E_ARG, "too many chunks");
    if (n_chunks && !lens_ok(h_chunk_len, n_chunks))
        return fail(BOA_E_ARG, "chunk length beyond 2^31 - 1 bytes or total beyond 2^48");
    return BOA_OK;
}
}  // namespace

namespace boa {
// The fused decoder on a caller-provided region only (never allocates).
int decode_into_region(const boa_model* m, const uint8_t* d_payload, const uint64_t* h_pay_off,
                       const uint64_t* h_pay_len, const uint8_t* h_first, const uint64_t* h_chunk_off,
                       const uint64_t* h_chunk_len, uint64_t n_chunks, const boa_run_opts* opts, uint8_t* d_out,
                       void* region, size_t region_bytes, void* stream) {
    boa_run_opts o{};
    if (opts) o = *opts;
    int rc = decode_args_ok(m, d_payload, h_pay_off, h_pay_len, h_first, h_chunk_off, h_chunk_len, n_chunks, o, d_out);
    if (rc) return rc;
    if (o.decode_kernel == 2) return fail(BOA_E_ARG, "the per-step decoder allocates; use the fused decoder");
    if (n_chunks == 0) return BOA_OK;
    if (!region) return fail(BOA_E_ARG, "null region");
    HIPCHK(hipSetDevice(m->device));
    DecHost H(h_pay_off, h_pay_len, h_first, h_chunk_off, h_chunk_len, n_chunks);
    return decode_fused(m, o, H, d_payload, d_out, region, region_bytes, false, as_stream(stream));
}
}  // namespace boa

extern "C" int boa_decode_dev(const boa_model* m, const uint8_t* d_payload, const uint64_t* h_pay_off,
                              const uint64_t* h_pay_len, const uint8_t* h_first, const uint64_t* h_chunk_off,
                              const uint64_t* h_chunk_len, uint64_t n_chunks, const boa_run_opts* opts,
                              uint8_t* d_out, void* d_ws, uint64_t ws_bytes, void* stream) {
    boa_run_opts o{};
    if (opts) o = *opts;
    int rc0 = decode_args_ok(m, d_payload, h_pay_off, h_pay_len, h_first, h_chunk_off, h_chunk_len, n_chunks, o, d_out);
    if (rc0) return rc0;
    if (n_chunks == 0) return BOA_OK;
    if (m->lay.H && o.decode_kernel == 0) o.decode_kernel = 2;   // automatic choice: the per-step decoder
    hipStream_t s = as_stream(stream);
    HIPCHK(hipSetDevice(m->device));
    DecHost H(h_pay_off, h_pay_len, h_first, h_chunk_off, h_chunk_len, n_chunks);
    if (o.decode_kernel != 2) return decode_fused(m, o, H, d_payload, d_out, d_ws, ws_bytes, true, s);
    // the per-step decoder allocates its own buffers (d_ws is not used)
    const std::vector<long long>&off = H.off, &len = H.len, &steps = H.steps, &poff = H.poff, &plen = H.plen;
    const std::vector<uint8_t>& first = H.first;
    DevBuf d_first, d_off, d_len, d_poff, d_plen;
    HIPCHK(upload(d_first, first, s));
    HIPCHK(upload(d_off, off, s));
    HIPCHK(upload(d_len, len, s));
    HIPCHK(upload(d_poff, poff, s));
    HIPCHK(upload(d_plen, plen, s));
    HIPCHK(launch_prefill(d_first.as<uint8_t>(), d_off.as<long long>(), d_len.as<long long>(), (int)n_chunks,
                          d_out, s));
    // Lanes are split into independent groups, each with its own schedule,
    // buffers, captured step graph and stream: a decoder step is a chain of
    // small latency-bound kernels, and the groups' chains overlap on the GPU.
    // Every lane runs the same arithmetic whatever group it is in.
    const int max_lanes = plan_lanes(o, steps);
    std::vector<int> idx;
    for (uint64_t i = 0; i < n_chunks; ++i)
        if (steps[i] > 0) idx.push_back((int)i);
    if (idx.empty()) { HIPCHK(hipStreamSynchronize(s)); return BOA_OK; }
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return steps[a] > steps[b]; });
    int G = o.decode_groups ? (int)o.decode_groups : 1;
    G = std::max(1, std::min<int>(G, (int)idx.size()));
    struct Group {
        HostPlan P;
        PlanDev PD;
        Work W;
        hipStream_t st = nullptr;
        hipEvent_t done = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        ~Group() {
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            if (done) (void)hipEventDestroy(done);
            if (st) (void)hipStreamDestroy(st);
        }
    };
    std::vector<std::unique_ptr<Group>> groups;
    hipEvent_t ready;
    HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    struct EvG { hipEvent_t e; ~EvG() { (void)hipEventDestroy(e); } } ready_guard{ready};
    HIPCHK(hipEventRecord(ready, s));                       // prefill done
    const int unroll = 8;
    long long max_steps = 0;
    for (int g = 0; g < G; ++g) {
        std::vector<long long> gsteps(n_chunks, 0);
        for (size_t i = g; i < idx.size(); i += G) gsteps[idx[i]] = steps[idx[i]];
        auto grp = std::make_unique<Group>();
        grp->P = build_plan(gsteps, std::max(1, max_lanes / G));
        if (grp->P.lanes == 0) continue;
        int rc = upload_plan(grp->P, off, gsteps, grp->PD, s);
        if (rc) return rc;
        rc = grp->W.alloc(m, grp->P.lanes, 1);
        if (rc) return rc;
        HIPCHK(hipStreamCreateWithFlags(&grp->st, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&grp->done, hipEventDisableTiming));
        HIPCHK(hipStreamWaitEvent(grp->st, ready, 0));
        Work& W = grp->W;
        HIPCHK(hipMemsetAsync(W.coder.p, 0, W.coder.n, grp->st));
        const Plan p = grp->PD.view();
        // rows and embeddings of step 0; every later step's are written by the decoder
        HIPCHK(launch_embed(m->d_w + m->lay.embed, d_out, p, W.lanes, 1, 0, nullptr, m->lay.D,
                            W.row_chunk.as<int>(), W.row_pos.as<int>(), W.r.as<float>(), grp->st));
        if (o.use_graph != 2) {
            hipStream_t cs;
            HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            int rc2 = BOA_OK;
            if (e == hipSuccess) {
                for (int u = 0; u < unroll && rc2 == BOA_OK; ++u)
                    rc2 = enqueue_decode_step(m, W, (int)o.dtype, p, d_out, d_payload, d_poff.as<long long>(),
                                              d_plen.as<long long>(), cs);
                hipError_t e2 = hipStreamEndCapture(cs, &grp->graph);
                if (e2 != hipSuccess && rc2 == BOA_OK) rc2 = fail(BOA_E_DEVICE, hipGetErrorString(e2));
            } else {
                rc2 = fail(BOA_E_DEVICE, hipGetErrorString(e));
            }
            if (rc2 == BOA_OK) {
                e = hipGraphInstantiate(&grp->exec, grp->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) rc2 = fail(BOA_E_DEVICE, hipGetErrorString(e));
            }
            (void)hipStreamDestroy(cs);
            if (rc2) return rc2;
        }
        max_steps = std::max(max_steps, grp->P.total_steps);
        groups.push_back(std::move(grp));
    }
    if (o.use_graph != 2) {
        for (long long st = 0; st < max_steps; st += unroll)
            for (auto& grp : groups)
                if (st < grp->P.total_steps) HIPCHK(hipGraphLaunch(grp->exec, grp->st));
    } else {
        for (long long st = 0; st < max_steps; ++st)
            for (auto& grp : groups)
                if (st < grp->P.total_steps) {
                    int rc = enqueue_decode_step(m, grp->W, (int)o.dtype, grp->PD.view(), d_out, d_payload,
                                                 d_poff.as<long long>(), d_plen.as<long long>(), grp->st);
                    if (rc) return rc;
                }
    }
    for (auto& grp : groups) {
        HIPCHK(hipEventRecord(grp->done, grp->st));
        HIPCHK(hipStreamWaitEvent(s, grp->done, 0));
    }
    HIPCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

// =================================================================== workspace and host helpers
extern "C" int boa_workspace_size(const boa_model* m, const uint64_t* h_chunk_len, uint64_t n_chunks,
                                  const boa_run_opts* opts, uint32_t mode, uint64_t* bytes) {
    if (!m || !bytes || (n_chunks && !h_chunk_len)) return fail(BOA_E_ARG, "null argument");
    if (mode != BOA_WS_ENCODE && mode != BOA_WS_DECODE) return fail(BOA_E_ARG, "mode must be BOA_WS_ENCODE or BOA_WS_DECODE");
    boa_run_opts o{};
    if (opts) o = *opts;
    if (!dtype_ok(o.dtype)) return fail(BOA_E_UNSUPPORTED, "dtype not supported by this library");
    if (n_chunks > (1u << 30)) return fail(BOA_E_ARG, "too many chunks");
    if (n_chunks && !lens_ok(h_chunk_len, n_chunks))
        return fail(BOA_E_ARG, "chunk length beyond 2^31 - 1 bytes or total beyond 2^48");
    *bytes = 0;
    if (n_chunks == 0) return BOA_OK;
    const std::vector<long long> steps = chunk_steps(h_chunk_len, n_chunks);
    if (mode == BOA_WS_ENCODE) {
        *bytes = encode_ws_bytes(m, steps, o);
        return BOA_OK;
    }
    if (o.decode_kernel == 2 || (m->lay.H && o.decode_kernel == 0))
        return BOA_OK;                           // the per-step decoder allocates its own buffers
    FusedShape F;
    int rc = fused_shape(m, o, steps, F);
    if (rc) return rc;
    *bytes = decode_ws_bytes(m, o, steps);
    return BOA_OK;
}

extern "C" int boa_plan_lanes(const uint64_t* h_chunk_len, uint64_t n_chunks, uint32_t max_lanes, uint32_t* lanes) {
    if (!lanes || (n_chunks && !h_chunk_len)) return fail(BOA_E_ARG, "null argument");
    if (!lens_ok(h_chunk_len, n_chunks)) return fail(BOA_E_ARG, "chunk length beyond 2^31 - 1 bytes or total beyond 2^48");
    boa_run_opts o{};
    o.max_lanes = max_lanes;
    const std::vector<long long> steps = chunk_steps(h_chunk_len, n_chunks);
    const HostPlan P = build_plan(steps, plan_lanes(o, steps));
    *lanes = (uint32_t)P.lanes;
    return BOA_OK;
}

extern "C" int boa_split_fixed(uint64_t n, uint64_t chunk_len, uint64_t* h_lens, uint64_t cap, uint64_t* n_chunks) {
    if (!n_chunks || chunk_len == 0) return fail(BOA_E_ARG, "chunk_len must be positive");
    const uint64_t k = n / chunk_len + (n % chunk_len ? 1 : 0);
    *n_chunks = k;
    if (!h_lens) return BOA_OK;
    if (cap < k) return fail(BOA_E_ARG, "h_lens holds fewer entries than chunks");
    for (uint64_t i = 0; i < k; ++i) h_lens[i] = (i + 1 < k || n % chunk_len == 0) ? chunk_len : n % chunk_len;
    return BOA_OK;
}

extern "C" int boa_payload_layout(const uint64_t* h_chunk_len, uint64_t n, uint64_t* h_chunk_off, uint64_t* h_pay_off,
                                  uint64_t* h_pay_cap, uint64_t* total_cap) {
    if (n && (!h_chunk_len || !h_chunk_off || !h_pay_off || !h_pay_cap)) return fail(BOA_E_ARG, "null argument");
    if (!total_cap) return fail(BOA_E_ARG, "null argument");
    if (n && !lens_ok(h_chunk_len, n)) return fail(BOA_E_ARG, "chunk length beyond 2^31 - 1 bytes or total beyond 2^48");
    uint64_t off = 0, po = 0;
    for (uint64_t i = 0; i < n; ++i) {
        h_chunk_off[i] = off;
        h_pay_off[i] = po;
        h_pay_cap[i] = 2 * h_chunk_len[i] + 64;
        off += h_chunk_len[i];
        po += h_pay_cap[i];
    }
    *total_cap = po;
    return BOA_OK;
}

extern "C" int boa_diagnostics_summary(const uint32_t* h_rank_hist, const uint64_t* h_calib, uint32_t n_bins,
                                       double* h_topk, double* ece, uint64_t* positions) {
    if (!h_rank_hist || !h_calib || !h_topk || !ece || !positions) return fail(BOA_E_ARG, "null argument");
    if (n_bins < 1 || n_bins > 1024) return fail(BOA_E_ARG, "n_bins must be in [1, 1024]");
    uint64_t n = 0;
    for (int r = 0; r < 256; ++r) n += h_rank_hist[r];
    *positions = n;
    uint64_t cum = 0;
    for (int k = 0; k < 256; ++k) {
        cum += h_rank_hist[k];
        h_topk[k] = n ? (double)cum / (double)n : 0.0;     // Top-(k+1): rank < k + 1
    }
    // ECE = sum_b (n_b / N) |acc_b - conf_b| with conf_b = (sum of conf 2^32) / 2^32 / n_b,
    // N the binned positions
    uint64_t nb = 0;
    for (uint32_t b = 0; b < n_bins; ++b) nb += h_calib[3 * b];
    double e = 0.0;
    for (uint32_t b = 0; b < n_bins; ++b) {
        const uint64_t cnt = h_calib[3 * b], cor = h_calib[3 * b + 1], cs = h_calib[3 * b + 2];
        if (!cnt) continue;
        const double acc = (double)cor / (double)cnt, conf = (double)cs / 4294967296.0 / (double)cnt;
        e += (double)cnt / (double)nb * std::fabs(acc - conf);
    }
    *ece = e;
    return BOA_OK;
}

// =================================================================== parity helpers
extern "C" int boa_logits_dev(const boa_model* m, const uint8_t* d_seqs, uint32_t n_lanes, uint32_t T,
                              uint32_t dtype, uint32_t tile_t, float* d_logits, float* d_probs,
                              uint16_t* d_tables, void* stream) {
    if (!m || !d_seqs || !d_logits) return fail(BOA_E_ARG, "null argument");
    if (!dtype_ok(dtype)) return fail(BOA_E_UNSUPPORTED, "dtype not supported by this library");
    if (n_lanes == 0 || T < 2) return BOA_OK;
    hipStream_t s = as_stream(stream);
    HIPCHK(hipSetDevice(m->device));
    std::vector<long long> off(n_lanes), steps(n_lanes, (long long)T - 1);
    for (uint32_t i = 0; i < n_lanes; ++i) off[i] = (long long)i * T;
    HostPlan P = build_plan(steps, (int)n_lanes);
    PlanDev PD;
    int rc = upload_plan(P, off, steps, PD, s);
    if (rc) return rc;
    const int Tt = pick_tile(P.lanes, P.total_steps, tile_t);
    Work W;
    rc = W.alloc(m, P.lanes, Tt);
    if (rc) return rc;
    DevBuf probs, tables;
    if (d_probs) ALLOC(probs, (size_t)P.lanes * Tt * 256 * 4);
    if (d_tables) ALLOC(tables, (size_t)P.lanes * Tt * 256 * 2);
    const Plan p = PD.view();
    const int M = P.lanes * Tt;
    // lanes of build_plan are sorted by length (all equal here), lane i <-> chunk ent_chunk[i]
    for (uint32_t i = 0; i < n_lanes; ++i)
        if (P.ent_chunk[P.lane_first[i]] != (int)i) return fail(BOA_E_DEVICE, "unexpected lane order");
    for (long long s0 = 0; s0 < P.total_steps; s0 += Tt) {
        rc = forward_tile(m, W, (int)dtype, d_seqs, p, s0, nullptr, s);
        if (rc) return rc;
        HIPCHK(launch_scatter_rows(W.logits.as<float>(), P.lanes, Tt, 256, s0, (long long)T - 1, d_logits, s));
        if (d_probs || d_tables) {
            HIPCHK(launch_quant_sym(W.logits.as<float>(), M, d_seqs, p, W.row_chunk.as<int>(), W.row_pos.as<int>(),
                                    nullptr, d_probs ? probs.as<float>() : nullptr,
                                    d_tables ? tables.as<uint16_t>() : nullptr, s));
            if (d_probs)
                HIPCHK(launch_scatter_rows(probs.as<float>(), P.lanes, Tt, 256, s0, (long long)T - 1, d_probs, s));
            if (d_tables)
                HIPCHK(launch_scatter_rows_u16(tables.as<uint16_t>(), P.lanes, Tt, 256, s0, (long long)T - 1,
                                               d_tables, s));
        }
    }
    HIPCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

extern "C" int boa_diagnostics_dev(const boa_model* m, const uint8_t* d_seqs, uint32_t n_lanes, uint32_t T,
                                   uint32_t dtype, uint32_t tile_t, uint32_t n_bins, uint32_t* d_confusion,
                                   uint32_t* d_rank_hist, uint64_t* d_calib, void* stream) {
    if (!m || !d_confusion || !d_rank_hist || !d_calib) return fail(BOA_E_ARG, "null argument");
    if (n_bins < 1 || n_bins > 1024) return fail(BOA_E_ARG, "n_bins must be in [1, 1024]");
    if (!dtype_ok(dtype)) return fail(BOA_E_UNSUPPORTED, "dtype not supported by this library");
    hipStream_t s = as_stream(stream);
    HIPCHK(hipSetDevice(m->device));
    HIPCHK(hipMemsetAsync(d_confusion, 0, 256 * 256 * sizeof(uint32_t), s));
    HIPCHK(hipMemsetAsync(d_rank_hist, 0, 256 * sizeof(uint32_t), s));
    HIPCHK(hipMemsetAsync(d_calib, 0, (size_t)3 * n_bins * sizeof(uint64_t), s));
    if (n_lanes == 0 || T < 2) {
        HIPCHK(hipStreamSynchronize(s));
        return BOA_OK;
    }
    if (!d_seqs) return fail(BOA_E_ARG, "null argument");
    std::vector<long long> off(n_lanes), steps(n_lanes, (long long)T - 1);
    for (uint32_t i = 0; i < n_lanes; ++i) off[i] = (long long)i * T;
    HostPlan P = build_plan(steps, (int)n_lanes);
    PlanDev PD;
    int rc = upload_plan(P, off, steps, PD, s);
    if (rc) return rc;
    const int Tt = pick_tile(P.lanes, P.total_steps, tile_t);
    Work W;
    rc = W.alloc(m, P.lanes, Tt);
    if (rc) return rc;
    const Plan p = PD.view();
    const int M = P.lanes * Tt;
    for (long long s0 = 0; s0 < P.total_steps; s0 += Tt) {
        rc = forward_tile(m, W, (int)dtype, d_seqs, p, s0, nullptr, s);
        if (rc) return rc;
        HIPCHK(launch_diag(W.logits.as<float>(), M, d_seqs, p, W.row_chunk.as<int>(), W.row_pos.as<int>(),
                           (int)n_bins, d_confusion, d_rank_hist, reinterpret_cast<unsigned long long*>(d_calib), s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

extern "C" int boa_code_tables_dev(const uint8_t* d_sym, const uint16_t* d_freq, const uint64_t* h_nsym,
                                   uint64_t n_lanes, uint8_t* d_payload, const uint64_t* h_pay_off,
                                   const uint64_t* h_pay_cap, uint32_t* d_pay_len, void* stream) {
    if (n_lanes == 0) return BOA_OK;
    if (!d_sym || !d_freq || !h_nsym || !d_payload || !h_pay_off || !h_pay_cap || !d_pay_len)
        return fail(BOA_E_ARG, "null argument");
    hipStream_t s = as_stream(stream);
    std::vector<long long> so(n_lanes), ns(n_lanes), po(n_lanes), pc(n_lanes);
    long long acc = 0;
    for (uint64_t i = 0; i < n_lanes; ++i) {
        so[i] = acc; ns[i] = (long long)h_nsym[i]; acc += ns[i];
        po[i] = (long long)h_pay_off[i]; pc[i] = (long long)std::min<uint64_t>(h_pay_cap[i], 0xFFFFFFF0ULL);
    }
    DevBuf a, b, c, d;
    HIPCHK(upload(a, so, s)); HIPCHK(upload(b, ns, s)); HIPCHK(upload(c, po, s)); HIPCHK(upload(d, pc, s));
    HIPCHK(launch_code_tables(d_sym, d_freq, a.as<long long>(), b.as<long long>(), (int)n_lanes, d_payload,
                              c.as<long long>(), d.as<long long>(), d_pay_len, s));
    HIPCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

extern "C" int boa_decode_tables_dev(const uint8_t* d_payload, const uint64_t* h_pay_off,
                                     const uint64_t* h_pay_len, const uint16_t* d_freq, const uint64_t* h_nsym,
                                     uint64_t n_lanes, uint8_t* d_sym, void* stream) {
    if (n_lanes == 0) return BOA_OK;
    if (!d_payload || !h_pay_off || !h_pay_len || !d_freq || !h_nsym || !d_sym)
        return fail(BOA_E_ARG, "null argument");
    hipStream_t s = as_stream(stream);
    std::vector<long long> so(n_lanes), ns(n_lanes), po(n_lanes), pl(n_lanes);
    long long acc = 0;
    for (uint64_t i = 0; i < n_lanes; ++i) {
        so[i] = acc; ns[i] = (long long)h_nsym[i]; acc += ns[i];
        po[i] = (long long)h_pay_off[i]; pl[i] = (long long)std::min<uint64_t>(h_pay_len[i], 0xFFFFFFF0ULL);
    }
    DevBuf a, b, c, d;
    HIPCHK(upload(a, so, s)); HIPCHK(upload(b, ns, s)); HIPCHK(upload(c, po, s)); HIPCHK(upload(d, pl, s));
    HIPCHK(launch_decode_tables(d_payload, c.as<long long>(), d.as<long long>(), d_freq, a.as<long long>(),
                                b.as<long long>(), (int)n_lanes, d_sym, s));
    HIPCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

// =================================================================== order-2
namespace {
constexpr size_t O2_TABLE_BYTES = 65536ull * 256ull * 2ull;   // per concurrently coded chunk
int o2_batch(uint64_t n) { return (int)std::min<uint64_t>(n, 256); }
}  // namespace

extern "C" int boa_order2_encode_dev(const uint8_t* d_data, const uint64_t* h_chunk_off,
                                     const uint64_t* h_chunk_len, uint64_t n_chunks, uint8_t* d_payload,
                                     const uint64_t* h_pay_off, const uint64_t* h_pay_cap, uint32_t* d_pay_len,
                                     double* d_ideal_bits, void* stream) {
    if (n_chunks == 0) return BOA_OK;
    if (!d_data || !h_chunk_off || !h_chunk_len || !d_payload || !h_pay_off || !h_pay_cap || !d_pay_len)
        return fail(BOA_E_ARG, "null argument");
    hipStream_t s = as_stream(stream);
    std::vector<long long> off(n_chunks), len(n_chunks), po(n_chunks), pc(n_chunks);
    for (uint64_t i = 0; i < n_chunks; ++i) {
        off[i] = (long long)h_chunk_off[i]; len[i] = (long long)h_chunk_len[i];
        po[i] = (long long)h_pay_off[i]; pc[i] = (long long)std::min<uint64_t>(h_pay_cap[i], 0xFFFFFFF0ULL);
    }
    DevBuf a, b, c, d, counts;
    HIPCHK(upload(a, off, s)); HIPCHK(upload(b, len, s)); HIPCHK(upload(c, po, s)); HIPCHK(upload(d, pc, s));
    const int B = o2_batch(n_chunks);
    ALLOC(counts, O2_TABLE_BYTES * B);
    for (uint64_t c0 = 0; c0 < n_chunks; c0 += B) {
        int nb = (int)std::min<uint64_t>(B, n_chunks - c0);
        HIPCHK(hipMemsetAsync(counts.p, 0, O2_TABLE_BYTES * nb, s));
        HIPCHK(launch_order2_encode(d_data, a.as<long long>() + c0, b.as<long long>() + c0, nb,
                                    counts.as<uint16_t>(), d_payload, c.as<long long>() + c0,
                                    d.as<long long>() + c0, d_pay_len + c0, d_ideal_bits ? d_ideal_bits + c0 : nullptr,
                                    s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

extern "C" int boa_order2_decode_dev(const uint8_t* d_payload, const uint64_t* h_pay_off,
                                     const uint64_t* h_pay_len, const uint8_t* h_first,
                                     const uint64_t* h_chunk_off, const uint64_t* h_chunk_len, uint64_t n_chunks,
                                     uint8_t* d_out, void* stream) {
    if (n_chunks == 0) return BOA_OK;
    if (!d_payload || !h_pay_off || !h_pay_len || !h_first || !h_chunk_off || !h_chunk_len || !d_out)
        return fail(BOA_E_ARG, "null argument");
    hipStream_t s = as_stream(stream);
    std::vector<long long> off(n_chunks), len(n_chunks), po(n_chunks), pl(n_chunks);
    std::vector<uint8_t> first(h_first, h_first + n_chunks);
    for (uint64_t i = 0; i < n_chunks; ++i) {
        off[i] = (long long)h_chunk_off[i]; len[i] = (long long)h_chunk_len[i];
        po[i] = (long long)h_pay_off[i]; pl[i] = (long long)std::min<uint64_t>(h_pay_len[i], 0xFFFFFFF0ULL);
    }
    DevBuf a, b, c, d, f, counts;
    HIPCHK(upload(a, off, s)); HIPCHK(upload(b, len, s)); HIPCHK(upload(c, po, s)); HIPCHK(upload(d, pl, s));
    HIPCHK(upload(f, first, s));
    HIPCHK(launch_prefill(f.as<uint8_t>(), a.as<long long>(), b.as<long long>(), (int)n_chunks, d_out, s));
    const int B = o2_batch(n_chunks);
    ALLOC(counts, O2_TABLE_BYTES * B);
    for (uint64_t c0 = 0; c0 < n_chunks; c0 += B) {
        int nb = (int)std::min<uint64_t>(B, n_chunks - c0);
        HIPCHK(hipMemsetAsync(counts.p, 0, O2_TABLE_BYTES * nb, s));
        HIPCHK(launch_order2_decode(d_payload, c.as<long long>() + c0, d.as<long long>() + c0,
                                    a.as<long long>() + c0, b.as<long long>() + c0, nb, counts.as<uint16_t>(), d_out,
                                    s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return BOA_OK;
}

// =================================================================== container
// Layout (little-endian):
//   header 64 B: "BOA1", u32 version, u64 fingerprint, u32 numerics id,
//     u8 w, u8 B, u16 0, u64 total length, u64 nominal chunk length,
//     u64 final chunk length, u64 n_chunks, u32 CRC32(header[0:56] + index), u32 0
//   index n_chunks x 32 B: u64 length, u64 payload offset, u32 payload bytes,
//     u32 CRC32 of the chunk's bytes, u8 first byte, u8 coder id, 6 B zero
//   payloads.
namespace {
constexpr size_t HDR = 64, IDX = 32;
template <typename T> void put(std::vector<uint8_t>& v, size_t at, T x) { std::memcpy(v.data() + at, &x, sizeof(T)); }
template <typename T> T get(const uint8_t* p, size_t at) { T x; std::memcpy(&x, p + at, sizeof(T)); return x; }
}  // namespace

extern "C" int boa_compress(const boa_model* m, const uint8_t* h_data, const uint64_t* h_chunk_len,
                            uint64_t n_chunks, const boa_run_opts* opts, uint8_t** out, uint64_t* out_len) {
    if (!m || !out || !out_len || (n_chunks && (!h_chunk_len))) return fail(BOA_E_ARG, "null argument");
    boa_run_opts o{};
    if (opts) o = *opts;
    if (n_chunks && !lens_ok(h_chunk_len, n_chunks))
        return fail(BOA_E_ARG, "chunk length beyond 2^31 - 1 bytes or total beyond 2^48");
    uint64_t total = 0;
    for (uint64_t i = 0; i < n_chunks; ++i) total += h_chunk_len[i];
    if (total && !h_data) return fail(BOA_E_ARG, "null data");
    HIPCHK(hipSetDevice(m->device));
    std::vector<uint64_t> off(n_chunks), poff(n_chunks), pcap(n_chunks);
    uint64_t acc = 0, pacc = 0;
    for (uint64_t i = 0; i < n_chunks; ++i) {
        off[i] = acc; acc += h_chunk_len[i];
        poff[i] = pacc; pcap[i] = 2 * h_chunk_len[i] + 64; pacc += pcap[i];
    }
    hipStream_t s;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct SG { hipStream_t s; ~SG() { (void)hipStreamDestroy(s); } } sg{s};
    DevBuf d_data, d_pay, d_len, d_crc, d_off, d_clen;
    ALLOC(d_data, total);
    if (total) HIPCHK(hipMemcpyAsync(d_data.p, h_data, total, hipMemcpyHostToDevice, s));
    ALLOC(d_pay, pacc);
    ALLOC(d_len, n_chunks * 4);
    int rc;
    if (o.dtype == BOA_DTYPE_INT8) {
        boa_qmodel* q = nullptr;
        rc = boa_qmodel_create(m, &q);
        if (rc) return rc;
        rc = boa_int_encode_dev(q, d_data.as<uint8_t>(), off.data(), h_chunk_len, n_chunks, d_pay.as<uint8_t>(),
                                poff.data(), pcap.data(), d_len.as<uint32_t>(), s);
        boa_qmodel_free(q);
    } else {
        rc = boa_encode_dev(m, d_data.as<uint8_t>(), off.data(), h_chunk_len, n_chunks, &o, d_pay.as<uint8_t>(),
                            poff.data(), pcap.data(), d_len.as<uint32_t>(), nullptr, nullptr, 0, s);
    }
    if (rc) return rc;
    std::vector<uint32_t> plen(n_chunks), ccrc(n_chunks);
    std::vector<uint32_t> coder(n_chunks, BOA_CODER_MAMBA);
    DevBuf d_len2, d_pay2;
    std::vector<uint32_t> plen2;
    if (o.fallback) {
        ALLOC(d_pay2, pacc);
        ALLOC(d_len2, n_chunks * 4);
        rc = boa_order2_encode_dev(d_data.as<uint8_t>(), off.data(), h_chunk_len, n_chunks, d_pay2.as<uint8_t>(),
                                   poff.data(), pcap.data(), d_len2.as<uint32_t>(), nullptr, s);
        if (rc) return rc;
        plen2.resize(n_chunks);
        if (n_chunks) HIPCHK(hipMemcpyAsync(plen2.data(), d_len2.p, n_chunks * 4, hipMemcpyDeviceToHost, s));
    }
    std::vector<long long> off_ll(off.begin(), off.end()), len_ll(h_chunk_len, h_chunk_len + n_chunks);
    HIPCHK(upload(d_off, off_ll, s));
    HIPCHK(upload(d_clen, len_ll, s));
    ALLOC(d_crc, n_chunks * 4);
    if (n_chunks) HIPCHK(launch_crc32(d_data.as<uint8_t>(), d_off.as<long long>(), d_clen.as<long long>(),
                                      (int)n_chunks, d_crc.as<uint32_t>(), s));
    if (n_chunks) {
        HIPCHK(hipMemcpyAsync(plen.data(), d_len.p, n_chunks * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(ccrc.data(), d_crc.p, n_chunks * 4, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    // per chunk: coded bytes and coder; raw when the coded form is not smaller
    std::vector<uint64_t> csize(n_chunks);
    uint64_t pay_total = 0;
    for (uint64_t i = 0; i < n_chunks; ++i) {
        uint64_t n = h_chunk_len[i];
        uint64_t raw = n > 0 ? n - 1 : 0;
        uint64_t best = plen[i] == 0xFFFFFFFFu ? UINT64_MAX : plen[i];
        coder[i] = BOA_CODER_MAMBA;
        if (o.fallback && plen2[i] != 0xFFFFFFFFu && plen2[i] < best) { best = plen2[i]; coder[i] = BOA_CODER_ORDER2; }
        if (best > raw) { best = raw; coder[i] = BOA_CODER_RAW; }
        csize[i] = best;
        pay_total += best;
    }
    const uint64_t size = HDR + IDX * n_chunks + pay_total;
    std::vector<uint8_t> buf(size, 0);
    uint64_t pa = 0;
    for (uint64_t i = 0; i < n_chunks; ++i) {
        size_t at = HDR + IDX * i;
        put<uint64_t>(buf, at, h_chunk_len[i]);
        put<uint64_t>(buf, at + 8, pa);
        put<uint32_t>(buf, at + 16, (uint32_t)csize[i]);
        put<uint32_t>(buf, at + 20, ccrc[i]);
        buf[at + 24] = h_chunk_len[i] ? h_data[off[i]] : 0;
        buf[at + 25] = (uint8_t)coder[i];
        uint8_t* dst = buf.data() + HDR + IDX * n_chunks + pa;
        if (csize[i]) {
            if (coder[i] == BOA_CODER_RAW) {
                std::memcpy(dst, h_data + off[i] + 1, csize[i]);
            } else {
                const DevBuf& src = coder[i] == BOA_CODER_MAMBA ? d_pay : d_pay2;
                HIPCHK(hipMemcpyAsync(dst, src.as<uint8_t>() + poff[i], csize[i], hipMemcpyDeviceToHost, s));
            }
        }
        pa += csize[i];
    }
    std::memcpy(buf.data(), "BOA1", 4);
    put<uint32_t>(buf, 4, 1);
    put<uint64_t>(buf, 8, model_fingerprint(m));
    put<uint32_t>(buf, 16, boa_numerics_id(o.dtype));
    buf[20] = 32;
    buf[21] = 16;
    put<uint64_t>(buf, 24, total);
    put<uint64_t>(buf, 32, n_chunks ? h_chunk_len[0] : 0);
    put<uint64_t>(buf, 40, n_chunks ? h_chunk_len[n_chunks - 1] : 0);
    put<uint64_t>(buf, 48, n_chunks);
    HIPCHK(hipStreamSynchronize(s));
    uint32_t c = crc32_host(buf.data(), 56);
    c = ~crc32_host(buf.data() + HDR, IDX * n_chunks, c);
    put<uint32_t>(buf, 56, c);
    uint8_t* res = static_cast<uint8_t*>(std::malloc(size ? size : 1));
    if (!res) return fail(BOA_E_OOM, "container");
    std::memcpy(res, buf.data(), size);
    *out = res;
    *out_len = size;
    g_last_pay.assign(csize.begin(), csize.end());
    g_last_coder = coder;
    return BOA_OK;
}

extern "C" int boa_last_chunk_stats(uint64_t* h_payload_bytes, uint32_t* h_coder, uint64_t n) {
    if (n != g_last_pay.size()) return fail(BOA_E_ARG, "chunk count differs from the last compress");
    for (uint64_t i = 0; i < n; ++i) {
        if (h_payload_bytes) h_payload_bytes[i] = g_last_pay[i];
        if (h_coder) h_coder[i] = g_last_coder[i];
    }
    return BOA_OK;
}

namespace {
// The parsed index of a container: per chunk its length, offset in the
// output, payload offset and size, CRC32, first byte and coder id.
struct Index {
    uint64_t n = 0, total = 0, fp = 0, pay_bytes = 0;
    uint32_t nid = 0;
    const uint8_t* pay = nullptr;
    std::vector<uint64_t> clen, off, poff, plen;
    std::vector<uint8_t> first, coder;
    std::vector<uint32_t> crc;
};

// Header, index CRC and every index record: coder ids known, payloads inside
// the container, raw chunks of the right size, lengths adding up to the
// header's total without wrapping, each within the decoder's step counter.
// The index is untrusted input: nothing here may overflow.
int parse_container(const uint8_t* p, uint64_t len, Index& ix, bool records) {
    if (!p || len < HDR) return fail(BOA_E_FORMAT, "container too short");
    if (std::memcmp(p, "BOA1", 4) != 0 || get<uint32_t>(p, 4) != 1) return fail(BOA_E_FORMAT, "bad magic/version");
    const uint64_t n = get<uint64_t>(p, 48);
    if (n > (len - HDR) / IDX) return fail(BOA_E_FORMAT, "index does not fit");
    uint32_t c = crc32_host(p, 56);
    c = ~crc32_host(p + HDR, IDX * n, c);
    if (c != get<uint32_t>(p, 56)) return fail(BOA_E_CRC, "index CRC mismatch");
    ix.n = n;
    ix.total = get<uint64_t>(p, 24);
    ix.fp = get<uint64_t>(p, 8);
    ix.nid = get<uint32_t>(p, 16);
    if (ix.total > MAX_TOTAL) return fail(BOA_E_CORRUPT, "total length beyond the supported maximum");
    if (!records) return BOA_OK;
    const uint8_t* idx = p + HDR;
    ix.pay = p + HDR + IDX * n;
    ix.pay_bytes = len - HDR - IDX * n;
    ix.clen.resize(n); ix.off.resize(n); ix.poff.resize(n); ix.plen.resize(n);
    ix.first.resize(n); ix.coder.resize(n); ix.crc.resize(n);
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t cl = get<uint64_t>(idx, IDX * i), po = get<uint64_t>(idx, IDX * i + 8);
        const uint64_t pl = get<uint32_t>(idx, IDX * i + 16);
        const uint8_t cd = idx[IDX * i + 25];
        if (cd > BOA_CODER_RAW) return fail(BOA_E_FORMAT, "unknown coder id");
        if (po > ix.pay_bytes || pl > ix.pay_bytes - po) return fail(BOA_E_CORRUPT, "payload truncated");
        if (cd == BOA_CODER_RAW && pl != (cl ? cl - 1 : 0)) return fail(BOA_E_CORRUPT, "raw chunk size mismatch");
        if (cl > MAX_CHUNK) return fail(BOA_E_CORRUPT, "chunk length beyond the supported maximum");
        if (cl > ix.total - acc) return fail(BOA_E_CORRUPT, "chunk lengths exceed the total length");
        ix.clen[i] = cl; ix.poff[i] = po; ix.plen[i] = pl;
        ix.crc[i] = get<uint32_t>(idx, IDX * i + 20);
        ix.first[i] = idx[IDX * i + 24];
        ix.coder[i] = cd;
        ix.off[i] = acc;
        acc += cl;
    }
    if (acc != ix.total) return fail(BOA_E_CORRUPT, "chunk lengths do not add up");
    return BOA_OK;
}
}  // namespace

extern "C" int boa_container_info(const uint8_t* h_container, uint64_t len, uint64_t* n_chunks,
                                  uint64_t* total_len, uint64_t* fingerprint, uint32_t* numerics_id) {
    Index ix;
    int rc = parse_container(h_container, len, ix, true);
    if (rc) return rc;
    if (n_chunks) *n_chunks = ix.n;
    if (total_len) *total_len = ix.total;
    if (fingerprint) *fingerprint = ix.fp;
    if (numerics_id) *numerics_id = ix.nid;
    return BOA_OK;
}

extern "C" int boa_decompress(const boa_model* m, const uint8_t* h_c, uint64_t len, const boa_run_opts* opts,
                              uint8_t** out, uint64_t* out_len) {
    if (!m || !h_c || !out || !out_len) return fail(BOA_E_ARG, "null argument");
    Index ix;
    int rc = parse_container(h_c, len, ix, true);
    if (rc) return rc;
    if (ix.fp != model_fingerprint(m)) return fail(BOA_E_MODEL, "container was written with another model");
    const uint32_t nid = ix.nid;
    uint32_t dtype = nid & 0xFF;
    if (nid != boa_numerics_id(dtype)) return fail(BOA_E_MODEL, "container numerics id differs from this library");
    boa_run_opts o{};
    if (opts) o = *opts;
    o.dtype = dtype;
    const uint64_t n = ix.n, total = ix.total, pay_bytes = ix.pay_bytes;
    const uint8_t* pay = ix.pay;
    const std::vector<uint64_t>&clen = ix.clen, &off = ix.off, &poff = ix.poff, &plen = ix.plen;
    const std::vector<uint8_t>&first = ix.first, &coder = ix.coder;
    const std::vector<uint32_t>& crc = ix.crc;
    HIPCHK(hipSetDevice(m->device));
    hipStream_t s;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct SG { hipStream_t s; ~SG() { (void)hipStreamDestroy(s); } } sg{s};
    DevBuf d_pay, d_out, d_crc, d_off, d_clen;
    ALLOC(d_pay, pay_bytes);
    if (pay_bytes) HIPCHK(hipMemcpyAsync(d_pay.p, pay, pay_bytes, hipMemcpyHostToDevice, s));
    ALLOC(d_out, total);
    // split by coder: model chunks, order-2 chunks; raw chunks are copied
    std::vector<uint64_t> mlen(n), o2len(n);
    for (uint64_t i = 0; i < n; ++i) {
        mlen[i] = coder[i] == BOA_CODER_MAMBA ? clen[i] : std::min<uint64_t>(clen[i], 1);
        o2len[i] = coder[i] == BOA_CODER_ORDER2 ? clen[i] : std::min<uint64_t>(clen[i], 1);
    }
    if (dtype == BOA_DTYPE_INT8) {
        boa_qmodel* q = nullptr;
        rc = boa_qmodel_create(m, &q);
        if (rc) return rc;
        rc = boa_int_decode_dev(q, d_pay.as<uint8_t>(), poff.data(), plen.data(), first.data(), off.data(),
                                mlen.data(), n, d_out.as<uint8_t>(), s);
        boa_qmodel_free(q);
    } else {
        rc = boa_decode_dev(m, d_pay.as<uint8_t>(), poff.data(), plen.data(), first.data(), off.data(), mlen.data(),
                            n, &o, d_out.as<uint8_t>(), nullptr, 0, s);
    }
    if (rc) return rc;
    bool any_o2 = std::any_of(coder.begin(), coder.end(), [](uint8_t c) { return c == BOA_CODER_ORDER2; });
    if (any_o2) {
        rc = boa_order2_decode_dev(d_pay.as<uint8_t>(), poff.data(), plen.data(), first.data(), off.data(),
                                   o2len.data(), n, d_out.as<uint8_t>(), s);
        if (rc) return rc;
    }
    for (uint64_t i = 0; i < n; ++i)
        if (coder[i] == BOA_CODER_RAW && plen[i])
            HIPCHK(hipMemcpyAsync(d_out.as<uint8_t>() + off[i] + 1, d_pay.as<uint8_t>() + poff[i], plen[i],
                                  hipMemcpyDeviceToDevice, s));
    std::vector<long long> off_ll(off.begin(), off.end()), len_ll(clen.begin(), clen.end());
    HIPCHK(upload(d_off, off_ll, s));
    HIPCHK(upload(d_clen, len_ll, s));
    ALLOC(d_crc, n * 4);
    std::vector<uint32_t> got(n);
    if (n) {
        HIPCHK(launch_crc32(d_out.as<uint8_t>(), d_off.as<long long>(), d_clen.as<long long>(), (int)n,
                            d_crc.as<uint32_t>(), s));
        HIPCHK(hipMemcpyAsync(got.data(), d_crc.p, n * 4, hipMemcpyDeviceToHost, s));
    }
    uint8_t* res = static_cast<uint8_t*>(std::malloc(total ? total : 1));
    if (!res) return fail(BOA_E_OOM, "output");
    if (total) HIPCHK(hipMemcpyAsync(res, d_out.p, total, hipMemcpyDeviceToHost, s));
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) { std::free(res); return fail(BOA_E_DEVICE, hipGetErrorString(e)); }
    for (uint64_t i = 0; i < n; ++i)
        if (got[i] != crc[i]) { std::free(res); return fail(BOA_E_CORRUPT, "chunk CRC mismatch after decode"); }
    *out = res;
    *out_len = total;
    return BOA_OK;
}
