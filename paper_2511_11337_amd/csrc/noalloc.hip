// Allocation-free decode: boa_decode_noalloc_dev, the fused decoder of
// boa_decode_dev with every device buffer of the call (per-chunk arrays, lane
// schedule, and any lane state kept outside LDS) carved from a fixed scratch
// array that the library defines once per device, for callers that cannot
// allocate device memory (code under stream capture, serving loops,
// harnesses that forbid allocation).
//
// The array is a file-scope __device__ variable: each GPU the library runs
// on holds its own copy until the process ends.  In host code its name is
// only a host-side stand-in, so its device address is looked up once per
// device with hipGetSymbolAddress and only that address is used.  Every call
// on one GPU shares the array; calls that overlap on one GPU race.  Nothing
// in it needs to start at zero: the decoder writes every piece before
// reading it.
#include <mutex>
#include <string>

#include "boa_internal.h"

namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(2) << 20;    // 2 MiB per device
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// device address of this device's scratch array (looked up once per device,
// with that device current)
int scratch_of(int dev, void** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return boa::set_error(BOA_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return boa::set_error(BOA_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BOA_OK;
}
}  // namespace

extern "C" int boa_decode_noalloc_dev(const boa_model* m, const uint8_t* d_payload, const uint64_t* h_pay_off,
                                      const uint64_t* h_pay_len, const uint8_t* h_first, const uint64_t* h_chunk_off,
                                      const uint64_t* h_chunk_len, uint64_t n_chunks, const boa_run_opts* opts,
                                      uint8_t* d_out, void* stream) {
    if (!m) return boa::set_error(BOA_E_ARG, "null model");
    hipError_t e = hipSetDevice(m->device);
    if (e != hipSuccess) return boa::set_error(BOA_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    void* ws = nullptr;
    int rc = scratch_of(m->device, &ws);
    if (rc) return rc;
    return boa::decode_into_region(m, d_payload, h_pay_off, h_pay_len, h_first, h_chunk_off, h_chunk_len, n_chunks,
                                   opts, d_out, ws, NOALLOC_SCRATCH_BYTES, stream);
}
