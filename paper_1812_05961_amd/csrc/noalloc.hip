// The allocation-free variant of cpd_mttkrp: every temporary of the call (the
// tile table when the tree has none cached for the width, the rank-ordered
// copy of the leaf factor, the per-XCD output copies) is carved from one
// fixed device array, so the call makes no device allocation.
#include <mutex>

#include "csf.h"

namespace cpd {
namespace {

constexpr size_t STATIC_SCRATCH_BYTES = size_t(64) << 20;

// One copy per device, held until the process ends.  Host code never uses
// this name as an address: it takes the device address from
// hipGetSymbolAddress, once per device.
__device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with it current).
cpd_status scratch_address(void **out) {
    int dev = 0;
    CPD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) CPD_FAIL(CPD_EUNSUPPORTED, "device %d beyond %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            CPD_FAIL(CPD_EHIP, "hipGetSymbolAddress of the static workspace failed: %s", hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return CPD_OK;
}

}  // namespace
}  // namespace cpd

extern "C" {

size_t cpd_mttkrp_noalloc_workspace_bytes(void) { return cpd::STATIC_SCRATCH_BYTES; }

cpd_status cpd_mttkrp_noalloc(cpd_csf csf, const void *const *factors, int32_t ld, int32_t rank, int32_t mode,
                              float *out, int32_t ldo, const cpd_mttkrp_opts *opts, void *stream) {
    cpd::clear_error();
    void *base = nullptr;
    CPD_TRY(cpd::scratch_address(&base));
    cpd::Workspace ws;
    ws.base = static_cast<char *>(base);
    ws.bytes = cpd::STATIC_SCRATCH_BYTES;
    return cpd::mttkrp_ws(csf, factors, ld, rank, mode, out, ldo, opts, (hipStream_t)stream, nullptr, nullptr, &ws);
}

}  // extern "C"
