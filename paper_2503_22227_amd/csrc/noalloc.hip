// HMult+Relin for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc): the
// key-switching workspace is a static device array instead of a caller buffer.
//
// The array holds kScratchBytes on every device the library runs on, until the
// process ends.  Host code never passes the array's name to a kernel (in host
// code it is only a stand-in for the symbol): its device address is looked up
// once per device with hipGetSymbolAddress and that address is what the
// kernels receive.  Every call on one device shares the array, so calls that
// overlap on one device (different streams, or threads) race.  Nothing in the
// array needs to start at zero: every region of the workspace is written before
// it is read within one call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "rf_internal.hpp"

namespace {

// Enough for HMult+Relin at N = 2^16 with 24 Q-primes and 4 special primes at
// alpha = 8 (106 MiB) and at alpha = 4 (148 MiB).
constexpr size_t kScratchBytes = (size_t)160 << 20;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) uint64_t scratch[kScratchBytes / 8];

namespace {

// Device address of the current device's copy of `scratch` (device `device`
// must be current); looked up once per device.
int scratch_address(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return rf::fail(RF_EUNSUPPORTED, "rf_hmult_relin_noalloc: device index");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return rf::fail(RF_EHIP, std::string("rf_hmult_relin_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return RF_OK;
}

}  // namespace

extern "C" int rf_hmult_relin_noalloc(const rf_ctx *c, const uint64_t *a, const uint64_t *b, const uint64_t *rlk,
                                      uint64_t *out, uint32_t nl, void *stream) {
    if (!c) return rf::fail(RF_EINVAL, "rf_hmult_relin_noalloc: null context");
    const size_t need = rf_workspace_bytes(c, RF_OP_HMULT_RELIN, nl);
    if (need == 0) return rf::fail(RF_ELEVEL, "rf_hmult_relin_noalloc: limb count out of range for this chain");
    if (need > kScratchBytes)
        return rf::fail(RF_EUNSUPPORTED, "rf_hmult_relin_noalloc: needs " + std::to_string(need) +
                                             " bytes of scratch, the static array holds " +
                                             std::to_string(kScratchBytes));
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != c->device && hipSetDevice(c->device) != hipSuccess)
        return rf::fail(RF_EHIP, "rf_hmult_relin_noalloc: hipSetDevice");
    void *ws = nullptr;
    int rc = scratch_address(c->device, &ws);
    if (rc == RF_OK) rc = rf_hmult_relin(c, a, b, rlk, out, nl, ws, kScratchBytes, stream);
    if (prev >= 0 && prev != c->device) (void)hipSetDevice(prev);
    return rc;
}
