// Fixed device scratch for the entry point that allocates nothing
// (ig_score_noalloc): pruned scoring's per-call work lives in one file-scope
// device array instead of library-allocated memory.  Each GPU the library runs on
// holds its own copy of the array until the process ends; host code reaches it
// only through the address hipGetSymbolAddress reports for the current device
// (the array's name in host code is a host-side stand-in, not a device address).
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace ig {

constexpr size_t kNoallocWords = IG_NOALLOC_SCRATCH_BYTES / 4;

static __device__ __align__(256) uint32_t scratch[kNoallocWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
uint32_t *g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

size_t noalloc_scratch_words() { return kNoallocWords; }

// The current device's copy of the array, looked up once per device.
uint32_t *noalloc_scratch() {
    int dev = 0;
    IG_HIP(hipGetDevice(&dev));
    IG_REQUIRE(dev >= 0 && dev < kMaxDevices, IG_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        IG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        IG_REQUIRE(p != nullptr, IG_E_DEVICE, "no device address for the fixed scratch array");
        g_noalloc_ptr[dev] = static_cast<uint32_t *>(p);
    }
    return g_noalloc_ptr[dev];
}

}  // namespace ig
