// The fixed device array behind mapdec_decode_noalloc, and its address.
#include <mutex>
#include <map>

#include "kernels.h"

namespace mapdec {

namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
}

// Workspace of the allocation-free decode: every call on a device shares
// that device's copy, held until the process ends.  On the host the name
// `scratch` is a stand-in, not the device address: host code passes only
// the address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

size_t scratch_bytes() { return kScratchBytes; }

hipError_t scratch_address(void **out) {
    static std::mutex mu;
    static std::map<int, void *> addr;   // device ordinal -> address of its copy
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        it = addr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return hipSuccess;
}

}  // namespace mapdec
