// noalloc.hip -- the scratch memory of the allocation-free entry point
// (pdmp_occupancy_bwd_noalloc): a file-scope device array that every GPU the library
// runs on holds until the process ends, instead of a caller workspace or hipMalloc.
//
// In host code the array's name is only a stand-in for the symbol, not a device
// address; the address of each device's copy comes from hipGetSymbolAddress, taken
// once per device (with that device current) on the first call there, and kept.
#include <mutex>

#include "pdmp_common.h"

namespace pdmp {

constexpr size_t kNoallocScratchBytes = (size_t)32 << 20;
constexpr int kNoallocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kNoallocMaxDevices];

size_t noalloc_scratch_bytes() { return kNoallocScratchBytes; }

// The current device's copy of the scratch array (its device address).
int32_t noalloc_scratch(void **ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("hipGetDevice: %s", hipGetErrorString(e));
        return PDMP_EDEVICE;
    }
    if (dev < 0 || dev >= kNoallocMaxDevices) {
        set_error("device %d beyond the %d the static scratch is kept for", dev,
                  kNoallocMaxDevices);
        return PDMP_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev,
                      hipGetErrorString(e));
            return PDMP_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return PDMP_OK;
}

}  // namespace pdmp
