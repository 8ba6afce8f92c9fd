// Static device scratch for the allocation-free entry point (rpa_apply_coulomb_noalloc).
//
// The array lives in the library's code object: every GPU the library runs on holds its own
// copy, at its own address, from the first use on that device until the process ends.  Host
// code never passes the array's name to a kernel or a copy (on the host it is only a stand-in
// symbol); the device address comes from hipGetSymbolAddress, taken once per device with that
// device current and kept here.  Every call on one GPU shares that GPU's array, so calls that
// overlap on one GPU (other streams, other host threads) race on it.
#include <mutex>

#include "internal.h"

namespace rpa {

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

int noalloc_scratch(void** out) {
    int dev = 0;
    RPA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index " + std::to_string(dev) + " beyond the scratch table (" +
                  std::to_string(kMaxDevices) + " devices)");
        return RPA_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        RPA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned a null scratch address");
            return RPA_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RPA_OK;
}

}  // namespace rpa
