// Fixed device scratch for the entry point that allocates nothing (sko_orth_block_noalloc).
//
// The array below is a file-scope device variable: the runtime places one copy on every
// device that loads the library, for the life of the process.  In host code its name is
// a host-side stand-in, not a device address, so host code never hands the name itself
// to a kernel or a copy: noalloc_init() looks up the device address once per device (with
// that device current, from sko_create) and every use goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "context.h"

namespace sko {
namespace {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

sko_status noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return SKO_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return SKO_OK;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return SKO_EDEVICE;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SKO_EDEVICE;
    g_ptr[device] = ptr;
    return SKO_OK;
}

void* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace sko
