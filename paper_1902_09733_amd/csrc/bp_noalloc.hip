// Fixed device scratch of bp_run_noalloc: callers that cannot allocate device
// memory (code under stream capture, serving loops, harnesses that forbid it)
// run bp_run's launch sequence on this array instead of a caller workspace.
//
// The array is a file-scope device variable, so every GPU the library runs on
// holds its own copy (of kNoallocScratchBytes) from the moment this file's
// code object is loaded on that device until the process ends.  Host code
// never passes the array's name to a kernel: the name is a host-side stand-in
// whose address is not a device address.  Its device address is resolved once
// per device with hipGetSymbolAddress (with that device current) and cached.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bp_internal.h"

namespace bpk {

static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices];
}  // namespace

void *noalloc_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_addr[dev] = p;
    }
    return g_addr[dev];
}

}  // namespace bpk
