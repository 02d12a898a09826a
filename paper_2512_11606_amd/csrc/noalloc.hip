// Allocation-free scratch of ahpp_query_noalloc.
//
// Callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc) get a single-source
// query whose per-query buffers (residues, reserves, V / attribute residues,
// partials, control block, top-k scratch) live in one file-scope device
// array instead of memory the library allocates.  Each GPU holds its own copy
// of the array, at its own address, for the life of the process.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress (at
// graph load, with the graph's device current) and only that address is
// handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ahpp_internal.h"

namespace ahpp {

namespace {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

void noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices)
        throw Failure{AHPP_ERR_DEVICE, "noalloc scratch: device ordinal " + std::to_string(device) + " unsupported"};
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return;
    void *p = nullptr;
    check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "noalloc scratch address");
    if (!p) throw Failure{AHPP_ERR_DEVICE, "noalloc scratch address: null"};
    g_ptr[device] = p;
}

void *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

}  // namespace ahpp
