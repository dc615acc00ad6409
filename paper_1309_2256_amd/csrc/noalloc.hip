// Device scratch for the allocation-free entry point tm_dslash_noalloc.
//
// The intermediate half fields of the composite operator kinds (the odd
// field of the Schur complement, the middle field of the normal operator,
// the even/odd halves of the full-lattice kinds) live in one file-scope
// device array instead of context workspace.  Each device that loads the
// library holds its own copy of the array for the life of the process; its
// device address is looked up once per device when the first context is
// created there (hipGetSymbolAddress with that device current) and only that
// address is handed to kernels and copies afterwards.
#include <mutex>

#include "runtime.h"

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_mutex;
void *g_ptr[kMaxDevices] = {};

}  // namespace

int noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return TM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_ptr[device]) return TM_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return TM_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return TM_ERR_HIP;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return TM_ERR_HIP;
    }
    g_ptr[device] = p;
    return TM_OK;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mutex);
    return g_ptr[device];
}
