// noalloc.hip -- the fixed device scratch of the entry point that allocates
// nothing (pft_mul_relin_batch_noalloc), for callers that cannot allocate
// device memory (graph capture, tight serving loops, allocation-free
// harnesses).
//
// `scratch` is a file-scope device array: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address is resolved once per device
// with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pft_kernels.h"

static __device__ __align__(256) uint64_t scratch[PFT_NOALLOC_SCRATCH_BYTES / 8];

namespace {
std::mutex g_mu;
uint64_t* g_ptr[PFT_NOALLOC_MAX_DEVICES] = {};
}  // namespace

int noalloc_scratch_init(int device, uint64_t** out) {
    *out = nullptr;
    if (device < 0 || device >= PFT_NOALLOC_MAX_DEVICES) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != device) return -1;  // the device must be current
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return -1;
        }
        g_ptr[device] = static_cast<uint64_t*>(p);
    }
    *out = g_ptr[device];
    return 0;
}
