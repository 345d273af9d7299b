// Device scratch of the allocation-free decode entry point: one file-scope
// array per GPU that the library runs on, held until the process ends.  Host
// code never uses the array's name as an address (on the host it is only a
// stand-in): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>
#include <unordered_map>

#include "kernels.h"

namespace bch {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static std::unordered_map<int, void *> g_scratch_ptr;  // device -> address of its scratch

hipError_t noalloc_scratch(void **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return e;
    g_scratch_ptr[dev] = p;
    *ptr = p;
    return hipSuccess;
}

}  // namespace bch
