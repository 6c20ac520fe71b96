// Device scratch of the sequence entry point that allocates nothing
// (bwr_sequence_dev_noalloc): a file-scope device array that every call on a
// device carves its buffers from, instead of allocating.  Host code never
// passes the array's name to a kernel or a copy: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <vector>

#include "engine.h"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)256 << 20;

}  // namespace

// Each GPU the library runs on holds its own copy of this array until the process ends.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace bwr {

namespace {

struct DeviceScratch {
    void* ptr = nullptr;  // device address of `scratch` on this device
    std::mutex use;       // calls on one device take turns (they share the array)
};

std::mutex g_scratch_mu;
std::vector<std::unique_ptr<DeviceScratch>> g_scratch;  // by device

}  // namespace

size_t noalloc_scratch_bytes() { return SCRATCH_BYTES; }

// The current device's scratch (its address resolved on the first call on that device, with the device
// current) and the lock its users hold.
Error noalloc_scratch(void** ptr, std::mutex** use) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return Error::device(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1);
    if (!g_scratch[dev]) {
        auto d = std::make_unique<DeviceScratch>();
        e = hipGetSymbolAddress(&d->ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !d->ptr) return Error::device(e, "hipGetSymbolAddress (scratch)");
        g_scratch[dev] = std::move(d);
    }
    *ptr = g_scratch[dev]->ptr;
    *use = &g_scratch[dev]->use;
    return {};
}

}  // namespace bwr
