// noalloc.hip -- the fixed device workspace of pdhg_setup_noalloc.
//
// One file-scope device array per GPU holds the whole workspace of the one
// handle that pdhg_setup_noalloc may keep live on that GPU (matrices, vectors,
// check partials, active lists and the done flags), so that call allocates no
// device memory and no pinned host memory.  Host code never names the array:
// its device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and the cached address is what the setup carves.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/pdhg.h"
#include "pdhg_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[PDHG_NOALLOC_MAX_BYTES];

constexpr int MAX_DEV = 64;

std::mutex g_mu;
void *g_ptr[MAX_DEV] = {};        // device address of `scratch` on each device
const void *g_owner[MAX_DEV] = {};  // the live no-alloc handle of each device

}  // namespace

namespace pdhg {

// Claims device `dev`'s array for `owner` and returns its device address in
// *ptr.  hipSuccess, or hipErrorInvalidDevice for a bad id, hipErrorInvalidValue
// if another live handle holds the array (*busy = 1), or the lookup's error.
hipError_t noalloc_claim(int dev, const void *owner, void **ptr, int *busy)
{
    *busy = 0;
    *ptr = nullptr;
    if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_owner[dev]) {
        *busy = 1;
        return hipErrorInvalidValue;
    }
    if (!g_ptr[dev]) {
        // the device is current (the caller's stream belongs to it)
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    g_owner[dev] = owner;
    *ptr = g_ptr[dev];
    return hipSuccess;
}

// Releases device `dev`'s array if `owner` holds it.
void noalloc_release(int dev, const void *owner)
{
    if (dev < 0 || dev >= MAX_DEV) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_owner[dev] == owner) g_owner[dev] = nullptr;
}

}  // namespace pdhg
