// numa_step_batch_noalloc: the batched steps of numa_step_batch with every
// item's stage scratch (stage states, element contributions, partial sums or
// the colour accumulator) taken from a static device array of the library
// instead of a caller buffer.  The kernels are numa_step_batch's; they take
// the array's device address as they take a caller's scratch.
#include <mutex>

#include "numa_internal.h"

using numa::set_error;

namespace {

constexpr uint64_t kScratchBytes = NUMA_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, at its own address on each; host code never names it
// except through HIP_SYMBOL (the name is a host-side stand-in, not a device
// address).
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char *g_addr[kMaxDevices];  // device address of scratch, per device, once looked up

// the array's address on the current device, looked up on the first call there
int32_t device_scratch(char **out, const char *fn)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("%s: hipGetDevice failed: %s", fn, hipGetErrorString(e));
        return NUMA_EDEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("%s: device %d beyond the %d the library tracks", fn, dev, kMaxDevices);
        return NUMA_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("%s: hipGetSymbolAddress of the static scratch failed on device %d: %s", fn, dev,
                      hipGetErrorString(e));
            return NUMA_EDEVICE;
        }
        g_addr[dev] = static_cast<char *>(p);
    }
    *out = g_addr[dev];
    return NUMA_OK;
}

}  // namespace

extern "C" int32_t numa_step_batch_noalloc(const numa_batch_item *items, int32_t n, int32_t prec, int32_t nsteps,
                                           void *stream)
{
    static const char fn[] = "numa_step_batch_noalloc";
    char *pool = nullptr;
    int32_t rc = device_scratch(&pool, fn);
    if (rc) return rc;
    if (nsteps == 0) return NUMA_OK;  // set-up only: the address is known from here on
    if (nsteps < 0) {
        set_error("%s: negative step count", fn);
        return NUMA_EINVAL;
    }
    if (n > NUMA_NOALLOC_MAX_ITEMS) {
        set_error("%s: %d items, at most %d per call", fn, n, NUMA_NOALLOC_MAX_ITEMS);
        return NUMA_EINVAL;
    }
    if ((rc = numa::check_batch(items, n, prec, false, fn))) return rc;
    const uint64_t need = numa::batch_pool_bytes(items, n, prec);
    if (need > kScratchBytes) {
        set_error("%s: the items need %llu bytes of scratch, the static scratch holds %llu", fn,
                  (unsigned long long)need, (unsigned long long)kScratchBytes);
        return NUMA_ENOMEM;
    }
    numa::StepItem st[5 * NUMA_NOALLOC_MAX_ITEMS];  // stages (at most 5) x items, on the stack
    return numa::run_step_batch(items, n, prec, nsteps, pool, st, reinterpret_cast<hipStream_t>(stream));
}
