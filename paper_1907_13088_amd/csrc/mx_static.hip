// The allocation-free stepping entry point: mx_step on a scratch area that
// is a file-scope device array of this library (one copy per GPU, held
// until the process ends) instead of a caller workspace.  Each device's
// copy has its own address, looked up once per device with that device
// current and kept; host code uses only that address, never the array's
// name (in host code the name stands for a host-side shadow, not device
// memory).
#include <atomic>

#include "mx_internal.h"

namespace {

__device__ __align__(256) char scratch[MX_STATIC_SCRATCH_BYTES];

std::atomic<void *> scratch_ptr[mx::MX_MAX_DEVICES];

}  // namespace

namespace mx {
int api_fail(int code, const char *msg);
}

extern "C" int mx_step_static(const mx_config *cfg, void *stream, void *const E[3], void *const B[3],
                              void *const J0[3], int nsteps, const double *env, const int *replay,
                              mx_step_stats *stats)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return mx::api_fail(MX_EDEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= mx::MX_MAX_DEVICES) return mx::api_fail(MX_EDEVICE, "device index out of range");
    void *p = scratch_ptr[dev].load(std::memory_order_acquire);
    if (p == nullptr) {
        // first call on this device (threads racing here look up the same address)
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return mx::api_fail(MX_EDEVICE, "the static scratch has no device address on this device");
        scratch_ptr[dev].store(p, std::memory_order_release);
    }
    return mx::step_on_scratch(cfg, stream, dev, p, MX_STATIC_SCRATCH_BYTES, E, B, J0, nsteps, env, replay, stats);
}
