#pragma once
// Grid-wide barrier of the cooperative (persistent) launches.
#include "mx_internal.h"

namespace mx {

// Grid-wide barrier for a cooperative launch.  bar[0] counts arrivals over
// the whole launch (never reset), bar[1] is the generation, bar[2] the work
// counter of the phase that ends here: the last workgroup to arrive resets
// it for the next phase before it releases the others.  A workgroup's
// generation is derived from the value its own arrival returns
// (prev / nblocks), so no separate read of bar[1] has to be ordered before
// the arrival.  Every wave first waits for its own memory operations; then
// one thread per workgroup makes the workgroup's writes visible at device
// scope (other XCDs have their own L2), arrives, polls the generation with
// plain device-scope loads (no cache invalidation per poll, which would
// evict the data of workgroups still computing on the same XCD), and
// acquires once.  The wait is bounded; returns false (every thread) after a
// time-out.  bar[0] wraps after 2^32 arrivals: far beyond one launch.
__device__ __forceinline__ bool grid_barrier(unsigned *bar, unsigned nblocks, int *err, int *sflag)
{
    __builtin_amdgcn_s_waitcnt(0);   // this wave's loads and stores have completed
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        // release fence + relaxed arrival: one L2 write-back per workgroup
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned prev = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned gen = prev / nblocks;   // barriers completed before this one
        if (prev % nblocks == nblocks - 1) {
            // the last arriver read every arrival: it acquires them before it
            // releases the next generation (so the chain of releases reaches
            // every waiter's acquire)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(&bar[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            // the generation only moves past gen once every workgroup has
            // arrived at this barrier, this one included
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1u << 25)) {   // the sleeps alone: over 1.8 s at 2.4 GHz
                    __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
        *sflag = ok;
    }
    __syncthreads();
    return *sflag != 0;
}

}  // namespace mx
