// Device-wide barrier of the persistent relaxation launches (2D and 3D
// tiles): an occupancy-sized grid walks each round's active tiles and
// separates rounds with this barrier.  Its wait is bounded: a workgroup that
// waits longer than kBarrierWaitTicks (or sees another's abort) raises the
// abort word and leaves, so every wave exits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chert {

constexpr uint64_t kBarrierWaitTicks = 200000000ull;  // 2 s of the 100 MHz real-time clock

struct PersistArgs {
  int max_rounds;
  uint32_t* bar;    // [0] arrivals, [1] generation, [2] abort, [3] work tickets
  int32_t* result;  // [phase]: rounds to convergence, -1 cap reached, -2 barrier timed out,
                    // -3 the caller's abort word was raised
};

// Dynamic hand-out of a round's n_act list entries to the persistent grid:
// each workgroup draws tickets from one counter that is never reset.  A
// round issues exactly n_act + gridDim.x tickets (every workgroup stops at
// its first ticket past the list), so all workgroups advance `base` alike;
// the differences are taken modulo 2^32.  Returns the next entry, or -1.
__device__ __forceinline__ int next_item(const PersistArgs& p, uint32_t base, int n_act) {
  __shared__ uint32_t s_ticket;
  if (threadIdx.x == 0)
    s_ticket = __hip_atomic_fetch_add(&p.bar[3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const uint32_t d = s_ticket - base;
  __syncthreads();  // every thread has read the ticket before the next draw
  return d < (uint32_t)n_act ? (int)d : -1;
}

// Device-wide barrier; false if aborted.  Release before arriving and
// acquire after leaving, at agent scope (the L2s of the XCDs are not
// coherent with each other for plain accesses).
__device__ __forceinline__ bool grid_barrier(const PersistArgs& p) {
  __shared__ int s_ok;
  // every wave's stores have left it; then one agent-scope release (an L2
  // write-back of this XCD, which covers every wave of the workgroup)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    int ok = 1;
    const uint32_t gen =
        __hip_atomic_load(&p.bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t arrived =
        __hip_atomic_fetch_add(&p.bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == gridDim.x - 1) {
      __hip_atomic_store(&p.bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&p.bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&p.bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(&p.bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            wall_clock64() - t0 > kBarrierWaitTicks) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    if (!ok) __hip_atomic_store(&p.bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_ok = ok;
    __threadfence();  // acquire: invalidates this CU's L1 and this XCD's L2
  }
  __syncthreads();
  return s_ok != 0;
}

}  // namespace chert
