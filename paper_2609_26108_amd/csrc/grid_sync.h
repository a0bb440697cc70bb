// Device-wide barrier of the persistent relaxation launches (2D and 3D
// tiles): an occupancy-sized grid walks each round's active tiles and
// separates rounds with this barrier.  Its wait is bounded: a workgroup that
// waits longer than kBarrierWaitTicks (or sees another's abort) raises the
// abort word and leaves, so every wave exits.  Also the ticket hand-out of
// a round's active tiles used by the persistent and the per-round list
// walks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chert {

constexpr uint64_t kBarrierWaitTicks = 200000000ull;  // 2 s of the 100 MHz real-time clock

// Work-ticket counters of the list walks: one 128-byte line per shard, so
// that draws spread over several addresses (atomics on one address
// serialise across the chip).
constexpr int kTickShards = 8;
constexpr int kTickStride = 32;  // 32-bit words between shards
constexpr int kTickWords = kTickShards * kTickStride;

// Round counters of a launch: [max_rounds + 2] list lengths, padded to a
// 128-byte line, then the ticket counters (all zeroed together).
__host__ __device__ inline size_t tick_offset(int max_rounds) {
  return ((size_t)max_rounds + 2 + 31) / 32 * 32;
}
__host__ __device__ inline size_t counter_words(int max_rounds) {
  return tick_offset(max_rounds) + 2 * kTickWords;  // per-round launches: by round parity
}

struct PersistArgs {
  int max_rounds;
  uint32_t* bar;    // [0] arrivals, [1] generation, [2] abort
  int32_t* result;  // [phase]: rounds to convergence, -1 cap reached, -2 barrier timed out,
                    // -3 the caller's abort word was raised
  uint32_t* tick;   // [kTickWords] zeroed before the launch, never reset during it
};

// Dynamic hand-out of a round's n_act list entries to the grid.
// The entries and workgroups are split into S = min(kTickShards, gridDim.x)
// shards by index mod S.  Within its shard a workgroup of rank r takes entry
// r first (no atomic, so a round does not start with every workgroup
// queueing on one address); when the shard has more entries than
// workgroups, each draws one ticket per entry it visits from the shard's
// counter for the remaining ones, and stops at its first ticket past them.
// Such a shard issues exactly as many tickets per round as it has entries,
// a shorter one none.  The persistent launch never resets its counters, so
// every workgroup advances its shard's `base` alike (round_tickets),
// differences taken modulo 2^32; the per-round launches use a zeroed set of
// counters per round (base 0).
struct Shard {
  int s, S, rank, workers;  // shard, shard count, rank in it, its workgroups
};
__device__ __forceinline__ Shard shard_of() {
  Shard h;
  h.S = (int)gridDim.x < kTickShards ? (int)gridDim.x : kTickShards;
  h.s = (int)blockIdx.x % h.S;
  h.rank = (int)blockIdx.x / h.S;
  h.workers = ((int)gridDim.x - h.s + h.S - 1) / h.S;
  return h;
}
__device__ __forceinline__ int shard_len(const Shard& h, int n_act) {
  return n_act > h.s ? (n_act - h.s + h.S - 1) / h.S : 0;
}
__device__ __forceinline__ int first_item(const Shard& h, int n_act) {
  return h.rank < shard_len(h, n_act) ? h.s + h.S * h.rank : -1;
}
// Thread 0 draws the ticket for the entry after the current one before
// visiting it, so the atomic's round trip overlaps the visit; ticket_item
// then turns it into that entry (or -1).  Draws happen only where the shard
// hands out tickets this round.
__device__ __forceinline__ uint32_t draw_ticket(uint32_t* tick, const Shard& h, int n_act) {
  uint32_t t = 0;
  if (threadIdx.x == 0 && shard_len(h, n_act) > h.workers)
    t = __hip_atomic_fetch_add(&tick[h.s * kTickStride], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
  return t;
}
__device__ __forceinline__ int ticket_item(const Shard& h, uint32_t base, int n_act, uint32_t t) {
  const int n = shard_len(h, n_act);
  if (n <= h.workers) return -1;  // every entry of the shard was a first one
  __shared__ uint32_t s_ticket;
  if (threadIdx.x == 0) s_ticket = t;
  __syncthreads();
  const uint32_t d = s_ticket - base;
  __syncthreads();  // every thread has read the ticket before the next one lands
  return d < (uint32_t)(n - h.workers) ? h.s + h.S * (h.workers + (int)d) : -1;
}
__device__ __forceinline__ uint32_t round_tickets(const Shard& h, int n_act) {
  const int n = shard_len(h, n_act);
  return n > h.workers ? (uint32_t)n : 0u;
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
