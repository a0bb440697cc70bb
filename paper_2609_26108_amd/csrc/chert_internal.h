// Host-side helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "chert.h"

namespace chert {

constexpr uint32_t kCacheMagic = 0x54524843u;  // 'CHRT'
constexpr uint32_t kCacheVersion = 1u;
constexpr size_t kHeaderBytes = 256;
constexpr int kMaxSweep = 4096;  // sweep table staged in LDS: 64 KiB
constexpr int kMaxRadius = 8;
constexpr int kMaxSubset = 512;  // direction columns of a subset cache
constexpr int kMaxOffsets = 288;  // (2R+1)^2 - 1 bound on |O_R| in 2D for R <= 8
constexpr int kMaxRadius3 = 4;    // 3D star radius limit
constexpr int kMaxOffsets3 = 728; // (2R+1)^3 - 1 bound on |O_R| in 3D for R <= 4
constexpr int kMaxFibonacci = 1 << 20;

// Statistics counters sharded over kStatSlots slots of 128 bytes: device-
// scope atomics on one address serialise across the chip (tens of ns each
// when thousands of workgroups hit it in a launch), so a workgroup adds into
// the slot of its index and the host reduces the slots.
constexpr int kStatSlots = 256;
constexpr int kStatSlotU64 = 16;  // counters per slot (128 bytes)
constexpr size_t kStatBytes = (size_t)kStatSlots * kStatSlotU64 * sizeof(unsigned long long);

__device__ __forceinline__ unsigned long long* stat_slot(unsigned long long* base) {
  return base + (size_t)(blockIdx.x & (kStatSlots - 1)) * kStatSlotU64;
}

// out[i] = sum over slots of counter i, or the maximum for the bits set in
// max_mask; n <= kStatSlotU64.
inline void stats_reduce(const unsigned long long* slots, int n, uint32_t max_mask,
                         unsigned long long* out) {
  for (int i = 0; i < n; ++i) {
    unsigned long long v = 0;
    for (int q = 0; q < kStatSlots; ++q) {
      const unsigned long long x = slots[(size_t)q * kStatSlotU64 + i];
      v = ((max_mask >> i) & 1u) ? (x > v ? x : v) : v + x;
    }
    out[i] = v;
  }
}

// Record a failure message for chert_last_error() and return the code.
int fail(int code, const char* msg);

// Forward star of radius R (offsets ordered by (oz, ox) ascending, primitive
// only), lengths and direction bins.  Returns the count.
int star_2d(int R, double hx, double hz, int n_dirs, int32_t* ox, int32_t* oz, double* L,
            int32_t* bin);

// Bin of one offset (x, z) != 0 under the star's rule (nearest tabulated
// direction, half-plane tie rounding); also for non-primitive offsets.
int32_t star_bin_2d(int x, int z, double hx, double hz, int n_dirs);

// Fibonacci ray directions f[3 N] (x, y, z) and the 3D forward star: offsets
// with max norm <= R, gcd 1, ordered by (oy, oz, ox); lengths; bins = the
// nearest Fibonacci direction (largest dot product, lowest index on ties).
void fibonacci(int N, double* f);
int star_3d(int R, double hx, double hy, double hz, int N, int32_t* ox, int32_t* oy, int32_t* oz,
            double* L, int32_t* bin);

// Cache column of every offset's bin (bin[o] in 0..n_dirs-1): the bin itself,
// or its position in the cache's direction subset.  INVALID_ARG when the
// subset lacks a bin.
int star_columns(const chert_cache_desc* d, const int32_t* bin, int n_off, int32_t* col);

// Node-frontier batches (frontier.hip): every 3D batch, and 2D batches run
// with CHERT_LAUNCH_FRONTIER.
inline bool is_3d_batch(const chert_trace_job* jobs, int n_jobs) {
  return jobs && n_jobs > 0 && jobs[0].g && jobs[0].g->dim == 3;
}
inline bool uses_frontier(const chert_trace_job* jobs, int n_jobs, const chert_trace_opts* o) {
  return is_3d_batch(jobs, n_jobs) || (o && o->launch == CHERT_LAUNCH_FRONTIER);
}
int trace_batch_frontier(const chert_trace_job* jobs, int n_jobs, const chert_trace_opts* o,
                         void* workspace_dev, size_t workspace_bytes, hipStream_t s);
size_t trace_batch_frontier_bytes(const chert_trace_job* jobs, int n_jobs,
                                  const chert_trace_opts* o);

// Smallest positive finite weight per field (wmin[2]) over weight tables laid
// out [2][per_field]: init once, then one call per table (frontier.hip).
int enqueue_wmin_init(double* wmin, hipStream_t s);
int enqueue_wmin(const double* W, int64_t per_field, double* wmin, hipStream_t s);

// 3D tiles for the traveltime phase of a 3D batch (tile3d.hip): one job per
// grid (class map, class-pair table [2][K][K][n_off] on the device), one
// problem per (source, field).  The star offsets are device arrays.  Runs the
// rounds to convergence on s (host checks every 8 rounds, or every round in
// one persistent launch when `persistent`); tau must hold its initial values
// (0 at the source, +inf elsewhere).
struct Tile3Job {
  int nx, ny, nz, K;
  const int32_t* cls;
  const double* W;
};
struct Tile3Prob {
  double* tau;
  int64_t src;
  int job, field;
};
int tiles3d_bytes(const Tile3Job* jobs, int n_jobs, const Tile3Prob* probs, int n_prob, int R,
                  int n_off, int tile_x, int tile_z, int max_rounds, size_t* bytes);
int relax_tiles_3d(const Tile3Job* jobs, int n_jobs, const Tile3Prob* probs, int n_prob,
                   const int32_t* ox_dev, const int32_t* oy_dev, const int32_t* oz_dev, int n_off,
                   int R, int tile_x, int tile_z, int push_group, int max_rounds, void* ws,
                   size_t ws_bytes, hipStream_t s, const volatile int32_t* abort_flag,
                   bool persistent, int* rounds, int64_t* visits, int64_t* edges);

// Raise *err if any of the n class ids lies outside [0, K) (trace.hip).
int enqueue_class_check(const int32_t* cls, int64_t n, int K, int32_t* err, hipStream_t s);

// 2D job checks shared by the tile and frontier paths (trace.hip).
int validate_job_2d(const chert_trace_job& j, uint32_t outs);
// Per-node weight table of a 2D job: W[f][j][o] = the edge j - o -> j
// (eqs 27-30), +inf off the grid or on an unusable entry (trace.hip).
int enqueue_weights_node_2d(double* W, int nx, int nz, int n_off, const int32_t* ox_dev,
                            const int32_t* oz_dev, const double* L_dev, const int32_t* col_dev,
                            int n_cols, const double* V, const double* A, const int32_t* st,
                            hipStream_t s);

// Class-pair weights W[f][ki][kj][o] (eqs 28-30) over an offset list whose
// lengths L and cache columns col live on the device; best (nullable): per
// (class, offset) column of a slowness-sampled cache, read instead of col
// (trace.hip).
int enqueue_pair_weights(double* W, int K, int n_off, const double* V, const double* A,
                         const int32_t* st, int n_cols, const double* L_dev,
                         const int32_t* col_dev, const int32_t* best, hipStream_t s);
// The closest stored ray direction of every class to every offset of a
// list (slowness-sampled caches, trace.hip).
int enqueue_slow_lookup(int32_t* best, int K, int n_cols, const double* RX, const double* RZ,
                        const int32_t* st, int n_off, const int32_t* ox_dev,
                        const int32_t* oz_dev, double hx, double hz, hipStream_t s);

// MSPM's local tables (cache_build.hip): for each job q (class job_class[q],
// or q itself when job_class is null; the job count is *n_jobs_dev times
// n_jobs_mul when n_jobs_dev is given, else n_jobs_fixed) a fresh theta_R
// sweep of n_sweep samples and one solve per target global ray angle
// psi_dev[t]: V, A, status [q][t].  grid: workgroups (one job each at a time).
int enqueue_mspm_solve(const chert_class* classes_dev, int mode, int kernel, int n_sweep,
                       const int32_t* job_class, const int32_t* n_jobs_dev, int n_jobs_mul,
                       int64_t n_jobs_fixed, int64_t grid, const double* psi_dev, int n_tgt,
                       double* V, double* A, int32_t* st, hipStream_t s);

// Kernel timing for chert_prof_*: returns a slot (or -1 when profiling is
// off) after recording a start event on the stream; prof_end records the stop.
int prof_begin(const char* name, hipStream_t s);
void prof_end(int slot, hipStream_t s);
// Turn event bracketing off (returns the previous state) and back on, around
// work that is captured into a graph.
bool prof_suspend();
void prof_resume(bool was);

}  // namespace chert

// Launch with optional event bracketing (see chert_prof_enable).
#define CHERT_LAUNCH(NAME, KERN, GRID, BLOCK, LDS, STREAM, ...)      \
  do {                                                               \
    int chert_slot_ = ::chert::prof_begin(NAME, STREAM);             \
    hipLaunchKernelGGL(KERN, GRID, BLOCK, LDS, STREAM, __VA_ARGS__); \
    ::chert::prof_end(chert_slot_, STREAM);                          \
  } while (0)
