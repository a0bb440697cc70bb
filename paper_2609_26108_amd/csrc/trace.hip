// First-arrival traveltime fields on 2D forward-star graphs (eqs 18-19,
// 22-34; Algorithm 2, tracing) for gfx950.
//
// A call carries one or more jobs (grid + cache mode + sources).  Each
// (job, source, field) triple is an independent min-plus problem: tau_R with
// the propagation increments, tau_I with the attenuation increments (eqs 24,
// 29-31).  All problems advance together in the same launches:
//   - every grid is cut into TX x TZ tiles; a workgroup owns one (problem,
//     tile) per round, stages the tile plus an R-wide halo of the field and
//     the class ids in LDS, pulls the interior nodes within R of the halo
//     parts that changed (all of them on a full visit) over the star, then
//     runs push iterations over a compacted frontier of improved nodes
//     (LDS 64-bit atomic min) until the tile is locally converged;
//   - changed nodes within R of a tile border activate the neighbouring
//     tile for the next round with the side they changed (double-buffered
//     flags, one counter per round);
//   - rounds repeat until a round activates nothing.
// Every value ever written is the left-to-right FP64 sum along some path and
// values only decrease, so the fixed point is the minimum over paths --
// bitwise what Dijkstra computes from the same weights, for any schedule.
//
// Predecessors (eq 33) are schedule-independent: once tau is final, the
// tight edges (tau_i + w_ij == tau_j) are fixed; a second tiled relaxation
// over them takes, per node, the smallest (hop_i + 1, offset index) over
// its tight in-edges (BFS layers with eq 33's tie rule) and, on the
// propagation problems, folds t* (the attenuation increments) along the
// predecessor tree in the same pass.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "chert.h"
#include "chert_internal.h"
#include "grid_sync.h"

#pragma clang fp contract(off)

namespace chert {

constexpr int kRelaxThreads = 1024;  // one node per thread: tiles <= 1024 nodes
// threads of a tile workgroup: the tile's nodes rounded up to whole wavefronts
static inline int tile_threads(int tx, int tz) { return (tx * tz + 63) / 64 * 64; }
constexpr int kLocalIterCap = 4096;
constexpr unsigned long long kKeyUnset = ~0ull;  // tree phase: node not reached
constexpr int kFieldR = 0, kFieldI = 1;
constexpr size_t kWLdsBytes = 48 * 1024;  // class-pair table staged in LDS up to this
// Tile flag bits.  Between two visits of a tile only its halo can change
// (interior nodes are written by the owning tile alone, which leaves them
// locally converged), so a visit pulls just the R-wide border band unless a
// full pull is requested.
constexpr int kFlagActive = 1;  // a neighbour changed nodes in our halo
constexpr int kFlagFull = 2;    // pull every interior node (iteration cap hit)
constexpr int kFlagSeed = 4;    // first visit of the source tile: push the source
// bits kSideShift + s, s = (sz + 1) * 3 + (sx + 1): the halo part facing the
// neighbour at (sx, sz) changed, so the nodes within R of that side re-pull
constexpr int kSideShift = 3;
constexpr int kPullGroup = 8;  // offsets per item of a tile's distributed pull
// LDS class ids of halo cells carry this bit (push targets must be interior)
constexpr int32_t kHaloBit = 0x40000000;
constexpr int32_t kClassMask = 0x3fffffff;

struct JobDev {
  int nx, nz;     // nodes (nx * nz < 2^31)
  int ntx, ntz;   // tiles per axis
  int K;          // classes of the job's cache (class mode)
  int w_in_lds;   // stage W in LDS
  int per_node;   // cache indexed by node: weights per (node, offset)
  int pad;
  const int32_t* class_id;
  const double* W;  // class mode: [2][K][K][n_off]; per-node: [2][n_nodes][n_off],
                    // entry (j, o) = weight of the edge between j and j - o
};

// Weight of the edge i -> j = i + o (pull side: j is known; push side: i is
// known and, by symmetry, row i at the reversed offset holds the same edge).
__device__ __forceinline__ double w_pull(const JobDev& jb, const double* Wp, int field, int ki,
                                         int kj, int o, int n_off, int64_t gj) {
  if (jb.per_node)
    return jb.W[((int64_t)field * jb.nx * jb.nz + gj) * n_off + o];
  return Wp[(ki * jb.K + kj) * n_off + o];
}
__device__ __forceinline__ double w_push(const JobDev& jb, const double* Wp, int field, int ki,
                                         int kj, int o, int n_off, int64_t gi) {
  if (jb.per_node)
    return jb.W[((int64_t)field * jb.nx * jb.nz + gi) * n_off + (n_off - 1 - o)];
  return Wp[(ki * jb.K + kj) * n_off + o];
}

// Per-node weights of offsets g*G .. g*G+G-1 read from row `row` of a
// table whose rows hold the edge i -> i + o at entry n_off - 1 - o (the push
// side: row i).  The block is contiguous and, since a 2D star's size is a
// multiple of 8 and rows start 64-byte aligned, 16-byte aligned: it is read
// with 16-byte loads.  w[u] = weight of offset g*G + u.
template <int G>
__device__ __forceinline__ void row_block_rev(const double* W, int64_t row, int n_off, int g,
                                              double* w) {
  const double* p = W + row * n_off + (n_off - (g + 1) * G);
  if constexpr (G == 1) {
    w[0] = p[0];
  } else {
#pragma unroll
    for (int q = 0; q < G / 2; ++q) {
      const double2 v = reinterpret_cast<const double2*>(p)[q];
      w[G - 1 - 2 * q] = v.x;
      w[G - 2 - 2 * q] = v.y;
    }
  }
}

// The same for the pull side (row j holds the edge j - o -> j at entry o):
// w[u] = weight of offset g*G + u.
template <int G>
__device__ __forceinline__ void row_block(const double* W, int64_t row, int n_off, int g,
                                          double* w) {
  const double2* p = reinterpret_cast<const double2*>(W + row * n_off + g * G);
#pragma unroll
  for (int q = 0; q < G / 2; ++q) {
    const double2 v = p[q];
    w[2 * q] = v.x;
    w[2 * q + 1] = v.y;
  }
}

struct ProbDev {
  double* tau;     // [n_nodes] this problem's field
  unsigned long long* key;  // [n_nodes] hop << 32 | predecessor offset index
  uint32_t* tight;  // [nw][n_nodes] tight out-edge masks
  int32_t* pred;   // [n_nodes] or nullptr (no tree phase for the problem)
  double* tstar;   // [n_nodes] or nullptr (propagation problems only)
  int64_t src;
  int job;
  int field;       // 0 = propagation (w_R), 1 = attenuation (w_I)
  int tile_base;   // first global tile index of this problem
  int pad;
};

struct RelaxArgs {
  int tx, tz, R, n_off, lw, lh;
  int nw;               // 32-bit words of a tight-edge mask (n_off bits)
  int n_prob, n_tiles;  // problems, tiles over all problems
  const JobDev* jobs;
  const ProbDev* probs;
  const int32_t* ox;
  const int32_t* oz;
  int32_t* flags;    // [2][n_tiles]
  int32_t* list;     // [2][n_tiles] tiles active in a round (by round parity)
  int32_t* counter;  // [max_rounds + 2] tiles active in each round
  uint32_t* tick;    // [2][kTickWords] work tickets of the per-round list walk, by round parity
  int32_t* err;      // out-of-range class ids seen
  unsigned long long* stats;  // [kStatSlots][16] shards of: [phase][visits, edges],
                              // levels sum [6 + phase], levels max [9 + phase]
  int w_lds_doubles; // LDS room for W
  // Tile ordering (bucket > 0): a tile activated with key k (the smallest
  // value among the changed border nodes that woke it: tau, or the hop
  // count in the tree phase) is visited in a round only if k <= its problem's smallest
  // pending key + bucket * wmin (tree phase: + bucket hops); otherwise it
  // waits, still active, for a later round.
  unsigned long long* key;   // [2][n_tiles] keys (double bits) by round parity
  unsigned long long* pmin;  // [3][n_prob] smallest key per problem, by round mod 3
  const double* wmin;        // [2] smallest positive edge weight per field
  double bucket;             // 0: every active tile is visited
  // Caller's abort word (device view of pinned host memory, nullable) and
  // the device word that records it was seen: rounds after that leave at
  // once.
  const int32_t* abort_host;
  int32_t* abort_seen;
};

constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;

__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

// one tile visit of a phase: count it, the edges it examined and its push
// levels (stats layout: [phase][visits, edges], then levels sum, levels max)
__device__ __forceinline__ void count_visit(const RelaxArgs& a, int phase, long long edges,
                                            int levels) {
  if (threadIdx.x == 0) {
    unsigned long long* st = stat_slot(a.stats);
    atomicAdd(&st[2 * phase], 1ull);
    atomicAdd(&st[2 * phase + 1], (unsigned long long)edges);
    atomicAdd(&st[6 + phase], (unsigned long long)levels);
    atomicMax(&st[9 + phase], (unsigned long long)levels);
  }
}

// ------------------------------------------------------------- weights ---

__global__ void k_check_classes(const int32_t* cls, int64_t n, int K, int32_t* err);

// W[f][ki][kj][o]: eqs 28-30 in this operation order, no contraction.
// Slowness-sampled caches: column of each endpoint from `best` [K][n_off]
// (the class's closest stored ray direction, -1: none) instead of col[o].
__global__ void k_weights(double* W, int K, int n_off, const double* V, const double* A,
                          const int32_t* st, int n_cols, const double* L,
                          const int32_t* col, const int32_t* best) {
  int64_t total = 2LL * K * K * n_off;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int o = (int)(t % n_off);
    int64_t r = t / n_off;
    int kj = (int)(r % K);
    r /= K;
    int ki = (int)(r % K);
    int f = (int)(r / K);
    const int bi = best ? best[(int64_t)ki * n_off + o] : col[o];
    const int bj = best ? best[(int64_t)kj * n_off + o] : col[o];
    const int bad = CHERT_ST_NO_BRACKET | CHERT_ST_FLUID | CHERT_ST_NONPHYS | CHERT_ST_NOCONV;
    int64_t ei = (int64_t)ki * n_cols + bi, ej = (int64_t)kj * n_cols + bj;
    double w;
    if (bi < 0 || bj < 0 || (st[ei] & bad) || (st[ej] & bad)) {
      w = INFINITY;
    } else if (f == kFieldR) {
      w = __ddiv_rn(L[o], __dmul_rn(0.5, __dadd_rn(V[ei], V[ej])));
    } else {
      w = __dmul_rn(L[o], __dmul_rn(0.5, __dadd_rn(A[ei], A[ej])));
    }
    W[t] = w;
  }
}

// The closest stored ray direction of class k to offset o (text after eq
// 27): the column whose RX/RZ has the largest dot product with o's unit
// vector (IEEE operations in the order of the definition), lowest column on
// ties, skipping columns without a ray direction; -1 if none.  One thread
// per (class, offset).
__global__ void k_slow_lookup(int32_t* best, int K, int n_cols, const double* RX,
                              const double* RZ, const int32_t* st, int n_off,
                              const int32_t* ox, const int32_t* oz, double hx, double hz) {
  const int64_t total = (int64_t)K * n_off;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(t % n_off);
    const int64_t k = t / n_off;
    const double ex = __dmul_rn((double)ox[o], hx), ez = __dmul_rn((double)oz[o], hz);
    const double len = __dsqrt_rn(__dadd_rn(__dmul_rn(ex, ex), __dmul_rn(ez, ez)));
    const double dx = __ddiv_rn(ex, len), dz = __ddiv_rn(ez, len);
    int b = -1;
    double bd = 0.0;
    for (int q = 0; q < n_cols; ++q) {
      const int64_t e = k * n_cols + q;
      if (st[e] & (CHERT_ST_NO_BRACKET | CHERT_ST_FLUID)) continue;
      const double dd = __dadd_rn(__dmul_rn(RX[e], dx), __dmul_rn(RZ[e], dz));
      if (b < 0 || dd > bd) {
        b = q;
        bd = dd;
      }
    }
    best[(int64_t)k * n_off + o] = b;
  }
}

// Per-node weights: W[f][j][o] for the edge between j - o and j (eqs 28-30),
// with V, A, status indexed [node][column] and col[o] the cache column of
// the offset's bin; out-of-grid neighbours give +inf.
__global__ void k_weights_node(double* W, int nx, int nz, int n_off, const int32_t* ox,
                               const int32_t* oz, const double* L, const int32_t* col,
                               int n_cols, const double* V, const double* A,
                               const int32_t* st) {
  const int64_t n = (int64_t)nx * nz;
  const int64_t total = n * n_off;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(t % n_off);
    const int64_t j = t / n_off;
    const int jx = (int)(j % nx), jz = (int)(j / nx);
    const int ix = jx - ox[o], iz = jz - oz[o];
    double wr = INFINITY, wi = INFINITY;
    if (ix >= 0 && ix < nx && iz >= 0 && iz < nz) {
      const int64_t i = (int64_t)ix + (int64_t)nx * iz;
      const int64_t ei = i * n_cols + col[o], ej = j * n_cols + col[o];
      const int bad = CHERT_ST_NO_BRACKET | CHERT_ST_FLUID | CHERT_ST_NONPHYS | CHERT_ST_NOCONV;
      if (!(st[ei] & bad) && !(st[ej] & bad)) {
        wr = __ddiv_rn(L[o], __dmul_rn(0.5, __dadd_rn(V[ei], V[ej])));
        wi = __dmul_rn(L[o], __dmul_rn(0.5, __dadd_rn(A[ei], A[ej])));
      }
    }
    W[t] = wr;
    W[total + t] = wi;
  }
}

int enqueue_class_check(const int32_t* cls, int64_t n, int K, int32_t* err, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256 > 1024 ? 1024 : (n + 255) / 256;
  CHERT_LAUNCH("k_check_classes", k_check_classes, dim3((unsigned)(blocks < 1 ? 1 : blocks)),
               dim3(256), 0, s, cls, n, K, err);
  return CHERT_OK;
}

int enqueue_pair_weights(double* W, int K, int n_off, const double* V, const double* A,
                         const int32_t* st, int n_cols, const double* L_dev,
                         const int32_t* col_dev, const int32_t* best, hipStream_t s) {
  const int64_t tw = 2LL * K * K * n_off;
  const int64_t blocks = (tw + 255) / 256;
  CHERT_LAUNCH("k_weights", k_weights, dim3((unsigned)(blocks > 65536 ? 65536 : blocks)),
               dim3(256), 0, s, W, K, n_off, V, A, st, n_cols, L_dev, col_dev, best);
  return CHERT_OK;
}

int enqueue_slow_lookup(int32_t* best, int K, int n_cols, const double* RX, const double* RZ,
                        const int32_t* st, int n_off, const int32_t* ox_dev,
                        const int32_t* oz_dev, double hx, double hz, hipStream_t s) {
  const int64_t tl = (int64_t)K * n_off;
  const int64_t blocks = (tl + 255) / 256;
  CHERT_LAUNCH("k_slow_lookup", k_slow_lookup, dim3((unsigned)(blocks > 4096 ? 4096 : blocks)),
               dim3(256), 0, s, best, K, n_cols, RX, RZ, st, n_off, ox_dev, oz_dev, hx, hz);
  return CHERT_OK;
}

int enqueue_weights_node_2d(double* W, int nx, int nz, int n_off, const int32_t* ox_dev,
                            const int32_t* oz_dev, const double* L_dev, const int32_t* col_dev,
                            int n_cols, const double* V, const double* A, const int32_t* st,
                            hipStream_t s) {
  const int64_t tw = (int64_t)nx * nz * n_off;
  const int64_t blocks = (tw + 255) / 256;
  CHERT_LAUNCH("k_weights_node", k_weights_node, dim3((unsigned)(blocks > 65536 ? 65536 : blocks)),
               dim3(256), 0, s, W, nx, nz, n_off, ox_dev, oz_dev, L_dev, col_dev, n_cols, V, A,
               st);
  return CHERT_OK;
}

// ---------------------------------------------------------------- init ---

// First kernel of a trace: clear the error word, the counters, the phase
// results and the abort record.
__global__ void k_trace_begin(int32_t* err, unsigned long long* stats, int32_t* persist_result,
                              int32_t* abort_seen) {
  if (threadIdx.x == 0) {
    *err = 0;
    *abort_seen = 0;
  }
  if (threadIdx.x < 4) persist_result[threadIdx.x] = 0;
  for (int i = threadIdx.x; i < kStatSlots * kStatSlotU64; i += blockDim.x) stats[i] = 0ull;
}

// Class ids of a map outside [0, K): raise the error word, which every
// later kernel of the trace checks before touching an output.
__global__ void k_check_classes(const int32_t* cls, int64_t n, int K, int32_t* err) {
  bool bad = false;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k = cls[j];
    bad |= k < 0 || k >= K;
  }
  if (__ballot(bad) != 0ull && __lane_id() == 0) atomicOr(err, 1);
}

// blockIdx.y = problem; x strides over its nodes
__global__ void k_init_fields(const ProbDev* probs, const JobDev* jobs, const int32_t* err) {
  if (*err) return;  // bad class map: outputs stay untouched
  const ProbDev pr = probs[blockIdx.y];
  const int64_t n = (int64_t)jobs[pr.job].nx * jobs[pr.job].nz;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    pr.tau[j] = (j == pr.src) ? 0.0 : INFINITY;
    if (pr.key) pr.key[j] = (j == pr.src) ? 0ull : kKeyUnset;
    if (pr.tstar) pr.tstar[j] = (j == pr.src) ? 0.0 : NAN;
  }
}

__global__ void k_clear_flags(int32_t* flags, int64_t n_flags, int32_t* counter, int n_counter,
                              uint32_t* bar, unsigned long long* key, int64_t n_key,
                              unsigned long long* pmin, int n_pmin) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t t = tid; t < n_flags; t += (int64_t)gridDim.x * blockDim.x) flags[t] = 0;
  for (int64_t t = tid; t < n_counter; t += (int64_t)gridDim.x * blockDim.x) counter[t] = 0;
  for (int64_t t = tid; t < n_key; t += (int64_t)gridDim.x * blockDim.x) key[t] = kInfBits;
  for (int64_t t = tid; t < n_pmin; t += (int64_t)gridDim.x * blockDim.x) pmin[t] = kInfBits;
  if (tid < 3) bar[tid] = 0u;  // barrier arrivals, generation, abort
}

// activate the source tile of every problem (tree phase: only problems
// with predecessors)
__global__ void k_seed_flags(int32_t* flags, int32_t* list, int32_t* counter,
                             const ProbDev* probs, const JobDev* jobs, int n_prob, int tx, int tz,
                             int tree_phase, unsigned long long* key, unsigned long long* pmin,
                             const int32_t* err) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_prob || *err) return;  // bad class map: nothing runs
  const ProbDev pr = probs[p];
  if (tree_phase && pr.pred == nullptr) return;
  const JobDev jb = jobs[pr.job];
  int sx = (int)(pr.src % jb.nx), sz = (int)(pr.src / jb.nx);
  const int T = pr.tile_base + (sz / tz) * jb.ntx + (sx / tx);
  flags[T] = kFlagActive | kFlagSeed;
  list[atomicAdd(&counter[0], 1)] = T;
  key[T] = 0ull;  // the source's value: visited in round 0
  pmin[p] = 0ull;
}

// --------------------------------------------------------- tile helpers ---

struct TileCtx {
  int p, t, tx, tz;
  int x0, z0;    // first interior node
  int txe, tze;  // interior extent (ragged at the grid edge)
  int active;    // flag bits (0 = not active this round)
};

// Claim this workgroup's (problem, tile) for the round: find the problem by
// binary search over the tile bases, read and clear the tile's flag.
__device__ __forceinline__ double key_delta(const RelaxArgs& a, int phase, int field) {
  if (phase == 1) return a.bucket;  // hop counts
  const double w = a.wmin[field];
  return w < INFINITY ? a.bucket * w : INFINITY;
}

__device__ __forceinline__ TileCtx tile_begin(const RelaxArgs& a, int round, int T, int* s_flag,
                                              int* s_prob, int phase) {
  // Plain round-robin order: the active tiles of a round form a compact
  // wavefront band, and dealing consecutive tiles to different XCDs spreads
  // that band over all of them (banding tiles per XCD measured slower).
  int32_t* fin = a.flags + (int64_t)(round & 1) * a.n_tiles;
  if (threadIdx.x == 0) {
    int32_t f = fin[T];
    if (f) {
      fin[T] = 0;
      int lo = 0, hi = a.n_prob - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.probs[mid].tile_base <= T) lo = mid;
        else hi = mid - 1;
      }
      *s_prob = lo;
      if (a.bucket > 0.0) {
        unsigned long long* kin = a.key + (int64_t)(round & 1) * a.n_tiles;
        const unsigned long long k = kin[T];
        kin[T] = kInfBits;
        const double lim = __longlong_as_double((long long)a.pmin[(round % 3) * a.n_prob + lo]) +
                           key_delta(a, phase, a.probs[lo].field);
        if (!(__longlong_as_double((long long)k) <= lim)) {
          // not yet: still active next round, with the same key
          const int64_t nxt = (int64_t)((round + 1) & 1) * a.n_tiles;
          if (atomicOr(&a.flags[nxt + T], f) == 0)
            a.list[nxt + atomicAdd(&a.counter[round + 1], 1)] = T;
          atomicMin(&a.key[nxt + T], k);
          atomicMin(&a.pmin[((round + 1) % 3) * a.n_prob + lo], k);
          f = 0;
        }
      }
    }
    *s_flag = f;
  }
  __syncthreads();
  TileCtx c;
  c.active = *s_flag;
  if (!c.active) return c;
  c.p = *s_prob;
  const ProbDev& pr = a.probs[c.p];
  const JobDev& jb = a.jobs[pr.job];
  c.t = T - pr.tile_base;
  c.tx = c.t % jb.ntx;
  c.tz = c.t / jb.ntx;
  c.x0 = c.tx * a.tx;
  c.z0 = c.tz * a.tz;
  c.txe = min(a.tx, jb.nx - c.x0);
  c.tze = min(a.tz, jb.nz - c.z0);
  return c;
}

// which neighbour tiles see node (x, z) of this tile in their halo
__device__ __forceinline__ int border_bits(int x, int z, int tx, int tz, int R) {
  int m = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    bool okz = dz == 0 || (dz < 0 && z < R) || (dz > 0 && z >= tz - R);
    if (!okz) continue;
    for (int dx = -1; dx <= 1; ++dx) {
      if (dx == 0 && dz == 0) continue;
      bool okx = dx == 0 || (dx < 0 && x < R) || (dx > 0 && x >= tx - R);
      if (okx) m |= 1 << ((dz + 1) * 3 + (dx + 1));
    }
  }
  return m;
}

__device__ __forceinline__ void activate(const RelaxArgs& a, int round, const TileCtx& c,
                                         const ProbDev& pr, const JobDev& jb, int mask,
                                         unsigned long long key) {
  int32_t* fout = a.flags + (int64_t)((round + 1) & 1) * a.n_tiles;
  if (a.bucket > 0.0) {
    // this tile again (iteration cap): key 0 keeps it in the next round
    if (mask & (1 << 4)) key = 0ull;
    atomicMin(&a.pmin[((round + 1) % 3) * a.n_prob + c.p], key);
  }
  // set the flags, then reserve list slots for the newly activated tiles
  // with one atomic (the counter is one address for the whole chip)
  int fresh = 0;
  for (int bit = 0; bit < 9; ++bit) {
    if (!(mask & (1 << bit))) continue;
    int dx = bit % 3 - 1, dz = bit / 3 - 1;
    int nx_ = c.tx + dx, nz_ = c.tz + dz;
    if (nx_ < 0 || nx_ >= jb.ntx || nz_ < 0 || nz_ >= jb.ntz) continue;
    int32_t* f = &fout[pr.tile_base + nz_ * jb.ntx + nx_];
    // the neighbour's halo facing us, i.e. its side (-dx, -dz), changed
    const int32_t bits =
        (bit == 4) ? (kFlagActive | kFlagFull) : (kFlagActive | (1 << (kSideShift + 8 - bit)));
    if (a.bucket > 0.0)
      atomicMin(&a.key[(int64_t)((round + 1) & 1) * a.n_tiles + pr.tile_base + nz_ * jb.ntx + nx_],
                key);
    if (atomicOr(f, bits) == 0) fresh |= 1 << bit;
  }
  if (!fresh) return;
  int slot = atomicAdd(&a.counter[round + 1], __popc(fresh));
  for (int bit = 0; bit < 9; ++bit)
    if (fresh & (1 << bit))
      a.list[(int64_t)((round + 1) & 1) * a.n_tiles + slot++] =
          pr.tile_base + (c.tz + bit / 3 - 1) * jb.ntx + (c.tx + bit % 3 - 1);
}

// Smallest pending key of each problem for round + 2 starts over (round
// round + 1 fills it; it was last read in round - 1).  Block 0 of a round.
__device__ __forceinline__ void reset_pmin(const RelaxArgs& a, int round) {
  if (a.bucket <= 0.0) return;
  unsigned long long* pm = a.pmin + (int64_t)((round + 2) % 3) * a.n_prob;
  for (int p = threadIdx.x; p < a.n_prob; p += blockDim.x) pm[p] = kInfBits;
}

struct Smem {
  double* val;    // [lw*lh] field values
  int32_t* cls;   // [lw*lh] class ids (| kHaloBit in the halo); -1 outside, -2 bad id
  int32_t* off;   // [n_off] LDS offsets of the star
  double* W;      // staged class-pair table
  int32_t* l0;    // frontier buffers (interior LDS indices)
  int32_t* l1;
  int32_t* inq;   // [lw*lh] 1 while queued
};

__device__ __forceinline__ Smem carve(const RelaxArgs& a, void* base) {
  Smem s;
  const int n = a.lw * a.lh;
  char* p = (char*)base;
  s.val = (double*)p;
  p += sizeof(double) * n;
  s.W = (double*)p;
  p += sizeof(double) * a.w_lds_doubles;
  s.cls = (int32_t*)p;
  p += sizeof(int32_t) * n;
  s.inq = (int32_t*)p;
  p += sizeof(int32_t) * n;
  s.off = (int32_t*)p;
  p += sizeof(int32_t) * ((a.n_off + 1) & ~1);
  s.l0 = (int32_t*)p;
  p += sizeof(int32_t) * a.tx * a.tz;
  s.l1 = (int32_t*)p;
  return s;
}

static size_t lds_bytes(int lw, int lh, int w_doubles, int n_off, int tx, int tz) {
  const size_t n = (size_t)lw * lh;
  return sizeof(double) * (n + w_doubles) + sizeof(int32_t) * 2 * n +
         sizeof(int32_t) * ((n_off + 1) & ~1) + sizeof(int32_t) * 2 * tx * tz;
}

// Stage class ids and star offsets of tile + halo.
__device__ __forceinline__ void load_common(const RelaxArgs& a, const TileCtx& c, const JobDev& jb,
                                            int32_t* cls, int32_t* inq, int32_t* off) {
  const int R = a.R, lw = a.lw, n = lw * a.lh;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    int gx = c.x0 + (q % lw) - R, gz = c.z0 + (q / lw) - R;
    int32_t k = -1;
    if (gx >= 0 && gx < jb.nx && gz >= 0 && gz < jb.nz) {
      k = jb.per_node ? 0 : jb.class_id[(int64_t)gx + (int64_t)jb.nx * gz];
      if (k < 0 || k >= jb.K) {
        atomicAdd(a.err, 1);
        k = -2;
      } else {
        const int lx = q % lw - R, lz = q / lw - R;
        if (lx < 0 || lx >= c.txe || lz < 0 || lz >= c.tze) k |= kHaloBit;
      }
    }
    cls[q] = k;
    inq[q] = 0;
  }
  for (int o = threadIdx.x; o < a.n_off; o += blockDim.x) off[o] = a.ox[o] + a.oz[o] * lw;
}

__device__ __forceinline__ const double* stage_w(const RelaxArgs& a, const JobDev& jb, int field,
                                                 const Smem& s) {
  if (jb.per_node) return jb.W;  // read per (node, offset) from HBM
  const int kk = jb.K * jb.K * a.n_off;
  const double* Wf = jb.W + (int64_t)field * kk;
  if (!jb.w_in_lds) return Wf;
  for (int q = threadIdx.x; q < kk; q += blockDim.x) s.W[q] = Wf[q];
  return s.W;
}

// Wavefront-aggregated append: one LDS atomic per wavefront (ballot +
// popcount), lane slots from the mask of lower lanes.
__device__ __forceinline__ void frontier_add(bool flag, int node, int32_t* list, int* count) {
  unsigned long long b = __ballot(flag);
  if (b == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)b) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(b));
  base = __shfl(base, leader);
  if (flag) list[base + __popcll(b & ((1ull << lane) - 1ull))] = node;
}



// frontier_add for G flags per lane: one LDS atomic per wavefront for all.
template <int G>
__device__ __forceinline__ void frontier_add_n(const bool* flag, const int* node, int32_t* list,
                                               int* count) {
  unsigned long long b[G];
  int tot = 0;
#pragma unroll
  for (int u = 0; u < G; ++u) {
    b[u] = __ballot(flag[u]);
    tot += __popcll(b[u]);
  }
  if (tot == 0) return;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)__ballot(true)) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, tot);
  base = __shfl(base, leader);
  const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int u = 0; u < G; ++u) {
    if (flag[u]) list[base + __popcll(b[u] & lt)] = node[u];
    base += __popcll(b[u]);
  }
}

// Does this visit pull node ml (LDS index)?  The R-wide strips facing the
// neighbours whose halo part changed (side bits), or all on kFlagFull.
__device__ __forceinline__ bool pulls(const RelaxArgs& a, const TileCtx& c, int ml) {
  if (c.active & kFlagFull) return true;
  const int x = ml % a.lw - a.R, z = ml / a.lw - a.R;
  const bool near[2][3] = {{x < a.R, true, x >= a.tx - a.R}, {z < a.R, true, z >= a.tz - a.R}};
  const int sides = (c.active >> kSideShift) & 0x1ff;
  for (int sz = 0; sz < 3; ++sz)
    for (int sx = 0; sx < 3; ++sx)
      if (((sides >> (sz * 3 + sx)) & 1) && near[0][sx] && near[1][sz]) return true;
  return false;
}

// LDS index of the problem's source if this visit seeds it, else -1.
__device__ __forceinline__ int seed_node(const RelaxArgs& a, const TileCtx& c, int64_t src,
                                         int nx) {
  if (!(c.active & kFlagSeed)) return -1;
  const int sx = (int)(src % nx) - c.x0, sz = (int)(src / nx) - c.z0;
  if (sx < 0 || sx >= c.txe || sz < 0 || sz >= c.tze) return -1;
  return (sz + a.R) * a.lw + (sx + a.R);
}

// Global node index of LDS cell l.
__device__ __forceinline__ int64_t gnode(const RelaxArgs& a, const TileCtx& c, const JobDev& jb,
                                         int l) {
  return (int64_t)(c.x0 + l % a.lw - a.R) + (int64_t)jb.nx * (c.z0 + l / a.lw - a.R);
}

// LDS index of this thread's interior node, or -1.
__device__ __forceinline__ int my_node(const RelaxArgs& a, const TileCtx& c) {
  const int q = threadIdx.x;
  if (q >= a.tx * a.tz) return -1;
  const int x = q % a.tx, z = q / a.tx;
  if (x >= c.txe || z >= c.tze) return -1;
  return (z + a.R) * a.lw + (x + a.R);
}


// ----------------------------------------------------- relaxation phases ---

// Phase TAU: tau_j <- min(tau_j, tau_i + w_ij) (eq 31).
template <int G>
__device__ __forceinline__ void relax_tau(const RelaxArgs& a, int round, int T) {
  extern __shared__ double smem_d[];
  __shared__ int s_flag, s_prob, s_mask, s_cnt[3];
  __shared__ unsigned long long s_key;
  __shared__ int s_npull;
  const TileCtx c = tile_begin(a, round, T, &s_flag, &s_prob, 0);
  if (!c.active) return;
  const Smem s = carve(a, smem_d);
  const int R = a.R, lw = a.lw, n = lw * a.lh, n_off = a.n_off;
  const ProbDev pr = a.probs[c.p];
  const JobDev jb = a.jobs[pr.job];
  if (threadIdx.x == 0) {
    s_mask = 0;
    s_key = kInfBits;
    s_npull = 0;
    s_cnt[0] = 0;
    s_cnt[1] = 0;
    s_cnt[2] = 0;
  }
  load_common(a, c, jb, s.cls, s.inq, s.off);
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    int gx = c.x0 + (q % lw) - R, gz = c.z0 + (q / lw) - R;
    bool in = gx >= 0 && gx < jb.nx && gz >= 0 && gz < jb.nz;
    s.val[q] = in ? pr.tau[(int64_t)gx + (int64_t)jb.nx * gz] : INFINITY;
  }
  const double* Wp = stage_w(a, jb, pr.field, s);
  __syncthreads();
  const int ml = my_node(a, c);
  long long raw = 0;
  const double orig = ml >= 0 ? s.val[ml] : 0.0;

  // Pull over the border band (or every node), then seed the source.  The
  // pulled nodes' in-edges are spread over the block as items (node, group
  // of kPullGroup offsets) -- not one node's whole star per thread, which
  // kept a wavefront waiting on its few pulling lanes -- each lowering its
  // node with the 64-bit LDS atomic min; a node whose value dropped enters
  // the first frontier.  (In-neighbours lowered meanwhile enter it too.)
  {
    const bool pl = ml >= 0 && pulls(a, c, ml) && s.cls[ml] >= 0;
    if (pl) atomicAdd(&s_npull, 1);
    frontier_add(pl, ml, s.l1, &s_cnt[1]);  // l1 is free until the first level
    __syncthreads();
    const int np = s_cnt[1];
    const int npg = (n_off + kPullGroup - 1) / kPullGroup;
    const int total = np * npg;
    for (int item = threadIdx.x; item < total; item += blockDim.x) {
      const int j = s.l1[item / npg], g = item % npg;
      const int kj = s.cls[j];
      const int64_t gj = gnode(a, c, jb, j);
      double best = s.val[j];
      if (jb.per_node) {
        // the group's eight consecutive entries of row j (|O| is a multiple
        // of 8, so the group is whole)
        double wv[kPullGroup];
        row_block<kPullGroup>(jb.W, (int64_t)pr.field * jb.nx * jb.nz + gj, n_off, g, wv);
#pragma unroll
        for (int u = 0; u < kPullGroup; ++u) {
          const int o = g * kPullGroup + u;
          if (o >= n_off) break;
          const int ii = j - s.off[o];
          if (s.cls[ii] < 0) continue;
          const double cand = __dadd_rn(s.val[ii], wv[u]);
          if (cand < best) best = cand;
        }
      } else {
#pragma unroll
        for (int u = 0; u < kPullGroup; ++u) {
          const int o = g * kPullGroup + u;
          if (o >= n_off) break;
          const int ii = j - s.off[o];
          const int ki = s.cls[ii];
          if (ki < 0) continue;
          const double cand =
              __dadd_rn(s.val[ii], w_pull(jb, Wp, pr.field, ki & kClassMask, kj, o, n_off, gj));
          if (cand < best) best = cand;
        }
      }
      if (best < s.val[j]) atomicMin((unsigned long long*)&s.val[j], dbits(best));
    }
    __syncthreads();
    if (threadIdx.x == 0) s_cnt[1] = 0;  // every thread has read np
    const bool improved = pl && s.val[ml] < orig;
    if (improved) s.inq[ml] = 1;
    frontier_add(improved, ml, s.l0, &s_cnt[0]);
  }
  if (threadIdx.x == 0) {
    const int sn = seed_node(a, c, pr.src, jb.nx);
    if (sn >= 0 && s.cls[sn] >= 0 && atomicExch(&s.inq[sn], 1) != 1)
      s.l0[atomicAdd(&s_cnt[0], 1)] = sn;
  }
  __syncthreads();

  // push iterations over the frontier: one barrier per level; counters
  // rotate over three slots, the dedupe stamp is the level number
  int ci = 0, it = 1;
  int nf = s_cnt[0];
  const int ngroups = (n_off + G - 1) / G;
  const int nt = blockDim.x;
  // Work items = (frontier node, group of G offsets).  When the block
  // holds whole groups, each thread keeps one group for the whole visit
  // (its star offsets in registers) and walks the frontier in steps of
  // `per` nodes; otherwise the items rotate over the block.
  const int per = nt / ngroups;
  const int my_g = per > 0 ? (int)threadIdx.x % ngroups : 0;
  const int my_f = per > 0 ? (int)threadIdx.x / ngroups : 0;
  int offr[G];
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const int o = my_g * G + u;
    offr[u] = o < n_off ? s.off[o] : 0;
  }
  const int q_step = nt / ngroups, r_step = nt % ngroups;

  // one item; "plain read first": most pushes do not improve and skip
  // the atomic.  Per-node weights: every load of the G edges first
  // (independent chains in flight together), then the atomics, then one
  // append for all of them.
  auto push_item = [&](bool live, int i, int g, const int* offs, int32_t* lnxt, int* cnt) {
    const double vi = s.val[i];
    const int ki0 = s.cls[i];
    const int ki = ki0 >= 0 ? (ki0 & kClassMask) : 0;
    const int64_t gi = gnode(a, c, jb, i);
    if (!jb.per_node) {
      // class-pair weights in LDS: edge by edge (measured faster here than
      // batching the loads, which adds live registers)
#pragma unroll
      for (int u = 0; u < G; ++u) {
        bool improved = false;
        int jj = 0;
        const int o = g * G + u;
        if (live && o < n_off) {
          const int j = i + offs[u];
          const int kj = s.cls[j];
          if (kj >= 0 && !(kj & kHaloBit)) {
            const double cand = __dadd_rn(vi, Wp[(ki * jb.K + kj) * n_off + o]);
            if (cand < s.val[j]) {
              const unsigned long long old =
                  atomicMin((unsigned long long*)&s.val[j], dbits(cand));
              if (dbits(cand) < old) {
                improved = atomicExch(&s.inq[j], it + 1) != it + 1;
                jj = j;
              }
            }
          }
        }
        frontier_add(improved, jj, lnxt, cnt);
      }
      return;
    }
    // per-node weights from HBM: the group's G entries of row i in 16-byte
    // loads, issued before any atomic
    int jv[G];
    double cv[G];
    bool tv[G];
    double wv[G];
    if (live) row_block_rev<G>(jb.W, (int64_t)pr.field * jb.nx * jb.nz + gi, n_off, g, wv);
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int o = g * G + u;
      jv[u] = 0;
      cv[u] = 0.0;
      tv[u] = false;
      if (live && o < n_off) {
        const int j = i + offs[u];
        const int kj = s.cls[j];
        if (kj >= 0 && !(kj & kHaloBit)) {
          const double cand = __dadd_rn(vi, wv[u]);
          jv[u] = j;
          cv[u] = cand;
          tv[u] = cand < s.val[j];
        }
      }
    }
    bool imp[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      imp[u] = false;
      if (tv[u]) {
        const unsigned long long old =
            atomicMin((unsigned long long*)&s.val[jv[u]], dbits(cv[u]));
        if (dbits(cv[u]) < old) imp[u] = atomicExch(&s.inq[jv[u]], it + 1) != it + 1;
      }
    }
    frontier_add_n<G>(imp, jv, lnxt, cnt);
  };

  while (nf > 0 && it <= kLocalIterCap) {
    const int cn = ci == 2 ? 0 : ci + 1, cz = cn == 2 ? 0 : cn + 1;
    int32_t* const lcur = (it & 1) ? s.l0 : s.l1;
    int32_t* const lnxt = (it & 1) ? s.l1 : s.l0;
    if (threadIdx.x == 0) s_cnt[cz] = 0;
    raw += (long long)nf * n_off;
    const int idle = R * lw + R;  // idle lanes stand on the first interior node
    // every thread runs the same trip count so the appends see whole waves
    if (per > 0) {
      const int sweeps = (nf + per - 1) / per;
      for (int sw = 0; sw < sweeps; ++sw) {
        const int f = sw * per + my_f;
        const bool live = my_f < per && f < nf;
        push_item(live, live ? lcur[f] : idle, my_g, offr, lnxt, &s_cnt[cn]);
      }
    } else {
      const int total = nf * ngroups;
      const int bound = (total + nt - 1) / nt * nt;
      int f = threadIdx.x / ngroups, g = threadIdx.x % ngroups;
      for (int item = threadIdx.x; item < bound; item += nt) {
        const bool live = item < total;
        int offs[G];
#pragma unroll
        for (int u = 0; u < G; ++u) offs[u] = g * G + u < n_off ? s.off[g * G + u] : 0;
        push_item(live, live ? lcur[f] : idle, g, offs, lnxt, &s_cnt[cn]);
        f += q_step;
        g += r_step;
        if (g >= ngroups) {
          g -= ngroups;
          ++f;
        }
      }
    }
    __syncthreads();
    nf = s_cnt[cn];
    ci = cn;
    ++it;
  }

  int mask = (nf > 0) ? (1 << 4) : 0;  // bit 4 = this tile again
  if (ml >= 0 && s.val[ml] < orig) {
    int x = ml % lw - R, z = ml / lw - R;
    pr.tau[(int64_t)(c.x0 + x) + (int64_t)jb.nx * (c.z0 + z)] = s.val[ml];
    const int bb = border_bits(x, z, a.tx, a.tz, R);
    mask |= bb;
    if (bb && a.bucket > 0.0) atomicMin(&s_key, dbits(s.val[ml]));
  }
  count_visit(a, 0, raw + (long long)s_npull * n_off, it - 1);
  if (mask) atomicOr(&s_mask, mask);
  __syncthreads();
  if (threadIdx.x == 0 && s_mask) activate(a, round, c, pr, jb, s_mask, s_key);
}

// ------------------------------------------- predecessor tree phase ---
// Tight out-edges, once tau is final: bit (o & 31) of word o / 32 at node i
// is set when j = i + o lies in the grid, both classes are valid, tau_j is
// finite and tau_i + w_ij == tau_j (eq 33's candidate set).  The set never
// changes afterwards, so the tree phase reads neither tau nor w_R again.
// Layout [problem][word][node].  One workgroup per (problem, tile), tau and
// class ids of tile + halo staged in LDS (and the class-pair table when it
// fits), one thread per interior node; problems without predecessors leave.
__global__ void __launch_bounds__(kRelaxThreads) k_tight_out(RelaxArgs a) {
  extern __shared__ double smem_d[];
  __shared__ int s_prob;
  const int T = blockIdx.x;
  if (*a.err) return;  // bad class map: the fields were never initialised
  if (threadIdx.x == 0) {
    int lo = 0, hi = a.n_prob - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.probs[mid].tile_base <= T) lo = mid;
      else hi = mid - 1;
    }
    s_prob = lo;
  }
  __syncthreads();
  const ProbDev pr = a.probs[s_prob];
  if (!pr.pred) return;  // block-uniform
  const JobDev jb = a.jobs[pr.job];
  const int R = a.R, lw = a.lw, n = lw * a.lh, n_off = a.n_off, nw = a.nw;
  const int t = T - pr.tile_base;
  TileCtx c;
  c.p = s_prob;
  c.t = t;
  c.tx = t % jb.ntx;
  c.tz = t / jb.ntx;
  c.x0 = c.tx * a.tx;
  c.z0 = c.tz * a.tz;
  c.txe = min(a.tx, jb.nx - c.x0);
  c.tze = min(a.tz, jb.nz - c.z0);
  c.active = 1;
  const int w_lds = (!jb.per_node && jb.w_in_lds) ? jb.K * jb.K * n_off : 0;
  double* Ws = smem_d;
  double* val = Ws + a.w_lds_doubles;
  int32_t* cls = (int32_t*)(val + n);
  int32_t* off = cls + n;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const int gx = c.x0 + (q % lw) - R, gz = c.z0 + (q / lw) - R;
    double v = INFINITY;
    int32_t k = -1;
    if (gx >= 0 && gx < jb.nx && gz >= 0 && gz < jb.nz) {
      const int64_t g = (int64_t)gx + (int64_t)jb.nx * gz;
      v = pr.tau[g];
      k = jb.per_node ? 0 : jb.class_id[g];
      if (k < 0 || k >= jb.K) k = -1;
    }
    val[q] = v;
    cls[q] = k;
  }
  for (int o = threadIdx.x; o < n_off; o += blockDim.x) off[o] = a.ox[o] + a.oz[o] * lw;
  const double* Wp = jb.per_node ? jb.W : jb.W + (int64_t)pr.field * jb.K * jb.K * n_off;
  if (w_lds) {
    for (int q = threadIdx.x; q < w_lds; q += blockDim.x) Ws[q] = Wp[q];
    Wp = Ws;
  }
  __syncthreads();
  const int ml = my_node(a, c);
  if (ml < 0) return;
  const int ki = cls[ml];
  const double ti = val[ml];
  const bool ok = ki >= 0 && ti < INFINITY;
  const int64_t gi = gnode(a, c, jb, ml);
  const int64_t gn = (int64_t)jb.nx * jb.nz;
  if (jb.per_node) {
    // row i holds the edge i -> i + o at entry n_off - 1 - o: eight
    // consecutive entries (64 B) are loaded together, then tested
    for (int w = 0; w < nw; ++w) {
      uint32_t m = 0u;
      for (int b0 = 0; b0 < 32 && w * 32 + b0 < n_off; b0 += 8) {
        const int o0 = w * 32 + b0;
        double wv[8];
        if (ok) {
          row_block_rev<8>(jb.W, (int64_t)pr.field * gn + gi, n_off, o0 / 8, wv);
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u) wv[u] = INFINITY;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int o = o0 + u;
          if (o >= n_off) break;
          const int j = ml + off[o];
          const double tj = val[j];
          if (cls[j] >= 0 && tj < INFINITY && __dadd_rn(ti, wv[u]) == tj) m |= 1u << (b0 + u);
        }
      }
      pr.tight[(int64_t)w * gn + gi] = m;
    }
    return;
  }
  for (int w = 0; w < nw; ++w) {
    uint32_t m = 0u;
    for (int b = 0; ok && b < 32; ++b) {
      const int o = w * 32 + b;
      if (o >= n_off) break;
      const int j = ml + off[o];
      const int kj = cls[j];
      if (kj < 0) continue;
      const double tj = val[j];
      if (tj < INFINITY && __dadd_rn(ti, w_push(jb, Wp, pr.field, ki, kj, o, n_off, gi)) == tj)
        m |= 1u << b;
    }
    pr.tight[(int64_t)w * gn + gi] = m;
  }
}

static size_t tight_lds_bytes(int lw, int lh, int w_doubles, int n_off) {
  const size_t n = (size_t)lw * lh;
  return sizeof(double) * (w_doubles + n) + sizeof(int32_t) * (n + n_off);
}

// key of j when reached from i over offset o: (hop_i + 1, o), compared as
// one 64-bit word, so min over the tight in-edges is eq 33's choice
__device__ __forceinline__ unsigned long long tree_key(unsigned long long ki, int o) {
  return (((ki >> 32) + 1ull) << 32) | (unsigned long long)(unsigned)o;
}

struct TreeSmem {
  unsigned long long* key;  // [lw*lh] hop << 32 | predecessor offset index
  double* ts;               // [lw*lh] t* (NaN while unknown)
  uint32_t* om;             // [nw][lw*lh] tight out-masks
  int32_t* cls;
  int32_t* inq;             // (level + 1) << 1 | key changed at that level
  int32_t* off;
  int32_t* l0;              // frontiers (interior LDS indices)
  int32_t* l1;
  int32_t* lc;              // candidates of a level before the t* check
};

__device__ __forceinline__ TreeSmem carve_tree(const RelaxArgs& a, void* base) {
  TreeSmem s;
  const int n = a.lw * a.lh, T = a.tx * a.tz;
  char* p = (char*)base;
  s.key = (unsigned long long*)p;
  p += sizeof(unsigned long long) * n;
  s.ts = (double*)p;
  p += sizeof(double) * n;
  s.om = (uint32_t*)p;
  p += sizeof(uint32_t) * a.nw * n;
  s.cls = (int32_t*)p;
  p += sizeof(int32_t) * n;
  s.inq = (int32_t*)p;
  p += sizeof(int32_t) * n;
  s.off = (int32_t*)p;
  p += sizeof(int32_t) * ((a.n_off + 1) & ~1);
  s.l0 = (int32_t*)p;
  p += sizeof(int32_t) * T;
  s.l1 = (int32_t*)p;
  p += sizeof(int32_t) * T;
  s.lc = (int32_t*)p;
  return s;
}

static size_t tree_lds_bytes(int lw, int lh, int nw, int n_off, int tx, int tz) {
  const size_t n = (size_t)lw * lh;
  return (2 * sizeof(double) + sizeof(uint32_t) * nw + 2 * sizeof(int32_t)) * n +
         sizeof(int32_t) * ((n_off + 1) & ~1) + sizeof(int32_t) * 3 * tx * tz;
}

// Phase TREE: hop counts, predecessors (eq 33) and t* in one relaxation.
// key_j = min over tight in-edges i -> j of (hop_i + 1, offset index): BFS
// layers over the tight edges with eq 33's tie rule built in.  With t*,
// t*_j = t*_p + w_I(p -> j) for the predecessor p the key names; a node
// whose key or t* changed pushes to its tight children, and a child that
// the push names its predecessor again re-reads the parent's t*.  Keys only
// decrease, t* follows the (acyclic) predecessor tree, so the fixed point
// is the ordered fold along that tree for any schedule.
__device__ __forceinline__ void relax_tree(const RelaxArgs& a, int round, int T) {
  extern __shared__ double smem_d[];
  __shared__ int s_flag, s_prob, s_mask, s_cnt[3], s_cand[2];
  __shared__ unsigned long long s_key;
  __shared__ int s_npull;
  const TileCtx c = tile_begin(a, round, T, &s_flag, &s_prob, 1);
  if (!c.active) return;
  const TreeSmem s = carve_tree(a, smem_d);
  const int R = a.R, lw = a.lw, n = lw * a.lh, n_off = a.n_off, nw = a.nw;
  const ProbDev pr = a.probs[c.p];
  const JobDev jb = a.jobs[pr.job];
  const bool fold = pr.tstar != nullptr;  // block-uniform
  const int64_t gn = (int64_t)jb.nx * jb.nz;
  const double* WI = jb.per_node ? jb.W : jb.W + (int64_t)kFieldI * jb.K * jb.K * n_off;
  if (threadIdx.x == 0) {
    s_mask = 0;
    s_key = kInfBits;
    s_npull = 0;
    s_cnt[0] = 0;
    s_cnt[1] = 0;
    s_cnt[2] = 0;
    s_cand[1] = 0;
  }
  load_common(a, c, jb, s.cls, s.inq, s.off);
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    int gx = c.x0 + (q % lw) - R, gz = c.z0 + (q / lw) - R;
    bool in = gx >= 0 && gx < jb.nx && gz >= 0 && gz < jb.nz;
    int64_t g = (int64_t)gx + (int64_t)jb.nx * gz;
    s.key[q] = in ? pr.key[g] : kKeyUnset;
    s.ts[q] = (in && fold) ? pr.tstar[g] : NAN;
    for (int w = 0; w < nw; ++w) s.om[w * n + q] = in ? pr.tight[(int64_t)w * gn + g] : 0u;
  }
  __syncthreads();
  const int ml = my_node(a, c);
  long long raw = 0;
  const unsigned long long okey = ml >= 0 ? s.key[ml] : 0ull;
  const double ots = ml >= 0 ? s.ts[ml] : 0.0;

  // t*_j from the predecessor its key names; true if t*_j changed
  auto refold = [&](int j) -> bool {
    const unsigned long long k = s.key[j];
    if (k == kKeyUnset || (k >> 32) == 0ull) return false;  // unreached, or the source
    const int o = (int)(k & 0xffffffffull);
    const int p = j - s.off[o];
    const double t = __dadd_rn(s.ts[p], w_pull(jb, WI, kFieldI, s.cls[p] & kClassMask,
                                               s.cls[j] & kClassMask, o, n_off,
                                               gnode(a, c, jb, j)));
    if (dbits(t) == dbits(s.ts[j])) return false;
    s.ts[j] = t;
    return true;
  };

  // pull over the border band (or every node), then seed the source: the
  // pulled nodes' in-edges as (node, kPullGroup offsets) items over the
  // block (64-bit LDS atomic min on the key), then each pulled node
  // re-reads its t*
  {
    const bool pl = ml >= 0 && pulls(a, c, ml);
    if (pl) atomicAdd(&s_npull, 1);
    frontier_add(pl, ml, s.l1, &s_cnt[1]);  // l1 is free until the first level
    __syncthreads();
    const int np = s_cnt[1];
    const int npg = (n_off + kPullGroup - 1) / kPullGroup;
    const int total = np * npg;
    for (int item = threadIdx.x; item < total; item += blockDim.x) {
      const int j = s.l1[item / npg], g = item % npg;
      unsigned long long best = s.key[j];
#pragma unroll
      for (int u = 0; u < kPullGroup; ++u) {
        const int o = g * kPullGroup + u;
        if (o >= n_off) break;
        const int ii = j - s.off[o];
        if (!((s.om[(o >> 5) * n + ii] >> (o & 31)) & 1u)) continue;
        const unsigned long long ki = s.key[ii];
        if (ki == kKeyUnset) continue;
        const unsigned long long cand = tree_key(ki, o);
        if (cand < best) best = cand;
      }
      if (best < s.key[j]) atomicMin(&s.key[j], best);
    }
    __syncthreads();
    if (threadIdx.x == 0) s_cnt[1] = 0;  // every thread has read np
    bool changed = pl && s.key[ml] != okey;
    if (pl && fold && refold(ml)) changed = true;
    if (changed) s.inq[ml] = 2;
    frontier_add(changed, ml, s.l0, &s_cnt[0]);
  }
  if (threadIdx.x == 0) {
    const int sn = seed_node(a, c, pr.src, jb.nx);
    if (sn >= 0 && s.cls[sn] >= 0 && atomicExch(&s.inq[sn], 2) != 2)
      s.l0[atomicAdd(&s_cnt[0], 1)] = sn;
  }
  __syncthreads();

  // push levels over the tight out-edges of the frontier nodes only
  int ci = 0, it = 1;
  int nf = s_cnt[0];
  const int nt = blockDim.x;
  while (nf > 0 && it <= kLocalIterCap) {
    const int cn = ci == 2 ? 0 : ci + 1, cz = cn == 2 ? 0 : cn + 1;
    int32_t* const lcur = (it & 1) ? s.l0 : s.l1;
    int32_t* const lnxt = (it & 1) ? s.l1 : s.l0;
    // candidate counts alternate by level: the other slot was last read
    // before the previous level's final barrier
    int* const cand_cnt = &s_cand[it & 1];
    if (threadIdx.x == 0) {
      s_cnt[cz] = 0;
      s_cand[(it + 1) & 1] = 0;
    }
    const int32_t stamp = (it + 1) << 1;
    for (int b0 = 0; b0 < nf; b0 += nt) {
      const int f = b0 + (int)threadIdx.x;
      const bool live = f < nf;
      const int i = live ? lcur[f] : 0;
      const unsigned long long ki = live ? s.key[i] : kKeyUnset;
      const bool has = ki != kKeyUnset;
      // the wavefront's tight out-edges dealt one per lane: a lane's count,
      // inclusive prefix over the wavefront, then edge e goes to the lane
      // holding it (first lane whose inclusive prefix exceeds e)
      int cnt = 0;
      for (int w = 0; w < nw; ++w) cnt += has ? __popc(s.om[w * n + i]) : 0;
      const int lane = __lane_id();
      int incl = cnt;
      for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
      }
      const int excl = incl - cnt;
      const int total = __shfl(incl, 63);
      for (int e0 = 0; e0 < total; e0 += 64) {
        const int e = e0 + lane;
        int owner = 0;
        for (int step = 32; step > 0; step >>= 1)
          if (__shfl(incl, owner + step - 1) <= e) owner += step;
        owner = owner > 63 ? 63 : owner;
        const int ex_o = __shfl(excl, owner);
        const int io = __shfl(i, owner);
        const unsigned long long ko = __shfl(ki, owner);
        bool mark = false;
        int jj = 0;
        if (e < total) {
          int k = e - ex_o, o = -1;  // the owner's k-th set bit
          for (int w = 0; w < nw; ++w) {
            uint32_t m = s.om[w * n + io];
            const int pc = __popc(m);
            if (o < 0 && k < pc) {
              for (int t = 0; t < k; ++t) m &= m - 1u;
              o = w * 32 + __ffs(m) - 1;
            } else if (o < 0) {
              k -= pc;
            }
          }
          const int j = io + s.off[o];
          const int kj = s.cls[j];
          ++raw;
          if (kj >= 0 && !(kj & kHaloBit)) {
            const unsigned long long cand = tree_key(ko, o);
            if (cand < s.key[j] || (fold && cand == s.key[j])) {
              const unsigned long long old = atomicMin(&s.key[j], cand);
              if (cand < old) {
                mark = (atomicMax(&s.inq[j], stamp | 1) >> 1) != it + 1;
                jj = j;
              } else if (fold && cand == old) {
                mark = (atomicMax(&s.inq[j], stamp) >> 1) != it + 1;
                jj = j;
              }
            }
          }
        }
        if (fold) frontier_add(mark, jj, s.lc, cand_cnt);
        else frontier_add(mark, jj, lnxt, &s_cnt[cn]);
      }
    }
    __syncthreads();
    if (fold) {
      // keep the candidates whose key changed or whose t* changes
      const int nc = *cand_cnt;
      for (int b0 = 0; b0 < nc; b0 += nt) {
        const int q = b0 + (int)threadIdx.x;
        const bool live = q < nc;
        const int j = live ? s.lc[q] : 0;
        bool keep = false;
        if (live) {
          const bool kchg = (s.inq[j] & 1) != 0;
          keep = refold(j) || kchg;
        }
        frontier_add(keep, j, lnxt, &s_cnt[cn]);
      }
      __syncthreads();
    }
    nf = s_cnt[cn];
    ci = cn;
    ++it;
  }

  int mask = (nf > 0) ? (1 << 4) : 0;
  if (ml >= 0) {
    const bool kc = s.key[ml] != okey;
    const bool tc = fold && dbits(s.ts[ml]) != dbits(ots);
    if (kc || tc) {
      int x = ml % lw - R, z = ml / lw - R;
      const int64_t g = (int64_t)(c.x0 + x) + (int64_t)jb.nx * (c.z0 + z);
      if (kc) pr.key[g] = s.key[ml];
      if (tc) pr.tstar[g] = s.ts[ml];
      const int bb = border_bits(x, z, a.tx, a.tz, R);
      mask |= bb;
      if (bb && a.bucket > 0.0) atomicMin(&s_key, dbits((double)(s.key[ml] >> 32)));
    }
  }
  count_visit(a, 1, raw + (long long)s_npull * n_off, it - 1);
  if (mask) atomicOr(&s_mask, mask);
  __syncthreads();
  if (threadIdx.x == 0 && s_mask) activate(a, round, c, pr, jb, s_mask, s_key);
}

// pred_j = j - (the offset its key names); -1 for the source and unreached
// nodes.  blockIdx.y = problem.
__global__ void k_pred(RelaxArgs a) {
  const ProbDev pr = a.probs[blockIdx.y];
  if (!pr.pred || *a.err) return;
  const JobDev jb = a.jobs[pr.job];
  const int64_t n = (int64_t)jb.nx * jb.nz;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = pr.key[j];
    int32_t p = -1;
    if (k != kKeyUnset && (k >> 32) != 0ull) {
      const int o = (int)(k & 0xffffffffull);
      p = (int32_t)(j - (a.ox[o] + (int64_t)jb.nx * a.oz[o]));
    }
    pr.pred[j] = p;
  }
}

// One launch per round.  With one workgroup per tile (grid = n_tiles) tile T
// is always visited by workgroup T, so it stays on one XCD and its interior
// values from the last visit can still be in that XCD's L2; with a smaller
// grid (large batches: fewer dispatches) the workgroups walk the round's
// active-tile list.
template <int G, int PH>
__device__ __forceinline__ void visit(const RelaxArgs& a, int round, int T) {
  if constexpr (PH == 0) relax_tau<G>(a, round, T);
  else relax_tree(a, round, T);
}
// Caller's abort word, read through the system scope (pinned host memory).
__device__ __forceinline__ bool host_abort(const RelaxArgs& a) {
  return __hip_atomic_load(a.abort_host, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
}

// Per-round launches with an abort word: workgroup 0 polls the word and
// records it for the following rounds; every workgroup leaves once the
// record is set.  True if this workgroup should leave now.
__device__ __forceinline__ bool round_aborted(const RelaxArgs& a) {
  if (!a.abort_host) return false;
  __shared__ int s_ab;
  if (threadIdx.x == 0) {
    int ab = __hip_atomic_load(a.abort_seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!ab && blockIdx.x == 0 && host_abort(a)) {
      __hip_atomic_store(a.abort_seen, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ab = 1;
    }
    s_ab = ab;
  }
  __syncthreads();
  return s_ab != 0;
}

template <int G, int PH>
__device__ __forceinline__ void round_tiles(const RelaxArgs& a, int round) {
  if (round_aborted(a)) return;
  if (blockIdx.x == 0) reset_pmin(a, round);
  if ((int)gridDim.x == a.n_tiles) {
    visit<G, PH>(a, round, blockIdx.x);  // inactive tiles leave at once
    return;
  }
  const int n_act = a.counter[round];
  const int32_t* lst = a.list + (int64_t)(round & 1) * a.n_tiles;
  if constexpr (PH == 0) {
    // tau visits differ in length by tens of levels: after its first entry
    // a workgroup takes the next by ticket as it frees up.  The next
    // round's ticket lines (last used a round ago) start from zero.
    if (blockIdx.x == 0)
      for (int q = threadIdx.x; q < kTickWords; q += blockDim.x)
        a.tick[((round + 1) & 1) * kTickWords + q] = 0u;
    uint32_t* tick = a.tick + (round & 1) * kTickWords;
    const Shard sh = shard_of();
    for (int i = first_item(sh, n_act); i >= 0;) {
      const uint32_t t = draw_ticket(tick, sh, n_act);  // the next entry's, in flight meanwhile
      visit<G, PH>(a, round, lst[i]);
      __syncthreads();  // LDS is reused by the next tile
      i = ticket_item(sh, 0u, n_act, t);
    }
  } else {
    // tree visits: dealt round-robin (tickets measured slower here)
    for (int i = blockIdx.x; i < n_act; i += gridDim.x) {
      visit<G, PH>(a, round, lst[i]);
      __syncthreads();  // LDS is reused by the next tile
    }
  }
}
// LEAN: at most 64 VGPRs (8 waves per SIMD; not for G = 4, which would
// spill), so two 1024-thread tile workgroups share a compute unit.  Pays
// when rounds have far more active tiles than compute units; otherwise
// the unconstrained build runs each visit faster.
template <int G, int LEAN>
__global__ void __launch_bounds__(kRelaxThreads)
__attribute__((amdgpu_waves_per_eu(LEAN && G < 4 ? 8 : 1))) k_relax_tau(RelaxArgs a, int round) {
  round_tiles<G, 0>(a, round);
}
template <int LEAN>
__global__ void __launch_bounds__(kRelaxThreads) __attribute__((amdgpu_waves_per_eu(LEAN ? 8 : 1)))
k_relax_tree(RelaxArgs a, int round) {
  round_tiles<1, 1>(a, round);
}

// ------------------------------------------------- persistent launch ---
// All rounds of a phase in one launch: a grid no larger than the device
// holds at once walks each round's active-tile list, and rounds are
// separated by a device-wide barrier.  The barrier's wait is bounded: a
// workgroup that waits longer than kBarrierWaitTicks (or sees another's
// abort) raises the abort word and leaves, so every wave exits.

template <int G, int PH>
__global__ void __launch_bounds__(kRelaxThreads) k_relax_persist(RelaxArgs a, PersistArgs p) {
  const Shard sh = shard_of();
  uint32_t base = 0;  // tickets of this workgroup's shard issued before this round
  for (int round = 0; round < p.max_rounds; ++round) {
    if (blockIdx.x == 0) reset_pmin(a, round);
    const int n_act =
        __hip_atomic_load(&a.counter[round], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t* lst = a.list + (int64_t)(round & 1) * a.n_tiles;
    // visits differ in length by tens of levels: tiles are handed out as
    // workgroups free up rather than dealt round-robin
    for (int i = first_item(sh, n_act); i >= 0;) {
      const int T = lst[i];
      uint32_t t;
      if constexpr (PH == 0) {
        t = draw_ticket(p.tick, sh, n_act);  // the next entry's, in flight during the visit
        relax_tau<G>(a, round, T);
      } else {
        relax_tree(a, round, T);  // short visits, tight on registers: drawn after
        t = draw_ticket(p.tick, sh, n_act);
      }
      __syncthreads();  // LDS is reused by the next tile
      i = ticket_item(sh, base, n_act, t);
    }
    base += round_tickets(sh, n_act);
    // the caller's abort word, polled once per round by workgroup 0 and
    // published by the barrier below, so every workgroup leaves together
    if (a.abort_host && blockIdx.x == 0 && threadIdx.x == 0 && host_abort(a))
      __hip_atomic_store(a.abort_seen, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!grid_barrier(p)) {
      if (threadIdx.x == 0) p.result[PH] = -2;
      return;
    }
    if (a.abort_host &&
        __hip_atomic_load(a.abort_seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
      if (blockIdx.x == 0 && threadIdx.x == 0) p.result[PH] = -3;
      return;
    }
    if (__hip_atomic_load(&a.counter[round + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
        0) {
      if (blockIdx.x == 0 && threadIdx.x == 0) p.result[PH] = round + 1;
      return;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) p.result[PH] = -1;
}

// A phase run for a fixed number of per-round launches (graph capture):
// rounds to convergence (the first round that activated nothing, + 1) or
// -1 if the budget was too short.  One thread.
__global__ void k_round_count(const int32_t* counter, int max_rounds, int32_t* result,
                              const int32_t* abort_seen) {
  if (*abort_seen) {
    *result = -3;
    return;
  }
  int r = -1;
  for (int q = 1; q <= max_rounds; ++q)
    if (counter[q] == 0) {
      r = q;
      break;
    }
  *result = r;
}

// unreachable nodes: t* = +inf.  blockIdx.y = problem.
__global__ void k_tstar_finish(const ProbDev* probs, const JobDev* jobs, const int32_t* err) {
  const ProbDev pr = probs[blockIdx.y];
  if (!pr.tstar || *err) return;
  const int64_t n = (int64_t)jobs[pr.job].nx * jobs[pr.job].nz;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x)
    if (isnan(pr.tstar[j])) pr.tstar[j] = INFINITY;
}

// ----------------------------------------------------------- host side ---

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static void tile_dims(const chert_trace_opts* o, int* tx, int* tz) {
  *tx = (o && o->tile_x > 0) ? o->tile_x : 32;
  *tz = (o && o->tile_z > 0) ? o->tile_z : 32;
}

static int problems_per_source(uint32_t outs) {
  int per = 0;
  if (outs & (CHERT_OUT_TAU_R | CHERT_OUT_PRED_P | CHERT_OUT_TSTAR)) ++per;
  if (outs & (CHERT_OUT_TAU_I | CHERT_OUT_PRED_A)) ++per;
  return per;
}

struct Plan {
  int tx, tz, R, n_off, lw, lh, nw;
  int n_prob = 0;
  int64_t n_tiles = 0;
  int max_rounds = 0;
  std::vector<int64_t> nodes;  // per job
  std::vector<int> ntx, ntz, K;
  size_t off_star = 0, off_lbin = 0, off_jobs = 0, off_probs = 0, off_flags = 0, off_list = 0,
         off_counter = 0, off_key = 0, off_pmin = 0, off_wmin = 0,
         off_err = 0, off_stats = 0, off_nkey = 0, off_tight = 0, total = 0;
  std::vector<size_t> off_W;  // per job
  std::vector<size_t> off_best;  // per job: closest-direction table (slowness caches)
  int w_lds_doubles = 0;
};

int validate_job_2d(const chert_trace_job& j, uint32_t outs) {
  chert_cache_layout lay;
  int rc = chert_cache_layout_of(j.d, j.n_classes, &lay);
  if (rc) return rc;
  const chert_grid* g = j.g;
  if (!g) return fail(CHERT_ERR_INVALID_ARG, "null grid");
  if (g->dim == 3) return fail(CHERT_ERR_INVALID_ARG, "2D and 3D jobs cannot share a batch");
  if (g->dim != 2 || g->ny != 1) return fail(CHERT_ERR_INVALID_ARG, "2D grid needs dim 2, ny 1");
  if (g->nx < 1 || g->nz < 1 || g->nx * g->nz >= 0x7fffffffLL)
    return fail(CHERT_ERR_INVALID_ARG, "grid size out of range");
  if (g->radius < 1 || g->radius > kMaxRadius)
    return fail(CHERT_ERR_INVALID_ARG, "radius must be 1..8");
  if (!(g->hx > 0.0) || !(g->hz > 0.0) || !isfinite(g->hx) || !isfinite(g->hz))
    return fail(CHERT_ERR_INVALID_ARG, "spacing must be positive");
  if (!g->class_id_dev && j.n_classes != g->nx * g->nz)
    return fail(CHERT_ERR_INVALID_ARG, "no class map: the cache must hold one class per node");
  if (j.mode < 0 || j.mode > 2 || !(j.d->mode_mask & (1u << j.mode)))
    return fail(CHERT_ERR_INVALID_ARG, "mode not in the cache");
  if (j.d->sampling == CHERT_SAMPLE_SLOWNESS && !g->class_id_dev)
    return fail(CHERT_ERR_UNSUPPORTED, "slowness-sampled caches are class caches");
  if (j.n_src < 1) return fail(CHERT_ERR_INVALID_ARG, "need at least one source");
  if (!j.cache_dev) return fail(CHERT_ERR_INVALID_ARG, "null cache");
  if (!j.src_nodes_host) return fail(CHERT_ERR_INVALID_ARG, "null sources");
  const int64_t n = g->nx * g->nz;
  for (int i = 0; i < j.n_src; ++i)
    if (j.src_nodes_host[i] < 0 || j.src_nodes_host[i] >= n)
      return fail(CHERT_ERR_INVALID_ARG, "source node out of range");
  if (((outs & CHERT_OUT_TAU_R) && !j.tau_r_dev) || ((outs & CHERT_OUT_TAU_I) && !j.tau_i_dev) ||
      ((outs & CHERT_OUT_TSTAR) && !j.tstar_dev) || ((outs & CHERT_OUT_PRED_P) && !j.pred_p_dev) ||
      ((outs & CHERT_OUT_PRED_A) && !j.pred_a_dev))
    return fail(CHERT_ERR_INVALID_ARG, "a selected output is NULL");
  // the tile kernels index a field's class-pair table [K][K][n_off] in 32 bits
  const int64_t n_off = star_2d(g->radius, 1.0, 1.0, 4, nullptr, nullptr, nullptr, nullptr);
  if (g->class_id_dev && (int64_t)j.n_classes * j.n_classes * n_off >= ((int64_t)1 << 31))
    return fail(CHERT_ERR_UNSUPPORTED, "class-pair table too large (use one class per node)");
  return CHERT_OK;
}

static int validate_opts(const chert_trace_opts* o) {
  if (!o) return fail(CHERT_ERR_INVALID_ARG, "null options");
  if (o->push_group != 0 && o->push_group != 1 && o->push_group != 2 && o->push_group != 4 &&
      o->push_group != 8)
    return fail(CHERT_ERR_INVALID_ARG, "push_group must be 0, 1, 2, 4 or 8");
  if (o->launch != CHERT_LAUNCH_PER_ROUND && o->launch != CHERT_LAUNCH_PERSISTENT)
    return fail(CHERT_ERR_INVALID_ARG, "launch must be CHERT_LAUNCH_PER_ROUND or _PERSISTENT");
  if (!(o->bucket_width >= 0.0) || !isfinite(o->bucket_width))
    return fail(CHERT_ERR_INVALID_ARG, "bucket_width must be finite and >= 0");
  uint32_t outs = o->outputs;
  if (outs == 0 || (outs & ~31u)) return fail(CHERT_ERR_INVALID_ARG, "bad output mask");
  if ((outs & CHERT_OUT_TSTAR) && !((outs & CHERT_OUT_TAU_R) && (outs & CHERT_OUT_PRED_P)))
    return fail(CHERT_ERR_INVALID_ARG, "TSTAR needs TAU_R and PRED_P");
  if ((outs & CHERT_OUT_PRED_P) && !(outs & CHERT_OUT_TAU_R))
    return fail(CHERT_ERR_INVALID_ARG, "PRED_P needs TAU_R");
  if ((outs & CHERT_OUT_PRED_A) && !(outs & CHERT_OUT_TAU_I))
    return fail(CHERT_ERR_INVALID_ARG, "PRED_A needs TAU_I");
  return CHERT_OK;
}

static int make_plan(const chert_trace_job* jobs, int n_jobs, const chert_trace_opts* o,
                     Plan* P) {
  if (!jobs || n_jobs < 1) return fail(CHERT_ERR_INVALID_ARG, "need at least one job");
  int rc = validate_opts(o);
  if (rc) return rc;
  for (int j = 0; j < n_jobs; ++j) {
    rc = validate_job_2d(jobs[j], o->outputs);
    if (rc) return rc;
    if (jobs[j].g->radius != jobs[0].g->radius)
      return fail(CHERT_ERR_INVALID_ARG, "all jobs of a batch need the same radius");
  }
  tile_dims(o, &P->tx, &P->tz);
  P->R = jobs[0].g->radius;
  if (P->tx < P->R || P->tz < P->R || P->tx * P->tz > kRelaxThreads)
    return fail(CHERT_ERR_INVALID_ARG, "tile must be >= radius per side and <= 1024 nodes");
  P->n_off = star_2d(P->R, 1.0, 1.0, 4, nullptr, nullptr, nullptr, nullptr);
  // the star is symmetric under the square's eight symmetries, so |O| is a
  // multiple of 8; the per-node kernels read whole 8-offset groups
  if (P->n_off % 8) return fail(CHERT_ERR_UNSUPPORTED, "forward star size not a multiple of 8");
  P->nw = (P->n_off + 31) / 32;
  P->lw = P->tx + 2 * P->R;
  P->lh = P->tz + 2 * P->R;
  const int per = problems_per_source(o->outputs);
  int64_t max_tile_span = 0, tree_nodes = 0;
  const int tree_per = ((o->outputs & CHERT_OUT_PRED_P) ? 1 : 0) + ((o->outputs & CHERT_OUT_PRED_A) ? 1 : 0);
  int w_lds = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const chert_grid* g = jobs[j].g;
    int ntx = (int)((g->nx + P->tx - 1) / P->tx), ntz = (int)((g->nz + P->tz - 1) / P->tz);
    P->ntx.push_back(ntx);
    P->ntz.push_back(ntz);
    P->K.push_back((int)jobs[j].n_classes);
    P->nodes.push_back(g->nx * g->nz);
    int np = per * jobs[j].n_src;
    P->n_prob += np;
    P->n_tiles += (int64_t)np * ntx * ntz;
    tree_nodes += (int64_t)tree_per * jobs[j].n_src * g->nx * g->nz;
    if (ntx + ntz > max_tile_span) max_tile_span = ntx + ntz;
    if (g->class_id_dev) {
      size_t wf = (size_t)jobs[j].n_classes * jobs[j].n_classes * P->n_off * sizeof(double);
      if (wf <= kWLdsBytes && (int)(wf / sizeof(double)) > w_lds)
        w_lds = (int)(wf / sizeof(double));
    }
  }
  if (P->n_tiles >= 0x7fffffffLL || P->n_prob > 65535)
    return fail(CHERT_ERR_UNSUPPORTED, "batch too large for one launch");
  P->w_lds_doubles = w_lds;
  // ordered tiles wait for their turn: more rounds, fewer visits
  P->max_rounds = (o->max_rounds > 0)
                      ? o->max_rounds
                      : 1024 + 64 * (int)max_tile_span + (o->bucket_width > 0.0 ? 8192 : 0);
  size_t off = 0;
  P->off_star = off;
  off += align256((size_t)kMaxOffsets * 2 * sizeof(int32_t));
  P->off_lbin = off;
  off += align256((size_t)n_jobs * kMaxOffsets * (sizeof(double) + 2 * sizeof(int32_t)));
  P->off_jobs = off;
  off += align256((size_t)n_jobs * sizeof(JobDev));
  P->off_probs = off;
  off += align256((size_t)P->n_prob * sizeof(ProbDev));
  P->off_flags = off;
  off += align256((size_t)2 * P->n_tiles * sizeof(int32_t));
  P->off_list = off;
  off += align256((size_t)2 * P->n_tiles * sizeof(int32_t));
  P->off_counter = off;
  off += align256(counter_words(P->max_rounds) * sizeof(int32_t));  // counts, tickets
  P->off_key = off;
  off += align256((size_t)2 * P->n_tiles * sizeof(uint64_t));
  P->off_pmin = off;
  off += align256((size_t)3 * P->n_prob * sizeof(uint64_t));
  P->off_wmin = off;
  off += 256;
  P->off_err = off;
  off += 256;
  P->off_stats = off;
  off += align256(kStatBytes);
  for (int j = 0; j < n_jobs; ++j) {
    P->off_best.push_back(off);
    if (jobs[j].d->sampling == CHERT_SAMPLE_SLOWNESS)
      off += align256((size_t)jobs[j].n_classes * P->n_off * sizeof(int32_t));
    P->off_W.push_back(off);
    const size_t rows = jobs[j].g->class_id_dev
                            ? (size_t)jobs[j].n_classes * jobs[j].n_classes
                            : (size_t)jobs[j].g->nx * jobs[j].g->nz;
    off += align256((size_t)2 * rows * P->n_off * sizeof(double));
  }
  P->off_nkey = off;
  off += align256((size_t)tree_nodes * sizeof(unsigned long long));
  P->off_tight = off;
  off += align256((size_t)tree_nodes * P->nw * sizeof(uint32_t));
  P->total = off;
  return CHERT_OK;
}

// Rounds go out in groups between host checks of the round counters:
// 16, then 32, then 64 at a time (a converged phase's extra launches find
// no active tile and leave at once; each check costs a stream drain).
static int run_rounds(hipStream_t s, const RelaxArgs& a, void (*kern)(RelaxArgs, int),
                      const char* name, int grid, size_t lds, int max_rounds,
                      const volatile int32_t* abort_flag, int* rounds) {
  constexpr int kMaxBatch = 64;
  int32_t counts[kMaxBatch];
  int batch = 16;
  for (int r = 0; r < max_rounds; r += batch, batch = std::min(2 * batch, kMaxBatch)) {
    int nb = batch;
    if (r + nb > max_rounds) nb = max_rounds - r;
    for (int q = 0; q < nb; ++q)
      CHERT_LAUNCH(name, kern, dim3((unsigned)grid), dim3((unsigned)tile_threads(a.tx, a.tz)), lds,
                   s, a, r + q);
    int32_t seen = 0;
    hipError_t e = hipMemcpyAsync(counts, a.counter + r + 1, sizeof(int32_t) * nb,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && abort_flag)
      e = hipMemcpyAsync(&seen, a.abort_seen, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
    // rounds the kernels skipped after seeing the word activate nothing, so
    // the word is checked before the counts
    if (abort_flag && (seen || *abort_flag)) {
      *rounds = r + nb;
      return fail(CHERT_ERR_ABORTED, "aborted by the caller");
    }
    for (int q = 0; q < nb; ++q)
      if (counts[q] == 0) {
        *rounds = r + q + 1;
        return CHERT_OK;
      }
  }
  *rounds = max_rounds;
  return fail(CHERT_ERR_NO_CONVERGENCE, "relaxation round cap reached");
}

typedef void (*RoundKern)(RelaxArgs, int);
typedef void (*PersistKern)(RelaxArgs, PersistArgs);

static RoundKern round_kernel(int ph, int G, bool lean) {
  if (ph == 0) {
    if (lean)
      return G == 1 ? k_relax_tau<1, 1>
                    : (G == 2 ? k_relax_tau<2, 1> : (G == 4 ? k_relax_tau<4, 1> : k_relax_tau<8, 1>));
    return G == 1 ? k_relax_tau<1, 0>
                  : (G == 2 ? k_relax_tau<2, 0> : (G == 4 ? k_relax_tau<4, 0> : k_relax_tau<8, 0>));
  }
  return lean ? k_relax_tree<1> : k_relax_tree<0>;  // one lane per frontier node: no push groups
}

static PersistKern persist_kernel(int ph, int G) {
  if (ph == 0)
    return G == 1 ? k_relax_persist<1, 0>
                  : (G == 2 ? k_relax_persist<2, 0>
                            : (G == 4 ? k_relax_persist<4, 0> : k_relax_persist<8, 0>));
  return k_relax_persist<1, 1>;  // tree phase: no push groups
}

// Persistent-launch grid: as many workgroups as the device holds at once
// (never more than the tiles), so every workgroup of the launch is resident.
static int persist_grid(const void* kern, int threads, size_t lds, int64_t n_tiles, int* grid) {
  int per_cu = 0, cus = 0, dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds);
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  if (per_cu < 1) return fail(CHERT_ERR_HIP, "relaxation kernel does not fit on a compute unit");
  int64_t g = (int64_t)per_cu * cus;
  if (g > n_tiles) g = n_tiles;
  *grid = (int)(g < 1 ? 1 : g);
  return CHERT_OK;
}

// A batch ready to run: plan, device tables uploaded, kernel arguments.
struct Prepared {
  Plan P;
  RelaxArgs a{};
  PersistArgs pa{};
  size_t lds[2] = {0, 0};  // dynamic LDS per phase (tau, tree)
  uint8_t* ws = nullptr;
  JobDev* djobs = nullptr;
  ProbDev* dprobs = nullptr;
  std::vector<JobDev> jd;
  int32_t* dox = nullptr;
  int32_t* doz = nullptr;
  double* dL = nullptr;
  int32_t* dcol = nullptr;
  int pgrid[2] = {0, 0};  // persistent-launch grid per phase
  int rgrid[2] = {0, 0};  // per-round launch grid per phase
  bool fixed_rounds = false;  // per-round launches without host checks (graphs)
  bool lean = false;          // occupancy-limited kernel builds (large batches)
};

// Plan the batch and upload its tables (synchronous on s).
static int prepare(const chert_trace_job* jobs, int n_jobs, const chert_trace_opts* o,
                   void* workspace_dev, size_t workspace_bytes, hipStream_t s, Prepared* Q) {
  Plan& P = Q->P;
  int rc = make_plan(jobs, n_jobs, o, &P);
  if (rc) return rc;
  if (!workspace_dev || workspace_bytes < P.total)
    return fail(CHERT_ERR_INVALID_ARG, "workspace too small");
  uint8_t* ws = (uint8_t*)workspace_dev;
  const uint32_t outs = o->outputs;

  // forward star (shared offsets) and per-job lengths/bins on the host
  std::vector<int32_t> star(2 * kMaxOffsets);
  std::vector<uint8_t> lbin((size_t)n_jobs * kMaxOffsets * (sizeof(double) + 2 * sizeof(int32_t)));
  double* hL = (double*)lbin.data();
  int32_t* hbin = (int32_t*)(hL + (size_t)n_jobs * kMaxOffsets);
  int32_t* hcol = hbin + (size_t)n_jobs * kMaxOffsets;
  for (int j = 0; j < n_jobs; ++j) {
    const chert_grid* g = jobs[j].g;
    const chert_cache_desc* d = jobs[j].d;
    star_2d(P.R, g->hx, g->hz, d->n_dirs, star.data(), star.data() + kMaxOffsets,
            hL + (size_t)j * kMaxOffsets, hbin + (size_t)j * kMaxOffsets);
    rc = star_columns(d, hbin + (size_t)j * kMaxOffsets, P.n_off, hcol + (size_t)j * kMaxOffsets);
    if (rc) return rc;
  }
  int32_t* dox = (int32_t*)(ws + P.off_star);
  int32_t* doz = dox + kMaxOffsets;
  double* dL = (double*)(ws + P.off_lbin);
  int32_t* dbin = (int32_t*)(dL + (size_t)n_jobs * kMaxOffsets);
  int32_t* dcol = dbin + (size_t)n_jobs * kMaxOffsets;
  (void)dbin;

  std::vector<JobDev>& jd = Q->jd;
  jd.assign(n_jobs, JobDev{});
  std::vector<ProbDev> probs;
  unsigned long long* nkey = (unsigned long long*)(ws + P.off_nkey);
  uint32_t* tight = (uint32_t*)(ws + P.off_tight);
  int64_t tree_off = 0;  // nodes of the tree-phase problems so far
  int tile_base = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const chert_trace_job& J = jobs[j];
    JobDev& d = jd[j];
    d.nx = (int)J.g->nx;
    d.nz = (int)J.g->nz;
    d.ntx = P.ntx[j];
    d.ntz = P.ntz[j];
    d.per_node = J.g->class_id_dev ? 0 : 1;
    d.K = d.per_node ? 1 : P.K[j];
    size_t wf = (size_t)d.K * d.K * P.n_off;
    d.w_in_lds = (!d.per_node && wf <= (size_t)P.w_lds_doubles) ? 1 : 0;
    d.class_id = J.g->class_id_dev;
    d.W = (const double*)(ws + P.off_W[j]);
    const int64_t n = P.nodes[j];
    const int ntiles = d.ntx * d.ntz;
    for (int i = 0; i < J.n_src; ++i) {
      if (outs & (CHERT_OUT_TAU_R | CHERT_OUT_PRED_P | CHERT_OUT_TSTAR)) {
        ProbDev p{};
        p.tau = J.tau_r_dev + (int64_t)i * n;
        p.pred = (outs & CHERT_OUT_PRED_P) ? J.pred_p_dev + (int64_t)i * n : nullptr;
        p.tstar = (outs & CHERT_OUT_TSTAR) ? J.tstar_dev + (int64_t)i * n : nullptr;
        p.src = J.src_nodes_host[i];
        p.job = j;
        p.field = kFieldR;
        p.tile_base = tile_base;
        if (p.pred) {
          p.key = nkey + tree_off;
          p.tight = tight + tree_off * P.nw;
          tree_off += n;
        }
        tile_base += ntiles;
        probs.push_back(p);
      }
      if (outs & (CHERT_OUT_TAU_I | CHERT_OUT_PRED_A)) {
        ProbDev p{};
        p.tau = J.tau_i_dev + (int64_t)i * n;
        p.pred = (outs & CHERT_OUT_PRED_A) ? J.pred_a_dev + (int64_t)i * n : nullptr;
        p.tstar = nullptr;
        p.src = J.src_nodes_host[i];
        p.job = j;
        p.field = kFieldI;
        p.tile_base = tile_base;
        if (p.pred) {
          p.key = nkey + tree_off;
          p.tight = tight + tree_off * P.nw;
          tree_off += n;
        }
        tile_base += ntiles;
        probs.push_back(p);
      }
    }
  }
  JobDev* djobs = (JobDev*)(ws + P.off_jobs);
  ProbDev* dprobs = (ProbDev*)(ws + P.off_probs);
  // the star, lengths/bins, job and problem tables lie in order at the
  // start of the workspace: one upload for all four
  std::vector<uint8_t> up(P.off_probs + probs.size() * sizeof(ProbDev), 0);
  memcpy(up.data() + P.off_star, star.data(), star.size() * sizeof(int32_t));
  memcpy(up.data() + P.off_lbin, lbin.data(), lbin.size());
  memcpy(up.data() + P.off_jobs, jd.data(), jd.size() * sizeof(JobDev));
  memcpy(up.data() + P.off_probs, probs.data(), probs.size() * sizeof(ProbDev));
  hipError_t e = hipMemcpyAsync(ws, up.data(), up.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host buffer is a local
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));

  RelaxArgs& a = Q->a;
  a.tx = P.tx;
  a.tz = P.tz;
  a.R = P.R;
  a.n_off = P.n_off;
  a.nw = P.nw;
  a.lw = P.lw;
  a.lh = P.lh;
  a.n_prob = P.n_prob;
  a.n_tiles = (int)P.n_tiles;
  a.jobs = djobs;
  a.probs = dprobs;
  a.ox = dox;
  a.oz = doz;
  a.flags = (int32_t*)(ws + P.off_flags);
  a.list = (int32_t*)(ws + P.off_list);
  a.counter = (int32_t*)(ws + P.off_counter);
  a.err = (int32_t*)(ws + P.off_err);
  a.stats = (unsigned long long*)(ws + P.off_stats);
  a.w_lds_doubles = P.w_lds_doubles;
  a.key = (unsigned long long*)(ws + P.off_key);
  a.pmin = (unsigned long long*)(ws + P.off_pmin);
  a.wmin = (const double*)(ws + P.off_wmin);
  a.bucket = o->bucket_width;
  a.abort_seen = (int32_t*)(ws + P.off_err + 224);
  a.abort_host = nullptr;
  if (o->abort_flag_host) {
    // only page-locked host memory the device can read is accepted
    hipPointerAttribute_t at{};
    const hipError_t pe = hipPointerGetAttributes(&at, (const void*)o->abort_flag_host);
    if (pe != hipSuccess || at.type != hipMemoryTypeHost || !at.devicePointer) {
      (void)hipGetLastError();
      return fail(CHERT_ERR_INVALID_ARG, "abort_flag_host must be pinned host memory");
    }
    a.abort_host = (const int32_t*)at.devicePointer;
  }
  Q->lds[0] = lds_bytes(P.lw, P.lh, P.w_lds_doubles, P.n_off, P.tx, P.tz);
  Q->lds[1] = tree_lds_bytes(P.lw, P.lh, P.nw, P.n_off, P.tx, P.tz);
  Q->pa.max_rounds = P.max_rounds;
  Q->pa.bar = (uint32_t*)(ws + P.off_err + 192);
  Q->pa.result = (int32_t*)(ws + P.off_err + 208);
  Q->pa.tick = (uint32_t*)(ws + P.off_counter) + tick_offset(P.max_rounds);
  Q->a.tick = Q->pa.tick;
  Q->ws = ws;
  Q->djobs = djobs;
  Q->dprobs = dprobs;
  Q->dox = dox;
  Q->doz = doz;
  Q->dL = dL;
  Q->dcol = dcol;
  const int G = o->push_group ? o->push_group : 2;
  {
    int dev = 0, cus = 0;
    hipError_t e2 = hipGetDevice(&dev);
    if (e2 == hipSuccess)
      e2 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e2 != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e2));
    Q->lean = P.n_tiles > 8 * (int64_t)cus;
  }
  for (int ph = 0; ph < 2; ++ph) {
    if (o->launch == CHERT_LAUNCH_PERSISTENT)
      rc = persist_grid((const void*)persist_kernel(ph, G), tile_threads(P.tx, P.tz), Q->lds[ph],
                        P.n_tiles, &Q->pgrid[ph]);
    else
      rc = persist_grid((const void*)round_kernel(ph, G, Q->lean), tile_threads(P.tx, P.tz), Q->lds[ph],
                        P.n_tiles, &Q->rgrid[ph]);
    if (rc) return rc;
    // per-round launches: one workgroup per tile (tile affinity) while that
    // is at most 4x the resident workgroups (tree phase: 8x), else a list
    // walk by twice the resident workgroups for the tau phase, whose tiles
    // go out by ticket, and eight times for the tree phase, dealt
    // round-robin and balanced by the dispatcher
    const int64_t res = Q->rgrid[ph];
    if (ph == 0)
      Q->rgrid[ph] = (int)(P.n_tiles <= 4 * res ? P.n_tiles : 2 * res);
    else
      Q->rgrid[ph] = (int)std::min<int64_t>(P.n_tiles, 8 * res);
  }
  return CHERT_OK;
}


// Enqueue every kernel of a prepared batch on s.  With the persistent
// launch nothing here waits for the device, so the sequence can be captured
// into a graph; the per-round launch synchronises s every 8 rounds to test
// for termination.
static int enqueue(const Prepared& Q, const chert_trace_job* jobs, int n_jobs,
                   const chert_trace_opts* o, hipStream_t s, int rounds[3]) {
  const Plan& P = Q.P;
  const RelaxArgs& a = Q.a;
  const PersistArgs& pa = Q.pa;
  uint8_t* ws = Q.ws;
  const uint32_t outs = o->outputs;
  CHERT_LAUNCH("k_trace_begin", k_trace_begin, dim3(1), dim3(64), 0, s, a.err, a.stats, pa.result,
               a.abort_seen);
  for (int j = 0; j < n_jobs; ++j)
    if (!Q.jd[j].per_node) enqueue_class_check(Q.jd[j].class_id, P.nodes[j], Q.jd[j].K, a.err, s);
  for (int j = 0; j < n_jobs; ++j) {
    const chert_trace_job& J = jobs[j];
    chert_cache_layout lay;
    chert_cache_layout_of(J.d, J.n_classes, &lay);
    const uint8_t* cache = (const uint8_t*)J.cache_dev;
    const int64_t K = J.n_classes;
    const int n_cols = J.d->n_subset ? J.d->n_subset : J.d->n_dirs;
    const int64_t ent = 3 * K * (int64_t)n_cols;
    const int64_t mslice = (int64_t)J.mode * K * n_cols;
    const double* fields = (const double*)(cache + lay.fields_offset);
    const double* Vm = fields + CHERT_F_V * ent + mslice;
    const double* Am = fields + CHERT_F_A * ent + mslice;
    const int32_t* Sm = (const int32_t*)(cache + lay.status_offset) + mslice;
    if (Q.jd[j].per_node) {
      int rc = enqueue_weights_node_2d((double*)(ws + P.off_W[j]), Q.jd[j].nx, Q.jd[j].nz,
                                       P.n_off, Q.dox, Q.doz, Q.dL + (size_t)j * kMaxOffsets,
                                       Q.dcol + (size_t)j * kMaxOffsets, n_cols, Vm, Am, Sm, s);
      if (rc) return rc;
    } else {
      const int32_t* best = nullptr;
      if (J.d->sampling == CHERT_SAMPLE_SLOWNESS) {
        const double* RXm = fields + CHERT_F_RX * ent + mslice;
        const double* RZm = fields + CHERT_F_RZ * ent + mslice;
        int32_t* bt = (int32_t*)(ws + P.off_best[j]);
        const int64_t tl = K * P.n_off;
        CHERT_LAUNCH("k_slow_lookup", k_slow_lookup,
                     dim3((unsigned)((tl + 255) / 256 > 4096 ? 4096 : (tl + 255) / 256)), dim3(256),
                     0, s, bt, (int)K, n_cols, RXm, RZm, Sm, P.n_off, (const int32_t*)Q.dox,
                     (const int32_t*)Q.doz, J.g->hx, J.g->hz);
        best = bt;
      }
      int64_t tw = 2 * K * K * P.n_off;
      int64_t blocks = (tw + 255) / 256;
      CHERT_LAUNCH("k_weights", k_weights, dim3((unsigned)(blocks > 65536 ? 65536 : blocks)),
                   dim3(256), 0, s, (double*)(ws + P.off_W[j]), (int)K, P.n_off, Vm, Am, Sm,
                   n_cols, Q.dL + (size_t)j * kMaxOffsets, Q.dcol + (size_t)j * kMaxOffsets, best);
    }
  }
  if (a.bucket > 0.0) {  // the ordering's unit: smallest edge weight per field
    enqueue_wmin_init((double*)a.wmin, s);
    for (int j = 0; j < n_jobs; ++j) {
      const int64_t rows = Q.jd[j].per_node ? P.nodes[j] : (int64_t)Q.jd[j].K * Q.jd[j].K;
      enqueue_wmin((const double*)(ws + P.off_W[j]), rows * P.n_off, (double*)a.wmin, s);
    }
  }
  int64_t max_nodes = 0;
  for (int64_t n : P.nodes) max_nodes = n > max_nodes ? n : max_nodes;
  const unsigned gx = (unsigned)((max_nodes + 255) / 256 > 1024 ? 1024 : (max_nodes + 255) / 256);
  const dim3 pgrid(gx, (unsigned)P.n_prob);
  CHERT_LAUNCH("k_init_fields", k_init_fields, pgrid, dim3(256), 0, s, Q.dprobs, Q.djobs, a.err);
  const int64_t n_flags = 2 * P.n_tiles;
  auto init_flags = [&](int tree_phase) {
    CHERT_LAUNCH("k_clear_flags", k_clear_flags, dim3(256), dim3(256), 0, s, a.flags, n_flags,
                 a.counter, (int)counter_words(P.max_rounds), pa.bar, a.key, 2 * P.n_tiles, a.pmin,
                 3 * P.n_prob);
    CHERT_LAUNCH("k_seed_flags", k_seed_flags, dim3((P.n_prob + 63) / 64), dim3(64), 0, s,
                 a.flags, a.list, a.counter, Q.dprobs, Q.djobs, P.n_prob, P.tx, P.tz,
                 tree_phase, a.key, a.pmin, (const int32_t*)a.err);
  };
  const int G = o->push_group ? o->push_group : 2;
  static const char* kname[2] = {"k_relax_tau", "k_relax_tree"};
  static const char* pname[2] = {"k_relax_persist_tau", "k_relax_persist_tree"};
  auto phase = [&](int ph) -> int {
    const size_t lds = Q.lds[ph];
    init_flags(ph);
    if (o->launch == CHERT_LAUNCH_PERSISTENT) {
      CHERT_LAUNCH(pname[ph], persist_kernel(ph, G), dim3((unsigned)Q.pgrid[ph]),
                   dim3((unsigned)tile_threads(a.tx, a.tz)), lds, s, a, pa);
      rounds[ph] = 0;  // read back by finish()
      return CHERT_OK;
    }
    if (Q.fixed_rounds) {  // every round of the budget, convergence read back by finish()
      for (int r = 0; r < P.max_rounds; ++r)
        CHERT_LAUNCH(kname[ph], round_kernel(ph, G, Q.lean), dim3((unsigned)Q.rgrid[ph]),
                     dim3((unsigned)tile_threads(a.tx, a.tz)), lds, s, a, r);
      CHERT_LAUNCH("k_round_count", k_round_count, dim3(1), dim3(1), 0, s, a.counter,
                   P.max_rounds, pa.result + ph, (const int32_t*)a.abort_seen);
      rounds[ph] = 0;
      return CHERT_OK;
    }
    return run_rounds(s, a, round_kernel(ph, G, Q.lean), kname[ph], Q.rgrid[ph], lds, P.max_rounds,
                      o->abort_flag_host, &rounds[ph]);
  };
  int rc = phase(0);
  if (rc) return rc;
  if (outs & (CHERT_OUT_PRED_P | CHERT_OUT_PRED_A)) {
    CHERT_LAUNCH("k_tight_out", k_tight_out, dim3((unsigned)P.n_tiles),
                 dim3((unsigned)tile_threads(a.tx, a.tz)),
                 tight_lds_bytes(P.lw, P.lh, P.w_lds_doubles, P.n_off), s, a);
    rc = phase(1);
    if (rc) return rc;
    CHERT_LAUNCH("k_pred", k_pred, pgrid, dim3(256), 0, s, a);
    if (outs & CHERT_OUT_TSTAR)
      CHERT_LAUNCH("k_tstar_finish", k_tstar_finish, pgrid, dim3(256), 0, s, Q.dprobs, Q.djobs,
                   (const int32_t*)a.err);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  return CHERT_OK;
}

// Wait for a batch enqueued on s and report its errors and counters.
static int finish(const Prepared& Q, const chert_trace_opts* o, hipStream_t s, int rounds[3],
                  chert_trace_stats* stats_host) {
  const RelaxArgs& a = Q.a;
  int32_t herr = 0;
  int32_t hres[4] = {0, 0, 0, 0};
  unsigned long long hstats[12];
  std::vector<unsigned long long> slots((size_t)kStatSlots * kStatSlotU64);
  hipError_t e = hipMemcpyAsync(&herr, a.err, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(slots.data(), a.stats, kStatBytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hres, Q.pa.result, sizeof(hres), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  stats_reduce(slots.data(), 12, 0xe00u, hstats);  // entries 9-11 are maxima
  const uint32_t outs = o->outputs;
  const bool ran[3] = {true, (outs & (CHERT_OUT_PRED_P | CHERT_OUT_PRED_A)) != 0, false};
  int status = CHERT_OK;
  if (o->launch == CHERT_LAUNCH_PERSISTENT || Q.fixed_rounds)
    for (int ph = 0; ph < 3; ++ph) {
      rounds[ph] = ran[ph] ? hres[ph] : 0;
      if (ran[ph] && hres[ph] == -2 && !status)
        status = fail(CHERT_ERR_HIP, "persistent relaxation: device-wide barrier timed out");
      if (ran[ph] && hres[ph] == -3 && !status)
        status = fail(CHERT_ERR_ABORTED, "aborted by the caller");
      if (ran[ph] && hres[ph] == -1 && !status)
        status = fail(CHERT_ERR_NO_CONVERGENCE, "relaxation round cap reached");
      if (rounds[ph] < 0) rounds[ph] = Q.P.max_rounds;
    }
  if (stats_host) {
    chert_trace_stats* st = stats_host;
    for (int ph = 0; ph < 3; ++ph) {
      st->rounds[ph] = rounds[ph];
      st->tile_visits[ph] = (int64_t)hstats[2 * ph];
      st->edge_relaxations[ph] = (int64_t)hstats[2 * ph + 1];
      st->levels_sum[ph] = (int64_t)hstats[6 + ph];
      st->levels_max[ph] = (int32_t)hstats[9 + ph];
    }
    st->reserved = 0;
  }
  if (status) return status;
  if (herr) return fail(CHERT_ERR_INVALID_ARG, "class id out of range");
  return CHERT_OK;
}

static int trace_batch(const chert_trace_job* jobs, int n_jobs, const chert_trace_opts* o,
                       void* workspace_dev, size_t workspace_bytes, hipStream_t s) {
  if (uses_frontier(jobs, n_jobs, o))
    return trace_batch_frontier(jobs, n_jobs, o, workspace_dev, workspace_bytes, s);
  Prepared Q;
  int rc = prepare(jobs, n_jobs, o, workspace_dev, workspace_bytes, s, &Q);
  if (rc) return rc;
  int rounds[3] = {0, 0, 0};
  rc = enqueue(Q, jobs, n_jobs, o, s, rounds);
  if (rc) return rc;
  return finish(Q, o, s, rounds, o->stats_host);
}

static chert_trace_job single_job(const chert_cache_desc* d, const void* cache_dev,
                                  int64_t n_classes, const chert_grid* g, int32_t mode,
                                  const int64_t* src, int32_t n_src, double* tau_r,
                                  double* tau_i, double* tstar, int32_t* pred_p,
                                  int32_t* pred_a) {
  chert_trace_job j{};
  j.d = d;
  j.cache_dev = cache_dev;
  j.n_classes = n_classes;
  j.g = g;
  j.mode = mode;
  j.src_nodes_host = src;
  j.n_src = n_src;
  j.tau_r_dev = tau_r;
  j.tau_i_dev = tau_i;
  j.tstar_dev = tstar;
  j.pred_p_dev = pred_p;
  j.pred_a_dev = pred_a;
  return j;
}

}  // namespace chert

using namespace chert;

extern "C" size_t chert_trace_batch_workspace_bytes(const chert_trace_job* jobs, int32_t n_jobs,
                                                    const chert_trace_opts* o) {
  if (uses_frontier(jobs, n_jobs, o)) return trace_batch_frontier_bytes(jobs, n_jobs, o);
  Plan P;
  if (make_plan(jobs, n_jobs, o, &P) != CHERT_OK) return 0;
  return P.total;
}

extern "C" int chert_trace_batch(const chert_trace_job* jobs, int32_t n_jobs,
                                 const chert_trace_opts* o, void* workspace_dev,
                                 size_t workspace_bytes, void* stream) {
  return trace_batch(jobs, n_jobs, o, workspace_dev, workspace_bytes, (hipStream_t)stream);
}

extern "C" size_t chert_trace_workspace_bytes(const chert_cache_desc* d, int64_t n_classes,
                                              const chert_grid* g, int32_t n_src,
                                              const chert_trace_opts* o) {
  if (!d || !g || !o) return 0;
  // sizes only: placeholders stand in for the device pointers and sources
  std::vector<int64_t> src((size_t)(n_src > 0 ? n_src : 0), 0);
  int mode = (d->mode_mask & 1u) ? 0 : ((d->mode_mask & 2u) ? 1 : 2);
  double dummy_d = 0.0;
  int32_t dummy_i = 0;
  chert_trace_job j = single_job(d, &dummy_d, n_classes, g, mode, src.data(), n_src, &dummy_d,
                                 &dummy_d, &dummy_d, &dummy_i, &dummy_i);
  if (uses_frontier(&j, 1, o)) return trace_batch_frontier_bytes(&j, 1, o);
  Plan P;
  if (make_plan(&j, 1, o, &P) != CHERT_OK) return 0;
  return P.total;
}

extern "C" int chert_trace_field(const chert_cache_desc* d, const void* cache_dev,
                                 int64_t n_classes, const chert_grid* g, int32_t mode,
                                 const int64_t* src_nodes_host, int32_t n_src,
                                 const chert_trace_opts* o, double* tau_r_dev,
                                 double* tau_i_dev, double* tstar_dev, int32_t* pred_p_dev,
                                 int32_t* pred_a_dev, void* workspace_dev,
                                 size_t workspace_bytes, void* stream) {
  chert_trace_job j = single_job(d, cache_dev, n_classes, g, mode, src_nodes_host, n_src,
                                 tau_r_dev, tau_i_dev, tstar_dev, pred_p_dev, pred_a_dev);
  return trace_batch(&j, 1, o, workspace_dev, workspace_bytes, (hipStream_t)stream);
}

// ------------------------------------------------------------- autotune --

namespace {
const int kTuneTiles[][2] = {{32, 32}, {64, 16}, {16, 64}, {32, 16}, {16, 32}, {128, 8}, {16, 16}};
const int kTuneTiles3D[][2] = {{8, 8}, {8, 16}, {16, 4}, {4, 16}};
const int kTuneGroups[] = {1, 2, 4};        // 3D tiles
const int kTuneGroups2D[] = {1, 2, 4, 8};   // 2D tiles
const int kTuneLaunch[] = {CHERT_LAUNCH_PER_ROUND, CHERT_LAUNCH_PERSISTENT};
constexpr int kTuneFinal = 3;  // probe winners timed again on the whole batch
}  // namespace

const double kTuneBuckets[] = {0.0, 4.0, 16.0, 32.0, 64.0, 128.0, 256.0};
const double kTuneBuckets2D[] = {16.0, 64.0};  // 2D: the tiles usually win; one bucket
                                               // can blow up on per-node media
const double kTuneTileBuckets[] = {16.0, 64.0, 256.0};

extern "C" size_t chert_trace_autotune_workspace_bytes(const chert_trace_job* jobs,
                                                       int32_t n_jobs,
                                                       const chert_trace_opts* o) {
  if (!o) return 0;
  // the bucketed frontier plan is the largest frontier plan
  chert_trace_opts f = *o;
  f.launch = CHERT_LAUNCH_FRONTIER;
  f.bucket_width = 1.0;
  size_t best = chert_trace_batch_workspace_bytes(jobs, n_jobs, &f);
  if (is_3d_batch(jobs, n_jobs)) {
    for (const auto& t : kTuneTiles3D) {
      chert_trace_opts c = *o;
      c.tile_x = t[0];
      c.tile_z = t[1];
      c.launch = CHERT_LAUNCH_PER_ROUND;
      c.bucket_width = 1.0;
      const size_t b = chert_trace_batch_workspace_bytes(jobs, n_jobs, &c);
      if (b > best) best = b;
    }
    return best;
  }
  for (const auto& t : kTuneTiles) {
    chert_trace_opts c = *o;
    c.tile_x = t[0];
    c.tile_z = t[1];
    c.launch = CHERT_LAUNCH_PER_ROUND;
    c.bucket_width = 1.0;  // ordered tiles: the larger round counter array
    const size_t b = chert_trace_batch_workspace_bytes(jobs, n_jobs, &c);
    if (b > best) best = b;
  }
  return best;
}

extern "C" int chert_trace_autotune(const chert_trace_job* jobs, int32_t n_jobs,
                                    chert_trace_opts* o, void* workspace_dev,
                                    size_t workspace_bytes, void* stream, double* best_ms) {
  if (!o || !jobs || n_jobs < 1) return fail(CHERT_ERR_INVALID_ARG, "null options or jobs");
  hipStream_t s = (hipStream_t)stream;
  // probe: the first source of every job
  std::vector<chert_trace_job> probe(jobs, jobs + n_jobs);
  for (auto& j : probe) j.n_src = j.n_src > 0 ? 1 : 0;
  std::vector<chert_trace_opts> cands;
  const bool three_d = is_3d_batch(jobs, n_jobs);
  const double* bws = three_d ? kTuneBuckets : kTuneBuckets2D;
  const int n_bws = three_d ? (int)(sizeof(kTuneBuckets) / sizeof(double))
                            : (int)(sizeof(kTuneBuckets2D) / sizeof(double));
  bool ray_caches = true;  // the frontier reads ray-direction caches only
  for (int j = 0; j < n_jobs; ++j)
    if (jobs[j].d && jobs[j].d->sampling != CHERT_SAMPLE_RAY) ray_caches = false;
  for (int q = 0; ray_caches && q < n_bws; ++q) {
    chert_trace_opts c = *o;
    c.launch = CHERT_LAUNCH_FRONTIER;
    c.bucket_width = bws[q];
    cands.push_back(c);
  }
  if (three_d)  // 3D tiles (tile_x x tile_x x tile_z), per-round or persistent
    for (const auto& t : kTuneTiles3D)
      for (int G : kTuneGroups)
        for (int L : kTuneLaunch) {
          chert_trace_opts c = *o;
          c.tile_x = t[0];
          c.tile_z = t[1];
          c.push_group = G;
          c.launch = L;
          c.bucket_width = 0.0;
          cands.push_back(c);
        }
  if (!three_d)
    for (const auto& t : kTuneTiles)
      for (int G : kTuneGroups2D)
        for (int L : kTuneLaunch) {
          chert_trace_opts c = *o;
          c.tile_x = t[0];
          c.tile_z = t[1];
          c.push_group = G;
          c.launch = L;
          c.bucket_width = 0.0;
          cands.push_back(c);
        }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(CHERT_ERR_HIP, "event creation failed");
  double best = -1.0;
  chert_trace_opts pick = *o;
  int tried = 0;
  std::vector<std::pair<float, chert_trace_opts>> timed;  // every candidate that ran
  // time c on a batch (HIP events, the second of two runs); false if it
  // does not fit the workspace or fails
  auto time_on = [&](const chert_trace_job* b, chert_trace_opts c, float* ms) {
    c.stats_host = nullptr;
    const size_t need = chert_trace_batch_workspace_bytes(b, n_jobs, &c);
    if (need == 0 || need > workspace_bytes) return false;  // shape not valid here
    int rc = CHERT_OK;
    for (int rep = 0; rep < 2 && rc == CHERT_OK; ++rep) {
      (void)hipEventRecord(e0, s);
      rc = trace_batch(b, n_jobs, &c, workspace_dev, workspace_bytes, s);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) rc = CHERT_ERR_HIP;
      if (rc == CHERT_OK) (void)hipEventElapsedTime(ms, e0, e1);
    }
    return rc == CHERT_OK;
  };
  auto consider = [&](chert_trace_opts c) {
    float ms = 0.f;
    if (!time_on(probe.data(), c, &ms)) return;
    ++tried;
    timed.emplace_back(ms, c);
    if (best < 0.0 || ms < best) {
      best = ms;
      pick = c;
    }
  };
  for (const chert_trace_opts& c : cands) consider(c);
  // 2D tiles: then the ordering width for the fastest shape (the 3D tiles
  // have no ordering)
  if (tried > 0 && pick.launch != CHERT_LAUNCH_FRONTIER && !three_d)
    for (double bw : kTuneTileBuckets) {
      chert_trace_opts c = pick;
      c.bucket_width = bw;
      consider(c);
    }
  // the probe's few fastest, timed again on the whole batch: a probe of one
  // source per job can rank shapes differently from many sources
  bool partial = false;
  for (int j = 0; j < n_jobs; ++j) partial |= jobs[j].n_src > 1;
  if (partial && tried > 1) {
    std::stable_sort(timed.begin(), timed.end(),
                     [](const std::pair<float, chert_trace_opts>& x,
                        const std::pair<float, chert_trace_opts>& y) { return x.first < y.first; });
    double whole = -1.0;
    for (size_t q = 0; q < timed.size() && q < (size_t)kTuneFinal; ++q) {
      float ms = 0.f;
      if (!time_on(jobs, timed[q].second, &ms)) continue;
      if (whole < 0.0 || ms < whole) {
        whole = ms;
        pick = timed[q].second;
      }
    }
    if (whole >= 0.0) best = whole;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (tried == 0) return fail(CHERT_ERR_INVALID_ARG, "no candidate fits the workspace");
  o->tile_x = pick.tile_x;
  o->tile_z = pick.tile_z;
  o->push_group = pick.push_group;
  o->launch = pick.launch;
  o->bucket_width = pick.bucket_width;
  if (best_ms) *best_ms = best;
  return CHERT_OK;
}

// ---------------------------------------------------------------- graphs --

struct chert_trace_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  chert::Prepared Q;
  chert_trace_opts o{};
};

extern "C" int chert_trace_graph_create(const chert_trace_job* jobs, int32_t n_jobs,
                                        const chert_trace_opts* o, void* workspace_dev,
                                        size_t workspace_bytes, void* stream,
                                        chert_trace_graph** out) {
  if (!out) return fail(CHERT_ERR_INVALID_ARG, "null graph handle");
  *out = nullptr;
  if (!o || !(o->launch == CHERT_LAUNCH_PERSISTENT ||
               (o->launch == CHERT_LAUNCH_PER_ROUND && o->max_rounds > 0)))
    return fail(CHERT_ERR_INVALID_ARG,
                "graph capture needs the persistent launch, or per-round launches with a "
                "round budget (max_rounds > 0)");
  if (!stream) return fail(CHERT_ERR_INVALID_ARG, "graph capture needs a non-null stream");
  hipStream_t s = (hipStream_t)stream;
  chert_trace_graph* G = new (std::nothrow) chert_trace_graph();
  if (!G) return fail(CHERT_ERR_CAPACITY, "out of host memory");
  int rc = chert::prepare(jobs, n_jobs, o, workspace_dev, workspace_bytes, s, &G->Q);
  if (rc) {
    delete G;
    return rc;
  }
  G->o = *o;
  G->o.stats_host = nullptr;
  G->Q.fixed_rounds = (o->launch == CHERT_LAUNCH_PER_ROUND);
  const bool prof = chert::prof_suspend();
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    chert::prof_resume(prof);
    delete G;
    return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  }
  int rounds[3];
  rc = chert::enqueue(G->Q, jobs, n_jobs, &G->o, s, rounds);
  e = hipStreamEndCapture(s, &G->graph);
  chert::prof_resume(prof);
  if (rc == CHERT_OK && e != hipSuccess) rc = fail(CHERT_ERR_HIP, hipGetErrorString(e));
  if (rc == CHERT_OK) {
    e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = fail(CHERT_ERR_HIP, hipGetErrorString(e));
  }
  if (rc) {
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return rc;
  }
  *out = G;
  return CHERT_OK;
}

extern "C" int chert_trace_graph_launch(chert_trace_graph* g, void* stream) {
  if (!g) return fail(CHERT_ERR_INVALID_ARG, "null graph");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  return CHERT_OK;
}

extern "C" int chert_trace_graph_finish(chert_trace_graph* g, void* stream,
                                        chert_trace_stats* stats_host) {
  if (!g) return fail(CHERT_ERR_INVALID_ARG, "null graph");
  int rounds[3] = {0, 0, 0};
  return chert::finish(g->Q, &g->o, (hipStream_t)stream, rounds, stats_host);
}

extern "C" int chert_trace_graph_destroy(chert_trace_graph* g) {
  if (!g) return CHERT_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return CHERT_OK;
}
