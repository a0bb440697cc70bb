// Node-frontier label-correcting traveltimes (eq 31 over the forward star,
// edge costs of eqs 27-30) for gfx950.  Every 3D batch runs here: its
// traveltimes on this node frontier (CHERT_LAUNCH_FRONTIER) or on the 3D
// tiles of tile3d.hip (CHERT_LAUNCH_PER_ROUND), its predecessors and t*
// always here.  2D batches that ask for CHERT_LAUNCH_FRONTIER run here too;
// trace.hip holds the 2D tile relaxation.  All reach the fixed point
// Dijkstra reaches from the same weights.
//
// Iteration it relaxes every out-edge of the (problem, node) items whose
// traveltime dropped in iteration it - 1, one thread per (item, offset): an
// improved head is claimed with a 64-bit atomicMin on the bits of the
// (non-negative) double, stamped so that it enters the next frontier once,
// and appended with one atomic per wavefront (ballot + prefix count).  With
// near/far buckets an improvement at or above the problem's threshold waits
// in a far pile until the near frontier is empty.
//
// Predecessors (eq 33): hop counts over tight edges (tau_i + w_ij == tau_j,
// bitwise) by BFS layers: layer k holds the nodes at hop k, each node
// entered once (the hop atomicMin is its own dedupe), all layers stored in
// order in one list.  pred_j is the tight in-neighbour at hop_j - 1 with the
// smallest offset index, and t* folds the attenuation weights along the
// propagation predecessors layer by layer: the rule and the fold of the 2D
// tile path's tree phase.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <vector>

#include "chert.h"
#include "chert_internal.h"

namespace chert {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

constexpr int kFieldR = 0;
constexpr int32_t kHopUnsetF = 0x7fffffff;
constexpr int kFrontierThreads = 256;
constexpr int kFrontierBlocks = 4096;
constexpr int kLutSide = 2 * kMaxRadius + 1;  // (dx, dy, dz) -> offset index table side

// W[f][ki][kj][o] (eqs 28-30 in this operation order, no contraction) from a
// mode's slice of a cache: col[o] is the cache column of offset o's bin
__global__ void k_front_weights(double* W, int K, int n_off, const double* V, const double* A,
                                const int32_t* st, int n_cols, const double* L,
                                const int32_t* col) {
  const int64_t total = 2LL * K * K * n_off;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(t % n_off);
    int64_t r = t / n_off;
    const int kj = (int)(r % K);
    r /= K;
    const int ki = (int)(r % K);
    const int f = (int)(r / K);
    const int b = col[o];
    const int bad = CHERT_ST_NO_BRACKET | CHERT_ST_FLUID | CHERT_ST_NONPHYS | CHERT_ST_NOCONV;
    const int64_t ei = (int64_t)ki * n_cols + b, ej = (int64_t)kj * n_cols + b;
    double w;
    if ((st[ei] & bad) || (st[ej] & bad)) w = INFINITY;
    else if (f == kFieldR) w = __ddiv_rn(L[o], __dmul_rn(0.5, __dadd_rn(V[ei], V[ej])));
    else w = __dmul_rn(L[o], __dmul_rn(0.5, __dadd_rn(A[ei], A[ej])));
    W[t] = w;
  }
}

struct JobF {
  int nx, ny, nz, K;  // ny = 1 in 2D
  int per_node;       // one cache row per node, weights per (node, offset)
  int pad;
  int64_t n;          // nodes
  const int32_t* cls; // class map (class mode)
  const double* W;    // class mode [2][K][K][n_off]; per node [2][n][n_off] where
                      // row j, offset o holds the edge j - o -> j
};

// Weight of the edge i -> j = i + o read on the head's side (per node: row j).
__device__ __forceinline__ bool w_head(const JobF& J, int n_off, int field, int i, int j, int o,
                                       double* w) {
  if (J.per_node) {
    *w = J.W[((int64_t)field * J.n + j) * n_off + o];
    return true;
  }
  const int ci = J.cls[i], cj = J.cls[j];
  if (ci < 0 || ci >= J.K || cj < 0 || cj >= J.K) return false;
  *w = J.W[(((int64_t)field * J.K + ci) * J.K + cj) * n_off + o];
  return true;
}

struct ProbF {
  double* tau;
  int32_t* stamp;   // near-frontier stamps (iteration numbers); hop counts later
  int32_t* fstamp;  // far-pile stamps (epoch numbers)
  int32_t* pred;    // predecessors (nullable)
  double* tstar;    // t* along this field's tree (nullable; propagation field)
  int job, field;
  int64_t src;
};

struct RF {
  const JobF* jobs;
  const ProbF* probs;
  int n_prob, n_off;
  const int32_t* ox;
  const int32_t* oy;
  const int32_t* oz;
  int64_t* lists;   // [2][cap] items (problem << 32 | node), by iteration parity
  int64_t cap;
  int32_t* counts;  // [max_iter + 2] frontier size of each iteration
  int32_t* err;
  unsigned long long* stats;  // [kStatSlots][16] shards of: [0] iterations run with
                              // work, [1] edges examined
  double* thr;        // [n_prob] current threshold (+inf: one bucket)
  double* thr_min;    // [n_prob] far-pile minimum (scratch of the split)
  double* wmin;       // [2] smallest positive edge weight per field
  double bucket;      // bucket width in units of wmin (0: one bucket)
  int64_t* far;       // [2][cap] far piles by epoch parity
  int32_t* far_count; // [2]
  int32_t* seg;       // [max_iter + 2] start of each BFS layer in the order list
  const int16_t* lut; // offset index of (dx, dy, dz), (2R+1)^3 entries, -1 if none
  int R;
};

__device__ __forceinline__ void append64(bool flag, int64_t item, int64_t* list, int32_t* count) {
  const unsigned long long b = __ballot(flag);
  if (b == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)b) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(b));
  base = __shfl(base, leader);
  if (flag) list[base + __popcll(b & ((1ull << lane) - 1ull))] = item;
}

// neighbour of node i at offset o (sign +1) or -o (sign -1); -1 outside the grid
__device__ __forceinline__ int step(const JobF& J, const RF& a, int i, int o, int sign) {
  const int x = i % J.nx, r = i / J.nx, y = r % J.ny, z = r / J.ny;
  const int X = x + sign * a.ox[o], Y = y + sign * a.oy[o], Z = z + sign * a.oz[o];
  if (X < 0 || X >= J.nx || Y < 0 || Y >= J.ny || Z < 0 || Z >= J.nz) return -1;
  return X + J.nx * (Y + J.ny * Z);
}

__global__ void k_front_clear(int32_t* counts, int n_counts, int32_t* err,
                              unsigned long long* stats, int32_t* far_count) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_counts; t += gridDim.x * blockDim.x)
    counts[t] = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < kStatSlots * kStatSlotU64;
       t += gridDim.x * blockDim.x)
    stats[t] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x < 4) {
    if (threadIdx.x == 0) *err = 0;
    far_count[threadIdx.x] = 0;  // far-pile counts
  }
}

// blockIdx.y = problem: tau = inf (0 at the source), stamps 0, source queued
__global__ void k_front_init(RF a) {
  const int p = blockIdx.y;
  const ProbF P = a.probs[p];
  const int64_t n = a.jobs[P.job].n;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    P.tau[j] = (j == P.src) ? 0.0 : INFINITY;
    P.stamp[j] = 0;
    P.fstamp[j] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.lists[atomicAdd(&a.counts[0], 1)] = ((int64_t)p << 32) | (int64_t)P.src;
    const double w = a.wmin[P.field];
    a.thr[p] = (a.bucket > 0.0 && w < INFINITY) ? a.bucket * w : INFINITY;
    a.thr_min[p] = INFINITY;
  }
}

// smallest positive finite weight of each field over a job's table
__global__ void k_front_wmin(const double* W, int64_t per_field, double* wmin) {
  const int f = blockIdx.y;
  double m = INFINITY;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < per_field;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double w = W[f * per_field + t];
    if (w > 0.0 && w < m) m = w;
  }
  for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off));
  if (__lane_id() == 0 && m < INFINITY) atomicMin((unsigned long long*)&wmin[f], dbits(m));
}

__global__ void k_front_wmin_init(double* wmin) {
  if (threadIdx.x < 2) wmin[threadIdx.x] = INFINITY;
}

// split, step 1: smallest traveltime of each problem's far pile; per-block
// minima in LDS (few problems, many items: one global atomic per problem
// and block instead of one per item)
constexpr int kFarMinLds = 2048;
__global__ void __launch_bounds__(256) k_front_far_min(RF a, int epoch) {
  __shared__ unsigned long long s_min[kFarMinLds];
  const bool lds = a.n_prob <= kFarMinLds;
  if (lds)
    for (int p = threadIdx.x; p < a.n_prob; p += blockDim.x) s_min[p] = dbits(INFINITY);
  __syncthreads();
  const int nf = a.far_count[epoch & 1];
  const int64_t* fl = a.far + (int64_t)(epoch & 1) * a.cap;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nf; q += gridDim.x * blockDim.x) {
    const int64_t item = fl[q];
    const int p = (int)(item >> 32);
    const double t = a.probs[p].tau[item & 0xffffffffLL];
    if (lds) atomicMin(&s_min[p], dbits(t));
    else atomicMin((unsigned long long*)&a.thr_min[p], dbits(t));
  }
  __syncthreads();
  if (lds)
    for (int p = threadIdx.x; p < a.n_prob; p += blockDim.x)
      if (s_min[p] != dbits(INFINITY)) atomicMin((unsigned long long*)&a.thr_min[p], s_min[p]);
}

// split, step 2: thresholds move to the far minimum plus one bucket
__global__ void k_front_far_thr(RF a, int epoch) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < a.n_prob; p += gridDim.x * blockDim.x) {
    const double m = a.thr_min[p];
    if (m < INFINITY) a.thr[p] = m + a.bucket * a.wmin[a.probs[p].field];
    a.thr_min[p] = INFINITY;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.far_count[(epoch + 1) & 1] = 0;
}

// split, step 3: far items under the new threshold form iteration it's
// frontier; the rest move to the next epoch's pile
__global__ void k_front_far_split(RF a, int epoch, int it) {
  const int nf = a.far_count[epoch & 1];
  const int64_t* fl = a.far + (int64_t)(epoch & 1) * a.cap;
  int64_t* fo = a.far + (int64_t)((epoch + 1) & 1) * a.cap;
  int64_t* lout = a.lists + (int64_t)(it & 1) * a.cap;
  for (int base = blockIdx.x * blockDim.x; base < nf; base += gridDim.x * blockDim.x) {
    const int q = base + threadIdx.x;
    bool near = false, far = false;
    int64_t item = 0;
    if (q < nf) {
      item = fl[q];
      const int p = (int)(item >> 32);
      const int64_t j = item & 0xffffffffLL;
      const ProbF P = a.probs[p];
      if (P.tau[j] < a.thr[p]) near = atomicExch(&P.stamp[j], it) != it;
      else far = atomicExch(&P.fstamp[j], epoch + 2) != epoch + 2;
    }
    append64(near, item, lout, &a.counts[it]);
    append64(far, item, fo, &a.far_count[(epoch + 1) & 1]);
  }
}

// Weight of the edge i -> j = i + o read on the tail's side: class mode from
// the tail's class ci; per node from row i at the reversed offset (the star
// is symmetric: index n_off-1-o is -o), whose entry is the edge j -> i --
// equal bitwise, since the cache holds direction d + n_dirs/2 as the exact
// copy of d and L_o is even in o.  False when a class id is out of range.
__device__ __forceinline__ bool w_out(const JobF& J, int n_off, int field, int i, int ci, int j,
                                      int o, double* w) {
  if (J.per_node) {
    *w = J.W[((int64_t)field * J.n + i) * n_off + (n_off - 1 - o)];
    return true;
  }
  const int cj = J.cls[j];
  if (ci < 0 || ci >= J.K || cj < 0 || cj >= J.K) return false;
  *w = J.W[(((int64_t)field * J.K + ci) * J.K + cj) * n_off + o];
  return true;
}

// One wavefront per frontier item, its lanes over the star offsets: the
// item is decoded once and its traveltime read once per wavefront.
__global__ void __launch_bounds__(kFrontierThreads) k_front_relax(RF a, int it, int epoch) {
  const int n_near = a.counts[it];
  if (n_near == 0) return;
  const int64_t* lin = a.lists + (int64_t)(it & 1) * a.cap;
  int64_t* lout = a.lists + (int64_t)((it + 1) & 1) * a.cap;
  int64_t* far = a.far + (int64_t)(epoch & 1) * a.cap;
  const int lane = __lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  long long raw = 0;
  for (int64_t f = wave; f < n_near; f += n_waves) {
    const int64_t item = lin[f];
    const int p = (int)(item >> 32);
    const int i = (int)(item & 0xffffffffLL);
    const ProbF P = a.probs[p];
    const JobF J = a.jobs[P.job];
    const int x = i % J.nx, r = i / J.nx, y = r % J.ny, z = r / J.ny;
    const double ti = P.tau[i];
    const double thr = a.thr[p];
    const int ci = J.per_node ? 0 : J.cls[i];
    raw += a.n_off;
    for (int o0 = 0; o0 < a.n_off; o0 += 64) {
      const int o = o0 + lane;
      bool want = false, later = false;
      int64_t out = 0;
      if (o < a.n_off) {
        const int X = x + a.ox[o], Y = y + a.oy[o], Z = z + a.oz[o];
        if (X >= 0 && X < J.nx && Y >= 0 && Y < J.ny && Z >= 0 && Z < J.nz) {
          const int j = X + J.nx * (Y + J.ny * Z);
          double w;
          if (!w_out(J, a.n_off, P.field, i, ci, j, o, &w)) {
            *a.err = 1;
          } else {
            const double cand = __dadd_rn(ti, w);
            if (cand < P.tau[j]) {
              const unsigned long long old =
                  atomicMin((unsigned long long*)&P.tau[j], dbits(cand));
              if (dbits(cand) < old) {
                out = ((int64_t)p << 32) | (int64_t)j;
                if (cand < thr) want = atomicExch(&P.stamp[j], it + 1) != it + 1;
                else later = atomicExch(&P.fstamp[j], epoch + 1) != epoch + 1;
              }
            }
          }
        }
      }
      append64(want, out, lout, &a.counts[it + 1]);
      append64(later, out, far, &a.far_count[epoch & 1]);
    }
  }
  if (lane == 0 && raw) atomicAdd(&stat_slot(a.stats)[1], (unsigned long long)raw);
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.stats[0], 1ull);
}

// ------------------------------------------------ predecessors and t* ---

__global__ void k_front_zero(int32_t* counts, int32_t* seg, int n) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    counts[t] = 0;
    seg[t] = 0;
  }
}

// blockIdx.y = problem; only problems with predecessors take part
__global__ void k_front_hop_init(RF a) {
  const int p = blockIdx.y;
  const ProbF P = a.probs[p];
  if (!P.pred) return;
  const int64_t n = a.jobs[P.job].n;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    P.stamp[j] = (j == P.src) ? 0 : kHopUnsetF;
    if (P.tstar) P.tstar[j] = (j == P.src) ? 0.0 : INFINITY;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    a.lists[atomicAdd(&a.counts[0], 1)] = ((int64_t)p << 32) | (int64_t)P.src;
}

__global__ void __launch_bounds__(kFrontierThreads) k_front_hop(RF a, int k) {
  const int start = a.seg[k], cnt = a.counts[k];
  if (blockIdx.x == 0 && threadIdx.x == 0) a.seg[k + 1] = start + cnt;
  if (cnt == 0) return;
  int64_t* out = a.lists + start + cnt;
  const int lane = __lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t f = wave; f < cnt; f += n_waves) {  // one wavefront per item
    const int64_t item = a.lists[start + f];
    const int p = (int)(item >> 32);
    const int i = (int)(item & 0xffffffffLL);
    const ProbF P = a.probs[p];
    const JobF J = a.jobs[P.job];
    const int x = i % J.nx, r = i / J.nx, y = r % J.ny, z = r / J.ny;
    const double ti = P.tau[i];
    const int ci = J.per_node ? 0 : J.cls[i];
    for (int o0 = 0; o0 < a.n_off; o0 += 64) {
      const int o = o0 + lane;
      bool want = false;
      int64_t item_j = 0;
      if (o < a.n_off) {
        const int X = x + a.ox[o], Y = y + a.oy[o], Z = z + a.oz[o];
        if (X >= 0 && X < J.nx && Y >= 0 && Y < J.ny && Z >= 0 && Z < J.nz) {
          const int j = X + J.nx * (Y + J.ny * Z);
          const double tj = P.tau[j];
          double w;
          if (tj < INFINITY && w_out(J, a.n_off, P.field, i, ci, j, o, &w) &&
              __dadd_rn(ti, w) == tj && atomicMin(&P.stamp[j], k + 1) > k + 1) {
            want = true;
            item_j = ((int64_t)p << 32) | (int64_t)j;
          }
        }
      }
      append64(want, item_j, out, &a.counts[k + 1]);
    }
  }
}

// blockIdx.y = problem
__global__ void k_front_pred(RF a) {
  const int p = blockIdx.y;
  const ProbF P = a.probs[p];
  if (!P.pred) return;
  const JobF J = a.jobs[P.job];
  for (int64_t jj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; jj < J.n;
       jj += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)jj;
    const int h = P.stamp[j];
    int best = -1;
    if (h != kHopUnsetF && h > 0) {
      const double tj = P.tau[j];
      for (int o = 0; o < a.n_off && best < 0; ++o) {
        const int i = step(J, a, j, o, -1);
        if (i < 0 || P.stamp[i] != h - 1) continue;
        double w;
        if (w_head(J, a.n_off, P.field, i, j, o, &w) && __dadd_rn(P.tau[i], w) == tj) best = i;
      }
    }
    P.pred[j] = best;
  }
}

// t* of BFS layer k (k >= 1) of the propagation problems
__global__ void k_front_tstar(RF a, int k) {
  const int start = a.seg[k], cnt = a.counts[k];
  const int side = 2 * a.R + 1;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
    const int64_t item = a.lists[start + q];
    const ProbF P = a.probs[(int)(item >> 32)];
    if (!P.tstar) continue;
    const JobF J = a.jobs[P.job];
    const int j = (int)(item & 0xffffffffLL);
    const int i = P.pred[j];
    if (i < 0) continue;  // only if the two rows of a per-node edge disagree
    const int dx = j % J.nx - i % J.nx;
    const int dy = (j / J.nx) % J.ny - (i / J.nx) % J.ny;
    const int dz = j / (J.nx * J.ny) - i / (J.nx * J.ny);
    const int o = a.lut[((dz + a.R) * side + (dy + a.R)) * side + (dx + a.R)];
    if (o < 0) continue;
    double w = INFINITY;
    w_head(J, a.n_off, 1, i, j, o, &w);
    P.tstar[j] = __dadd_rn(P.tstar[i], w);
  }
}

// smallest positive weight of each field of a weight table (also for the
// tile path's ordering): init once per call, then once per table
int enqueue_wmin_init(double* wmin, hipStream_t s) {
  CHERT_LAUNCH("k_front_wmin_init", k_front_wmin_init, dim3(1), dim3(64), 0, s, wmin);
  return CHERT_OK;
}
int enqueue_wmin(const double* W, int64_t per_field, double* wmin, hipStream_t s) {
  const int64_t blocks = (per_field + 255) / 256;
  CHERT_LAUNCH("k_front_wmin", k_front_wmin, dim3((unsigned)(blocks > 1024 ? 1024 : blocks), 2),
               dim3(256), 0, s, W, per_field, wmin);
  return CHERT_OK;
}

// ------------------------------------------------------------------ plan --

struct PlanF {
  int dim = 0, R = 0, n_off = 0, n_prob = 0, max_iter = 0;
  int64_t cap = 0;
  bool tiles = false;  // 3D traveltimes on tiles (tile3d.hip) instead of the frontier
  size_t off_stats = 0;
  size_t off_star = 0, off_lcol = 0, off_jobs = 0, off_probs = 0, off_counts = 0, off_err = 0,
         off_lists = 0, off_far = 0, off_thr = 0, off_lut = 0, off_tiles = 0, total = 0;
  std::vector<size_t> off_W, off_stamp;  // per job, per problem (near and far stamps)
};

static bool per_node_job(const chert_trace_job& j) { return j.g->dim == 2 && !j.g->class_id_dev; }

static int validate_job3(const chert_trace_job& j, uint32_t outs) {
  chert_cache_layout lay;
  int rc = chert_cache_layout_of(j.d, j.n_classes, &lay);
  if (rc) return rc;
  const chert_grid* g = j.g;
  if (!g || g->dim != 3) return fail(CHERT_ERR_INVALID_ARG, "a 3D batch needs 3D grids");
  if (j.d->dim != 3) return fail(CHERT_ERR_INVALID_ARG, "a 3D grid needs a 3D cache");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx * g->ny * g->nz >= 0x7fffffffLL)
    return fail(CHERT_ERR_INVALID_ARG, "grid size out of range");
  if (g->radius < 1 || g->radius > kMaxRadius3)
    return fail(CHERT_ERR_INVALID_ARG, "3D radius must be 1..4");
  if (!(g->hx > 0.0) || !(g->hy > 0.0) || !(g->hz > 0.0) || !isfinite(g->hx) ||
      !isfinite(g->hy) || !isfinite(g->hz))
    return fail(CHERT_ERR_INVALID_ARG, "spacing must be positive");
  if (!g->class_id_dev) return fail(CHERT_ERR_UNSUPPORTED, "3D grids need a class map");
  if ((outs & CHERT_OUT_PRED_P) && !j.pred_p_dev) return fail(CHERT_ERR_INVALID_ARG, "null pred_p");
  if ((outs & CHERT_OUT_PRED_A) && !j.pred_a_dev) return fail(CHERT_ERR_INVALID_ARG, "null pred_a");
  if ((outs & CHERT_OUT_TSTAR) && !j.tstar_dev) return fail(CHERT_ERR_INVALID_ARG, "null tstar");
  if (j.mode < 0 || j.mode > 2 || !(j.d->mode_mask & (1u << j.mode)))
    return fail(CHERT_ERR_INVALID_ARG, "mode not in the cache");
  if (!j.cache_dev) return fail(CHERT_ERR_INVALID_ARG, "null cache");
  if (j.n_src < 1 || !j.src_nodes_host) return fail(CHERT_ERR_INVALID_ARG, "need sources");
  const int64_t n = g->nx * g->ny * g->nz;
  for (int i = 0; i < j.n_src; ++i)
    if (j.src_nodes_host[i] < 0 || j.src_nodes_host[i] >= n)
      return fail(CHERT_ERR_INVALID_ARG, "source out of range");
  if ((outs & CHERT_OUT_TAU_R) && !j.tau_r_dev) return fail(CHERT_ERR_INVALID_ARG, "null tau_r");
  if ((outs & CHERT_OUT_TAU_I) && !j.tau_i_dev) return fail(CHERT_ERR_INVALID_ARG, "null tau_i");
  return CHERT_OK;
}

static int make_plan_f(const chert_trace_job* jobs, int n_jobs, const chert_trace_opts* o,
                       PlanF* P) {
  if (!jobs || n_jobs < 1) return fail(CHERT_ERR_INVALID_ARG, "need at least one job");
  if (!o) return fail(CHERT_ERR_INVALID_ARG, "null options");
  if (!jobs[0].g) return fail(CHERT_ERR_INVALID_ARG, "null grid");
  const uint32_t outs = o->outputs;
  if (outs == 0 || !(outs & (CHERT_OUT_TAU_R | CHERT_OUT_TAU_I)))
    return fail(CHERT_ERR_INVALID_ARG, "bad output mask");
  if (!(o->bucket_width >= 0.0) || !isfinite(o->bucket_width))
    return fail(CHERT_ERR_INVALID_ARG, "bucket_width must be finite and >= 0");
  if (outs & ~31u) return fail(CHERT_ERR_INVALID_ARG, "bad output mask");
  if ((outs & CHERT_OUT_TSTAR) && !((outs & CHERT_OUT_TAU_R) && (outs & CHERT_OUT_PRED_P)))
    return fail(CHERT_ERR_INVALID_ARG, "TSTAR needs TAU_R and PRED_P");
  if ((outs & CHERT_OUT_PRED_P) && !(outs & CHERT_OUT_TAU_R))
    return fail(CHERT_ERR_INVALID_ARG, "PRED_P needs TAU_R");
  if ((outs & CHERT_OUT_PRED_A) && !(outs & CHERT_OUT_TAU_I))
    return fail(CHERT_ERR_INVALID_ARG, "PRED_A needs TAU_I");
  P->dim = jobs[0].g->dim;
  for (int j = 0; j < n_jobs; ++j) {
    int rc = P->dim == 3 ? validate_job3(jobs[j], outs) : validate_job_2d(jobs[j], outs);
    if (rc) return rc;
    if (jobs[j].d->sampling != CHERT_SAMPLE_RAY)
      return fail(CHERT_ERR_UNSUPPORTED, "the node frontier reads ray-direction caches only");
    if (jobs[j].g->radius != jobs[0].g->radius)
      return fail(CHERT_ERR_INVALID_ARG, "all jobs of a batch need the same radius");
  }
  P->R = jobs[0].g->radius;
  P->n_off = P->dim == 3
                 ? star_3d(P->R, 1.0, 1.0, 1.0, 2, nullptr, nullptr, nullptr, nullptr, nullptr)
                 : star_2d(P->R, 1.0, 1.0, 4, nullptr, nullptr, nullptr, nullptr);
  const int per = ((outs & CHERT_OUT_TAU_R) ? 1 : 0) + ((outs & CHERT_OUT_TAU_I) ? 1 : 0);
  int64_t span = 0;
  P->n_prob = 0;
  P->cap = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const chert_grid* g = jobs[j].g;
    const int64_t n = g->nx * g->ny * g->nz;
    P->n_prob += per * jobs[j].n_src;
    P->cap += (int64_t)per * jobs[j].n_src * n;
    const int64_t sp = g->nx + g->ny + g->nz;
    if (sp > span) span = sp;
  }
  if (P->n_prob > 65535 || P->cap >= 0x7fffffffLL)
    return fail(CHERT_ERR_UNSUPPORTED, "batch too large for one launch");
  P->max_iter = (o->max_rounds > 0) ? o->max_rounds : 4096 + 64 * (int)span;
  size_t off = 0;
  P->off_star = off;
  off += align256((size_t)3 * kMaxOffsets3 * sizeof(int32_t));
  P->off_lcol = off;
  off += align256((size_t)n_jobs * P->n_off * (sizeof(double) + sizeof(int32_t)));
  P->off_jobs = off;
  off += align256((size_t)n_jobs * sizeof(JobF));
  P->off_probs = off;
  off += align256((size_t)P->n_prob * sizeof(ProbF));
  P->off_counts = off;
  off += 2 * align256((size_t)(P->max_iter + 2) * sizeof(int32_t));  // counts, BFS layer starts
  P->off_lut = off;
  off += align256((size_t)kLutSide * kLutSide * kLutSide * sizeof(int16_t));
  P->off_err = off;
  off += 256;
  P->off_stats = off;
  off += align256(kStatBytes);
  P->off_W.clear();
  for (int j = 0; j < n_jobs; ++j) {
    P->off_W.push_back(off);
    const chert_grid* g = jobs[j].g;
    const size_t rows = per_node_job(jobs[j]) ? (size_t)(g->nx * g->nz)
                                              : (size_t)jobs[j].n_classes * jobs[j].n_classes;
    off += align256((size_t)2 * rows * P->n_off * sizeof(double));
  }
  P->off_stamp.clear();
  for (int j = 0; j < n_jobs; ++j) {
    const chert_grid* g = jobs[j].g;
    for (int q = 0; q < per * jobs[j].n_src; ++q) {
      P->off_stamp.push_back(off);
      off += 2 * align256((size_t)(g->nx * g->ny * g->nz) * sizeof(int32_t));
    }
  }
  P->off_lists = off;
  off += align256((size_t)2 * P->cap * sizeof(int64_t));
  P->off_far = off;
  off += (o->bucket_width > 0.0) ? align256((size_t)2 * P->cap * sizeof(int64_t)) : 0;
  P->off_thr = off;
  off += align256((size_t)2 * P->n_prob * sizeof(double) + 4 * sizeof(double));
  P->tiles = P->dim == 3 &&
             (o->launch == CHERT_LAUNCH_PER_ROUND || o->launch == CHERT_LAUNCH_PERSISTENT);
  if (P->tiles) {
    if (o->push_group != 0 && o->push_group != 1 && o->push_group != 2 && o->push_group != 4)
      return fail(CHERT_ERR_INVALID_ARG, "push_group must be 0, 1, 2 or 4");
    std::vector<Tile3Job> tj(n_jobs);
    std::vector<Tile3Prob> tp;
    for (int j = 0; j < n_jobs; ++j) {
      const chert_grid* g = jobs[j].g;
      tj[j] = Tile3Job{(int)g->nx, (int)g->ny, (int)g->nz, (int)jobs[j].n_classes, nullptr, nullptr};
      for (int q = 0; q < per * jobs[j].n_src; ++q) tp.push_back(Tile3Prob{nullptr, 0, j, 0});
    }
    size_t tb = 0;
    const int rc = tiles3d_bytes(tj.data(), n_jobs, tp.data(), (int)tp.size(), P->R, P->n_off,
                                 o->tile_x, o->tile_z, P->max_iter, &tb);
    if (rc) return rc;
    P->off_tiles = off;
    off += align256(tb);
  }
  P->total = off;
  return CHERT_OK;
}

// ---------------------------------------------------------------- driver --

int trace_batch_frontier(const chert_trace_job* jobs, int n_jobs, const chert_trace_opts* o,
                         void* workspace_dev, size_t workspace_bytes, hipStream_t s) {
  PlanF P;
  int rc = make_plan_f(jobs, n_jobs, o, &P);
  if (rc) return rc;
  if (!workspace_dev || workspace_bytes < P.total)
    return fail(CHERT_ERR_INVALID_ARG, "workspace too small");
  uint8_t* ws = (uint8_t*)workspace_dev;
  const uint32_t outs = o->outputs;
  // star (shared offsets; oy = 0 in 2D), per-job lengths and cache columns
  std::vector<int32_t> star((size_t)3 * kMaxOffsets3, 0);
  std::vector<uint8_t> lcol((size_t)n_jobs * P.n_off * (sizeof(double) + sizeof(int32_t)));
  double* hL = (double*)lcol.data();
  int32_t* hcol = (int32_t*)(hL + (size_t)n_jobs * P.n_off);
  std::vector<int32_t> bin(P.n_off);
  for (int j = 0; j < n_jobs; ++j) {
    const chert_grid* g = jobs[j].g;
    int32_t* ox = star.data();
    int32_t* oy = star.data() + kMaxOffsets3;
    int32_t* oz = star.data() + 2 * kMaxOffsets3;
    double* L = hL + (size_t)j * P.n_off;
    int32_t* col = hcol + (size_t)j * P.n_off;
    if (P.dim == 3) {
      star_3d(P.R, g->hx, g->hy, g->hz, jobs[j].d->n_dirs, ox, oy, oz, L, col);
    } else {
      star_2d(P.R, g->hx, g->hz, jobs[j].d->n_dirs, ox, oz, L, bin.data());
      rc = star_columns(jobs[j].d, bin.data(), P.n_off, col);
      if (rc) return rc;
    }
  }
  std::vector<JobF> jd(n_jobs);
  std::vector<ProbF> pd;
  for (int j = 0; j < n_jobs; ++j) {
    const chert_trace_job& J = jobs[j];
    jd[j].nx = (int)J.g->nx;
    jd[j].ny = P.dim == 3 ? (int)J.g->ny : 1;
    jd[j].nz = (int)J.g->nz;
    jd[j].K = (int)J.n_classes;
    jd[j].per_node = per_node_job(J) ? 1 : 0;
    jd[j].n = (int64_t)jd[j].nx * jd[j].ny * jd[j].nz;
    jd[j].cls = J.g->class_id_dev;
    jd[j].W = (const double*)(ws + P.off_W[j]);
    const int64_t n = jd[j].n;
    for (int i = 0; i < J.n_src; ++i) {
      for (int field = 0; field < 2; ++field) {
        if (!(outs & (field ? CHERT_OUT_TAU_I : CHERT_OUT_TAU_R))) continue;
        ProbF q{};
        q.tau = (field ? J.tau_i_dev : J.tau_r_dev) + (int64_t)i * n;
        q.stamp = (int32_t*)(ws + P.off_stamp[pd.size()]);
        q.fstamp = (int32_t*)(ws + P.off_stamp[pd.size()] +
                              align256((size_t)n * sizeof(int32_t)));
        q.job = j;
        q.field = field;
        q.src = J.src_nodes_host[i];
        if (field == 0 && (outs & CHERT_OUT_PRED_P)) q.pred = J.pred_p_dev + (int64_t)i * n;
        if (field == 1 && (outs & CHERT_OUT_PRED_A)) q.pred = J.pred_a_dev + (int64_t)i * n;
        if (field == 0 && (outs & CHERT_OUT_TSTAR)) q.tstar = J.tstar_dev + (int64_t)i * n;
        pd.push_back(q);
      }
    }
  }
  std::vector<int16_t> lut((size_t)kLutSide * kLutSide * kLutSide, (int16_t)-1);
  {
    const int side = 2 * P.R + 1;
    for (int q = 0; q < P.n_off; ++q)
      lut[((star[2 * kMaxOffsets3 + q] + P.R) * side + (star[kMaxOffsets3 + q] + P.R)) * side +
          (star[q] + P.R)] = (int16_t)q;
  }
  int32_t* dstar = (int32_t*)(ws + P.off_star);
  double* dL = (double*)(ws + P.off_lcol);
  int32_t* dcol = (int32_t*)(dL + (size_t)n_jobs * P.n_off);
  JobF* djobs = (JobF*)(ws + P.off_jobs);
  ProbF* dprobs = (ProbF*)(ws + P.off_probs);
  hipError_t e = hipMemcpyAsync(dstar, star.data(), star.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dL, lcol.data(), lcol.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(djobs, jd.data(), jd.size() * sizeof(JobF), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dprobs, pd.data(), pd.size() * sizeof(ProbF), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + P.off_lut, lut.data(), lut.size() * sizeof(int16_t),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // host buffers are locals
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));

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
    double* W = (double*)(ws + P.off_W[j]);
    if (jd[j].per_node) {
      rc = enqueue_weights_node_2d(W, jd[j].nx, jd[j].nz, P.n_off, dstar,
                                   dstar + 2 * kMaxOffsets3, dL + (size_t)j * P.n_off,
                                   dcol + (size_t)j * P.n_off, n_cols, Vm, Am, Sm, s);
      if (rc) return rc;
    } else {
      const int64_t tw = 2 * K * K * P.n_off;
      const int64_t blocks = (tw + 255) / 256;
      CHERT_LAUNCH("k_front_weights", k_front_weights,
                   dim3((unsigned)(blocks > 65536 ? 65536 : blocks)), dim3(256), 0, s, W, (int)K,
                   P.n_off, Vm, Am, Sm, n_cols, dL + (size_t)j * P.n_off,
                   dcol + (size_t)j * P.n_off);
    }
  }
  RF a{};
  a.jobs = djobs;
  a.probs = dprobs;
  a.n_prob = (int)pd.size();
  a.n_off = P.n_off;
  a.ox = dstar;
  a.oy = dstar + kMaxOffsets3;
  a.oz = dstar + 2 * kMaxOffsets3;
  a.lists = (int64_t*)(ws + P.off_lists);
  a.cap = P.cap;
  a.counts = (int32_t*)(ws + P.off_counts);
  a.err = (int32_t*)(ws + P.off_err);
  a.stats = (unsigned long long*)(ws + P.off_stats);
  a.far_count = (int32_t*)(ws + P.off_err + 128);
  a.thr = (double*)(ws + P.off_thr);
  a.thr_min = a.thr + P.n_prob;
  a.wmin = a.thr_min + P.n_prob;
  a.bucket = o->bucket_width;
  a.far = o->bucket_width > 0.0 ? (int64_t*)(ws + P.off_far) : nullptr;
  a.seg = a.counts + align256((size_t)(P.max_iter + 2) * sizeof(int32_t)) / sizeof(int32_t);
  a.lut = (const int16_t*)(ws + P.off_lut);
  a.R = P.R;
  CHERT_LAUNCH("k_front_clear", k_front_clear, dim3(64), dim3(256), 0, s, a.counts,
               P.max_iter + 2, a.err, a.stats, a.far_count);
  // class ids checked before any output is written
  {
    bool any_map = false;
    for (int j = 0; j < n_jobs; ++j)
      if (!jd[j].per_node) {
        enqueue_class_check(jd[j].cls, jd[j].n, jd[j].K, a.err, s);
        any_map = true;
      }
    if (any_map) {
      int32_t herr0 = 0;
      e = hipMemcpyAsync(&herr0, a.err, sizeof(int32_t), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
      if (herr0) return fail(CHERT_ERR_INVALID_ARG, "class id out of range");
    }
  }
  enqueue_wmin_init(a.wmin, s);
  if (a.far) {
    for (int j = 0; j < n_jobs; ++j) {
      const int64_t rows = jd[j].per_node ? jd[j].n : jobs[j].n_classes * jobs[j].n_classes;
      enqueue_wmin((const double*)(ws + P.off_W[j]), rows * (int64_t)P.n_off, a.wmin, s);
    }
  }
  int64_t max_nodes = 0;
  for (int j = 0; j < n_jobs; ++j)
    if (jd[j].n > max_nodes) max_nodes = jd[j].n;
  const unsigned gx = (unsigned)((max_nodes + 255) / 256 > 1024 ? 1024 : (max_nodes + 255) / 256);
  CHERT_LAUNCH("k_front_init", k_front_init, dim3(gx, (unsigned)a.n_prob), dim3(256), 0, s, a);
  // iterations in groups of 8 between host checks of the frontier sizes;
  // an empty near frontier with a non-empty far pile starts the next bucket
  const int group = 8;
  int iters = -1, epoch = 0;
  int32_t counts[group + 2];
  int64_t tile_visits = 0, tile_edges = 0;
  if (P.tiles) {  // 3D: the traveltimes on tiles, from the initial fields above
    std::vector<Tile3Job> tj(n_jobs);
    for (int j = 0; j < n_jobs; ++j)
      tj[j] = Tile3Job{jd[j].nx, jd[j].ny, jd[j].nz, jd[j].K, jd[j].cls, jd[j].W};
    std::vector<Tile3Prob> tp(pd.size());
    for (size_t q = 0; q < pd.size(); ++q)
      tp[q] = Tile3Prob{pd[q].tau, pd[q].src, pd[q].job, pd[q].field};
    int rounds = 0;
    rc = relax_tiles_3d(tj.data(), n_jobs, tp.data(), (int)tp.size(), a.ox, a.oy, a.oz, P.n_off,
                        P.R, o->tile_x, o->tile_z, o->push_group, P.max_iter, ws + P.off_tiles,
                        P.total - P.off_tiles, s, o->abort_flag_host,
                        o->launch == CHERT_LAUNCH_PERSISTENT, &rounds, &tile_visits, &tile_edges);
    if (rc) return rc;
    iters = rounds;
  }
  for (int it = 0; it < P.max_iter && iters < 0;) {
    const int nb = it + group > P.max_iter ? P.max_iter - it : group;
    for (int q = 0; q < nb; ++q)
      CHERT_LAUNCH("k_front_relax", k_front_relax, dim3(kFrontierBlocks), dim3(kFrontierThreads),
                   0, s, a, it + q, epoch);
    e = hipMemcpyAsync(counts, a.counts + it + 1, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && a.far)
      e = hipMemcpyAsync(counts + group, a.far_count + (epoch & 1), sizeof(int32_t),
                         hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
    if (o->abort_flag_host && *o->abort_flag_host)
      return fail(CHERT_ERR_ABORTED, "aborted by the caller");
    int empty = -1;
    for (int q = 0; q < nb && empty < 0; ++q)
      if (counts[q] == 0) empty = it + q + 1;
    if (empty < 0) {
      it += nb;
      continue;
    }
    if (!a.far || counts[group] == 0) {
      iters = empty;
      break;
    }
    // next bucket: its frontier becomes iteration `empty`'s input
    const int nfar = counts[group];
    const unsigned fb = (unsigned)((nfar + 255) / 256 > 4096 ? 4096 : (nfar + 255) / 256);
    const unsigned fmb = fb > 512 ? 512 : fb;  // few blocks: fewer global merges
    CHERT_LAUNCH("k_front_far_min", k_front_far_min, dim3(fmb), dim3(256), 0, s, a, epoch);
    CHERT_LAUNCH("k_front_far_thr", k_front_far_thr, dim3((a.n_prob + 255) / 256), dim3(256), 0,
                 s, a, epoch);
    CHERT_LAUNCH("k_front_far_split", k_front_far_split, dim3(fb), dim3(256), 0, s, a, epoch,
                 empty);
    ++epoch;
    it = empty;
  }
  int layers = 0;
  if (iters >= 0 && (outs & (CHERT_OUT_PRED_P | CHERT_OUT_PRED_A | CHERT_OUT_TSTAR))) {
    CHERT_LAUNCH("k_front_zero", k_front_zero, dim3(64), dim3(256), 0, s, a.counts, a.seg,
                 P.max_iter + 2);
    CHERT_LAUNCH("k_front_hop_init", k_front_hop_init, dim3(gx, (unsigned)a.n_prob), dim3(256), 0,
                 s, a);
    for (int k = 0; k < P.max_iter && layers == 0; k += group) {
      const int nb = k + group > P.max_iter ? P.max_iter - k : group;
      for (int q = 0; q < nb; ++q)
        CHERT_LAUNCH("k_front_hop", k_front_hop, dim3(kFrontierBlocks), dim3(kFrontierThreads), 0,
                     s, a, k + q);
      e = hipMemcpyAsync(counts, a.counts + k + 1, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
      if (o->abort_flag_host && *o->abort_flag_host)
        return fail(CHERT_ERR_ABORTED, "aborted by the caller");
      for (int q = 0; q < nb && layers == 0; ++q)
        if (counts[q] == 0) layers = k + q + 1;
    }
    if (layers == 0) return fail(CHERT_ERR_NO_CONVERGENCE, "hop layers exceed the iteration cap");
    CHERT_LAUNCH("k_front_pred", k_front_pred, dim3(gx, (unsigned)a.n_prob), dim3(256), 0, s, a);
    if (outs & CHERT_OUT_TSTAR)
      for (int k = 1; k < layers; ++k)
        CHERT_LAUNCH("k_front_tstar", k_front_tstar, dim3(1024), dim3(256), 0, s, a, k);
  }
  int32_t herr = 0;
  unsigned long long hstats[2] = {0, 0};
  std::vector<unsigned long long> slots((size_t)kStatSlots * kStatSlotU64);
  e = hipMemcpyAsync(&herr, a.err, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(slots.data(), a.stats, kStatBytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  stats_reduce(slots.data(), 2, 0u, hstats);
  if (o->stats_host) {
    chert_trace_stats* st = o->stats_host;
    *st = chert_trace_stats{};
    st->rounds[0] = iters < 0 ? P.max_iter : iters;
    st->rounds[1] = layers;
    st->tile_visits[0] = P.tiles ? tile_visits : (int64_t)hstats[0];
    st->edge_relaxations[0] = P.tiles ? tile_edges : (int64_t)hstats[1];
  }
  if (iters < 0) return fail(CHERT_ERR_NO_CONVERGENCE, "relaxation iteration cap reached");
  if (herr) return fail(CHERT_ERR_INVALID_ARG, "class id out of range");
  return CHERT_OK;
}

size_t trace_batch_frontier_bytes(const chert_trace_job* jobs, int n_jobs,
                                  const chert_trace_opts* o) {
  PlanF P;
  if (make_plan_f(jobs, n_jobs, o, &P) != CHERT_OK) return 0;
  return P.total;
}

}  // namespace chert
