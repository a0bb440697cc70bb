// First-arrival traveltime fields on a 2D forward-star graph (eqs 18-19,
// 22-34; Algorithm 2, tracing) for gfx950.
//
// Each (source, field) pair is an independent min-plus problem: tau_R with
// the propagation increments, tau_I with the attenuation increments (eqs 24,
// 29-31).  The solver is a tiled, frontier-driven label-correcting
// relaxation:
//   - the grid is cut into TX x TZ tiles; a workgroup owns one (problem,
//     tile), stages the tile plus an R-wide halo of tau and the class ids in
//     LDS, and pulls every interior node over the star until the tile is
//     locally converged (chaotic in-place updates are safe: every value ever
//     written is the fold of some path, and values only decrease);
//   - changed nodes within R of a tile border activate the neighbouring
//     tile for the next round (double-buffered flags, one counter per round);
//   - rounds repeat until a round activates nothing.
// The fixed point equals Dijkstra's result bitwise because both are the
// minimum over paths of the left-to-right FP64 sum of the same weights.
//
// Predecessors (eq 33) are made schedule-independent: BFS hop counts over
// the tight edges (tau_i + w_ij == tau_j) by the same tiled relaxation, then
// pred_j = tight neighbour with the smallest (hop, offset index).  t* folds
// the attenuation increments along the propagation predecessor tree.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <vector>

#include "chert.h"
#include "chert_internal.h"

#pragma clang fp contract(off)

namespace chert {

constexpr int kRelaxThreads = 256;
constexpr int kMaxNodesPerThread = 4;
constexpr int kLocalIterCap = 512;
constexpr int32_t kHopUnset = 0x7fffffff;
constexpr int kFieldR = 0, kFieldI = 1;

struct ProbDev {
  double* tau;     // [n_nodes] this problem's traveltime field
  int32_t* hop;    // [n_nodes] hop counts, then predecessor offset index
  int32_t* pred;   // [n_nodes] or nullptr
  double* tstar;   // [n_nodes] or nullptr (propagation problems only)
  int64_t src;
  int32_t field;   // 0 = propagation (w_R), 1 = attenuation (w_I)
  int32_t tstar_of; // for t*: index of the propagation problem, else -1
};

struct Geom {
  int64_t nx, nz;
  int tx, tz;      // tile size
  int ntx, ntz;    // tiles per axis
  int R;
  int n_off;
  int lw, lh;      // LDS tile + halo extent
  int K;           // classes
};

struct RelaxArgs {
  Geom g;
  const int32_t* class_id;
  const int32_t* ox;
  const int32_t* oz;
  const double* W;  // [2][K][K][n_off]
  ProbDev* probs;
  int n_prob;
  int32_t* flags;   // [2][n_prob][n_tiles]
  int32_t* counter; // [max_rounds + 2]
  int32_t* err;     // [1] out-of-range class ids seen
  int w_in_lds;
};

// ------------------------------------------------------------- weights ---

// W[f][ki][kj][o]: eqs 28-30 in this operation order, no contraction.
__global__ void k_weights(double* W, int K, int n_off, const double* V, const double* A,
                          const int32_t* st, int n_dirs, const double* L,
                          const int32_t* bin) {
  int64_t total = 2LL * K * K * n_off;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int o = (int)(t % n_off);
    int64_t r = t / n_off;
    int kj = (int)(r % K);
    r /= K;
    int ki = (int)(r % K);
    int f = (int)(r / K);
    int b = bin[o];
    const int bad = CHERT_ST_NO_BRACKET | CHERT_ST_FLUID | CHERT_ST_NONPHYS;
    int64_t ei = (int64_t)ki * n_dirs + b, ej = (int64_t)kj * n_dirs + b;
    double w;
    if ((st[ei] & bad) || (st[ej] & bad)) {
      w = INFINITY;
    } else if (f == kFieldR) {
      w = __ddiv_rn(L[o], __dmul_rn(0.5, __dadd_rn(V[ei], V[ej])));
    } else {
      w = __dmul_rn(L[o], __dmul_rn(0.5, __dadd_rn(A[ei], A[ej])));
    }
    W[t] = w;
  }
}

// ---------------------------------------------------------------- init ---

__global__ void k_init_fields(ProbDev* probs, int n_prob, int64_t n_nodes, int32_t* err) {
  int64_t total = (int64_t)n_prob * n_nodes;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int p = (int)(t / n_nodes);
    int64_t j = t % n_nodes;
    ProbDev pr = probs[p];
    if (t == 0) *err = 0;
    pr.tau[j] = (j == pr.src) ? 0.0 : INFINITY;
    pr.hop[j] = (j == pr.src) ? 0 : kHopUnset;
    if (pr.tstar) pr.tstar[j] = (j == pr.src) ? 0.0 : NAN;
  }
}

// Clear flags and counters, then activate each problem's source tile.
__global__ void k_init_flags(int32_t* flags, int64_t n_flags, int32_t* counter,
                             int n_counter) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t t = tid; t < n_flags; t += (int64_t)gridDim.x * blockDim.x) flags[t] = 0;
  for (int64_t t = tid; t < n_counter; t += (int64_t)gridDim.x * blockDim.x) counter[t] = 0;
}

__global__ void k_seed_flags(int32_t* flags, int32_t* counter, const ProbDev* probs, int n_prob,
                             Geom g, int phase_tstar) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_prob) return;
  if (phase_tstar && probs[p].tstar == nullptr) return;
  int64_t s = probs[p].src;
  int tx = (int)((s % g.nx) / g.tx), tz = (int)((s / g.nx) / g.tz);
  int n_tiles = g.ntx * g.ntz;
  flags[(int64_t)p * n_tiles + tz * g.ntx + tx] = 1;
  atomicAdd(&counter[0], 1);
}

// --------------------------------------------------------- tile helpers ---

struct TileCtx {
  int p, t, tx, tz;
  int64_t x0, z0;  // first interior node
  int txe, tze;    // interior extent (ragged at the grid edge)
};

__device__ __forceinline__ bool tile_begin(const RelaxArgs& a, int round, TileCtx* c,
                                           int* s_flag) {
  const int n_tiles = a.g.ntx * a.g.ntz;
  c->p = blockIdx.x / n_tiles;
  c->t = blockIdx.x % n_tiles;
  int32_t* fin = a.flags + (int64_t)(round & 1) * a.n_prob * n_tiles;
  if (threadIdx.x == 0) {
    int32_t f = fin[(int64_t)c->p * n_tiles + c->t];
    *s_flag = f;
    if (f) fin[(int64_t)c->p * n_tiles + c->t] = 0;
  }
  __syncthreads();
  if (!*s_flag) return false;
  c->tx = c->t % a.g.ntx;
  c->tz = c->t / a.g.ntx;
  c->x0 = (int64_t)c->tx * a.g.tx;
  c->z0 = (int64_t)c->tz * a.g.tz;
  c->txe = (int)min((int64_t)a.g.tx, a.g.nx - c->x0);
  c->tze = (int)min((int64_t)a.g.tz, a.g.nz - c->z0);
  return true;
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
                                         int mask) {
  const int n_tiles = a.g.ntx * a.g.ntz;
  int32_t* fout = a.flags + (int64_t)((round + 1) & 1) * a.n_prob * n_tiles;
  for (int bit = 0; bit < 9; ++bit) {
    if (!(mask & (1 << bit))) continue;
    int dx = bit % 3 - 1, dz = bit / 3 - 1;
    int nx_ = c.tx + dx, nz_ = c.tz + dz;
    if (nx_ < 0 || nx_ >= a.g.ntx || nz_ < 0 || nz_ >= a.g.ntz) continue;
    int32_t* f = &fout[(int64_t)c.p * n_tiles + nz_ * a.g.ntx + nx_];
    if (atomicOr(f, 1) == 0) atomicAdd(&a.counter[round + 1], 1);
  }
}

// Stage class ids of tile + halo; out-of-grid = -1, out-of-range ids = -2.
__device__ __forceinline__ void load_classes(const RelaxArgs& a, const TileCtx& c,
                                             int32_t* cls_l) {
  const int R = a.g.R, lw = a.g.lw, n = lw * a.g.lh;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    int64_t gx = c.x0 + (q % lw) - R, gz = c.z0 + (q / lw) - R;
    int32_t k = -1;
    if (gx >= 0 && gx < a.g.nx && gz >= 0 && gz < a.g.nz) {
      k = a.class_id[gx + a.g.nx * gz];
      if (k < 0 || k >= a.g.K) {
        atomicAdd(a.err, 1);
        k = -2;
      }
    }
    cls_l[q] = k;
  }
}

__device__ __forceinline__ void load_offsets(const RelaxArgs& a, int32_t* off_l) {
  for (int o = threadIdx.x; o < a.g.n_off; o += blockDim.x)
    off_l[o] = a.ox[o] + a.oz[o] * a.g.lw;
}

struct Smem {
  double* val;     // [lw*lh]
  int32_t* ival;   // [lw*lh]
  int32_t* cls;    // [lw*lh]
  int32_t* off;    // [n_off]
  double* W;       // [K*K*n_off] when staged
};

__device__ __forceinline__ Smem carve(const RelaxArgs& a, void* base) {
  Smem s;
  const int n = a.g.lw * a.g.lh;
  char* p = (char*)base;
  s.val = (double*)p;
  p += sizeof(double) * n;
  s.ival = (int32_t*)p;
  p += sizeof(int32_t) * n;
  s.cls = (int32_t*)p;
  p += sizeof(int32_t) * n;
  s.off = (int32_t*)p;
  p += sizeof(int32_t) * ((a.g.n_off + 1) & ~1);
  s.W = (double*)p;
  return s;
}

// ----------------------------------------------------- relaxation phases ---

// Phase TAU: tau_j <- min(tau_j, tau_i + w_ij) over the star (eq 31, pull).
__global__ void __launch_bounds__(kRelaxThreads) k_relax_tau(RelaxArgs a, int round) {
  extern __shared__ double smem_d[];
  __shared__ int s_flag, s_mask;
  TileCtx c;
  if (!tile_begin(a, round, &c, &s_flag)) return;
  Smem s = carve(a, smem_d);
  const int R = a.g.R, lw = a.g.lw, n = lw * a.g.lh, K = a.g.K, n_off = a.g.n_off;
  const ProbDev pr = a.probs[c.p];
  const double* Wf = a.W + (int64_t)pr.field * K * K * n_off;
  if (threadIdx.x == 0) s_mask = 0;
  load_classes(a, c, s.cls);
  load_offsets(a, s.off);
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    int64_t gx = c.x0 + (q % lw) - R, gz = c.z0 + (q / lw) - R;
    bool in = gx >= 0 && gx < a.g.nx && gz >= 0 && gz < a.g.nz;
    s.val[q] = in ? pr.tau[gx + a.g.nx * gz] : INFINITY;
  }
  if (a.w_in_lds)
    for (int q = threadIdx.x; q < K * K * n_off; q += blockDim.x) s.W[q] = Wf[q];
  __syncthreads();
  const double* Wp = a.w_in_lds ? s.W : Wf;

  int li[kMaxNodesPerThread];
  double orig[kMaxNodesPerThread];
  int mine = 0;
  for (int q = threadIdx.x; q < a.g.tx * a.g.tz && mine < kMaxNodesPerThread; q += blockDim.x) {
    int x = q % a.g.tx, z = q / a.g.tx;
    if (x >= c.txe || z >= c.tze) continue;
    li[mine] = (z + R) * lw + (x + R);
    orig[mine] = s.val[li[mine]];
    ++mine;
  }
  int it = 0, changed;
  do {
    changed = 0;
    for (int m = 0; m < mine; ++m) {
      const int l = li[m];
      const int kj = s.cls[l];
      if (kj < 0) continue;
      const double cur = s.val[l];
      double best = cur;
      for (int o = 0; o < n_off; ++o) {
        const int ii = l - s.off[o];
        const int ki = s.cls[ii];
        if (ki < 0) continue;
        const double cand = __dadd_rn(s.val[ii], Wp[((int64_t)ki * K + kj) * n_off + o]);
        if (cand < best) best = cand;
      }
      if (best < cur) {
        s.val[l] = best;
        changed = 1;
      }
    }
    ++it;
  } while (__syncthreads_or(changed) && it < kLocalIterCap);

  int mask = (it >= kLocalIterCap) ? (1 << 4) : 0;  // bit 4 = this tile again
  for (int m = 0; m < mine; ++m) {
    const int l = li[m];
    if (s.val[l] < orig[m]) {
      int x = l % lw - R, z = l / lw - R;
      pr.tau[(c.x0 + x) + a.g.nx * (c.z0 + z)] = s.val[l];
      mask |= border_bits(x, z, a.g.tx, a.g.tz, R);
    }
  }
  if (mask) atomicOr(&s_mask, mask);
  __syncthreads();
  if (threadIdx.x == 0 && s_mask) activate(a, round, c, s_mask);
}

// Phase HOP: BFS hop counts over tight edges, h_j <- min(h_j, h_i + 1).
__global__ void __launch_bounds__(kRelaxThreads) k_relax_hop(RelaxArgs a, int round) {
  extern __shared__ double smem_d[];
  __shared__ int s_flag, s_mask;
  TileCtx c;
  if (!tile_begin(a, round, &c, &s_flag)) return;
  Smem s = carve(a, smem_d);
  const int R = a.g.R, lw = a.g.lw, n = lw * a.g.lh, K = a.g.K, n_off = a.g.n_off;
  const ProbDev pr = a.probs[c.p];
  const double* Wf = a.W + (int64_t)pr.field * K * K * n_off;
  if (threadIdx.x == 0) s_mask = 0;
  load_classes(a, c, s.cls);
  load_offsets(a, s.off);
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    int64_t gx = c.x0 + (q % lw) - R, gz = c.z0 + (q / lw) - R;
    bool in = gx >= 0 && gx < a.g.nx && gz >= 0 && gz < a.g.nz;
    int64_t g = gx + a.g.nx * gz;
    s.val[q] = in ? pr.tau[g] : INFINITY;
    s.ival[q] = in ? pr.hop[g] : kHopUnset;
  }
  if (a.w_in_lds)
    for (int q = threadIdx.x; q < K * K * n_off; q += blockDim.x) s.W[q] = Wf[q];
  __syncthreads();
  const double* Wp = a.w_in_lds ? s.W : Wf;

  int li[kMaxNodesPerThread];
  int32_t orig[kMaxNodesPerThread];
  int mine = 0;
  for (int q = threadIdx.x; q < a.g.tx * a.g.tz && mine < kMaxNodesPerThread; q += blockDim.x) {
    int x = q % a.g.tx, z = q / a.g.tx;
    if (x >= c.txe || z >= c.tze) continue;
    li[mine] = (z + R) * lw + (x + R);
    orig[mine] = s.ival[li[mine]];
    ++mine;
  }
  int it = 0, changed;
  do {
    changed = 0;
    for (int m = 0; m < mine; ++m) {
      const int l = li[m];
      const int kj = s.cls[l];
      const double tj = s.val[l];
      if (kj < 0 || !(tj < INFINITY)) continue;
      const int32_t cur = s.ival[l];
      int32_t best = cur;
      for (int o = 0; o < n_off; ++o) {
        const int ii = l - s.off[o];
        const int ki = s.cls[ii];
        const int32_t hi = s.ival[ii];
        if (ki < 0 || hi == kHopUnset || hi + 1 >= best) continue;
        if (__dadd_rn(s.val[ii], Wp[((int64_t)ki * K + kj) * n_off + o]) == tj) best = hi + 1;
      }
      if (best < cur) {
        s.ival[l] = best;
        changed = 1;
      }
    }
    ++it;
  } while (__syncthreads_or(changed) && it < kLocalIterCap);

  int mask = (it >= kLocalIterCap) ? (1 << 4) : 0;
  for (int m = 0; m < mine; ++m) {
    const int l = li[m];
    if (s.ival[l] < orig[m]) {
      int x = l % lw - R, z = l / lw - R;
      pr.hop[(c.x0 + x) + a.g.nx * (c.z0 + z)] = s.ival[l];
      mask |= border_bits(x, z, a.g.tx, a.g.tz, R);
    }
  }
  if (mask) atomicOr(&s_mask, mask);
  __syncthreads();
  if (threadIdx.x == 0 && s_mask) activate(a, round, c, s_mask);
}

// pred_j = tight in-neighbour with hop_j - 1 and the smallest offset index.
// Afterwards hop[] holds the predecessor's offset index (or -1) for t*.
__global__ void k_pred(RelaxArgs a) {
  const int64_t n_nodes = a.g.nx * a.g.nz;
  const int K = a.g.K, n_off = a.g.n_off;
  int64_t total = (int64_t)a.n_prob * n_nodes;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(t / n_nodes);
    const int64_t j = t % n_nodes;
    const ProbDev pr = a.probs[p];
    const double* Wf = a.W + (int64_t)pr.field * K * K * n_off;
    const int32_t hj = pr.hop[j];
    int32_t best = -1, best_o = -1;
    const int64_t jx = j % a.g.nx, jz = j / a.g.nx;
    const int32_t kj = a.class_id[j];
    if (j != pr.src && hj != kHopUnset && kj >= 0 && kj < K) {
      const double tj = pr.tau[j];
      for (int o = 0; o < n_off; ++o) {
        int64_t ix = jx - a.ox[o], iz = jz - a.oz[o];
        if (ix < 0 || ix >= a.g.nx || iz < 0 || iz >= a.g.nz) continue;
        int64_t i = ix + a.g.nx * iz;
        if (pr.hop[i] != hj - 1) continue;
        int32_t ki = a.class_id[i];
        if (ki < 0 || ki >= K) continue;
        if (__dadd_rn(pr.tau[i], Wf[((int64_t)ki * K + kj) * n_off + o]) == tj) {
          best = (int32_t)i;
          best_o = o;
          break;
        }
      }
    }
    (void)best_o;
    if (pr.pred) pr.pred[j] = best;
  }
}

// pred offsets must be written only after every hop read: separate pass
__global__ void k_pred_offsets(RelaxArgs a) {
  const int64_t n_nodes = a.g.nx * a.g.nz;
  int64_t total = (int64_t)a.n_prob * n_nodes;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(t / n_nodes);
    const int64_t j = t % n_nodes;
    const ProbDev pr = a.probs[p];
    if (!pr.pred) continue;
    int32_t i = pr.pred[j];
    int32_t o_idx = -1;
    if (i >= 0) {
      int dx = (int)(j % a.g.nx - i % a.g.nx), dz = (int)(j / a.g.nx - i / a.g.nx);
      for (int o = 0; o < a.g.n_off; ++o)
        if (a.ox[o] == dx && a.oz[o] == dz) {
          o_idx = o;
          break;
        }
    }
    pr.hop[j] = o_idx;
  }
}

// Phase TSTAR: t*_j = t*_pred + w_I(pred -> j) once t*_pred is known.
__global__ void __launch_bounds__(kRelaxThreads) k_relax_tstar(RelaxArgs a, int round) {
  extern __shared__ double smem_d[];
  __shared__ int s_flag, s_mask;
  TileCtx c;
  if (!tile_begin(a, round, &c, &s_flag)) return;
  Smem s = carve(a, smem_d);
  const int R = a.g.R, lw = a.g.lw, n = lw * a.g.lh, K = a.g.K, n_off = a.g.n_off;
  const ProbDev pr = a.probs[c.p];
  if (!pr.tstar) return;  // block-uniform
  const ProbDev pp = a.probs[pr.tstar_of];  // the propagation problem (pred source)
  const double* WI = a.W + (int64_t)kFieldI * K * K * n_off;
  if (threadIdx.x == 0) s_mask = 0;
  load_classes(a, c, s.cls);
  load_offsets(a, s.off);
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    int64_t gx = c.x0 + (q % lw) - R, gz = c.z0 + (q / lw) - R;
    bool in = gx >= 0 && gx < a.g.nx && gz >= 0 && gz < a.g.nz;
    s.val[q] = in ? pr.tstar[gx + a.g.nx * gz] : NAN;
  }
  __syncthreads();

  int li[kMaxNodesPerThread];
  int32_t po[kMaxNodesPerThread];
  int mine = 0;
  for (int q = threadIdx.x; q < a.g.tx * a.g.tz && mine < kMaxNodesPerThread; q += blockDim.x) {
    int x = q % a.g.tx, z = q / a.g.tx;
    if (x >= c.txe || z >= c.tze) continue;
    li[mine] = (z + R) * lw + (x + R);
    po[mine] = pp.hop[(c.x0 + x) + a.g.nx * (c.z0 + z)];  // pred offset index
    ++mine;
  }
  int it = 0, changed;
  do {
    changed = 0;
    for (int m = 0; m < mine; ++m) {
      const int l = li[m];
      const int o = po[m];
      if (o < 0 || !isnan(s.val[l])) continue;
      const int ii = l - s.off[o];
      const double tp = s.val[ii];
      if (isnan(tp)) continue;
      const int ki = s.cls[ii], kj = s.cls[l];
      s.val[l] = __dadd_rn(tp, WI[((int64_t)ki * K + kj) * n_off + o]);
      changed = 1;
    }
    ++it;
  } while (__syncthreads_or(changed) && it < kLocalIterCap);

  int mask = (it >= kLocalIterCap) ? (1 << 4) : 0;
  for (int m = 0; m < mine; ++m) {
    const int l = li[m];
    if (po[m] >= 0 && !isnan(s.val[l])) {
      int x = l % lw - R, z = l / lw - R;
      int64_t g = (c.x0 + x) + a.g.nx * (c.z0 + z);
      if (isnan(pr.tstar[g])) {
        pr.tstar[g] = s.val[l];
        mask |= border_bits(x, z, a.g.tx, a.g.tz, R);
      }
    }
  }
  if (mask) atomicOr(&s_mask, mask);
  __syncthreads();
  if (threadIdx.x == 0 && s_mask) activate(a, round, c, s_mask);
}

// unreachable nodes: t* = +inf
__global__ void k_tstar_finish(ProbDev* probs, int n_prob, int64_t n_nodes) {
  int64_t total = (int64_t)n_prob * n_nodes;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    ProbDev pr = probs[t / n_nodes];
    if (pr.tstar && isnan(pr.tstar[t % n_nodes])) pr.tstar[t % n_nodes] = INFINITY;
  }
}

// ----------------------------------------------------------- host side ---

struct WsLayout {
  size_t star, W, probs, flags, counter, err, hop, total;
  int n_off, n_prob, n_tiles, max_rounds;
};

static int count_problems(uint32_t outs, int n_src) {
  int per = 0;
  if (outs & (CHERT_OUT_TAU_R | CHERT_OUT_PRED_P | CHERT_OUT_TSTAR)) ++per;
  if (outs & (CHERT_OUT_TAU_I | CHERT_OUT_PRED_A)) ++per;
  return per * n_src;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int tile_dims(const chert_trace_opts* o, int* tx, int* tz) {
  *tx = (o && o->tile_x > 0) ? o->tile_x : 32;
  *tz = (o && o->tile_z > 0) ? o->tile_z : 16;
  return (*tx) * (*tz) <= kRelaxThreads * kMaxNodesPerThread;
}

static WsLayout ws_layout(int64_t K, const chert_grid* g, int n_src, const chert_trace_opts* o,
                          int n_dirs) {
  WsLayout L{};
  int tx, tz;
  tile_dims(o, &tx, &tz);
  L.n_off = star_2d(g->radius, g->hx, g->hz, n_dirs, nullptr, nullptr, nullptr, nullptr);
  L.n_prob = count_problems(o ? o->outputs : 0, n_src);
  int ntx = (int)((g->nx + tx - 1) / tx), ntz = (int)((g->nz + tz - 1) / tz);
  L.n_tiles = ntx * ntz;
  L.max_rounds = (o && o->max_rounds > 0) ? o->max_rounds : 1024 + 64 * (ntx + ntz);
  size_t off = 0;
  L.star = off;
  off += align256((size_t)kMaxOffsets * (3 * sizeof(int32_t) + sizeof(double)));
  L.W = off;
  off += align256((size_t)2 * K * K * L.n_off * sizeof(double));
  L.probs = off;
  off += align256((size_t)L.n_prob * sizeof(ProbDev));
  L.flags = off;
  off += align256((size_t)2 * L.n_prob * L.n_tiles * sizeof(int32_t));
  L.counter = off;
  off += align256((size_t)(L.max_rounds + 2) * sizeof(int32_t));
  L.err = off;
  off += 256;
  L.hop = off;
  off += align256((size_t)L.n_prob * g->nx * g->nz * sizeof(int32_t));
  L.total = off;
  return L;
}

static int validate(const chert_cache_desc* d, int64_t K, const chert_grid* g, int mode,
                    int n_src, const chert_trace_opts* o) {
  chert_cache_layout lay;
  int rc = chert_cache_layout_of(d, K, &lay);
  if (rc) return rc;
  if (!g || !o) return fail(CHERT_ERR_INVALID_ARG, "null grid or options");
  if (g->dim == 3) return fail(CHERT_ERR_UNSUPPORTED, "3D grids are not traced yet");
  if (g->dim != 2 || g->ny != 1) return fail(CHERT_ERR_INVALID_ARG, "2D grid needs dim 2, ny 1");
  if (g->nx < 1 || g->nz < 1 || g->nx * g->nz > 0x7fffffffLL)
    return fail(CHERT_ERR_INVALID_ARG, "grid size out of range");
  if (g->radius < 1 || g->radius > kMaxRadius) return fail(CHERT_ERR_INVALID_ARG, "radius must be 1..8");
  if (!(g->hx > 0.0) || !(g->hz > 0.0) || !isfinite(g->hx) || !isfinite(g->hz))
    return fail(CHERT_ERR_INVALID_ARG, "spacing must be positive");
  if (!g->class_id_dev) return fail(CHERT_ERR_INVALID_ARG, "null class ids");
  if (mode < 0 || mode > 2 || !(d->mode_mask & (1u << mode)))
    return fail(CHERT_ERR_INVALID_ARG, "mode not in the cache");
  if (n_src < 1) return fail(CHERT_ERR_INVALID_ARG, "need at least one source");
  uint32_t outs = o->outputs;
  if (outs == 0 || (outs & ~31u)) return fail(CHERT_ERR_INVALID_ARG, "bad output mask");
  if ((outs & CHERT_OUT_TSTAR) && !((outs & CHERT_OUT_TAU_R) && (outs & CHERT_OUT_PRED_P)))
    return fail(CHERT_ERR_INVALID_ARG, "TSTAR needs TAU_R and PRED_P");
  if ((outs & CHERT_OUT_PRED_P) && !(outs & CHERT_OUT_TAU_R))
    return fail(CHERT_ERR_INVALID_ARG, "PRED_P needs TAU_R");
  if ((outs & CHERT_OUT_PRED_A) && !(outs & CHERT_OUT_TAU_I))
    return fail(CHERT_ERR_INVALID_ARG, "PRED_A needs TAU_I");
  int tx, tz;
  if (!tile_dims(o, &tx, &tz) || tx < g->radius || tz < g->radius)
    return fail(CHERT_ERR_INVALID_ARG, "tile must hold >= radius and <= 1024 nodes");
  return CHERT_OK;
}

}  // namespace chert

using namespace chert;

extern "C" size_t chert_trace_workspace_bytes(const chert_cache_desc* d, int64_t n_classes,
                                              const chert_grid* g, int32_t n_src,
                                              const chert_trace_opts* o) {
  if (!d || !g || !o) return 0;
  int mode = (d->mode_mask & 1u) ? 0 : ((d->mode_mask & 2u) ? 1 : 2);
  if (validate(d, n_classes, g, mode, n_src, o) != CHERT_OK) return 0;
  return ws_layout(n_classes, g, n_src, o, d->n_dirs).total;
}

static int run_rounds(hipStream_t s, const RelaxArgs& a, void (*kern)(RelaxArgs, int),
                      size_t lds, int max_rounds) {
  const int n_tiles = a.g.ntx * a.g.ntz;
  const int64_t grid = (int64_t)a.n_prob * n_tiles;
  const int batch = 8;
  int32_t counts[batch];
  for (int r = 0; r < max_rounds; r += batch) {
    int nb = batch;
    if (r + nb > max_rounds) nb = max_rounds - r;
    for (int q = 0; q < nb; ++q)
      hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kRelaxThreads), lds, s, a, r + q);
    hipError_t e = hipMemcpyAsync(counts, a.counter + r + 1, sizeof(int32_t) * nb,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
    for (int q = 0; q < nb; ++q)
      if (counts[q] == 0) return CHERT_OK;
  }
  return fail(CHERT_ERR_NO_CONVERGENCE, "relaxation round cap reached");
}

extern "C" int chert_trace_field(const chert_cache_desc* d, const void* cache_dev,
                                 int64_t n_classes, const chert_grid* g, int32_t mode,
                                 const int64_t* src_nodes_host, int32_t n_src,
                                 const chert_trace_opts* o, double* tau_r_dev,
                                 double* tau_i_dev, double* tstar_dev, int32_t* pred_p_dev,
                                 int32_t* pred_a_dev, void* workspace_dev,
                                 size_t workspace_bytes, void* stream) {
  int rc = validate(d, n_classes, g, mode, n_src, o);
  if (rc) return rc;
  if (!cache_dev) return fail(CHERT_ERR_INVALID_ARG, "null cache");
  if (!src_nodes_host) return fail(CHERT_ERR_INVALID_ARG, "null sources");
  const int64_t n_nodes = g->nx * g->nz;
  for (int i = 0; i < n_src; ++i)
    if (src_nodes_host[i] < 0 || src_nodes_host[i] >= n_nodes)
      return fail(CHERT_ERR_INVALID_ARG, "source node out of range");
  const uint32_t outs = o->outputs;
  if (((outs & CHERT_OUT_TAU_R) && !tau_r_dev) || ((outs & CHERT_OUT_TAU_I) && !tau_i_dev) ||
      ((outs & CHERT_OUT_TSTAR) && !tstar_dev) || ((outs & CHERT_OUT_PRED_P) && !pred_p_dev) ||
      ((outs & CHERT_OUT_PRED_A) && !pred_a_dev))
    return fail(CHERT_ERR_INVALID_ARG, "a selected output is NULL");
  const int64_t K = n_classes;
  WsLayout L = ws_layout(K, g, n_src, o, d->n_dirs);
  if (!workspace_dev || workspace_bytes < L.total)
    return fail(CHERT_ERR_INVALID_ARG, "workspace too small");
  if (K * K * (int64_t)L.n_off > (int64_t)1 << 28)
    return fail(CHERT_ERR_UNSUPPORTED, "class-pair table too large");

  hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)workspace_dev;
  chert_cache_layout lay;
  chert_cache_layout_of(d, K, &lay);
  const uint8_t* cache = (const uint8_t*)cache_dev;
  const int64_t ent = 3 * K * (int64_t)d->n_dirs;
  const int64_t mslice = (int64_t)mode * K * d->n_dirs;
  const double* fields = (const double*)(cache + lay.fields_offset);
  const double* Vm = fields + CHERT_F_V * ent + mslice;
  const double* Am = fields + CHERT_F_A * ent + mslice;
  const int32_t* Sm = (const int32_t*)(cache + lay.status_offset) + mslice;

  // forward star on the host (IEEE sqrt/atan2), uploaded once per call
  std::vector<uint8_t> star(align256((size_t)kMaxOffsets * (3 * sizeof(int32_t) + sizeof(double))));
  int32_t* hox = (int32_t*)star.data();
  int32_t* hoz = hox + kMaxOffsets;
  int32_t* hbin = hoz + kMaxOffsets;
  double* hL = (double*)(hbin + kMaxOffsets);
  star_2d(g->radius, g->hx, g->hz, d->n_dirs, hox, hoz, hL, hbin);
  int32_t* dox = (int32_t*)(ws + L.star);
  int32_t* doz = dox + kMaxOffsets;
  int32_t* dbin = doz + kMaxOffsets;
  double* dL = (double*)(dbin + kMaxOffsets);

  // problems: per source, propagation then attenuation
  std::vector<ProbDev> probs;
  int32_t* hop = (int32_t*)(ws + L.hop);
  for (int i = 0; i < n_src; ++i) {
    int prop_idx = -1;
    if (outs & (CHERT_OUT_TAU_R | CHERT_OUT_PRED_P | CHERT_OUT_TSTAR)) {
      ProbDev p{};
      p.tau = tau_r_dev + (int64_t)i * n_nodes;
      p.pred = (outs & CHERT_OUT_PRED_P) ? pred_p_dev + (int64_t)i * n_nodes : nullptr;
      p.tstar = (outs & CHERT_OUT_TSTAR) ? tstar_dev + (int64_t)i * n_nodes : nullptr;
      p.src = src_nodes_host[i];
      p.field = kFieldR;
      prop_idx = (int)probs.size();
      p.tstar_of = prop_idx;
      p.hop = hop + (int64_t)probs.size() * n_nodes;
      probs.push_back(p);
    }
    if (outs & (CHERT_OUT_TAU_I | CHERT_OUT_PRED_A)) {
      ProbDev p{};
      p.tau = tau_i_dev + (int64_t)i * n_nodes;
      p.pred = (outs & CHERT_OUT_PRED_A) ? pred_a_dev + (int64_t)i * n_nodes : nullptr;
      p.tstar = nullptr;
      p.src = src_nodes_host[i];
      p.field = kFieldI;
      p.tstar_of = -1;
      p.hop = hop + (int64_t)probs.size() * n_nodes;
      probs.push_back(p);
    }
  }
  ProbDev* dprobs = (ProbDev*)(ws + L.probs);
  hipError_t e = hipMemcpyAsync(dox, star.data(), star.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dprobs, probs.data(), probs.size() * sizeof(ProbDev), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // host buffers are locals
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));

  Geom G{};
  G.nx = g->nx;
  G.nz = g->nz;
  tile_dims(o, &G.tx, &G.tz);
  G.ntx = (int)((g->nx + G.tx - 1) / G.tx);
  G.ntz = (int)((g->nz + G.tz - 1) / G.tz);
  G.R = g->radius;
  G.n_off = L.n_off;
  G.lw = G.tx + 2 * G.R;
  G.lh = G.tz + 2 * G.R;
  G.K = (int)K;

  RelaxArgs a{};
  a.g = G;
  a.class_id = g->class_id_dev;
  a.ox = dox;
  a.oz = doz;
  a.W = (const double*)(ws + L.W);
  a.probs = dprobs;
  a.n_prob = (int)probs.size();
  a.flags = (int32_t*)(ws + L.flags);
  a.counter = (int32_t*)(ws + L.counter);
  a.err = (int32_t*)(ws + L.err);
  const size_t lds_base = (size_t)G.lw * G.lh * (sizeof(double) + 2 * sizeof(int32_t)) +
                          sizeof(int32_t) * ((G.n_off + 1) & ~1);
  const size_t wbytes = (size_t)K * K * G.n_off * sizeof(double);
  a.w_in_lds = (lds_base + wbytes <= 48 * 1024) ? 1 : 0;
  const size_t lds = lds_base + (a.w_in_lds ? wbytes : 0);

  {
    int64_t tw = 2 * K * K * G.n_off;
    int64_t blocks = (tw + 255) / 256;
    hipLaunchKernelGGL(k_weights, dim3((unsigned)(blocks > 65536 ? 65536 : blocks)), dim3(256),
                       0, s, (double*)(ws + L.W), (int)K, G.n_off, Vm, Am, Sm, d->n_dirs, dL,
                       dbin);
    int64_t tn = (int64_t)a.n_prob * n_nodes;
    int64_t nb = (tn + 255) / 256;
    hipLaunchKernelGGL(k_init_fields, dim3((unsigned)(nb > 65536 ? 65536 : nb)), dim3(256), 0, s,
                       dprobs, a.n_prob, n_nodes, a.err);
  }
  const int64_t n_flags = 2LL * a.n_prob * L.n_tiles;
  auto init_flags = [&](int tstar_phase) {
    hipLaunchKernelGGL(k_init_flags, dim3(64), dim3(256), 0, s, a.flags, n_flags, a.counter,
                       L.max_rounds + 2);
    hipLaunchKernelGGL(k_seed_flags, dim3((a.n_prob + 63) / 64), dim3(64), 0, s, a.flags,
                       a.counter, dprobs, a.n_prob, G, tstar_phase);
  };
  init_flags(0);
  rc = run_rounds(s, a, k_relax_tau, lds, L.max_rounds);
  if (rc) return rc;
  bool need_pred = (outs & (CHERT_OUT_PRED_P | CHERT_OUT_PRED_A)) != 0;
  if (need_pred) {
    init_flags(0);
    rc = run_rounds(s, a, k_relax_hop, lds, L.max_rounds);
    if (rc) return rc;
    int64_t tn = (int64_t)a.n_prob * n_nodes;
    int64_t nb = (tn + 255) / 256;
    unsigned gb = (unsigned)(nb > 65536 ? 65536 : nb);
    hipLaunchKernelGGL(k_pred, dim3(gb), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_pred_offsets, dim3(gb), dim3(256), 0, s, a);
  }
  if (outs & CHERT_OUT_TSTAR) {
    init_flags(1);
    rc = run_rounds(s, a, k_relax_tstar, lds, L.max_rounds);
    if (rc) return rc;
    int64_t tn = (int64_t)a.n_prob * n_nodes;
    int64_t nb = (tn + 255) / 256;
    hipLaunchKernelGGL(k_tstar_finish, dim3((unsigned)(nb > 65536 ? 65536 : nb)), dim3(256), 0,
                       s, dprobs, a.n_prob, n_nodes);
  }
  int32_t herr = 0;
  e = hipMemcpyAsync(&herr, a.err, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  if (herr) return fail(CHERT_ERR_INVALID_ARG, "class id out of range");
  return CHERT_OK;
}
