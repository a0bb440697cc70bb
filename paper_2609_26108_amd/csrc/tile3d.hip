// 3D traveltime tiles (eq 31 over the 3D forward star, class-pair edge costs
// of eqs 27-30) for gfx950: the tile relaxation of trace.hip carried to 3D.
//
// Every grid of the batch is cut into TX x TX x TZ tiles.  A workgroup (one
// thread per tile node) owns one (problem, tile) per round: it stages the
// tile plus an R-wide halo of traveltimes and class ids in LDS, pulls the
// strips facing the neighbour tiles whose halo part changed (all nodes when
// asked), then pushes over a frontier of improved nodes (64-bit LDS atomic
// min, wavefront ballot compaction) until the tile is locally converged.
// Changed nodes within R of a face, edge or corner wake the neighbour tile
// across it (26 neighbours, the side travels with the flag); rounds repeat
// until one wakes nothing.  Every value written is the left-to-right FP64
// sum along some path and values only decrease, so the fixed point is the
// minimum over paths, bitwise what Dijkstra computes from the same weights.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <vector>

#include "chert.h"
#include "chert_internal.h"
#include "grid_sync.h"

#pragma clang fp contract(off)

namespace chert {

namespace {

constexpr int kT3Threads = 1024;        // tiles of at most 1024 nodes
constexpr int kT3IterCap = 4096;        // push levels per visit before a full re-visit
constexpr int kT3Active = 1, kT3Full = 2, kT3Seed = 4;
constexpr int kT3SideShift = 3;         // bits 3 + s, s = (dz+1)*9 + (dy+1)*3 + (dx+1)
constexpr int kT3Self = 13;             // s of (0, 0, 0)
constexpr int32_t kT3Halo = 0x40000000; // LDS class ids of halo cells carry this bit
constexpr int32_t kT3ClassMask = 0x3fffffff;
constexpr size_t kT3WLdsBytes = 48 * 1024;

struct T3JobDev {
  int nx, ny, nz, K;
  int ntx, nty, ntz, pad;
  const int32_t* cls;
  const double* W;  // [2][K][K][n_off]
};

struct T3ProbDev {
  double* tau;
  int64_t src;
  int job, field, tile_base, pad;
};

struct T3Args {
  int tx, tz, R, n_off;
  int lx, lz;          // LDS box: lx x lx x lz (tile + 2R per axis)
  int n_prob, n_tiles;
  int w_lds;           // doubles of the class-pair table staged in LDS (0: read from L2)
  int pad;
  const T3JobDev* jobs;
  const T3ProbDev* probs;
  const int32_t* ox;
  const int32_t* oy;
  const int32_t* oz;
  int32_t* flags;    // [2][n_tiles] by round parity
  int32_t* list;     // [2][n_tiles] tiles active in a round
  int32_t* counter;  // [counter_words(max_rounds)]: list lengths, then tickets
  uint32_t* tick;    // [2][kTickWords] tickets of the per-round list walk, by round parity
  int32_t* err;
  unsigned long long* stats;  // [kStatSlots][16] shards of: [0] visits, [1] edges examined
  // the caller's abort word (device view of pinned host memory, nullable)
  // and the device word recording that it was seen (persistent launch)
  const int32_t* abort_host;
  int32_t* abort_seen;
};

__device__ __forceinline__ unsigned long long dbits3(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

__device__ __forceinline__ void frontier_add3(bool flag, int node, int32_t* list, int* count) {
  const unsigned long long b = __ballot(flag);
  if (b == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)b) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(b));
  base = __shfl(base, leader);
  if (flag) list[base + __popcll(b & ((1ull << lane) - 1ull))] = node;
}

// which neighbour tiles see interior node (x, y, z) in their halo
__device__ __forceinline__ int border_bits3(int x, int y, int z, int tx, int tz, int R) {
  int m = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const bool okz = dz == 0 || (dz < 0 && z < R) || (dz > 0 && z >= tz - R);
    if (!okz) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const bool oky = dy == 0 || (dy < 0 && y < R) || (dy > 0 && y >= tx - R);
      if (!oky) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        const bool okx = dx == 0 || (dx < 0 && x < R) || (dx > 0 && x >= tx - R);
        if (okx) m |= 1 << ((dz + 1) * 9 + (dy + 1) * 3 + (dx + 1));
      }
    }
  }
  return m;
}

// Does this visit pull interior node (x, y, z)?  The strips facing the
// neighbours whose halo part changed, or every node on a full visit.
__device__ __forceinline__ bool pulls3(int flag, int x, int y, int z, int tx, int tz, int R) {
  if (flag & kT3Full) return true;
  const int sides = (flag >> kT3SideShift) & 0x7ffffff;
  if (!sides) return false;
  const bool nx[3] = {x < R, true, x >= tx - R};
  const bool ny[3] = {y < R, true, y >= tx - R};
  const bool nz[3] = {z < R, true, z >= tz - R};
  for (int s = 0; s < 27; ++s)
    if (((sides >> s) & 1) && nx[s % 3] && ny[(s / 3) % 3] && nz[s / 9]) return true;
  return false;
}

__global__ void k_tile3_clear(int32_t* flags, int64_t n_flags, int32_t* counter, int n_counter,
                              int32_t* err, unsigned long long* stats) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t t = tid; t < n_flags; t += (int64_t)gridDim.x * blockDim.x) flags[t] = 0;
  for (int64_t t = tid; t < n_counter; t += (int64_t)gridDim.x * blockDim.x) counter[t] = 0;
  if (tid < 64) err[tid] = 0;  // error word, barrier words, result, abort record
  for (int64_t t = tid; t < kStatSlots * kStatSlotU64; t += (int64_t)gridDim.x * blockDim.x)
    stats[t] = 0ull;
}

// activate the source tile of every problem
__global__ void k_tile3_seed(T3Args a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_prob) return;
  const T3ProbDev P = a.probs[p];
  const T3JobDev J = a.jobs[P.job];
  const int sx = (int)(P.src % J.nx), sy = (int)((P.src / J.nx) % J.ny),
            sz = (int)(P.src / ((int64_t)J.nx * J.ny));
  const int T = P.tile_base + ((sz / a.tz) * J.nty + sy / a.tx) * J.ntx + sx / a.tx;
  a.flags[T] = kT3Active | kT3Seed;
  a.list[atomicAdd(&a.counter[0], 1)] = T;
}

template <int G>
__device__ void visit3(const T3Args& a, int round, int T) {
  extern __shared__ double smem3[];
  __shared__ int s_flag, s_prob, s_mask, s_cnt[3], s_npull;
  if (threadIdx.x == 0) {
    int32_t* fin = a.flags + (int64_t)(round & 1) * a.n_tiles;
    const int32_t f = fin[T];
    if (f) {
      fin[T] = 0;
      int lo = 0, hi = a.n_prob - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.probs[mid].tile_base <= T) lo = mid;
        else hi = mid - 1;
      }
      s_prob = lo;
    }
    s_flag = f;
    s_mask = 0;
    s_npull = 0;
    s_cnt[0] = s_cnt[1] = s_cnt[2] = 0;
  }
  __syncthreads();
  const int flag = s_flag;
  if (!flag) return;  // block-uniform
  const T3ProbDev P = a.probs[s_prob];
  const T3JobDev J = a.jobs[P.job];
  const int R = a.R, lx = a.lx, lz = a.lz, n_off = a.n_off, tx = a.tx, tz = a.tz;
  const int t = T - P.tile_base;
  const int ttx = t % J.ntx, tty = (t / J.ntx) % J.nty, ttz = t / (J.ntx * J.nty);
  const int x0 = ttx * tx, y0 = tty * tx, z0 = ttz * tz;
  const int txe = min(tx, J.nx - x0), tye = min(tx, J.ny - y0), tze = min(tz, J.nz - z0);
  const int nbox = lx * lx * lz;
  // LDS carve: values, class-pair table, class ids, queue marks, offsets, frontiers
  double* val = smem3;
  double* Ws = val + nbox;
  int32_t* cls = (int32_t*)(Ws + a.w_lds);
  int32_t* inq = cls + nbox;
  int32_t* off = inq + nbox;
  int32_t* l0 = off + ((n_off + 1) & ~1);
  int32_t* l1 = l0 + tx * tx * tz;

  for (int q = threadIdx.x; q < nbox; q += blockDim.x) {
    const int qx = q % lx, qy = (q / lx) % lx, qz = q / (lx * lx);
    const int gx = x0 + qx - R, gy = y0 + qy - R, gz = z0 + qz - R;
    int32_t k = -1;
    double v = INFINITY;
    if (gx >= 0 && gx < J.nx && gy >= 0 && gy < J.ny && gz >= 0 && gz < J.nz) {
      const int64_t g = gx + (int64_t)J.nx * (gy + (int64_t)J.ny * gz);
      k = J.cls[g];
      v = P.tau[g];
      if (k < 0 || k >= J.K) {
        atomicAdd(a.err, 1);
        k = -2;
      } else if (qx - R >= txe || qy - R >= tye || qz - R >= tze || qx < R || qy < R || qz < R) {
        k |= kT3Halo;
      }
    }
    val[q] = v;
    cls[q] = k;
    inq[q] = 0;
  }
  for (int o = threadIdx.x; o < n_off; o += blockDim.x)
    off[o] = a.ox[o] + lx * (a.oy[o] + lx * a.oz[o]);
  const double* Wf = J.W + (int64_t)P.field * J.K * J.K * n_off;
  const double* Wp = Wf;
  if (a.w_lds) {
    const int kk = J.K * J.K * n_off;
    for (int q = threadIdx.x; q < kk; q += blockDim.x) Ws[q] = Wf[q];
    Wp = Ws;
  }
  __syncthreads();

  // this thread's interior node
  int ml = -1, ix = 0, iy = 0, iz = 0;
  if ((int)threadIdx.x < tx * tx * tz) {
    ix = threadIdx.x % tx;
    iy = (threadIdx.x / tx) % tx;
    iz = threadIdx.x / (tx * tx);
    if (ix < txe && iy < tye && iz < tze) ml = (ix + R) + lx * ((iy + R) + lx * (iz + R));
  }
  const double orig = ml >= 0 ? val[ml] : 0.0;
  {
    bool improved = false;
    if (ml >= 0 && pulls3(flag, ix, iy, iz, tx, tz, R)) {
      atomicAdd(&s_npull, 1);
      const int kj = cls[ml];
      if (kj >= 0) {
        const double cur = val[ml];
        double best = cur;
        for (int o = 0; o < n_off; ++o) {
          const int ii = ml - off[o];
          const int ki = cls[ii];
          if (ki < 0) continue;
          const double cand =
              __dadd_rn(val[ii], Wp[(int64_t)((ki & kT3ClassMask) * J.K + kj) * n_off + o]);
          if (cand < best) best = cand;
        }
        if (best < cur) {
          val[ml] = best;
          inq[ml] = 1;
          improved = true;
        }
      }
    }
    frontier_add3(improved, ml, l0, &s_cnt[0]);
  }
  if (threadIdx.x == 0 && (flag & kT3Seed)) {
    const int sx = (int)(P.src % J.nx) - x0, sy = (int)((P.src / J.nx) % J.ny) - y0,
              sz = (int)(P.src / ((int64_t)J.nx * J.ny)) - z0;
    if (sx >= 0 && sx < txe && sy >= 0 && sy < tye && sz >= 0 && sz < tze) {
      const int sn = (sx + R) + lx * ((sy + R) + lx * (sz + R));
      if (cls[sn] >= 0 && atomicExch(&inq[sn], 1) != 1) l0[atomicAdd(&s_cnt[0], 1)] = sn;
    }
  }
  __syncthreads();

  // push levels; counters rotate over three slots, the dedupe stamp is the level
  long long raw = 0;
  int ci = 0, it = 1;
  int nf = s_cnt[0];
  const int nt = blockDim.x;
  const int ngroups = (n_off + G - 1) / G;
  const int q_step = nt / ngroups, r_step = nt % ngroups;
  while (nf > 0 && it <= kT3IterCap) {
    const int cn = ci == 2 ? 0 : ci + 1, cz = cn == 2 ? 0 : cn + 1;
    int32_t* const lcur = (it & 1) ? l0 : l1;
    int32_t* const lnxt = (it & 1) ? l1 : l0;
    if (threadIdx.x == 0) s_cnt[cz] = 0;
    raw += (long long)nf * n_off;
    const int total = nf * ngroups;
    const int bound = (total + nt - 1) / nt * nt;
    int f = threadIdx.x / ngroups, g = threadIdx.x % ngroups;
    for (int item = threadIdx.x; item < bound; item += nt) {
      const bool live = item < total;
      const int i = live ? lcur[f] : 0;
#pragma unroll
      for (int u = 0; u < G; ++u) {
        bool improved = false;
        int jj = 0;
        const int o = g * G + u;
        if (live && o < n_off) {
          const int j = i + off[o];
          const int kj = cls[j];
          if (kj >= 0 && !(kj & kT3Halo)) {
            const int ki = cls[i] & kT3ClassMask;
            const double cand = __dadd_rn(val[i], Wp[(int64_t)(ki * J.K + kj) * n_off + o]);
            if (cand < val[j]) {
              const unsigned long long old = atomicMin((unsigned long long*)&val[j], dbits3(cand));
              if (dbits3(cand) < old) {
                improved = atomicExch(&inq[j], it + 1) != it + 1;
                jj = j;
              }
            }
          }
        }
        frontier_add3(improved, jj, lnxt, &s_cnt[cn]);
      }
      f += q_step;
      g += r_step;
      if (g >= ngroups) {
        g -= ngroups;
        ++f;
      }
    }
    __syncthreads();
    nf = s_cnt[cn];
    ci = cn;
    ++it;
  }

  int mask = (nf > 0) ? (1 << kT3Self) : 0;  // iteration cap: this tile again, in full
  if (ml >= 0 && val[ml] < orig) {
    P.tau[(x0 + ix) + (int64_t)J.nx * ((y0 + iy) + (int64_t)J.ny * (z0 + iz))] = val[ml];
    mask |= border_bits3(ix, iy, iz, tx, tz, R);
  }
  if (mask) atomicOr(&s_mask, mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long* st = stat_slot(a.stats);
    atomicAdd(&st[0], 1ull);
    atomicAdd(&st[1], (unsigned long long)(raw + (long long)s_npull * n_off));
    const int m = s_mask;
    if (m) {
      int32_t* fout = a.flags + (int64_t)((round + 1) & 1) * a.n_tiles;
      int32_t* lout = a.list + (int64_t)((round + 1) & 1) * a.n_tiles;
      int fresh = 0;
      for (int s = 0; s < 27; ++s) {
        if (!((m >> s) & 1)) continue;
        const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
        const int nx_ = ttx + dx, ny_ = tty + dy, nz_ = ttz + dz;
        if (nx_ < 0 || nx_ >= J.ntx || ny_ < 0 || ny_ >= J.nty || nz_ < 0 || nz_ >= J.ntz) continue;
        const int TN = P.tile_base + (nz_ * J.nty + ny_) * J.ntx + nx_;
        // the neighbour's halo part facing us (its side -d) changed
        const int32_t bits = (s == kT3Self) ? (kT3Active | kT3Full)
                                            : (kT3Active | (1 << (kT3SideShift + 26 - s)));
        if (atomicOr(&fout[TN], bits) == 0) fresh |= 1 << s;
      }
      // one reservation for the newly activated tiles (the counter is one
      // address for the whole chip)
      if (fresh) {
        int slot = atomicAdd(&a.counter[round + 1], __popc(fresh));
        for (int s = 0; s < 27; ++s)
          if ((fresh >> s) & 1)
            lout[slot++] = P.tile_base + ((ttz + s / 9 - 1) * J.nty + (tty + (s / 3) % 3 - 1)) * J.ntx +
                           (ttx + s % 3 - 1);
      }
    }
  }
}

// One launch per round: one workgroup per tile (affinity), or a smaller grid
// walking the round's active list on large batches.
template <int G>
__global__ void __launch_bounds__(kT3Threads) k_tile3_tau(T3Args a, int round) {
  if ((int)gridDim.x == a.n_tiles) {
    visit3<G>(a, round, blockIdx.x);
    return;
  }
  const int n_act = a.counter[round];
  const int32_t* lst = a.list + (int64_t)(round & 1) * a.n_tiles;
  // tiles by ticket as workgroups free up; the next round's ticket lines
  // (last used a round ago) start from zero
  if (blockIdx.x == 0)
    for (int q = threadIdx.x; q < kTickWords; q += blockDim.x)
      a.tick[((round + 1) & 1) * kTickWords + q] = 0u;
  uint32_t* tick = a.tick + (round & 1) * kTickWords;
  const Shard sh = shard_of();
  for (int i = first_item(sh, n_act); i >= 0;) {
    const uint32_t t = draw_ticket(tick, sh, n_act);  // the next entry's, in flight meanwhile
    visit3<G>(a, round, lst[i]);
    __syncthreads();  // LDS is reused by the next tile
    i = ticket_item(sh, 0u, n_act, t);
  }
}

// All rounds in one launch: an occupancy-sized grid walks each round's
// active list; rounds are separated by the bounded device-wide barrier.
// The caller's abort word is polled once per round by workgroup 0 and
// published by the barrier, so every workgroup leaves together.  Result:
// rounds to convergence, -1 cap reached, -2 barrier timed out, -3 aborted.
template <int G>
__global__ void __launch_bounds__(kT3Threads) k_tile3_persist(T3Args a, PersistArgs p) {
  const Shard sh = shard_of();
  uint32_t base = 0;  // tickets of this workgroup's shard issued before this round
  for (int round = 0; round < p.max_rounds; ++round) {
    const int n_act =
        __hip_atomic_load(&a.counter[round], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t* lst = a.list + (int64_t)(round & 1) * a.n_tiles;
    for (int i = first_item(sh, n_act); i >= 0;) {
      const uint32_t t = draw_ticket(p.tick, sh, n_act);  // the next entry's, in flight meanwhile
      visit3<G>(a, round, lst[i]);
      __syncthreads();  // LDS is reused by the next tile
      i = ticket_item(sh, base, n_act, t);
    }
    base += round_tickets(sh, n_act);
    if (a.abort_host && blockIdx.x == 0 && threadIdx.x == 0 &&
        __hip_atomic_load(a.abort_host, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0)
      __hip_atomic_store(a.abort_seen, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!grid_barrier(p)) {
      if (threadIdx.x == 0) p.result[0] = -2;
      return;
    }
    if (a.abort_host &&
        __hip_atomic_load(a.abort_seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
      if (blockIdx.x == 0 && threadIdx.x == 0) p.result[0] = -3;
      return;
    }
    if (__hip_atomic_load(&a.counter[round + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
        0) {
      if (blockIdx.x == 0 && threadIdx.x == 0) p.result[0] = round + 1;
      return;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) p.result[0] = -1;
}

size_t align256_t3(size_t x) { return (x + 255) & ~(size_t)255; }

struct T3Plan {
  int tx = 0, tz = 0, lx = 0, lz = 0, n_tiles = 0, w_lds = 0;
  size_t off_jobs = 0, off_probs = 0, off_flags = 0, off_list = 0, off_counter = 0, off_err = 0,
         off_stats = 0, total = 0;
  size_t lds = 0;
};

int plan_t3(const Tile3Job* jobs, int n_jobs, const Tile3Prob* probs, int n_prob, int R,
            int n_off, int tile_x, int tile_z, int max_rounds, T3Plan* P) {
  P->tx = tile_x > 0 ? tile_x : 8;
  P->tz = tile_z > 0 ? tile_z : 8;
  if (P->tx < R || P->tz < R || P->tx * P->tx * P->tz > kT3Threads)
    return fail(CHERT_ERR_INVALID_ARG, "3D tile must be >= radius per side and <= 1024 nodes");
  P->lx = P->tx + 2 * R;
  P->lz = P->tz + 2 * R;
  int64_t tiles = 0;
  int maxK = 0;
  for (int q = 0; q < n_prob; ++q) {
    const Tile3Job& J = jobs[probs[q].job];
    tiles += (int64_t)((J.nx + P->tx - 1) / P->tx) * ((J.ny + P->tx - 1) / P->tx) *
             ((J.nz + P->tz - 1) / P->tz);
  }
  for (int j = 0; j < n_jobs; ++j) maxK = jobs[j].K > maxK ? jobs[j].K : maxK;
  if (tiles >= 0x7fffffffLL) return fail(CHERT_ERR_UNSUPPORTED, "batch too large for one launch");
  P->n_tiles = (int)tiles;
  const size_t wbytes = (size_t)maxK * maxK * n_off * sizeof(double);
  P->w_lds = wbytes <= kT3WLdsBytes ? (int)(wbytes / sizeof(double)) : 0;
  const size_t nbox = (size_t)P->lx * P->lx * P->lz;
  P->lds = nbox * sizeof(double) + (size_t)P->w_lds * sizeof(double) + 2 * nbox * sizeof(int32_t) +
           (size_t)((n_off + 1) & ~1) * sizeof(int32_t) +
           2 * (size_t)P->tx * P->tx * P->tz * sizeof(int32_t);
  size_t off = 0;
  P->off_jobs = off;
  off += align256_t3((size_t)n_jobs * sizeof(T3JobDev));
  P->off_probs = off;
  off += align256_t3((size_t)n_prob * sizeof(T3ProbDev));
  P->off_flags = off;
  off += align256_t3((size_t)2 * P->n_tiles * sizeof(int32_t));
  P->off_list = off;
  off += align256_t3((size_t)2 * P->n_tiles * sizeof(int32_t));
  P->off_counter = off;
  off += align256_t3(counter_words(max_rounds) * sizeof(int32_t));  // counts, tickets
  P->off_err = off;
  off += 256;
  P->off_stats = off;
  off += align256_t3(kStatBytes);
  P->total = off;
  return CHERT_OK;
}

int threads_of(const T3Plan& P) { return (P.tx * P.tx * P.tz + 63) / 64 * 64; }

// Error word and the sharded statistics, after the relaxation (synchronous).
int read_back(const T3Args& a, hipStream_t s, int32_t* herr, int64_t* visits, int64_t* edges) {
  unsigned long long hs[2] = {0, 0};
  std::vector<unsigned long long> slots((size_t)kStatSlots * kStatSlotU64);
  hipError_t e = hipMemcpyAsync(herr, a.err, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(slots.data(), a.stats, kStatBytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  stats_reduce(slots.data(), 2, 0u, hs);
  *visits = (int64_t)hs[0];
  *edges = (int64_t)hs[1];
  return CHERT_OK;
}

// Every round in one launch of an occupancy-sized grid (all of its
// workgroups resident, which the device-wide barrier needs).
int run_persistent(const T3Plan& P, const T3Args& a, int push_group, int max_rounds, int threads,
                   hipStream_t s, int* rounds, int64_t* visits, int64_t* edges) {
  void (*kern)(T3Args, PersistArgs) =
      push_group == 1 ? k_tile3_persist<1> : (push_group == 4 ? k_tile3_persist<4>
                                                              : k_tile3_persist<2>);
  int per_cu = 0, cus = 0, dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, P.lds);
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  if (per_cu < 1) return fail(CHERT_ERR_UNSUPPORTED, "3D tile does not fit on a compute unit");
  const int64_t resident = (int64_t)per_cu * cus;
  const int grid = (int)(P.n_tiles < resident ? P.n_tiles : resident);
  PersistArgs pa{};
  pa.max_rounds = max_rounds;
  pa.bar = (uint32_t*)(a.err + 48);  // [0] arrivals, [1] generation, [2] abort
  pa.result = a.err + 52;
  pa.tick = (uint32_t*)a.counter + tick_offset(max_rounds);
  CHERT_LAUNCH("k_tile3_clear", k_tile3_clear, dim3(256), dim3(256), 0, s, a.flags,
               (int64_t)2 * P.n_tiles, a.counter, (int)counter_words(max_rounds), a.err, a.stats);
  CHERT_LAUNCH("k_tile3_seed", k_tile3_seed, dim3((a.n_prob + 63) / 64), dim3(64), 0, s, a);
  CHERT_LAUNCH("k_tile3_persist", kern, dim3((unsigned)grid), dim3((unsigned)threads), P.lds, s,
               a, pa);
  int32_t res = 0, herr = 0;
  e = hipMemcpyAsync(&res, pa.result, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  int rc = read_back(a, s, &herr, visits, edges);
  if (rc) return rc;
  *rounds = res > 0 ? res : max_rounds;
  if (res == -3) return fail(CHERT_ERR_ABORTED, "aborted by the caller");
  if (res == -2) return fail(CHERT_ERR_HIP, "device-wide barrier timed out");
  if (res <= 0) return fail(CHERT_ERR_NO_CONVERGENCE, "relaxation round cap reached");
  if (herr) return fail(CHERT_ERR_INVALID_ARG, "class id out of range");
  return CHERT_OK;
}

}  // namespace

int tiles3d_bytes(const Tile3Job* jobs, int n_jobs, const Tile3Prob* probs, int n_prob, int R,
                  int n_off, int tile_x, int tile_z, int max_rounds, size_t* bytes) {
  T3Plan P;
  const int rc = plan_t3(jobs, n_jobs, probs, n_prob, R, n_off, tile_x, tile_z, max_rounds, &P);
  *bytes = rc ? 0 : P.total;
  return rc;
}

int relax_tiles_3d(const Tile3Job* jobs, int n_jobs, const Tile3Prob* probs, int n_prob,
                   const int32_t* ox_dev, const int32_t* oy_dev, const int32_t* oz_dev, int n_off,
                   int R, int tile_x, int tile_z, int push_group, int max_rounds, void* ws,
                   size_t ws_bytes, hipStream_t s, const volatile int32_t* abort_flag,
                   bool persistent, int* rounds, int64_t* visits, int64_t* edges) {
  T3Plan P;
  int rc = plan_t3(jobs, n_jobs, probs, n_prob, R, n_off, tile_x, tile_z, max_rounds, &P);
  if (rc) return rc;
  if (!ws || ws_bytes < P.total) return fail(CHERT_ERR_INVALID_ARG, "workspace too small");
  uint8_t* w = (uint8_t*)ws;
  std::vector<T3JobDev> jd(n_jobs);
  for (int j = 0; j < n_jobs; ++j) {
    jd[j].nx = jobs[j].nx;
    jd[j].ny = jobs[j].ny;
    jd[j].nz = jobs[j].nz;
    jd[j].K = jobs[j].K;
    jd[j].ntx = (jobs[j].nx + P.tx - 1) / P.tx;
    jd[j].nty = (jobs[j].ny + P.tx - 1) / P.tx;
    jd[j].ntz = (jobs[j].nz + P.tz - 1) / P.tz;
    jd[j].cls = jobs[j].cls;
    jd[j].W = jobs[j].W;
  }
  std::vector<T3ProbDev> pd(n_prob);
  int base = 0;
  for (int q = 0; q < n_prob; ++q) {
    pd[q].tau = probs[q].tau;
    pd[q].src = probs[q].src;
    pd[q].job = probs[q].job;
    pd[q].field = probs[q].field;
    pd[q].tile_base = base;
    const T3JobDev& J = jd[probs[q].job];
    base += J.ntx * J.nty * J.ntz;
  }
  hipError_t e = hipMemcpyAsync(w + P.off_jobs, jd.data(), jd.size() * sizeof(T3JobDev),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(w + P.off_probs, pd.data(), pd.size() * sizeof(T3ProbDev),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // host buffers are locals
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  T3Args a{};
  a.tx = P.tx;
  a.tz = P.tz;
  a.R = R;
  a.n_off = n_off;
  a.lx = P.lx;
  a.lz = P.lz;
  a.n_prob = n_prob;
  a.n_tiles = P.n_tiles;
  a.w_lds = P.w_lds;
  a.jobs = (const T3JobDev*)(w + P.off_jobs);
  a.probs = (const T3ProbDev*)(w + P.off_probs);
  a.ox = ox_dev;
  a.oy = oy_dev;
  a.oz = oz_dev;
  a.flags = (int32_t*)(w + P.off_flags);
  a.list = (int32_t*)(w + P.off_list);
  a.counter = (int32_t*)(w + P.off_counter);
  a.err = (int32_t*)(w + P.off_err);
  a.stats = (unsigned long long*)(w + P.off_stats);
  a.tick = (uint32_t*)a.counter + tick_offset(max_rounds);
  a.abort_seen = a.err + 56;
  a.abort_host = nullptr;
  if (persistent && abort_flag) {
    // the persistent grid polls the word itself: page-locked host memory only
    hipPointerAttribute_t at{};
    const hipError_t pe = hipPointerGetAttributes(&at, (const void*)abort_flag);
    if (pe != hipSuccess || at.type != hipMemoryTypeHost || !at.devicePointer) {
      (void)hipGetLastError();
      return fail(CHERT_ERR_INVALID_ARG, "abort_flag_host must be pinned host memory");
    }
    a.abort_host = (const int32_t*)at.devicePointer;
  }
  if (persistent) return run_persistent(P, a, push_group, max_rounds, threads_of(P), s, rounds,
                                        visits, edges);
  void (*kern)(T3Args, int) = push_group == 1 ? k_tile3_tau<1> : (push_group == 4 ? k_tile3_tau<4>
                                                                                   : k_tile3_tau<2>);
  const int threads = threads_of(P);
  int per_cu = 0, cus = 0, dev = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, P.lds);
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  if (per_cu < 1) return fail(CHERT_ERR_UNSUPPORTED, "3D tile does not fit on a compute unit");
  const int64_t resident = (int64_t)per_cu * cus;
  // one workgroup per tile up to twice the resident workgroups, else twice
  // the resident walking each round's list by ticket (twice measured 5 %
  // faster than four times on the 3D layered batch)
  const int grid = (int)(P.n_tiles <= 2 * resident ? P.n_tiles : 2 * resident);
  CHERT_LAUNCH("k_tile3_clear", k_tile3_clear, dim3(256), dim3(256), 0, s, a.flags,
               (int64_t)2 * P.n_tiles, a.counter, (int)counter_words(max_rounds), a.err, a.stats);
  CHERT_LAUNCH("k_tile3_seed", k_tile3_seed, dim3((n_prob + 63) / 64), dim3(64), 0, s, a);
  const int batch = 8;
  int32_t counts[batch];
  int done = -1;
  for (int r = 0; r < max_rounds && done < 0; r += batch) {
    const int nb = r + batch > max_rounds ? max_rounds - r : batch;
    for (int q = 0; q < nb; ++q)
      CHERT_LAUNCH("k_tile3_tau", kern, dim3((unsigned)grid), dim3((unsigned)threads), P.lds, s, a,
                   r + q);
    e = hipMemcpyAsync(counts, a.counter + r + 1, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
    for (int q = 0; q < nb && done < 0; ++q)
      if (counts[q] == 0) done = r + q + 1;
    if (done < 0 && abort_flag && *abort_flag) {
      *rounds = r + nb;
      return fail(CHERT_ERR_ABORTED, "aborted by the caller");
    }
  }
  int32_t herr = 0;
  rc = read_back(a, s, &herr, visits, edges);
  if (rc) return rc;
  *rounds = done < 0 ? max_rounds : done;
  if (done < 0) return fail(CHERT_ERR_NO_CONVERGENCE, "relaxation round cap reached");
  if (herr) return fail(CHERT_ERR_INVALID_ARG, "class id out of range");
  return CHERT_OK;
}

}  // namespace chert
