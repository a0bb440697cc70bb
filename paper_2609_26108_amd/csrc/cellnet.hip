// The cell network of the grid and nodal ray-network section (eqs 23-24,
// 27-32) on gfx950: nodes on the edges of rectangular cells, every pair of
// boundary nodes of a cell joined by a straight segment, the traveltimes
// marched cell by cell.
//
// Traveltimes: one wave per (problem, cell) visit, one lane per boundary node
// (4 cn <= 64).  The wave loads its cell's traveltimes and classes once,
// stages the weights of the cell's ordered pairs in LDS, then relaxes every
// ordered pair (eq 31) from lane broadcasts until a pass changes nothing
// (Jacobi passes inside the cell), and lowers the improved
// nodes in HBM with a 64-bit atomicMin on the traveltime bits (traveltimes
// are >= 0, so their bit patterns order like the values).  A cell is woken
// with key = the smallest improved traveltime among its nodes (the block
// traveltime of eq 24 over what changed); with an ordering width each round
// takes only the woken cells whose key is within the width of its problem's
// smallest key (the heap of cells of eqs 23 and 32 widened to a bucket, so a
// round holds many cells).  The fixed point is the network's shortest-path
// traveltimes whatever the schedule.
//
// Predecessors and t*: level-synchronous BFS over tight segments
// (tau_i + w_ij == tau_j) from the source, one launch per level, threads
// over (node, boundary slot) pairs: pred_j = the tight neighbour one
// level up with the smallest node
// index (the smallest (hop, index) among all tight neighbours), t*_j =
// t*_pred + the attenuation weight of that segment, each parent's value
// final one level earlier.
//
// 3D (the paper's blocks): the same kernels instantiated for boxes of cn^3
// lattice intervals whose nodes are the face points, (cn + 1)^3 - (cn - 1)^3
// <= 64 of them for cn <= 3, one lane each; a block has up to 26 neighbours
// and a node lies on up to 8 blocks.  Segment columns are the closest
// Fibonacci direction of the 3D cache.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <vector>

#include "chert_internal.h"

namespace chert {
namespace {

constexpr int kCellMaxN = 16;  // 4 cn boundary nodes <= 64 lanes
constexpr int kBlockMaxN = 3;  // (cn + 1)^3 - (cn - 1)^3 face nodes <= 64 lanes
constexpr int kCellWaves = 4;  // waves per workgroup
constexpr int kCellThreads = 64 * kCellWaves;
constexpr int kRelaxGrid = 4096;  // most workgroups of a relax launch
constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

__device__ __forceinline__ double bcast_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// order one wave's LDS writes before its later LDS reads (other lanes')
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// boundary slot s of a cell of side cn -> local lattice point (lx, lz):
// top edge left to right, right edge downwards, bottom edge right to left,
// left edge upwards; each boundary point once
__device__ __forceinline__ void slot_xy(int s, int cn, int& lx, int& lz) {
  const int e = s / cn, r = s - e * cn;
  if (e == 0) {
    lx = r;
    lz = 0;
  } else if (e == 1) {
    lx = cn;
    lz = r;
  } else if (e == 2) {
    lx = cn - r;
    lz = cn;
  } else {
    lx = 0;
    lz = cn - r;
  }
}

// the cells whose boundary holds lattice point (gx, gz) (a node), at most 4
__device__ __forceinline__ int cells_of(int gx, int gz, int cn, int ncx, int ncz, int* cs) {
  int xs[2], zs[2], nx = 0, nz = 0;
  const int qx = gx / cn, qz = gz / cn;
  if (gx - qx * cn == 0) {
    if (qx - 1 >= 0) xs[nx++] = qx - 1;
    if (qx < ncx) xs[nx++] = qx;
  } else {
    xs[nx++] = qx;
  }
  if (gz - qz * cn == 0) {
    if (qz - 1 >= 0) zs[nz++] = qz - 1;
    if (qz < ncz) zs[nz++] = qz;
  } else {
    zs[nz++] = qz;
  }
  int n = 0;
  for (int a = 0; a < nx; ++a)
    for (int b = 0; b < nz; ++b) cs[n++] = xs[a] + ncx * zs[b];
  return n;
}

// the cell indices along one axis whose closed range holds coordinate q
__device__ __forceinline__ int cells_along(int q, int cn, int nc, int* out) {
  const int c = q / cn;
  if (q - c * cn != 0) {
    out[0] = c;
    return 1;
  }
  int n = 0;
  if (c - 1 >= 0) out[n++] = c - 1;
  if (c < nc) out[n++] = c;
  return n;
}

struct CellArgs;
template <bool D3>
__device__ __forceinline__ int node_cells(const CellArgs& a, int64_t u, int* cs);

struct CellArgs {
  int ncx, ncz, cn, side, NX, K, n_src, n_prob;
  int ncy, NY;         // 3D: blocks and lattice points along y (2D: 1, 1)
  int ns, n_off;       // boundary nodes per cell; segment offsets (side^dim)
  int64_t n, C;
  const int32_t* cls;  // lattice -> class
  const int32_t* slot; // 3D: [ns] local point of slot s, lx | ly << 8 | lz << 16
  const double* W;     // [2][K][K][n_off]
  double* tau[2];      // per field slot: rows [n_src][n]
  int field_of[2];     // field slot -> 0 (propagation) or 1 (attenuation)
  const int64_t* src;  // [n_src]
  int32_t* active;     // [P][C]
  unsigned long long* key;     // [P][C]
  unsigned long long* minkey;  // [3][P]: round r reads slot r % 3
  int32_t* list;               // [P C] selected (problem, cell) items
  int32_t* count;              // [2] (round parity)
  unsigned long long* stats;   // visits, pair relaxations, passes, MSPM corner jobs
  unsigned long long* part;    // [kRelaxGrid][3] per-workgroup visits, pairs, passes
  const double* wmin;          // [2]
  double bucket;               // ordering width in units of wmin (0: none)
  // level phase
  int32_t* hop;        // [P][n]
  int32_t* bfs;        // [P][n] BFS order
  int32_t* bid;        // [P][n] predecessor bids (atomicMin)
  int32_t* bnd;        // [3][P] end of level L in slot L % 3
  int32_t* cnt;        // [3][P] nodes appended during level L in slot L % 3
  int32_t* alive;      // most BFS levels over the problems
  int32_t* pred[2];    // per field slot, rows [n_src][n] (nullable)
  double* tstar;       // rows [n_src][n] for the propagation slot (nullable)
  int tree_mask;       // bit fi: problems of field slot fi need the tree
  // MSPM (no cache): corner tables [row][n_canon] of V, A, status per
  // canonical segment offset; the rounds read one row per visited cell
  // corner (row it * 4 + corner of the round's list), the tree phase one row
  // per class
  int mspm;
  int n_canon;
  const int32_t* canon;  // [side^2] canonical offset index (-1: centre)
  const double* L;       // [side^2] segment lengths
  const double *tV, *tA;
  const int32_t* tS;     // visit tables
  int w_lds;             // the class-pair table is staged in LDS by k_cell_relax
  const double *kV, *kA;
  const int32_t* kS;     // class table
  int32_t* job_class;    // [4 P C] class of each (visit, corner) solve job
};

// MSPM quantities of the node at local (lx, lz) of a cell along canonical
// offset ci: at a corner its own row; between the corners q1, q2 of its
// edge, at fraction t of the edge from q1, x = x1 + t (x2 - x1) for V and A.
// Corner q: 0 = (0, 0), 1 = (cn, 0), 2 = (0, cn), 3 = (cn, cn); row[q] is
// the table row of corner q.
struct Rows4 {
  int64_t r0, r1, r2, r3;
  __device__ __forceinline__ int64_t operator[](int q) const {
    return q == 0 ? r0 : (q == 1 ? r1 : (q == 2 ? r2 : r3));  // selects, no memory
  }
};

__device__ __forceinline__ int32_t mspm_node(int cn, const Rows4& row, int lx, int lz, int ci,
                                             const double* V, const double* A, const int32_t* S,
                                             double* v, double* at) {
  const bool ex = lx == 0 || lx == cn, ez = lz == 0 || lz == cn;
  if (ex && ez) {
    const int64_t r = row[(lx == cn) + 2 * (lz == cn)] + ci;
    *v = V[r];
    *at = A[r];
    return S[r];
  }
  int q1, q2;
  double t;
  if (ez) {  // horizontal edge: corners (0, lz) and (cn, lz)
    q1 = 2 * (lz == cn);
    q2 = q1 + 1;
    t = (double)lx / (double)cn;
  } else {   // vertical edge: corners (lx, 0) and (lx, cn)
    q1 = (lx == cn);
    q2 = q1 + 2;
    t = (double)lz / (double)cn;
  }
  const int64_t r1 = row[q1] + ci, r2 = row[q2] + ci;
  const double v1 = V[r1], v2 = V[r2], a1 = A[r1], a2 = A[r2];
  *v = v1 + t * (v2 - v1);
  *at = a1 + t * (a2 - a1);
  return S[r1] | S[r2];
}

// MSPM weight of the segment from local (ax, az) to (bx, bz) of one cell
// (eqs 28-30 with the reconstructed end quantities); +inf if unusable
__device__ __forceinline__ double mspm_w(const CellArgs& a, int f, const Rows4& row, int ax,
                                         int az, int bx, int bz, const double* V, const double* A,
                                         const int32_t* S) {
  const int cn = a.cn;
  const int off = (bz - az + cn) * a.side + (bx - ax + cn);
  const int ci = a.canon[off];
  double va, aa, vb, ab;
  const int32_t sa = mspm_node(cn, row, ax, az, ci, V, A, S, &va, &aa);
  const int32_t sb = mspm_node(cn, row, bx, bz, ci, V, A, S, &vb, &ab);
  const int32_t bad = CHERT_ST_NO_BRACKET | CHERT_ST_FLUID | CHERT_ST_NONPHYS | CHERT_ST_NOCONV;
  if ((sa | sb) & bad) return INFINITY;
  return f == 0 ? a.L[off] / (0.5 * (va + vb)) : a.L[off] * (0.5 * (aa + ab));
}

// Weight of segment i -> j of cell c (field f): the class-pair table of a
// cached network, or MSPM's reconstruction from the class table.
// cached network: weight of a segment of offset index off from class ki to
// class kj (field f)
__device__ __forceinline__ double pair_w(const CellArgs& a, int f, int ki, int kj, int off) {
  const int64_t no = a.n_off;
  return a.W[((int64_t)f * a.K * a.K + (int64_t)ki * a.K + kj) * no + off];
}

template <bool MSPM, bool D3>
__device__ __forceinline__ double seg_weight(const CellArgs& a, int f, int c, int64_t i,
                                             int64_t j) {
  const int cn = a.cn;
  if constexpr (!MSPM) {
    int ix, iy, iz, jx, jy, jz;
    node_xyz<D3>(a, i, ix, iy, iz);
    node_xyz<D3>(a, j, jx, jy, jz);
    return pair_w(a, f, a.cls[i], a.cls[j], off_of<D3>(a, jx - ix, jy - iy, jz - iz));
  } else {
    static_assert(!D3, "MSPM runs on the 2D cell network");
    const int ix = (int)(i % a.NX), iz = (int)(i / a.NX), jx = (int)(j % a.NX),
              jz = (int)(j / a.NX);
    const int x0 = (c % a.ncx) * cn, z0 = (c / a.ncx) * cn;
    const int64_t n00 = (int64_t)x0 + (int64_t)a.NX * z0, dz = (int64_t)a.NX * cn;
    const Rows4 row{(int64_t)a.cls[n00] * a.n_canon, (int64_t)a.cls[n00 + cn] * a.n_canon,
                    (int64_t)a.cls[n00 + dz] * a.n_canon, (int64_t)a.cls[n00 + dz + cn] * a.n_canon};
    return mspm_w(a, f, row, ix - x0, iz - z0, jx - x0, jz - z0, a.kV, a.kA, a.kS);
  }
}

// a cell whose boundary holds both lattice nodes i and j
__device__ __forceinline__ int common_cell(const CellArgs& a, int64_t i, int64_t j) {
  int cs[4];
  const int nc = cells_of((int)(j % a.NX), (int)(j / a.NX), a.cn, a.ncx, a.ncz, cs);
  const int ix = (int)(i % a.NX), iz = (int)(i / a.NX);
  for (int q = 0; q < nc; ++q) {
    const int x0 = (cs[q] % a.ncx) * a.cn, z0 = (cs[q] / a.ncx) * a.cn;
    if (ix >= x0 && ix <= x0 + a.cn && iz >= z0 && iz <= z0 + a.cn) return cs[q];
  }
  return cs[0];
}

// lattice node -> (x, y, z) and back (2D: y = 0); lattices hold fewer than
// 2^31 points, so 32-bit division suffices
template <bool D3>
__device__ __forceinline__ void node_xyz(const CellArgs& a, int64_t u, int& x, int& y, int& z) {
  const int v = (int)u;
  x = v % a.NX;
  const int r = v / a.NX;
  if constexpr (D3) {
    y = r % a.NY;
    z = r / a.NY;
  } else {
    y = 0;
    z = r;
  }
}
__device__ __forceinline__ int64_t node_at(const CellArgs& a, int x, int y, int z) {
  return (int64_t)x + (int64_t)a.NX * ((int64_t)y + (int64_t)a.NY * z);
}

// the cells (blocks) whose boundary holds lattice node u: at most 4 (8)
template <bool D3>
__device__ __forceinline__ int node_cells(const CellArgs& a, int64_t u, int* cs) {
  int x, y, z;
  node_xyz<D3>(a, u, x, y, z);
  if constexpr (!D3) {
    return cells_of(x, z, a.cn, a.ncx, a.ncz, cs);
  } else {
    int xs[2], ys[2], zs[2];
    const int nx = cells_along(x, a.cn, a.ncx, xs), ny = cells_along(y, a.cn, a.ncy, ys),
              nz = cells_along(z, a.cn, a.ncz, zs);
    int n = 0;
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < ny; ++j)
        for (int k = 0; k < nz; ++k) cs[n++] = xs[i] + a.ncx * (ys[j] + a.ncy * zs[k]);
    return n;
  }
}

// local point of boundary slot s of a cell (block)
template <bool D3>
__device__ __forceinline__ void slot_pos(const CellArgs& a, int s, int& lx, int& ly, int& lz) {
  if constexpr (!D3) {
    slot_xy(s, a.cn, lx, lz);
    ly = 0;
  } else {
    const int q = a.slot[s];
    lx = q & 255;
    ly = (q >> 8) & 255;
    lz = q >> 16;
  }
}

// origin (lattice point of the lowest corner) of cell (block) c
template <bool D3>
__device__ __forceinline__ void cell_origin(const CellArgs& a, int c, int& x0, int& y0, int& z0) {
  x0 = (c % a.ncx) * a.cn;
  if constexpr (D3) {
    const int r = c / a.ncx;
    y0 = (r % a.ncy) * a.cn;
    z0 = (r / a.ncy) * a.cn;
  } else {
    y0 = 0;
    z0 = (c / a.ncx) * a.cn;
  }
}

// segment offset index: (dz, dx) in 2D, (dz, dy, dx) in 3D, each in [-cn, cn]
template <bool D3>
__device__ __forceinline__ int off_of(const CellArgs& a, int dx, int dy, int dz) {
  if constexpr (D3)
    return ((dz + a.cn) * a.side + (dy + a.cn)) * a.side + (dx + a.cn);
  else
    return (dz + a.cn) * a.side + (dx + a.cn);
}

__device__ __forceinline__ double* tau_row(const CellArgs& a, int p) {
  const int fi = p / a.n_src, s = p - fi * a.n_src;
  return a.tau[fi] + (int64_t)s * a.n;
}

// fill the outputs: +inf traveltimes and t*, -1 predecessors and hops
__global__ void k_cell_fill(CellArgs a) {
  const int p = blockIdx.y;
  const int fi = p / a.n_src, s = p - fi * a.n_src;
  double* t = a.tau[fi] + (int64_t)s * a.n;
  int32_t* pr = a.pred[fi] ? a.pred[fi] + (int64_t)s * a.n : nullptr;
  double* ts = (a.tstar && a.field_of[fi] == 0) ? a.tstar + (int64_t)s * a.n : nullptr;
  int32_t* hp = a.hop + (int64_t)p * a.n;
  int32_t* bd = a.bid + (int64_t)p * a.n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    t[i] = INFINITY;
    hp[i] = -1;
    bd[i] = 0x7fffffff;
    if (pr) pr[i] = -1;
    if (ts) ts[i] = INFINITY;
  }
  if (p == 0)
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < 3 * kRelaxGrid;
         q += gridDim.x * blockDim.x)
      a.part[q] = 0ull;
  int32_t* act = a.active + (int64_t)p * a.C;
  unsigned long long* ky = a.key + (int64_t)p * a.C;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.C;
       c += (int64_t)gridDim.x * blockDim.x) {
    act[c] = 0;
    ky[c] = kInfBits;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.minkey[p] = 0ull;  // round 0 takes the source's cells (key 0)
    a.minkey[a.n_prob + p] = kInfBits;
    a.minkey[2 * a.n_prob + p] = kInfBits;
  }
  if (p == 0 && blockIdx.x == 0 && threadIdx.x < 8) {
    if (threadIdx.x < 2) a.count[threadIdx.x] = 0;
    if (threadIdx.x < 4) a.stats[threadIdx.x] = 0;
    if (threadIdx.x == 3) *a.alive = 0;
  }
}

// the source: tau = 0, its cells woken with key 0
__global__ void k_cell_seed(CellArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n_prob) return;
  const int fi = p / a.n_src, s = p - fi * a.n_src;
  const int64_t src = a.src[s];
  tau_row(a, p)[src] = 0.0;
  int cs[8];
  const int nc = a.NY > 1 ? node_cells<true>(a, src, cs)  // 3D blocks
                           : node_cells<false>(a, src, cs);
  for (int q = 0; q < nc; ++q) {
    a.active[(int64_t)p * a.C + cs[q]] = 1;
    a.key[(int64_t)p * a.C + cs[q]] = 0ull;
  }
  // level 0 of the BFS: the source alone (end of "level -1" = 0, one node)
  if ((a.tree_mask >> fi) & 1) {
    a.hop[(int64_t)p * a.n + src] = 0;
    a.bfs[(int64_t)p * a.n] = (int32_t)src;
    if (a.tstar && a.field_of[fi] == 0) a.tstar[(int64_t)s * a.n + src] = 0.0;
  }
  a.bnd[2 * a.n_prob + p] = 0;
  a.cnt[2 * a.n_prob + p] = ((a.tree_mask >> fi) & 1) ? 1 : 0;
  a.cnt[p] = 0;
  a.cnt[a.n_prob + p] = 0;
}

// round r, step 1: take the woken cells (when ordered: those whose key is
// within the width of the problem's smallest key, slot r % 3, which the
// previous round's select and relax filled) into this round's list; the
// cells left waiting bid their keys for the next round's minimum
__global__ void k_cell_select(CellArgs a, int r) {
  const int64_t total = (int64_t)a.n_prob * a.C;
  const unsigned long long* mk = a.minkey + (int64_t)(r % 3) * a.n_prob;
  unsigned long long* mk_next = a.minkey + (int64_t)((r + 1) % 3) * a.n_prob;
  int32_t* cnt = a.count + (r & 1);
  const int lane = __lane_id();
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total;
       base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = base + threadIdx.x;
    bool take = false;
    int p = -1;
    unsigned long long defer = kInfBits;
    if (t < total && a.active[t]) {
      take = true;
      if (a.bucket > 0.0) {
        p = (int)(t / a.C);
        const int f = a.field_of[p / a.n_src];
        const unsigned long long k = a.key[t];
        const double lim = __longlong_as_double((long long)mk[p]) + a.bucket * a.wmin[f];
        take = __longlong_as_double((long long)k) <= lim;
        if (!take) defer = k;
      }
    }
    if (a.bucket > 0.0) {
      // deferred keys bid for the next round's minimum; when the wave's
      // deferred cells share one problem it reduces first and bids once
      // (atomics on one address serialise)
      const unsigned long long dm = __ballot(defer != kInfBits);
      if (dm) {
        const int p0 = __shfl(p, __ffsll((long long)dm) - 1);
        if (__ballot(defer != kInfBits && p != p0) == 0) {
          unsigned long long m = defer;
          for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long m2 = __shfl_xor(m, o);
            m = m2 < m ? m2 : m;
          }
          if (lane == 0) atomicMin(&mk_next[p0], m);
        } else if (defer != kInfBits) {
          atomicMin(&mk_next[p], defer);
        }
      }
    }
    const unsigned long long m = __ballot(take);
    if (m) {
      int pos0 = 0;
      const int leader = __ffsll((long long)m) - 1;
      if (lane == leader) pos0 = atomicAdd(cnt, __popcll(m));
      pos0 = __shfl(pos0, leader);
      if (take) {
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        a.list[pos0 + rank] = (int32_t)t;
        a.active[t] = 0;
        a.key[t] = kInfBits;
      }
    }
  }
  // the next round's counter and the round after next's minima start afresh
  // (slot (r + 2) % 3 was last read by the previous round's select)
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) a.count[(r + 1) & 1] = 0;
    unsigned long long* nm = a.minkey + (int64_t)((r + 2) % 3) * a.n_prob;
    for (int p = threadIdx.x; p < a.n_prob; p += blockDim.x) nm[p] = kInfBits;
  }
}

// round r, step 3: relax the listed cells.  Each visit first stages the
// weights of its ns x ns ordered pairs in LDS (one batch of independent
// loads per lane), then runs the passes from LDS and lane broadcasts.
template <bool MSPM, bool D3>
__global__ void __launch_bounds__(kCellThreads) k_cell_relax(CellArgs a, int r) {
  static_assert(!(MSPM && D3), "MSPM runs on the 2D cell network");
  constexpr int NNB = D3 ? 26 : 8;  // neighbouring cells (blocks)
  // dynamic LDS: [the class-pair table, when it fits][waves][ns][ns]
  extern __shared__ double s_w[];
  __shared__ unsigned long long s_wake[kCellWaves][NNB];  // per neighbour cell
  __shared__ unsigned long long s_part[kCellWaves][3];
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int wave = blockIdx.x * wpb + wib;
  const int nw = gridDim.x * wpb;
  const int count = a.count[r & 1];
  const int cn = a.cn, ns = D3 ? a.ns : 4 * cn, K = a.K;
  const int64_t s2 = a.n_off;
  const int64_t tab_n = a.w_lds ? 2LL * K * K * s2 : 0;
  double* wl = s_w + tab_n + (size_t)wib * ns * ns;
  // the whole class-pair table of both fields in LDS, once per workgroup
  // with work (block-uniform), so a visit's weights are LDS reads
  if (a.w_lds && blockIdx.x * wpb < count) {
    for (int64_t q = threadIdx.x; q < tab_n; q += blockDim.x) s_w[q] = a.W[q];
    __syncthreads();
  }
  int lx = 0, ly = 0, lz = 0;
  if (lane < ns) slot_pos<D3>(a, lane, lx, ly, lz);
  unsigned long long visits = 0, pairs = 0, passes_all = 0;
  for (int it = wave; it < count; it += nw) {
    const int64_t item = a.list[it];
    const int p = (int)(item / a.C);
    const int c = (int)(item - (int64_t)p * a.C);
    int x0, y0, z0;
    cell_origin<D3>(a, c, x0, y0, z0);
    double* tau = tau_row(a, p);
    const double* W =
        a.W ? (a.w_lds ? s_w : a.W) + (int64_t)a.field_of[p / a.n_src] * K * K * s2 : nullptr;
    const int64_t node = node_at(a, x0 + lx, y0 + ly, z0 + lz);
    int k = 0;
    double t = INFINITY;
    if (lane < ns) {
      k = a.cls[node];
      t = tau[node];
    }
    // stage w(a -> lane) for every slot a (the diagonal is never read),
    // eight loads in flight per lane; slot a's class and position come from
    // lane a
    if constexpr (MSPM) {  // this visit's corner rows (solved for it this round)
      const int f = a.field_of[p / a.n_src];
      const int64_t r0 = (int64_t)it * 4 * a.n_canon;
      const Rows4 row{r0, r0 + a.n_canon, r0 + 2 * a.n_canon, r0 + 3 * a.n_canon};
      for (int sa = 0; sa < ns; ++sa) {
        const int ax = __builtin_amdgcn_readlane(lx, sa);
        const int az = __builtin_amdgcn_readlane(lz, sa);
        if (lane < ns && lane != sa)
          wl[sa * ns + lane] = mspm_w(a, f, row, ax, az, lx, lz, a.tV, a.tA, a.tS);
      }
    } else {
      const double* Wk = W + (int64_t)k * s2;  // column class = this lane's
      for (int sa0 = 0; sa0 < ns; sa0 += 8) {
        double w8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int sa = sa0 + u < ns ? sa0 + u : ns - 1;
          const int ka = __builtin_amdgcn_readlane(k, sa);
          const int ax = __builtin_amdgcn_readlane(lx, sa);
          const int ay = D3 ? __builtin_amdgcn_readlane(ly, sa) : 0;
          const int az = __builtin_amdgcn_readlane(lz, sa);
          const int off = off_of<D3>(a, lx - ax, ly - ay, lz - az);
          w8[u] = lane < ns ? Wk[(int64_t)ka * K * s2 + off] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (lane < ns && sa0 + u < ns) wl[(sa0 + u) * ns + lane] = w8[u];
      }
    }
    wave_sync_lds();
    const double t0 = t;
    int passes = 0;
    for (;;) {
      double best = t;
#pragma unroll 4
      for (int sa = 0; sa < ns; ++sa) {
        const double ta = bcast_d(t, sa);
        // +inf + w stays +inf, and slot sa's own lane reads the unused
        // diagonal, so every lane can add without a branch
        const double cand = ta + wl[sa * ns + (lane < ns ? lane : 0)];
        if (lane < ns && lane != sa && cand < best) best = cand;
      }
      ++passes;
      const bool ch = best < t;
      t = best;
      if (!__ballot(ch)) break;
    }
    wave_sync_lds();  // LDS reused by the wave's next item
    ++visits;
    pairs += (unsigned long long)passes * ns * (ns - 1);
    passes_all += passes;
    // lower the improved nodes; each of the neighbouring cells (8, or 26
    // blocks) is woken once, with the smallest new traveltime among the nodes
    // it shares
    if (lane < NNB) s_wake[wib][lane] = kInfBits;
    wave_sync_lds();
    // (the atomic's old value is not waited for: a node this visit lowered
    // wakes its other cells even if another visit lowered it further, which
    // costs at most a visit that changes nothing)
    constexpr int kSelf = D3 ? 13 : 4;  // index of the cell itself
    if (lane < ns && t < t0) {
      const unsigned long long nb = dbits(t);
      atomicMin((unsigned long long*)&tau[node], nb);
      {
        const int ex = lx == 0 ? -1 : (lx == cn ? 1 : 0);
        const int ey = D3 ? (ly == 0 ? -1 : (ly == cn ? 1 : 0)) : 0;
        const int ez = lz == 0 ? -1 : (lz == cn ? 1 : 0);
        // neighbour d = (dx + 1) + 3 (dy + 1) + 9 (dz + 1) (2D: (dx + 1) +
        // 3 (dz + 1)), skipping the cell itself
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = D3 ? -1 : 0; dy <= (D3 ? 1 : 0); ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              if ((dx == 0 && dy == 0 && dz == 0) || (dx != 0 && dx != ex) ||
                  (dy != 0 && dy != ey) || (dz != 0 && dz != ez))
                continue;
              const int d = D3 ? (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1) : (dx + 1) + 3 * (dz + 1);
              atomicMin(&s_wake[wib][d < kSelf ? d : d - 1], nb);
            }
      }
    }
    wave_sync_lds();
    unsigned long long woke = kInfBits;
    if (lane < NNB) {
      const unsigned long long v = s_wake[wib][lane];
      const int d = lane < kSelf ? lane : lane + 1;
      const int cx = x0 / cn, cy = y0 / cn, cz = z0 / cn;
      const int nx = cx + d % 3 - 1;
      const int ny = D3 ? cy + (d / 3) % 3 - 1 : 0;
      const int nz = D3 ? cz + d / 9 - 1 : cz + d / 3 - 1;
      if (v != kInfBits && nx >= 0 && nx < a.ncx && ny >= 0 && ny < a.ncy && nz >= 0 &&
          nz < a.ncz) {
        const int64_t e = (int64_t)p * a.C + nx + (int64_t)a.ncx * (ny + (int64_t)a.ncy * nz);
        atomicMin(&a.key[e], v);
        a.active[e] = 1;
        woke = v;
      }
    }
    // the next round's smallest key of the problem: one atomic per visit
    // (atomics on one address serialise, so the wave reduces first)
    if (a.bucket > 0.0) {
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w2 = __shfl_xor(woke, o);
        woke = w2 < woke ? w2 : woke;
      }
      if (lane == 0 && woke != kInfBits)
        atomicMin(&a.minkey[(int64_t)((r + 1) % 3) * a.n_prob + p], woke);
    }
    wave_sync_lds();
  }
  // statistics: per-workgroup partial sums in plain stores (no atomics on a
  // shared address), summed by the host
  if (lane == 0) {
    s_part[wib][0] = visits;
    s_part[wib][1] = pairs;
    s_part[wib][2] = passes_all;
  }
  __syncthreads();
  if (threadIdx.x == 0 && blockIdx.x < kRelaxGrid) {
    unsigned long long v0 = 0, v1 = 0, v2 = 0;
    for (int w = 0; w < wpb; ++w) {
      v0 += s_part[w][0];
      v1 += s_part[w][1];
      v2 += s_part[w][2];
    }
    if (v0) {
      unsigned long long* pp = a.part + 3 * (int64_t)blockIdx.x;
      pp[0] += v0;
      pp[1] += v1;
      pp[2] += v2;
    }
  }
}

// Predecessors and t*, level L of the BFS over tight segments, one launch
// per level, grid (x, problem).  Step 1 (level L): every thread takes a
// (node j of the level, boundary slot) pair and visits the slot's point v
// in each of j's cells: a tight v one level up (tau_v + w(v->j) == tau_j)
// bids for pred_j
// with an atomicMin on its index; a v not yet reached with
// tau_j + w(j->v) == tau_v joins level L + 1 (one winner per node through a
// compare-and-swap on its hop).  Step 2 (level L - 1, whose bids were final
// when the previous launch ended): pred_j and t*_j = t*_pred + the
// attenuation weight of that segment (the parent's value final one level
// earlier).  Level bounds rotate through three slots per problem.
constexpr int kLvlThreads = 256;
constexpr int kLvlBuf = 4096;  // appends staged per workgroup (16 KiB of LDS)
template <bool MSPM, bool D3>
__global__ void __launch_bounds__(kLvlThreads) k_cell_level(CellArgs a, int L) {
  static_assert(!(MSPM && D3), "MSPM runs on the 2D cell network");
  __shared__ int32_t s_buf[kLvlBuf];
  __shared__ int s_n, s_base, s_any;
  const int p = blockIdx.y;
  const int fi = p / a.n_src, s = p - fi * a.n_src;
  if (!((a.tree_mask >> fi) & 1)) return;
  const int P = a.n_prob;
  const int start = a.bnd[((L + 2) % 3) * P + p];
  const int end = start + a.cnt[((L + 2) % 3) * P + p];
  const int pstart = L >= 2 ? a.bnd[((L + 1) % 3) * P + p] : start;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.bnd[(L % 3) * P + p] = end;
    a.cnt[((L + 1) % 3) * P + p] = 0;
  }
  int32_t* cnt = a.cnt + (L % 3) * P + p;
  const int ns = D3 ? a.ns : 4 * a.cn;
  constexpr int kCells = D3 ? 8 : 4;  // cells (blocks) a node can lie on
  const int cn = a.cn;
  const int f = a.field_of[fi];
  const double* tau = a.tau[fi] + (int64_t)s * a.n;
  int32_t* hop = a.hop + (int64_t)p * a.n;
  int32_t* bfs = a.bfs + (int64_t)p * a.n;
  int32_t* bid = a.bid + (int64_t)p * a.n;
  int32_t* pred = a.pred[fi] ? a.pred[fi] + (int64_t)s * a.n : nullptr;
  double* ts = (a.tstar && f == 0) ? a.tstar + (int64_t)s * a.n : nullptr;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  // one thread per (node of the level, boundary slot), looping over the
  // node's cells; a slot point that also lies on an earlier cell of the
  // node was handled there by the thread of its slot in that cell (it is a
  // face point of every cell whose closed box holds it), so each neighbour
  // is examined once.  Appends to the next level are staged in LDS and
  // reserved in the global list once per workgroup flush (device-scope
  // atomics on one address serialise across the chip).
  if (threadIdx.x == 0) {
    s_n = 0;
    s_any = 0;
  }
  __syncthreads();
  const int64_t work = (int64_t)(end - start) * ns;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < work; base += nthr) {
    const int64_t t = base + threadIdx.x;
    const bool valid = t < work;
    int64_t j = 0;
    int lx = 0, ly = 0, lz = 0, jx = 0, jy = 0, jz = 0, kj = 0;
    // the node's cells per axis: origins o?[0..n?-1] (two on a cell
    // boundary plane, else one)
    int nxa = 0, nya = 1, nza = 0, ox[2] = {0, 0}, oy[2] = {0, 0}, oz[2] = {0, 0};
    double tj = 0.0;
    if (valid) {
      j = bfs[start + (int)(t / ns)];
      slot_pos<D3>(a, (int)(t % ns), lx, ly, lz);
      node_xyz<D3>(a, j, jx, jy, jz);
      tj = tau[j];
      kj = MSPM ? 0 : a.cls[j];
      int c3[2];
      nxa = cells_along(jx, cn, a.ncx, c3);
      ox[0] = c3[0] * cn;
      ox[1] = c3[nxa - 1] * cn;
      if constexpr (D3) {
        nya = cells_along(jy, cn, a.ncy, c3);
        oy[0] = c3[0] * cn;
        oy[1] = c3[nya - 1] * cn;
      }
      nza = cells_along(jz, cn, a.ncz, c3);
      oz[0] = c3[0] * cn;
      oz[1] = c3[nza - 1] * cn;
    }
    // three passes over the node's cells so that each pass's memory
    // operations are independent and overlap: (1) tightness tests (loads
    // only), (2) the bids and the claims of unreached nodes (atomics, issued
    // back to back), (3) appends of the claimed nodes.  A slot point that
    // also lies on the node's other cell along an axis (local coordinate 0
    // in the upper cell) is examined in the lower cell only, so each
    // neighbour is examined once.
    int32_t upv[kCells], dnv[kCells];
#pragma unroll
    for (int q = 0; q < kCells; ++q) {
      const int ia = D3 ? (q >> 2) : (q >> 1), ib = D3 ? ((q >> 1) & 1) : 0, ic = q & 1;
      upv[q] = -1;
      dnv[q] = -1;
      const bool have = ia < nxa && ib < nya && ic < nza;
      const bool dup = (ia == 1 && lx == 0) || (ib == 1 && ly == 0) || (ic == 1 && lz == 0);
      if (have && !dup) {
        const int vx = ox[ia] + lx, vy = oy[ib] + ly, vz = oz[ic] + lz;
        const int64_t v = node_at(a, vx, vy, vz);
        if (v != j) {
          const double tv = tau[v];
          const int hv = hop[v];
          const bool up = L > 0 && hv == L - 1, down = hv == -1 && tv < INFINITY;
          if (up || down) {
            const int kv = MSPM ? 0 : a.cls[v];
            // MSPM reads the cell (2D): cell index of (ia, ic)
            const int c = MSPM ? ox[ia] / cn + a.ncx * (oz[ic] / cn) : 0;
            if (up) {  // v -> j tight?
              const double w =
                  MSPM ? seg_weight<MSPM, D3>(a, f, c, v, j)
                       : pair_w(a, f, kv, kj, off_of<D3>(a, jx - vx, jy - vy, jz - vz));
              if (tv + w == tj) upv[q] = (int32_t)v;
            }
            if (down) {  // j -> v tight?
              const double w =
                  MSPM ? seg_weight<MSPM, D3>(a, f, c, j, v)
                       : pair_w(a, f, kj, kv, off_of<D3>(a, vx - jx, vy - jy, vz - jz));
              if (tj + w == tv) dnv[q] = (int32_t)v;
            }
          }
        }
      }
    }
    bool won[kCells];
#pragma unroll
    for (int q = 0; q < kCells; ++q) {
      if (upv[q] >= 0) atomicMin(&bid[j], upv[q]);
      won[q] = dnv[q] >= 0 && atomicCAS(&hop[dnv[q]], -1, L + 1) == -1;
    }
#pragma unroll
    for (int q = 0; q < kCells; ++q)
      if (won[q]) s_buf[atomicAdd(&s_n, 1)] = dnv[q];  // LDS atomic
    // flush when another pass could overflow the buffer (workgroup-uniform)
    __syncthreads();
    const int n_st = s_n;
    __syncthreads();  // every thread has read the count before the next pass adds to it
    if (n_st > kLvlBuf - kLvlThreads * kCells || (n_st > 0 && base + nthr >= work)) {
      if (threadIdx.x == 0) {
        s_base = atomicAdd(cnt, n_st);
        s_any = 1;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < n_st; i += blockDim.x) bfs[end + s_base + i] = s_buf[i];
      __syncthreads();
      if (threadIdx.x == 0) s_n = 0;
      __syncthreads();
    }
  }
  if (L >= 2) {
    for (int64_t idx = pstart + tid; idx < start; idx += nthr) {
      const int64_t j = bfs[idx];
      const int b = bid[j];
      // a node one level below the source always has a tight neighbour one
      // level up (the one that reached it); the check only keeps the reads
      // in bounds
      if (b == 0x7fffffff) continue;
      if (pred) pred[j] = b;
      if (ts) ts[j] = ts[b] + seg_weight<MSPM, D3>(a, 1, MSPM ? common_cell(a, b, j) : 0, b, j);
    }
  }
  // any append keeps the BFS going: the workgroups that appended raise the
  // level count to L + 2 (levels 0 .. L + 1 hold nodes)
  if (threadIdx.x == 0 && s_any) atomicMax(a.alive, L + 2);
}

__global__ void k_cell_zero(int32_t* x) { *x = 0; }

// 3D segment columns: one workgroup per offset o, the Fibonacci direction
// with the largest dot product f . u_o (IEEE operations in the order of the
// definition, no contraction), the lowest index among equals: each thread
// keeps its first strict maximum over a strided pass, then the waves and
// the workgroup merge (larger dot first, lower index on a tie), which is the
// sequential rule.
constexpr int kFibThreads = 1024;
__global__ void __launch_bounds__(kFibThreads) k_fib_nearest(const double* f, int N,
                                                             const double* u, int n_off,
                                                             int32_t* col) {
  __shared__ double s_d[kFibThreads / 64];
  __shared__ int s_i[kFibThreads / 64];
  const int o = blockIdx.x;  // grid = n_off
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double u0 = u[3 * o], u1 = u[3 * o + 1], u2 = u[3 * o + 2];
  double bd = -2.0;
  int bi = 0x7fffffff;
  for (int i = threadIdx.x; i < N; i += kFibThreads) {
    const double d = __dadd_rn(__dadd_rn(__dmul_rn(f[3 * i], u0), __dmul_rn(f[3 * i + 1], u1)),
                               __dmul_rn(f[3 * i + 2], u2));
    if (d > bd) {
      bd = d;
      bi = i;
    }
  }
  for (int w = 32; w > 0; w >>= 1) {
    const double od = __shfl_xor(bd, w);
    const int oi = __shfl_xor(bi, w);
    if (od > bd || (od == bd && oi < bi)) {
      bd = od;
      bi = oi;
    }
  }
  if (lane == 0) {
    s_d[wv] = bd;
    s_i[wv] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kFibThreads / 64; ++w)
      if (s_d[w] > bd || (s_d[w] == bd && s_i[w] < bi)) {
        bd = s_d[w];
        bi = s_i[w];
      }
    col[o] = bi;
  }
}

// ---------------------------------------------------------------- plan ----

// MSPM, round r: the class of each corner of each listed cell (the solve
// jobs of this round's visits, job it * 4 + corner)
__global__ void k_mspm_jobs(CellArgs a, int r) {
  const int count = a.count[r & 1];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 4LL * count;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int it = (int)(t >> 2), q = (int)(t & 3);
    const int64_t item = a.list[it];
    const int c = (int)(item % a.C);
    const int x0 = (c % a.ncx) * a.cn + (q & 1) * a.cn, z0 = (c / a.ncx) * a.cn + (q >> 1) * a.cn;
    a.job_class[t] = a.cls[(int64_t)x0 + (int64_t)a.NX * z0];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.stats[3], 4ull * count);
}

// MSPM ordering scale: per field the smallest positive L / V and L A over
// the class table (canonical segment lengths)
__global__ void k_mspm_wmin(CellArgs a, const double* Lc, int64_t rows) {
  double m0 = INFINITY, m1 = INFINITY;
  const int32_t bad = CHERT_ST_NO_BRACKET | CHERT_ST_FLUID | CHERT_ST_NONPHYS | CHERT_ST_NOCONV;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < rows * a.n_canon;
       t += (int64_t)gridDim.x * blockDim.x) {
    if (a.kS[t] & bad) continue;
    const double l = Lc[t % a.n_canon];
    const double w0 = l / a.kV[t], w1 = l * a.kA[t];
    if (w0 > 0.0 && w0 < m0) m0 = w0;
    if (w1 > 0.0 && w1 < m1) m1 = w1;
  }
  for (int o = 32; o > 0; o >>= 1) {
    m0 = fmin(m0, __shfl_xor(m0, o));
    m1 = fmin(m1, __shfl_xor(m1, o));
  }
  double* wmin = const_cast<double*>(a.wmin);
  if (__lane_id() == 0) {
    if (m0 < INFINITY) atomicMin((unsigned long long*)&wmin[0], dbits(m0));
    if (m1 < INFINITY) atomicMin((unsigned long long*)&wmin[1], dbits(m1));
  }
}

// Where the segment weights come from: a cache (the cached network) or
// MSPM's fresh corner solves.
struct CellSrc {
  bool mspm = false;
  const chert_cache_desc* d = nullptr;
  const void* cache_dev = nullptr;
  const chert_class* classes_dev = nullptr;
  int kernel = 0, n_sweep = 0;
};

// The network's geometry: 2D cells (chert_cell_grid) or 3D blocks
// (chert_block_grid); ncy = 1, hy = 0 in 2D.
struct CellGeo {
  int dim = 2;
  int ncx = 0, ncy = 1, ncz = 0, cn = 0;
  double hx = 0.0, hy = 0.0, hz = 0.0;
  const int32_t* cls = nullptr;
};

CellGeo geo_of(const chert_cell_grid* g) {
  CellGeo G;
  G.dim = 2;
  G.ncx = g->ncx;
  G.ncz = g->ncz;
  G.cn = g->cell_n;
  G.hx = g->hx;
  G.hz = g->hz;
  G.cls = g->class_id_dev;
  return G;
}

CellGeo geo_of(const chert_block_grid* g) {
  CellGeo G;
  G.dim = 3;
  G.ncx = g->ncx;
  G.ncy = g->ncy;
  G.ncz = g->ncz;
  G.cn = g->block_n;
  G.hx = g->hx;
  G.hy = g->hy;
  G.hz = g->hz;
  G.cls = g->class_id_dev;
  return G;
}

struct CellPlan {
  int dim = 2, cn = 0, side = 0, NX = 0, NY = 1, NZ = 0, n_prob = 0, nfs = 0, max_rounds = 0;
  int n_cols = 0, n_canon = 0, ns = 0, n_off = 0, N = 0;
  int64_t n = 0, C = 0, K = 0;
  int fields[2] = {0, 0};
  bool slow = false;
  size_t off_tab = 0, off_geo = 0, off_W = 0, off_best = 0, off_ctl = 0, off_src = 0,
         off_act = 0, off_key = 0, off_list = 0, off_hop = 0, off_bfs = 0, off_bid = 0,
         off_kt = 0, off_vt = 0, off_jobs = 0, off_part = 0, total = 0;
};

int cell_plan(const CellSrc& w, int64_t n_classes, const CellGeo& G, int32_t mode,
              const int64_t* src, int32_t n_src, const chert_trace_opts* o, CellPlan* P) {
  if (!o) return fail(CHERT_ERR_INVALID_ARG, "null options");
  P->dim = G.dim;
  if (!w.mspm) {
    const chert_cache_desc* d = w.d;
    if (!d) return fail(CHERT_ERR_INVALID_ARG, "null descriptor");
    chert_cache_layout lay;
    int rc = chert_cache_layout_of(d, n_classes, &lay);
    if (rc) return rc;
    if (d->dim != G.dim)
      return fail(CHERT_ERR_INVALID_ARG,
                  G.dim == 2 ? "cell networks take 2D caches" : "block networks take 3D caches");
    if (mode < 0 || mode > 2 || !(d->mode_mask & (1u << mode)))
      return fail(CHERT_ERR_INVALID_ARG, "mode not in the cache");
    P->slow = d->sampling == CHERT_SAMPLE_SLOWNESS;
    P->n_cols = d->n_subset ? d->n_subset : d->n_dirs;
    P->N = G.dim == 3 ? d->n_dirs : 0;
  } else {
    if (G.dim != 2) return fail(CHERT_ERR_UNSUPPORTED, "MSPM runs on the 2D cell network");
    if (mode < 0 || mode > 2) return fail(CHERT_ERR_INVALID_ARG, "mode must be 0..2");
    if (w.kernel != CHERT_KERNEL_MEV && w.kernel != CHERT_KERNEL_OEV)
      return fail(CHERT_ERR_INVALID_ARG, "kernel must be MEV or OEV");
    if (w.n_sweep < 8 || w.n_sweep > kMaxSweep)
      return fail(CHERT_ERR_INVALID_ARG, "n_sweep must be 8..4096");
  }
  if (G.ncx < 1 || G.ncy < 1 || G.ncz < 1)
    return fail(CHERT_ERR_INVALID_ARG, "need at least one cell");
  if (G.dim == 2 && (G.cn < 1 || G.cn > kCellMaxN))
    return fail(CHERT_ERR_INVALID_ARG, "cell_n must be 1..16");
  if (G.dim == 3 && (G.cn < 1 || G.cn > kBlockMaxN))
    return fail(CHERT_ERR_INVALID_ARG, "block_n must be 1..3");
  if (!(G.hx > 0.0) || !(G.hz > 0.0) || !isfinite(G.hx) || !isfinite(G.hz) ||
      (G.dim == 3 && (!(G.hy > 0.0) || !isfinite(G.hy))))
    return fail(CHERT_ERR_INVALID_ARG, "spacing must be positive and finite");
  if (!G.cls) return fail(CHERT_ERR_INVALID_ARG, "cell networks need a class map");
  P->cn = G.cn;
  P->side = 2 * P->cn + 1;
  P->n_canon = 2 * P->cn * (P->cn + 1);
  P->n_off = G.dim == 3 ? P->side * P->side * P->side : P->side * P->side;
  P->ns = G.dim == 3 ? (P->cn + 1) * (P->cn + 1) * (P->cn + 1) - (P->cn - 1) * (P->cn - 1) * (P->cn - 1)
                     : 4 * P->cn;
  const int64_t NX = (int64_t)G.ncx * P->cn + 1, NZ = (int64_t)G.ncz * P->cn + 1;
  const int64_t NY = G.dim == 3 ? (int64_t)G.ncy * P->cn + 1 : 1;
  if (NX * NY * NZ >= 0x7fffffffLL) return fail(CHERT_ERR_INVALID_ARG, "lattice too large");
  P->NX = (int)NX;
  P->NY = (int)NY;
  P->NZ = (int)NZ;
  P->n = NX * NY * NZ;
  P->C = (int64_t)G.ncx * G.ncy * G.ncz;
  P->K = n_classes;
  if (n_classes < 1) return fail(CHERT_ERR_INVALID_ARG, "need at least one class");
  if (n_classes * n_classes * P->n_off >= 0x7fffffffLL)
    return fail(CHERT_ERR_UNSUPPORTED, "class-pair table too large");
  const uint32_t outs = o->outputs;
  if (outs == 0 || (outs & ~31u) || !(outs & (CHERT_OUT_TAU_R | CHERT_OUT_TAU_I)))
    return fail(CHERT_ERR_INVALID_ARG, "bad output mask");
  if ((outs & CHERT_OUT_TSTAR) && !((outs & CHERT_OUT_TAU_R) && (outs & CHERT_OUT_PRED_P)))
    return fail(CHERT_ERR_INVALID_ARG, "TSTAR needs TAU_R and PRED_P");
  if ((outs & CHERT_OUT_PRED_P) && !(outs & CHERT_OUT_TAU_R))
    return fail(CHERT_ERR_INVALID_ARG, "PRED_P needs TAU_R");
  if ((outs & CHERT_OUT_PRED_A) && !(outs & CHERT_OUT_TAU_I))
    return fail(CHERT_ERR_INVALID_ARG, "PRED_A needs TAU_I");
  if (!(o->bucket_width >= 0.0) || !isfinite(o->bucket_width))
    return fail(CHERT_ERR_INVALID_ARG, "bucket_width must be finite and >= 0");
  if (n_src < 1 || !src) return fail(CHERT_ERR_INVALID_ARG, "need sources");
  for (int i = 0; i < n_src; ++i) {
    if (src[i] < 0 || src[i] >= P->n) return fail(CHERT_ERR_INVALID_ARG, "source out of range");
    const int64_t x = src[i] % NX, y = (src[i] / NX) % NY, z = src[i] / (NX * NY);
    if (x % P->cn != 0 && z % P->cn != 0 && (G.dim == 2 || y % P->cn != 0))
      return fail(CHERT_ERR_INVALID_ARG, "a source inside a cell is not a node");
  }
  P->nfs = 0;
  if (outs & CHERT_OUT_TAU_R) P->fields[P->nfs++] = 0;
  if (outs & CHERT_OUT_TAU_I) P->fields[P->nfs++] = 1;
  if ((int64_t)P->nfs * n_src > 65535) return fail(CHERT_ERR_UNSUPPORTED, "too many sources");
  P->n_prob = P->nfs * n_src;
  if ((int64_t)P->n_prob * P->C >= 0x7fffffffLL / 4 || (int64_t)P->n_prob * P->n >= (1LL << 40))
    return fail(CHERT_ERR_UNSUPPORTED, "batch too large for one call");
  P->max_rounds =
      o->max_rounds > 0 ? o->max_rounds : 4096 + 64 * (G.ncx + (G.dim == 3 ? G.ncy : 0) + G.ncz);
  const int s2 = P->n_off;
  const size_t q3 = 2 * sizeof(double) + sizeof(int32_t);  // V, A, status
  size_t off = 0;
  P->off_tab = off;  // L (double), ox, oz, col, canon (int32), psi (double)
  off += al256((size_t)s2 * (sizeof(double) + 4 * sizeof(int32_t)) +
               (size_t)P->n_canon * sizeof(double) + 8);
  P->off_geo = off;  // 3D: unit vectors [n_off][3], Fibonacci directions [N][3], slots [64]
  if (G.dim == 3) off += al256((size_t)3 * (s2 + P->N) * sizeof(double) + 64 * sizeof(int32_t));
  P->off_W = off;
  if (!w.mspm) off += al256((size_t)2 * n_classes * n_classes * s2 * sizeof(double));
  P->off_best = off;
  if (P->slow) off += al256((size_t)n_classes * s2 * sizeof(int32_t));
  P->off_kt = off;
  if (w.mspm) off += al256((size_t)n_classes * P->n_canon * q3);
  P->off_vt = off;
  if (w.mspm) off += al256((size_t)4 * P->n_prob * P->C * P->n_canon * q3);
  P->off_jobs = off;
  if (w.mspm) off += al256((size_t)4 * P->n_prob * P->C * sizeof(int32_t));
  P->off_ctl = off;  // count[2], err, alive, stats[4], wmin[2], minkey[3][P], bnd, cnt
  off += al256(256 + (size_t)3 * P->n_prob * sizeof(unsigned long long) +
               (size_t)6 * P->n_prob * sizeof(int32_t));
  P->off_part = off;
  off += al256((size_t)3 * kRelaxGrid * sizeof(unsigned long long));
  P->off_src = off;
  off += al256((size_t)n_src * sizeof(int64_t));
  P->off_act = off;
  off += al256((size_t)P->n_prob * P->C * sizeof(int32_t));
  P->off_key = off;
  off += al256((size_t)P->n_prob * P->C * sizeof(unsigned long long));
  P->off_list = off;
  off += al256((size_t)P->n_prob * P->C * sizeof(int32_t));
  P->off_hop = off;
  off += al256((size_t)P->n_prob * P->n * sizeof(int32_t));
  P->off_bfs = off;
  off += al256((size_t)P->n_prob * P->n * sizeof(int32_t));
  P->off_bid = off;
  off += al256((size_t)P->n_prob * P->n * sizeof(int32_t));
  P->total = off;
  return CHERT_OK;
}

size_t cell_workspace(const CellSrc& w, int64_t n_classes, const CellGeo& G, int32_t n_src,
                      const chert_trace_opts* o) {
  if (n_src < 1) return 0;
  // sources are checked by the trace call; a lattice corner stands in here
  std::vector<int64_t> src((size_t)n_src, 0);
  CellPlan P;
  for (int m = 0; m < 3; ++m)  // the mode is checked by the trace call
    if (cell_plan(w, n_classes, G, m, src.data(), n_src, o, &P) == CHERT_OK) return P.total;
  return 0;
}

int trace_cells_impl(const CellSrc& w, int64_t n_classes, const CellGeo& G, int32_t mode,
                     const int64_t* src_nodes_host, int32_t n_src, const chert_trace_opts* o,
                     double* tau_r_dev, double* tau_i_dev, double* tstar_dev, int32_t* pred_p_dev,
                     int32_t* pred_a_dev, void* workspace_dev, size_t workspace_bytes,
                     void* stream) {
  CellPlan P;
  int rc = cell_plan(w, n_classes, G, mode, src_nodes_host, n_src, o, &P);
  if (rc) return rc;
  const uint32_t outs = o->outputs;
  if (!w.mspm && !w.cache_dev) return fail(CHERT_ERR_INVALID_ARG, "null cache");
  if (w.mspm && !w.classes_dev) return fail(CHERT_ERR_INVALID_ARG, "null classes");
  if ((outs & CHERT_OUT_TAU_R) && !tau_r_dev) return fail(CHERT_ERR_INVALID_ARG, "null tau_r");
  if ((outs & CHERT_OUT_TAU_I) && !tau_i_dev) return fail(CHERT_ERR_INVALID_ARG, "null tau_i");
  if ((outs & CHERT_OUT_TSTAR) && !tstar_dev) return fail(CHERT_ERR_INVALID_ARG, "null tstar");
  if ((outs & CHERT_OUT_PRED_P) && !pred_p_dev) return fail(CHERT_ERR_INVALID_ARG, "null pred_p");
  if ((outs & CHERT_OUT_PRED_A) && !pred_a_dev) return fail(CHERT_ERR_INVALID_ARG, "null pred_a");
  if (!workspace_dev || workspace_bytes < P.total || ((uintptr_t)workspace_dev & 255u))
    return fail(CHERT_ERR_INVALID_ARG, "workspace too small or unaligned");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)workspace_dev;
  const int cn = P.cn, side = P.side, s2 = P.n_off;
  const int K = (int)P.K;

  // segment offsets (dx, dz) in [-cn, cn]^2 (the centre is never a segment:
  // a stand-in offset keeps the lookups finite), lengths (eq 27), columns;
  // MSPM: canonical offsets (direction angle in [0, pi)) and their exact
  // global ray angles.  3D: offsets (dx, dy, dz) in [-cn, cn]^3, lengths and
  // unit vectors (the columns come from k_fib_nearest), and the block's face
  // points as slots.
  std::vector<int32_t> tab((size_t)s2 * 4);
  std::vector<double> L((size_t)s2), psi((size_t)P.n_canon), Lc((size_t)P.n_canon);
  std::vector<double> geo;
  std::vector<int32_t> slots;
  if (P.dim == 3) {
    geo.assign((size_t)3 * (s2 + P.N), 0.0);
    for (int dz = -cn; dz <= cn; ++dz)
      for (int dy = -cn; dy <= cn; ++dy)
        for (int dx = -cn; dx <= cn; ++dx) {
          const int q = ((dz + cn) * side + (dy + cn)) * side + (dx + cn);
          tab[q] = 0;
          tab[s2 + q] = 0;
          tab[2 * s2 + q] = 0;
          tab[3 * s2 + q] = -1;
          if (dx == 0 && dy == 0 && dz == 0) {  // never a segment
            L[q] = 0.0;
            geo[3 * q + 2] = 1.0;
            continue;
          }
          const double ex = dx * G.hx, ey = dy * G.hy, ez = dz * G.hz;
          const double len = sqrt(ex * ex + ez * ez + ey * ey);  // eq 27 in 3D
          L[q] = len;
          geo[3 * q] = ex / len;
          geo[3 * q + 1] = ey / len;
          geo[3 * q + 2] = ez / len;
        }
    fibonacci(P.N, geo.data() + 3 * (size_t)s2);
    for (int z = 0; z <= cn; ++z)
      for (int y = 0; y <= cn; ++y)
        for (int x = 0; x <= cn; ++x)
          if (x == 0 || y == 0 || z == 0 || x == cn || y == cn || z == cn)
            slots.push_back(x | (y << 8) | (z << 16));
    if ((int)slots.size() != P.ns) return fail(CHERT_ERR_INVALID_ARG, "block slot count");
  }
  for (int dz = -cn; dz <= cn && P.dim == 2; ++dz)
    for (int dx = -cn; dx <= cn; ++dx) {
      const int q = (dz + cn) * side + (dx + cn);
      const int x = (dx == 0 && dz == 0) ? 1 : dx;
      tab[q] = x;
      tab[s2 + q] = dz;
      const double ex = x * G.hx, ez = dz * G.hz;
      L[q] = sqrt(ex * ex + ez * ez);
      tab[2 * s2 + q] = 0;
      tab[3 * s2 + q] = -1;
    }
  if (P.dim == 2) {
    int ci = 0;
    for (int dz = -cn; dz <= cn; ++dz)
      for (int dx = -cn; dx <= cn; ++dx) {
        if (!(dx > 0 || (dx == 0 && dz > 0))) continue;
        psi[ci] = atan2(dx * G.hx, dz * G.hz);
        Lc[ci] = L[(dz + cn) * side + (dx + cn)];
        tab[3 * s2 + (dz + cn) * side + (dx + cn)] = ci;
        tab[3 * s2 + (-dz + cn) * side + (-dx + cn)] = ci;
        ++ci;
      }
  }
  if (!w.mspm && !P.slow && P.dim == 2) {
    std::vector<int32_t> bin((size_t)s2);
    for (int q = 0; q < s2; ++q)
      bin[q] = star_bin_2d(tab[q], tab[s2 + q], G.hx, G.hz, w.d->n_dirs);
    rc = star_columns(w.d, bin.data(), s2, tab.data() + 2 * s2);
    if (rc) return rc;
  }
  double* dL = (double*)(ws + P.off_tab);  // lengths first: 8-byte aligned
  int32_t* dtab = (int32_t*)(dL + s2);
  double* dpsi = (double*)(dtab + 4 * s2);  // 24 s2 bytes in: 8-byte aligned
  int64_t* dsrc = (int64_t*)(ws + P.off_src);
  hipError_t e = hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dL, L.data(), L.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dsrc, src_nodes_host, (size_t)n_src * sizeof(int64_t),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess && w.mspm)
    e = hipMemcpyAsync(dpsi, psi.data(), psi.size() * sizeof(double), hipMemcpyHostToDevice, s);
  double* dgeo = (double*)(ws + P.off_geo);
  int32_t* dslot = (int32_t*)(dgeo + 3 * ((size_t)s2 + P.N));
  if (e == hipSuccess && P.dim == 3)
    e = hipMemcpyAsync(dgeo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && P.dim == 3)
    e = hipMemcpyAsync(dslot, slots.data(), slots.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                       s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // host buffers are locals
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  if (P.dim == 3)  // the closest Fibonacci direction of every offset
    CHERT_LAUNCH("k_fib_nearest", k_fib_nearest, dim3((unsigned)s2), dim3(kFibThreads), 0, s,
                 dgeo + 3 * (size_t)s2, P.N, dgeo, s2, dtab + 2 * s2);

  uint8_t* ctl = ws + P.off_ctl;
  CellArgs a{};
  a.ncx = G.ncx;
  a.ncy = G.ncy;
  a.ncz = G.ncz;
  a.cn = cn;
  a.side = side;
  a.NX = P.NX;
  a.NY = P.NY;
  a.ns = P.ns;
  a.n_off = P.n_off;
  a.slot = P.dim == 3 ? dslot : nullptr;
  a.K = K;
  a.n_src = n_src;
  a.n_prob = P.n_prob;
  a.n = P.n;
  a.C = P.C;
  a.cls = G.cls;
  a.W = w.mspm ? nullptr : (const double*)(ws + P.off_W);
  a.src = dsrc;
  a.count = (int32_t*)ctl;
  int32_t* err = (int32_t*)(ctl + 8);
  a.alive = (int32_t*)(ctl + 12);
  a.stats = (unsigned long long*)(ctl + 16);
  a.part = (unsigned long long*)(ws + P.off_part);
  double* wmin = (double*)(ctl + 48);
  a.wmin = wmin;
  a.minkey = (unsigned long long*)(ctl + 256);
  a.bnd = (int32_t*)(a.minkey + 3 * (size_t)P.n_prob);
  a.cnt = a.bnd + 3 * (size_t)P.n_prob;
  a.active = (int32_t*)(ws + P.off_act);
  a.key = (unsigned long long*)(ws + P.off_key);
  a.list = (int32_t*)(ws + P.off_list);
  a.hop = (int32_t*)(ws + P.off_hop);
  a.bfs = (int32_t*)(ws + P.off_bfs);
  a.bid = (int32_t*)(ws + P.off_bid);
  a.bucket = o->bucket_width;
  a.tree_mask = 0;
  for (int fi = 0; fi < P.nfs; ++fi) {
    const int f = P.fields[fi];
    a.field_of[fi] = f;
    a.tau[fi] = f ? tau_i_dev : tau_r_dev;
    a.pred[fi] = f ? ((outs & CHERT_OUT_PRED_A) ? pred_a_dev : nullptr)
                   : ((outs & CHERT_OUT_PRED_P) ? pred_p_dev : nullptr);
    if (a.pred[fi]) a.tree_mask |= 1 << fi;
  }
  a.tstar = (outs & CHERT_OUT_TSTAR) ? tstar_dev : nullptr;
  a.mspm = w.mspm ? 1 : 0;
  a.n_canon = P.n_canon;
  a.canon = dtab + 3 * s2;
  a.L = dL;
  if (w.mspm) {
    const int64_t kr = P.K * P.n_canon, vr = 4 * (int64_t)P.n_prob * P.C * P.n_canon;
    uint8_t* kt = ws + P.off_kt;
    a.kV = (const double*)kt;
    a.kA = (const double*)(kt + kr * sizeof(double));
    a.kS = (const int32_t*)(kt + 2 * kr * sizeof(double));
    uint8_t* vt = ws + P.off_vt;
    a.tV = (const double*)vt;
    a.tA = (const double*)(vt + vr * sizeof(double));
    a.tS = (const int32_t*)(vt + 2 * vr * sizeof(double));
    a.job_class = (int32_t*)(ws + P.off_jobs);
  }

  // class ids checked before any output is written
  CHERT_LAUNCH("k_cell_zero", k_cell_zero, dim3(1), dim3(1), 0, s, err);
  enqueue_class_check(G.cls, P.n, K, err, s);
  {
    int32_t herr = 0;
    e = hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
    if (herr) return fail(CHERT_ERR_INVALID_ARG, "class id out of range");
  }

  enqueue_wmin_init(wmin, s);
  if (!w.mspm) {
    // weights of both fields for every class pair and segment offset
    chert_cache_layout lay;
    chert_cache_layout_of(w.d, n_classes, &lay);
    const uint8_t* cache = (const uint8_t*)w.cache_dev;
    const int64_t ent = 3 * P.K * (int64_t)P.n_cols;
    const int64_t mslice = (int64_t)mode * P.K * P.n_cols;
    const double* fields = (const double*)(cache + lay.fields_offset);
    const int32_t* Sm = (const int32_t*)(cache + lay.status_offset) + mslice;
    int32_t* best = nullptr;
    if (P.slow) {
      best = (int32_t*)(ws + P.off_best);
      enqueue_slow_lookup(best, K, P.n_cols, fields + CHERT_F_RX * ent + mslice,
                          fields + CHERT_F_RZ * ent + mslice, Sm, s2, dtab, dtab + s2, G.hx,
                          G.hz, s);
    }
    enqueue_pair_weights((double*)(ws + P.off_W), K, s2, fields + CHERT_F_V * ent + mslice,
                         fields + CHERT_F_A * ent + mslice, Sm, P.n_cols, dL, dtab + 2 * s2,
                         best, s);
    if (a.bucket > 0.0) enqueue_wmin((const double*)(ws + P.off_W), P.K * P.K * s2, wmin, s);
  } else {
    // the class table (the tree phase and the ordering scale read it; the
    // rounds solve their own corners afresh on every visit)
    enqueue_mspm_solve(w.classes_dev, mode, w.kernel, w.n_sweep, nullptr, nullptr, 0, P.K, P.K,
                       dpsi, P.n_canon, (double*)a.kV, (double*)a.kA, (int32_t*)a.kS, s);
    if (a.bucket > 0.0) {
      // canonical lengths ride in the visit table's first row until the
      // rounds overwrite it
      double* dLc = (double*)a.tV;
      e = hipMemcpyAsync(dLc, Lc.data(), Lc.size() * sizeof(double), hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
      CHERT_LAUNCH("k_mspm_wmin", k_mspm_wmin, dim3(64), dim3(256), 0, s, a, dLc, P.K);
      e = hipStreamSynchronize(s);  // Lc is a local
      if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
    }
  }

  const unsigned gfill = (unsigned)((P.n + 255) / 256 > 256 ? 256 : (P.n + 255) / 256);
  CHERT_LAUNCH("k_cell_fill", k_cell_fill, dim3(gfill, (unsigned)P.n_prob), dim3(256), 0, s, a);
  const unsigned gp = (unsigned)((P.n_prob + 255) / 256);
  CHERT_LAUNCH("k_cell_seed", k_cell_seed, dim3(gp), dim3(256), 0, s, a);

  // traveltime rounds, the host checking the round's list size every group
  const int64_t items = (int64_t)P.n_prob * P.C;
  const unsigned gsel = (unsigned)((items + 255) / 256 > 2048 ? 2048 : (items + 255) / 256);
  // waves per workgroup: the staged pair weights (ns^2 doubles per wave)
  // within 64 KiB of LDS
  const int ns = P.ns;
  int wpb = (int)(65536 / ((size_t)ns * ns * sizeof(double)));
  if (wpb > kCellWaves) wpb = kCellWaves;
  if (wpb < 1) wpb = 1;
  // (staging the whole class-pair table in LDS per workgroup measured
  // slower: fewer resident workgroups, and the table load costs more than
  // the weight loads it saves)
  a.w_lds = 0;
  const size_t lds = (size_t)wpb * ns * ns * sizeof(double);
  const unsigned grelax =
      (unsigned)((items + wpb - 1) / wpb > kRelaxGrid ? kRelaxGrid : (items + wpb - 1) / wpb);
  const unsigned gjobs = (unsigned)((4 * items + 255) / 256 > 1024 ? 1024 : (4 * items + 255) / 256);
  const int64_t gsolve = 4 * items > 16384 ? 16384 : 4 * items;
  int rounds = -1;
  for (int r = 0; r < P.max_rounds && rounds < 0;) {
    const int group = r < 16 ? 16 : 32;
    const int nb = r + group > P.max_rounds ? P.max_rounds - r : group;
    for (int q = 0; q < nb; ++q) {
      CHERT_LAUNCH("k_cell_select", k_cell_select, dim3(gsel), dim3(256), 0, s, a, r + q);
      if (w.mspm) {  // Algorithm 1: the visited cells' corners solved afresh
        CHERT_LAUNCH("k_mspm_jobs", k_mspm_jobs, dim3(gjobs), dim3(256), 0, s, a, r + q);
        enqueue_mspm_solve(w.classes_dev, mode, w.kernel, w.n_sweep, a.job_class,
                           a.count + ((r + q) & 1), 4, 0, gsolve, dpsi, P.n_canon,
                           (double*)a.tV, (double*)a.tA, (int32_t*)a.tS, s);
      }
      if (w.mspm)
        CHERT_LAUNCH("k_cell_relax", (k_cell_relax<true, false>), dim3(grelax), dim3(64 * wpb),
                     lds, s, a, r + q);
      else if (P.dim == 3)
        CHERT_LAUNCH("k_block_relax", (k_cell_relax<false, true>), dim3(grelax), dim3(64 * wpb),
                     lds, s, a, r + q);
      else
        CHERT_LAUNCH("k_cell_relax", (k_cell_relax<false, false>), dim3(grelax), dim3(64 * wpb),
                     lds, s, a, r + q);
    }
    r += nb;
    int32_t cnt = 0;
    e = hipMemcpyAsync(&cnt, a.count + ((r - 1) & 1), sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
    if (o->abort_flag_host && *o->abort_flag_host)
      return fail(CHERT_ERR_ABORTED, "aborted by the caller");
    if (cnt == 0) rounds = r;
  }
  if (rounds < 0) return fail(CHERT_ERR_NO_CONVERGENCE, "round cap reached");

  // predecessors and t*: one launch per level, the host checking between
  // groups of levels
  int levels = 0;
  if (a.tree_mask) {
    // few workgroups per problem: each reserves its staged appends with one
    // atomic per flush
    unsigned gx = (unsigned)(1024 / P.n_prob);
    if (gx < 1) gx = 1;
    if (gx > 128) gx = 128;
    int deepest = 1;  // levels holding nodes (the source's level 0 at least)
    for (int Lv = 0;;) {
      // groups of 8, then 16, then 32 levels between host checks (a group
      // with no append ends the BFS; predecessors trail by one level, so
      // any group of at least two levels finalises the last one)
      const int group = Lv < 16 ? 8 : (Lv < 48 ? 16 : 32);
      CHERT_LAUNCH("k_cell_zero", k_cell_zero, dim3(1), dim3(1), 0, s, a.alive);
      for (int q = 0; q < group; ++q, ++Lv)
        if (w.mspm)
          CHERT_LAUNCH("k_cell_level", (k_cell_level<true, false>), dim3(gx, (unsigned)P.n_prob),
                       dim3(kLvlThreads), 0, s, a, Lv);
        else if (P.dim == 3)
          CHERT_LAUNCH("k_block_level", (k_cell_level<false, true>),
                       dim3(gx, (unsigned)P.n_prob), dim3(kLvlThreads), 0, s, a, Lv);
        else
          CHERT_LAUNCH("k_cell_level", (k_cell_level<false, false>),
                       dim3(gx, (unsigned)P.n_prob), dim3(kLvlThreads), 0, s, a, Lv);
      int32_t alive = 0;
      e = hipMemcpyAsync(&alive, a.alive, sizeof(int32_t), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
      if (o->abort_flag_host && *o->abort_flag_host)
        return fail(CHERT_ERR_ABORTED, "aborted by the caller");
      if (alive == 0) {
        levels = deepest;
        break;
      }
      deepest = alive > deepest ? alive : deepest;
      if (Lv > P.n + 16) return fail(CHERT_ERR_HIP, "BFS did not end");
    }
  }
  if (o->stats_host) {
    unsigned long long st[4] = {0, 0, 0, 0};
    std::vector<unsigned long long> part((size_t)3 * kRelaxGrid);
    e = hipMemcpyAsync(st, a.stats, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(part.data(), a.part, part.size() * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
    for (int b = 0; b < kRelaxGrid; ++b)
      for (int i = 0; i < 3; ++i) st[i] += part[3 * (size_t)b + i];
    chert_trace_stats* ts = o->stats_host;
    memset(ts, 0, sizeof(*ts));
    ts->rounds[0] = rounds;
    ts->rounds[1] = levels;
    ts->tile_visits[0] = (int64_t)st[0];
    ts->edge_relaxations[0] = (int64_t)st[1];
    ts->levels_sum[0] = (int64_t)st[2];
    // MSPM: (class, direction) solves of the rounds' corner tables
    ts->edge_relaxations[1] = (int64_t)st[3] * P.n_canon;
  }
  return CHERT_OK;
}

}  // namespace
}  // namespace chert

using namespace chert;

extern "C" size_t chert_trace_cells_workspace_bytes(const chert_cache_desc* d,
                                                    int64_t n_classes,
                                                    const chert_cell_grid* g, int32_t n_src,
                                                    const chert_trace_opts* o) {
  if (!g) return 0;
  CellSrc w;
  w.d = d;
  return cell_workspace(w, n_classes, geo_of(g), n_src, o);
}

extern "C" int chert_trace_cells(const chert_cache_desc* d, const void* cache_dev,
                                 int64_t n_classes, const chert_cell_grid* g, int32_t mode,
                                 const int64_t* src_nodes_host, int32_t n_src,
                                 const chert_trace_opts* o, double* tau_r_dev, double* tau_i_dev,
                                 double* tstar_dev, int32_t* pred_p_dev, int32_t* pred_a_dev,
                                 void* workspace_dev, size_t workspace_bytes, void* stream) {
  if (!g) return fail(CHERT_ERR_INVALID_ARG, "null grid");
  CellSrc w;
  w.d = d;
  w.cache_dev = cache_dev;
  return trace_cells_impl(w, n_classes, geo_of(g), mode, src_nodes_host, n_src, o, tau_r_dev,
                          tau_i_dev, tstar_dev, pred_p_dev, pred_a_dev, workspace_dev,
                          workspace_bytes, stream);
}

extern "C" size_t chert_trace_blocks_workspace_bytes(const chert_cache_desc* d,
                                                     int64_t n_classes,
                                                     const chert_block_grid* g, int32_t n_src,
                                                     const chert_trace_opts* o) {
  if (!g) return 0;
  CellSrc w;
  w.d = d;
  return cell_workspace(w, n_classes, geo_of(g), n_src, o);
}

extern "C" int chert_trace_blocks(const chert_cache_desc* d, const void* cache_dev,
                                  int64_t n_classes, const chert_block_grid* g, int32_t mode,
                                  const int64_t* src_nodes_host, int32_t n_src,
                                  const chert_trace_opts* o, double* tau_r_dev, double* tau_i_dev,
                                  double* tstar_dev, int32_t* pred_p_dev, int32_t* pred_a_dev,
                                  void* workspace_dev, size_t workspace_bytes, void* stream) {
  if (!g) return fail(CHERT_ERR_INVALID_ARG, "null grid");
  CellSrc w;
  w.d = d;
  w.cache_dev = cache_dev;
  return trace_cells_impl(w, n_classes, geo_of(g), mode, src_nodes_host, n_src, o, tau_r_dev,
                          tau_i_dev, tstar_dev, pred_p_dev, pred_a_dev, workspace_dev,
                          workspace_bytes, stream);
}

extern "C" size_t chert_trace_mspm_workspace_bytes(int64_t n_classes, const chert_cell_grid* g,
                                                   int32_t n_src, const chert_trace_opts* o) {
  CellSrc w;
  w.mspm = true;
  w.kernel = CHERT_KERNEL_MEV;
  w.n_sweep = 8;
  w.classes_dev = (const chert_class*)1;  // not dereferenced by the size query
  if (!g) return 0;
  return cell_workspace(w, n_classes, geo_of(g), n_src, o);
}

extern "C" int chert_trace_mspm(const chert_class* classes_dev, int64_t n_classes,
                                const chert_cell_grid* g, int32_t mode, int32_t kernel,
                                int32_t n_sweep, const int64_t* src_nodes_host, int32_t n_src,
                                const chert_trace_opts* o, double* tau_r_dev, double* tau_i_dev,
                                double* tstar_dev, int32_t* pred_p_dev, int32_t* pred_a_dev,
                                void* workspace_dev, size_t workspace_bytes, void* stream) {
  CellSrc w;
  w.mspm = true;
  w.classes_dev = classes_dev;
  w.kernel = kernel;
  w.n_sweep = n_sweep;
  if (!g) return fail(CHERT_ERR_INVALID_ARG, "null grid");
  return trace_cells_impl(w, n_classes, geo_of(g), mode, src_nodes_host, n_src, o, tau_r_dev,
                          tau_i_dev, tstar_dev, pred_p_dev, pred_a_dev, workspace_dev,
                          workspace_bytes, stream);
}
