// Directional cache builder (eq 26; Algorithm 2, cache construction) for
// gfx950.  Two launches per build:
//   k_sweep: one lane per (mode, class, theta_R sample); solves the inner
//            homogeneity root theta_I(theta_R) (eq 9) by the outward scan and
//            stores (theta_I, local ray angle) in the sweep table.
//   k_solve: one workgroup per (mode, class, 64 target directions); stages
//            the class's sweep table in LDS, brackets every theta_R whose ray
//            angle crosses the target, refines each root with a 2D Newton
//            iteration on (homogeneity residual, ray-direction miss), keeps
//            the largest ray velocity (first arrival) and writes the entry and
//            its centrosymmetric copy (eqs 10-11).
// Per-node caches (one class per node) run both steps per job in one
// workgroup (k_build_fused), or start from the surrogate's prediction:
// k_warm_predict (MLP on the matrix cores), k_warm_solve (Newton polish
// and the checks that the plain search would return the same root),
// k_warm_window and k_warm_fold (the plain search's brackets near fold
// directions), with k_build_fused re-solving any job that fails a check.
// Everything is FP64 except the MLP: qSV cusps and triplications need it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "chert.h"
#include "chert_internal.h"
#include "mlp.h"
#include "physics.h"
#include "solve.h"

namespace chert {

struct SweepArgs {
  const chert_class* classes;
  int64_t n_classes;
  int n_modes;
  int modes[3];
  int kernel;
  int n_sweep;
  double2* table;  // [n_modes][n_classes][n_sweep] = (theta_I, psi); psi NaN: none
};

__device__ __forceinline__ bool is_fluid_shear(const chert_class& c, int mode) {
  if (mode == CHERT_QP) return false;
  return c.a44 == 0.0 || (mode == CHERT_QSH && c.a66 == 0.0);
}

__device__ __forceinline__ bool class_invalid(const chert_class& c) {
  const double* p = &c.a11;
  for (int i = 0; i < 10; ++i)
    if (isnan(p[i])) return true;
  if (!(c.a11 > 0.0) || !(c.a33 > 0.0) || c.a44 < 0.0 || c.a66 < 0.0) return true;
  for (int i = 5; i < 10; ++i)
    if (!(p[i] > 0.0)) return true;
  return false;
}

__global__ void __launch_bounds__(256) k_sweep(SweepArgs a) {
  int64_t total = (int64_t)a.n_modes * a.n_classes * a.n_sweep;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int j = (int)(t % a.n_sweep);
    int64_t job = t / a.n_sweep;
    int64_t k = job % a.n_classes;
    int mode = a.modes[job / a.n_classes];
    chert_class c = a.classes[k];
    double2 out = make_double2(0.0, NAN);
    if (!class_invalid(c) && !is_fluid_shear(c, mode)) {
      Medium m = load_medium(c);
      double thR = (j + 0.5) * (kTwoPi / a.n_sweep);
      double thI, sr, cr;
      sincos(thR, &sr, &cr);
      if (theta_imag_sc(m, mode, a.kernel, sr, cr, &thI)) {
        double psi = ray_angle_sc(m, mode, a.kernel, sr, cr, thI);
        if (isfinite(psi)) out = make_double2(thI, psi);
      }
    }
    a.table[t] = out;
  }
}

struct SolveArgs : SolveParams {
  const chert_class* classes;
  int64_t n_classes;
  int n_modes;
  int modes[3];
  int n_dirs;
  const double2* table;
  double* fields;   // [CHERT_NF][3][n_classes][n_cols]
  int32_t* status;  // [3][n_classes][n_cols]
  int n_cols;       // stored direction columns per (mode, class)
  int n_solve;      // directions solved per (mode, class); the rest are copies
  int dim;          // 2, or 3: columns are Fibonacci ray directions
  double fib_ga;    // 3D: golden angle pi (3 - sqrt 5) of the direction set
  int subset;       // 0: every direction d < n_dirs/2, column d, copy at d + n_dirs/2
  int16_t dir[kMaxSubset / 2];   // solved direction (subset caches)
  int16_t col[kMaxSubset / 2];   // its column
  int16_t pcol[kMaxSubset / 2];  // column of the reversed direction
};

__device__ __forceinline__ void dir_cols(const SolveArgs& a, int s, int* d, int* c, int* pc) {
  if (!a.subset) {
    *d = s;
    *c = s;
    *pc = s + a.n_dirs / 2;
  } else {
    *d = a.dir[s];
    *c = a.col[s];
    *pc = a.pcol[s];
  }
}

// local target ray angle of 2D direction d (eq 36)
__device__ __forceinline__ double dir_psi(const SolveArgs& a, int d, double tilt) {
  return wrap_pi(d * (kTwoPi / a.n_dirs) - tilt);
}

// 3D: Fibonacci ray direction s of n_dirs, and its polar angle to the
// symmetry axis e_z' of eq 35 (the target angle of the sagittal solve)
__device__ __forceinline__ double3 fib_dir(const SolveArgs& a, int s) {
  const double z = 1.0 - (2.0 * s + 1.0) / a.n_dirs;
  const double r = sqrt(1.0 - z * z);
  double sp, cp;
  sincos(s * a.fib_ga, &sp, &cp);
  return make_double3(r * cp, r * sp, z);
}

__device__ __forceinline__ double polar_to_axis(const double3& f, const chert_class& c) {
  double st, ct, sa, ca;
  sincos(c.tilt, &st, &ct);
  sincos(c.azimuth, &sa, &ca);
  double d = f.x * (st * ca) + f.y * (st * sa) + f.z * ct;
  d = fmin(1.0, fmax(-1.0, d));
  return acos(d);
}

__device__ __forceinline__ void store_entry(const SolveArgs& a, int64_t base, int64_t stride,
                                            const Entry& e, double tilt, int32_t st) {
  double ct, stl;
  sincos(tilt, &stl, &ct);
  double gx = e.r1 * ct + e.r3 * stl;
  double gz = -e.r1 * stl + e.r3 * ct;
  double* f = a.fields;
  f[CHERT_F_V * stride + base] = e.V;
  f[CHERT_F_A * stride + base] = e.A;
  f[CHERT_F_Q * stride + base] = e.Q;
  f[CHERT_F_RX * stride + base] = gx;
  f[CHERT_F_RZ * stride + base] = gz;
  f[CHERT_F_THR * stride + base] = e.thR;
  f[CHERT_F_THI * stride + base] = e.thI;
  f[CHERT_F_RES * stride + base] = e.res;
  a.status[base] = st;
}

__device__ __forceinline__ void store_invalid(const SolveArgs& a, int64_t base, int64_t stride,
                                              int32_t st) {
  for (int f = 0; f < CHERT_NF; ++f) a.fields[f * stride + base] = NAN;
  a.status[base] = st;
}

// Write the solved entry and its centrosymmetric copy (same ray quantities,
// reversed direction, slowness direction turned by pi).
__device__ __forceinline__ void store_pair(const SolveArgs& a, int64_t row, int col, int pcol,
                                           const Entry& best, double tilt, int32_t st) {
  const int64_t stride = 3 * a.n_classes * (int64_t)a.n_cols;
  if (st & (CHERT_ST_NO_BRACKET | CHERT_ST_FLUID) || (st == CHERT_ST_NONPHYS && isnan(best.V))) {
    store_invalid(a, row + col, stride, st);
    store_invalid(a, row + pcol, stride, st);
    return;
  }
  if (!(best.res <= a.resid_tol)) st |= CHERT_ST_NOCONV;
  store_entry(a, row + col, stride, best, tilt, st);
  Entry r = best;
  r.thR = best.thR + kPi;
  if (r.thR >= kTwoPi) r.thR -= kTwoPi;
  store_entry(a, row + pcol, stride, r, tilt, st);
  a.fields[CHERT_F_RX * stride + row + pcol] = -a.fields[CHERT_F_RX * stride + row + col];
  a.fields[CHERT_F_RZ * stride + row + pcol] = -a.fields[CHERT_F_RZ * stride + row + col];
}

// 3D entry: one column per Fibonacci direction (no centrosymmetric copy);
// the stored ray direction is the direction itself (x and z components)
__device__ __forceinline__ void store_single(const SolveArgs& a, int64_t idx, int64_t stride,
                                             const Entry& best, const double3& f, int32_t st) {
  if (st & (CHERT_ST_NO_BRACKET | CHERT_ST_FLUID) || (st == CHERT_ST_NONPHYS && isnan(best.V))) {
    store_invalid(a, idx, stride, st);
    return;
  }
  if (!(best.res <= a.resid_tol)) st |= CHERT_ST_NOCONV;
  double* fl = a.fields;
  fl[CHERT_F_V * stride + idx] = best.V;
  fl[CHERT_F_A * stride + idx] = best.A;
  fl[CHERT_F_Q * stride + idx] = best.Q;
  fl[CHERT_F_RX * stride + idx] = f.x;
  fl[CHERT_F_RZ * stride + idx] = f.z;
  fl[CHERT_F_THR * stride + idx] = best.thR;
  fl[CHERT_F_THI * stride + idx] = best.thI;
  fl[CHERT_F_RES * stride + idx] = best.res;
  a.status[idx] = st;
}

// Entries of a class that cannot be solved (invalid parameters, or a shear
// mode without shear stiffness).
__device__ __forceinline__ int32_t class_block(const chert_class& c, int mode) {
  if (class_invalid(c)) return CHERT_ST_NONPHYS;
  if (is_fluid_shear(c, mode)) return CHERT_ST_FLUID;
  return 0;
}

// Two-launch path (few classes): one workgroup per (mode, class, 64
// directions), sweep table from k_sweep staged in LDS.
// Class caches: SPLIT lanes per target direction, 64 / SPLIT directions per
// workgroup (SPLIT = 4 when there are too few directions to fill the
// device, else 1).  Each lane scans its share of the sweep table for
// brackets and refines them; the direction's first lane then folds the
// roots in scan order (the plain search's choice, exactly), or, if a share
// held more than kSolveSlots brackets, runs the serial search itself.
constexpr int kSolveSlots = 3;
struct SolveCand {
  Entry e;
  int32_t ok, ill;
};
template <int SPLIT>
__global__ void __launch_bounds__(64) k_solve(SolveArgs a) {
  constexpr int kSolveSplit = SPLIT, kSolveDirs = 64 / SPLIT;
  extern __shared__ double2 tab[];
  __shared__ SolveCand s_c[kSolveDirs][kSolveSplit * kSolveSlots];
  __shared__ int s_nc[kSolveDirs][kSolveSplit];
  __shared__ int s_over[kSolveDirs];
  __shared__ int s_br[64 * kMaxBr];
  const int chunks = (a.n_solve + kSolveDirs - 1) / kSolveDirs;
  const int64_t job = blockIdx.x / chunks;
  const int chunk = blockIdx.x % chunks;
  const int64_t k = job % a.n_classes;
  const int mode = a.modes[job / a.n_classes];
  const double2* src = a.table + job * a.n_sweep;
  for (int j = threadIdx.x; j < a.n_sweep; j += blockDim.x) tab[j] = src[j];
  const int dl = threadIdx.x / kSolveSplit, q = threadIdx.x % kSolveSplit;
  if (q == 0) s_over[dl] = 0;
  __syncthreads();

  const int sidx = chunk * kSolveDirs + dl;
  const bool valid = sidx < a.n_solve;
  const int64_t row = ((int64_t)mode * a.n_classes + k) * a.n_cols;
  const chert_class c = a.classes[k];
  const int32_t blocked = class_block(c, mode);
  const Medium m = load_medium(c);
  const FullTable full{tab, a.n_sweep};
  double3 f = make_double3(0.0, 0.0, 0.0);
  int d = 0, col = 0, pcol = 0;
  double psi_star = 0.0;
  if (valid) {
    if (a.dim == 3) {
      f = fib_dir(a, sidx);
      psi_star = blocked ? 0.0 : polar_to_axis(f, c);
    } else {
      dir_cols(a, sidx, &d, &col, &pcol);
      psi_star = blocked ? 0.0 : dir_psi(a, d, m.tilt);
    }
  }
  const bool el = theta_i_zero(m, mode);
  if (valid && !blocked) {
    // this lane's share of the bracket scan, then its roots
    const int span = (a.n_sweep + kSolveSplit - 1) / kSolveSplit;
    const int lo = q * span, hi = min(a.n_sweep, lo + span);
    int brj[kSolveSlots];
    int nb = 0;
    for (int j = lo; j < hi; ++j) {
      if (!is_bracket(full, j, a.n_sweep, psi_star)) continue;
      if (nb < kSolveSlots) brj[nb] = j;
      ++nb;
    }
    if (nb > kSolveSlots) s_over[dl] = 1;
    const int nk = nb < kSolveSlots ? nb : kSolveSlots;
    for (int b = 0; b < nk; ++b) {
      SolveCand& sc = s_c[dl][q * kSolveSlots + b];
      bool ill = false;
      const int j = brj[b];
      sc.ok = bracket_root(a, m, mode, j, tab[j], tab[j + 1 == a.n_sweep ? 0 : j + 1], psi_star,
                           el, &sc.e, &ill) ? 1 : 0;
      sc.ill = ill ? 1 : 0;
    }
    s_nc[dl][q] = nk;
  }
  __syncthreads();
  if (!valid || q != 0) return;
  Entry best{};
  best.V = NAN;
  int32_t st = blocked;
  if (!blocked) {
    if (s_over[dl]) {
      st = solve_dir(a, m, mode, full, psi_star, s_br + threadIdx.x * kMaxBr, &best);
    } else {
      bool found = false, ill = false;
      for (int qq = 0; qq < kSolveSplit; ++qq)
        for (int b = 0; b < s_nc[dl][qq]; ++b) {
          const SolveCand& sc = s_c[dl][qq * kSolveSlots + b];
          if (sc.ok) fold_choice(sc.e, sc.ill != 0, psi_star, a.resid_tol, &found, &ill, &best);
        }
      st = solve_status(found, ill, best);
    }
  }
  if (a.dim == 3) {
    store_single(a, row + sidx, 3 * a.n_classes * (int64_t)a.n_cols, best, f, st);
    return;
  }
  store_pair(a, row, col, pcol, best, blocked ? 0.0 : m.tilt, st);
}

// Fused path (many classes, e.g. one per node): one workgroup per
// (mode, class) sweeps theta_R into LDS, then solves that class's
// directions; no sweep table in HBM.
constexpr int kNodeThreads = 256;
__global__ void __launch_bounds__(kNodeThreads) k_build_fused(SolveArgs a, const int32_t* list,
                                                              const int32_t* list_len,
                                                              int64_t n_jobs) {
  extern __shared__ double2 tab[];
  __shared__ int s_br[kNodeThreads * kMaxBr];
  const int64_t n = list ? (int64_t)*list_len : n_jobs;
  for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
    const int64_t job = list ? (int64_t)list[it] : it;
    const int64_t k = job % a.n_classes;
    const int mode = a.modes[job / a.n_classes];
    const chert_class c = a.classes[k];
    const int64_t row = ((int64_t)mode * a.n_classes + k) * a.n_cols;
    const int32_t blocked = class_block(c, mode);
    if (blocked) {
      Entry none{};
      none.V = NAN;
      for (int sidx = threadIdx.x; sidx < a.n_solve; sidx += blockDim.x) {
        int d, col, pcol;
        dir_cols(a, sidx, &d, &col, &pcol);
        store_pair(a, row, col, pcol, none, 0.0, blocked);
      }
      continue;  // block-uniform
    }
    const Medium m = load_medium(c);
    __syncthreads();  // the previous job's solves are done with tab
    for (int j = threadIdx.x; j < a.n_sweep; j += blockDim.x) {
      const double thR = (j + 0.5) * (kTwoPi / a.n_sweep);
      double thI, sr, cr;
      sincos(thR, &sr, &cr);
      double2 out = make_double2(0.0, NAN);
      if (theta_imag_sc(m, mode, a.kernel, sr, cr, &thI)) {
        const double psi = ray_angle_sc(m, mode, a.kernel, sr, cr, thI);
        if (isfinite(psi)) out = make_double2(thI, psi);
      }
      tab[j] = out;
    }
    __syncthreads();
    for (int sidx = threadIdx.x; sidx < a.n_solve; sidx += blockDim.x) {
      int d, col, pcol;
      dir_cols(a, sidx, &d, &col, &pcol);
      Entry best{};
      const int32_t st = solve_dir(a, m, mode, FullTable{tab, a.n_sweep}, dir_psi(a, d, m.tilt),
                                   s_br + threadIdx.x * kMaxBr, &best);
      store_pair(a, row, col, pcol, best, m.tilt, st);
    }
  }
}

// MSPM's local tables (Algorithm 1): for each job -- a class -- a fresh
// theta_R sweep into LDS, then one solve per target global ray angle.  No
// cache and nothing kept between calls: every call pays for its sweeps.
// Outputs V, A and the status of each (job, target), with the status rules
// of cache entries (NaN quantities where there is no usable root).
__global__ void __launch_bounds__(64) k_mspm_solve(SolveArgs a, const int32_t* job_class,
                                                   const int32_t* n_jobs_dev, int n_jobs_mul,
                                                   int64_t n_jobs_fixed, const double* psi,
                                                   int n_tgt, double* V, double* A,
                                                   int32_t* st) {
  extern __shared__ double2 tab[];
  __shared__ int s_br[64 * kMaxBr];
  const int64_t n = n_jobs_dev ? (int64_t)(*n_jobs_dev) * n_jobs_mul : n_jobs_fixed;
  const int mode = a.modes[0];
  for (int64_t q = blockIdx.x; q < n; q += gridDim.x) {
    const int64_t k = job_class ? (int64_t)job_class[q] : q;
    const chert_class c = a.classes[k];
    const int32_t blocked = class_block(c, mode);
    double* Vq = V + q * n_tgt;
    double* Aq = A + q * n_tgt;
    int32_t* Sq = st + q * n_tgt;
    if (blocked) {
      for (int t = threadIdx.x; t < n_tgt; t += blockDim.x) {
        Vq[t] = NAN;
        Aq[t] = NAN;
        Sq[t] = blocked;
      }
      continue;  // block-uniform
    }
    const Medium m = load_medium(c);
    __syncthreads();  // the previous job's solves are done with tab
    for (int j = threadIdx.x; j < a.n_sweep; j += blockDim.x) {
      const double thR = (j + 0.5) * (kTwoPi / a.n_sweep);
      double thI, sr, cr;
      sincos(thR, &sr, &cr);
      double2 out = make_double2(0.0, NAN);
      if (theta_imag_sc(m, mode, a.kernel, sr, cr, &thI)) {
        const double ps = ray_angle_sc(m, mode, a.kernel, sr, cr, thI);
        if (isfinite(ps)) out = make_double2(thI, ps);
      }
      tab[j] = out;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n_tgt; t += blockDim.x) {
      Entry best{};
      int32_t s = solve_dir(a, m, mode, FullTable{tab, a.n_sweep}, wrap_pi(psi[t] - m.tilt),
                            s_br + threadIdx.x * kMaxBr, &best);
      if ((s & (CHERT_ST_NO_BRACKET | CHERT_ST_FLUID)) || (s == CHERT_ST_NONPHYS && isnan(best.V))) {
        Vq[t] = NAN;
        Aq[t] = NAN;
      } else {
        if (!(best.res <= a.resid_tol)) s |= CHERT_ST_NOCONV;
        Vq[t] = best.V;
        Aq[t] = best.A;
      }
      Sq[t] = s;
    }
  }
}

int enqueue_mspm_solve(const chert_class* classes_dev, int mode, int kernel, int n_sweep,
                       const int32_t* job_class, const int32_t* n_jobs_dev, int n_jobs_mul,
                       int64_t n_jobs_fixed, int64_t grid, const double* psi_dev, int n_tgt,
                       double* V, double* A, int32_t* st, hipStream_t s) {
  SolveArgs so{};
  so.modes[0] = mode;
  so.n_modes = 1;
  so.classes = classes_dev;
  so.kernel = kernel;
  so.n_sweep = n_sweep;
  so.resid_tol = 1e-9;
  so.newton_iters = 12;
  so.bisect_iters = 200;
  const unsigned g = (unsigned)(grid < 1 ? 1 : (grid > 65535 ? 65535 : grid));
  CHERT_LAUNCH("k_mspm_solve", k_mspm_solve, dim3(g), dim3(64),
               (size_t)n_sweep * sizeof(double2), s, so, job_class, n_jobs_dev, n_jobs_mul,
               n_jobs_fixed, psi_dev, n_tgt, V, A, st);
  return CHERT_OK;
}

// ---------------------------------------------------------------- warm start
// Surrogate-started solve: the MLP (mlp.h) predicts (theta_R, theta_I) for
// each solved direction, an FP64 Newton iteration polishes it, and the root
// is kept only where it is provably the one the sweep-and-bracket search
// above would pick; other jobs go back to k_build_fused.

constexpr int kProxyN = 180;                        // elastic map samples on [0, pi)
constexpr double kFoldSlope = 0.2;                  // d psi / d theta_R below this: fold
constexpr double kFoldMargin = 2.0 * kPi / 180.0;   // guard band around a fold
constexpr int kFoldBins = 720;                      // 0.5-degree ray-angle bins
constexpr int kFoldWords = (kFoldBins + 31) / 32;
constexpr double kWarmSlope = 0.05;                 // accepted roots: slope at least this

// a bracket of a fold direction's windowed table: sweep sample j and the
// (theta_I, ray angle) pairs at j and j + 1
struct WinBracket {
  double2 sa, sb;
  int32_t j, pad[3];
};

struct WarmArgs {
  SolveArgs so;
  const void* blob;
  float2* pred;                 // [jobs][n_solve] (theta_R - psi, theta_I)
  int32_t* fb_list;             // jobs for the plain path
  int32_t* fb_len;
  int32_t* win_list;            // jobs with directions near a fold (k_warm_window)
  int32_t* win_len;
  int4* dirs;                   // fold directions: (job, sidx, first bracket, brackets)
  int32_t* dir_len;
  int64_t dir_cap;
  WinBracket* brs;              // their brackets, in scan order per direction
  int32_t* br_len;
  int64_t br_cap;
  unsigned long long* stats;    // CHERT_WARM_NSTATS counters (folded from shard)
  unsigned long long* shard;    // [kStatSlots][16] per-slot partial counters
  double resid_tol;
};

// surrogate predictions for every (job, solved direction): kInferRows per
// workgroup
__global__ void __launch_bounds__(mlp::kThreads) k_warm_predict(WarmArgs w, int64_t n_rows) {
  __shared__ mlp::InferTile t;
  const SolveArgs& a = w.so;
  const mlp::Net n = mlp::net_of(w.blob);
  const int64_t base = (int64_t)blockIdx.x * mlp::kInferRows;
  for (int r = threadIdx.x; r < mlp::kInferRows; r += blockDim.x) {
    const int64_t e = base + r;
    float f[mlp::kIn] = {};
    if (e < n_rows) {
      const int64_t job = e / a.n_solve;
      const int sidx = (int)(e % a.n_solve);
      const chert_class c = a.classes[job % a.n_classes];
      int d, col, pcol;
      dir_cols(a, sidx, &d, &col, &pcol);
      mlp::features(c, a.modes[job / a.n_classes], dir_psi(a, d, c.tilt), f);
    }
    mlp::stage_row(n, t.x, r, f, e >= n_rows);
  }
  __syncthreads();
  mlp::forward_infer(n, t, [&](int r, int col, float v) {
    if (col < 2 && base + r < n_rows) (&w.pred[base + r].x)[col] = v;
  });
}

__device__ __forceinline__ int fold_bin(double psi) {
  int b = (int)floor((psi + kPi) * (kFoldBins / kTwoPi));
  b %= kFoldBins;
  return b < 0 ? b + kFoldBins : b;
}

// sweep samples whose theta_R the elastic map sends within kFoldMargin of
// psi_star (either half of the circle), plus one sample on each side
__device__ __forceinline__ void mark_window(const SolveArgs& a, const double* psi, double psi_star,
                                            uint32_t* mask) {
  const double dth = kTwoPi / a.n_sweep;
  for (int j = threadIdx.x; j < kProxyN; j += blockDim.x) {
    const double pa = psi[j];
    const double pb = j + 1 < kProxyN ? psi[j + 1] : psi[0] + kPi;
    const double dp = wrap_pi(pb - pa);
    const double lo = fmin(pa, pa + dp) - kFoldMargin;
    const double width = fabs(dp) + 2.0 * kFoldMargin;
    for (int half = 0; half < 2; ++half) {
      double off = fmod(psi_star - half * kPi - lo, kTwoPi);
      if (off < 0.0) off += kTwoPi;
      if (off > width) continue;
      const double ta = (j + 0.5) * (kPi / kProxyN) + half * kPi;
      const double tb = ta + kPi / kProxyN;
      const int i0 = (int)floor(ta / dth - 0.5) - 1;
      const int i1 = (int)ceil(tb / dth - 0.5) + 1;
      for (int i = i0; i <= i1; ++i) {
        const int q = ((i % a.n_sweep) + a.n_sweep) % a.n_sweep;
        atomicOr(&mask[q >> 5], 1u << (q & 31));
      }
    }
  }
}

// Elastic stand-in of the ray-angle map psi(theta_R) on [0, pi) (the other
// half is its centrosymmetric image): folds and near-folds within the margin
// mark ray-angle bins where the map may have several branches.  All 64 lanes;
// s_fold and *s_all must be cleared (and a barrier passed) before the call;
// ends with a barrier.
// `work`: this lane takes part, as lane l of the L serving this job; every
// thread of the workgroup calls it (it holds two workgroup barriers)
__device__ __forceinline__ void proxy_folds(const Medium& me, int mode, int kernel, bool work,
                                            int l, int L, double* s_psi, uint32_t* s_fold,
                                            int* s_all) {
  for (int j = l; work && j < kProxyN; j += L) {
    double sr, cr;  // real angle: sinh 0 = 0, cosh 0 = 1
    sincos((j + 0.5) * (kPi / kProxyN), &sr, &cr);
    s_psi[j] = ray_angle(energy_velocity_t(me, mode, kernel, Trig{sr, cr, 0.0, 1.0}));
  }
  __syncthreads();
  for (int j = l; work && j < kProxyN; j += L) {
    const double pa = s_psi[j];
    const double pb = j + 1 < kProxyN ? s_psi[j + 1] : s_psi[0] + kPi;
    if (!isfinite(pa) || !isfinite(pb)) {
      *s_all = 1;
      continue;
    }
    const double dp = wrap_pi(pb - pa);
    if (dp * (kProxyN / kPi) >= kFoldSlope) continue;
    const double lo = fmin(pa, pa + dp) - kFoldMargin;
    const double hi = fmax(pa, pa + dp) + kFoldMargin;
    const int nb = (int)floor((hi - lo) * (kFoldBins / kTwoPi)) + 2;
    for (int half = 0; half < 2; ++half) {
      const int b0 = fold_bin(lo + half * kPi);
      for (int q = 0; q < nb && q < kFoldBins; ++q) {
        const int b = (b0 + q) % kFoldBins;
        atomicOr(&s_fold[b >> 5], 1u << (b & 31));
      }
    }
  }
  __syncthreads();
}

__device__ __forceinline__ Medium elastic_of(const Medium& m) {
  Medium me = m;
  me.a11.im = me.a13.im = me.a33.im = me.a44.im = me.a66.im = 0.0;
  me.elastic_ps = me.elastic_sh = true;
  return me;
}

// Several (mode, class) jobs per workgroup, L = min(n_solve, 64) lanes each
// (one lane per solved direction; with n_solve = 40 a job per wavefront
// left 24 lanes idle): every direction away from a fold is polished from
// its prediction.  A job with a rejected direction goes to the plain path
// (fb_list); a job whose other directions all passed and that has
// directions near a fold goes to k_warm_window (win_list).  Small static
// LDS only, so occupancy is set by registers.
constexpr int kWarmSolveThreads = 256;
constexpr int kWarmSolveJobs = 16;  // most jobs a workgroup holds
__host__ __device__ inline int warm_lanes(int n_solve) { return n_solve < 64 ? n_solve : 64; }
__host__ __device__ inline int warm_jobs(int n_solve) {
  const int j = kWarmSolveThreads / warm_lanes(n_solve);
  return j < kWarmSolveJobs ? j : kWarmSolveJobs;
}

__global__ void __launch_bounds__(kWarmSolveThreads) k_warm_solve(WarmArgs w, int64_t n_jobs) {
  __shared__ double s_psi[kWarmSolveJobs][kProxyN];
  __shared__ uint32_t s_fold[kWarmSolveJobs][kFoldWords];
  __shared__ int s_all[kWarmSolveJobs], s_nflag[kWarmSolveJobs], s_rej[kWarmSolveJobs];
  __shared__ uint32_t s_cnt[CHERT_WARM_NSTATS];

  const SolveArgs& a = w.so;
  const int L = warm_lanes(a.n_solve), J = warm_jobs(a.n_solve);
  const int q = (int)threadIdx.x / L, l = (int)threadIdx.x % L;
  const int64_t job = (int64_t)blockIdx.x * J + q;
  const bool on = q < J && job < n_jobs;  // this lane serves a job
  const int qs = q < J ? q : 0;           // its LDS slot (idle lanes: any)
  for (int i = threadIdx.x; i < CHERT_WARM_NSTATS; i += blockDim.x) s_cnt[i] = 0;
  for (int i = threadIdx.x; i < kWarmSolveJobs * kFoldWords; i += blockDim.x)
    (&s_fold[0][0])[i] = 0;
  if (threadIdx.x < kWarmSolveJobs) {
    s_all[threadIdx.x] = 0;
    s_nflag[threadIdx.x] = 0;
    s_rej[threadIdx.x] = 0;
  }
  const int64_t k = on ? job % a.n_classes : 0;
  const int mode = on ? a.modes[job / a.n_classes] : 0;
  const chert_class c = a.classes[k];
  const int64_t row = ((int64_t)mode * a.n_classes + k) * a.n_cols;
  const int32_t blocked = on ? class_block(c, mode) : 0;
  const bool work = on && !blocked;
  __syncthreads();  // LDS cleared
  if (on && l == 0) atomicAdd(&s_cnt[0], 1u);
  if (on && blocked) {
    Entry none{};
    none.V = NAN;
    for (int sidx = l; sidx < a.n_solve; sidx += L) {
      int d, col, pcol;
      dir_cols(a, sidx, &d, &col, &pcol);
      store_pair(a, row, col, pcol, none, 0.0, blocked);
    }
  }
  const Medium m = load_medium(c);
  const bool el = theta_i_zero(m, mode);
  proxy_folds(elastic_of(m), mode, a.kernel, work, l, L, s_psi[qs], s_fold[qs], &s_all[qs]);

  bool reject = false;
  for (int sidx = l; work && sidx < a.n_solve; sidx += L) {
    int d, col, pcol;
    dir_cols(a, sidx, &d, &col, &pcol);
    const double psi_star = dir_psi(a, d, m.tilt);
    atomicAdd(&s_cnt[2], 1u);
    const int fb = fold_bin(psi_star);
    if (s_all[qs]) {
      reject = true;
      continue;
    }
    if ((s_fold[qs][fb >> 5] >> (fb & 31)) & 1u) {  // near a fold: k_warm_window
      atomicAdd(&s_cnt[3], 1u);
      atomicAdd(&s_nflag[qs], 1);
      continue;
    }
    const float2 p = w.pred[job * a.n_solve + sidx];
    double x, y, slope;
    if (!warm_newton(m, mode, a.kernel, el, psi_star, psi_star + (double)p.x, (double)p.y, &x,
                     &y, &slope)) {
      atomicAdd(&s_cnt[4], 1u);
      reject = true;
      continue;
    }
    if (!(slope >= kWarmSlope)) {
      atomicAdd(&s_cnt[5], 1u);
      reject = true;
      continue;
    }
    if (!el && !thi_is_nearest(m, mode, a.kernel, x, y)) {
      atomicAdd(&s_cnt[6], 1u);
      reject = true;
      continue;
    }
    x = fmod(x, kTwoPi);
    if (x < 0.0) x += kTwoPi;
    const Vel v = energy_velocity(m, mode, a.kernel, x, y);
    Entry e;
    ray_quantities(v, &e);
    e.thR = x;
    e.thI = y;
    const double h = el ? 0.0 : homog_residual(v);
    e.res = fmax(fabs(h), fabs(wrap_pi(ray_angle(v) - psi_star)));
    if (!(e.res <= w.resid_tol) || !(e.V > 0.0) || !isfinite(e.V) || !(e.A >= 0.0)) {
      atomicAdd(&s_cnt[7], 1u);
      reject = true;
      continue;
    }
    store_pair(a, row, col, pcol, e, m.tilt, CHERT_ST_OK);
  }
  if (reject) s_rej[qs] = 1;
  __syncthreads();
  if (work && l == 0) {
    if (s_rej[qs]) {
      atomicAdd(&s_cnt[1], 1u);
      w.fb_list[atomicAdd(w.fb_len, 1)] = (int32_t)job;
    } else if (s_nflag[qs] > 0) {
      w.win_list[atomicAdd(w.win_len, 1)] = (int32_t)job;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < CHERT_WARM_NSTATS; i += blockDim.x)
    if (s_cnt[i]) atomicAdd(&stat_slot(w.shard)[i], (unsigned long long)s_cnt[i]);
}

// Directions near a fold, for the jobs k_warm_solve listed: the plain
// sweep-and-bracket search, evaluated only at the sweep samples the elastic
// map places within kFoldMargin of the target ray angle.  Samples left out
// read as NaN and so never bracket; the search is the plain one wherever the
// viscoelastic map stays within kFoldMargin of the elastic one, which is
// checked on every evaluated sample (half the margin; otherwise, or beyond
// kWinCap samples, the job goes to the plain path).  One wavefront per
// listed job, grid-strided; the marked samples are kept compact in LDS.
constexpr int kWinCap = 512;
// room for fold directions and their brackets, per job on average (more: the
// job is redone by the plain path)
constexpr int64_t kDirsPerJob = 4, kBracketsPerJob = 8;
__global__ void __launch_bounds__(64) k_warm_window(WarmArgs w) {
  extern __shared__ double2 s_ent[];  // [kWinCap] (theta_I, psi); then idx, pos
  int16_t* s_idx = reinterpret_cast<int16_t*>(s_ent + kWinCap);  // [kWinCap]
  __shared__ double s_psi[kProxyN];
  __shared__ uint32_t s_fold[kFoldWords];
  __shared__ uint32_t s_mask[kMaxSweep / 32];
  __shared__ int16_t s_flag[kMaxSubset / 2];
  __shared__ int s_all, s_nflag, s_bad;

  const SolveArgs& a = w.so;
  const int lane = threadIdx.x;
  int16_t* s_pos = s_idx + kWinCap;  // [n_sweep]
  const int n_words = (a.n_sweep + 31) / 32;
  const int n_list = *w.win_len;
  unsigned long long samples = 0, guard = 0;
  for (int q = blockIdx.x; q < n_list; q += gridDim.x) {
    const int64_t job = w.win_list[q];
    const int64_t k = job % a.n_classes;
    const int mode = a.modes[job / a.n_classes];
    const chert_class c = a.classes[k];
    const Medium m = load_medium(c);
    const Medium me = elastic_of(m);
    __syncthreads();  // the previous job is done with the shared arrays
    if (lane < kFoldWords) s_fold[lane] = 0;
    if (lane == 0) {
      s_all = 0;
      s_nflag = 0;
      s_bad = 0;
    }
    for (int i = lane; i < a.n_sweep; i += 64) s_pos[i] = -1;
    for (int i = lane; i < n_words; i += 64) s_mask[i] = 0u;
    __syncthreads();
    proxy_folds(me, mode, a.kernel, true, lane, 64, s_psi, s_fold, &s_all);
    for (int sidx = lane; sidx < a.n_solve; sidx += 64) {
      int d, col, pcol;
      dir_cols(a, sidx, &d, &col, &pcol);
      const int fb = fold_bin(dir_psi(a, d, m.tilt));
      if ((s_fold[fb >> 5] >> (fb & 31)) & 1u) s_flag[atomicAdd(&s_nflag, 1)] = (int16_t)sidx;
    }
    __syncthreads();
    const int nflag = s_nflag;
    for (int f = 0; f < nflag; ++f) {
      int d, col, pcol;
      dir_cols(a, s_flag[f], &d, &col, &pcol);
      mark_window(a, s_psi, dir_psi(a, d, m.tilt), s_mask);
    }
    __syncthreads();
    // marked samples in ascending order: one mask word per lane, prefix sum
    // of the word populations across the wavefront
    int nl = 0;
    for (int base = 0; base < n_words; base += 64) {
      const int wd = base + lane;
      uint32_t bits = wd < n_words ? s_mask[wd] : 0u;
      const int cnt = __popc(bits);
      int incl = cnt;
      for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
      }
      int slot = nl + incl - cnt;
      while (bits) {
        const int b = __builtin_ctz(bits);
        bits &= bits - 1u;
        if (slot < kWinCap) {
          s_idx[slot] = (int16_t)(wd * 32 + b);
          s_pos[wd * 32 + b] = (int16_t)slot;
        }
        ++slot;
      }
      nl += __shfl(incl, 63);
    }
    if (nl > kWinCap) {  // wavefront-uniform
      if (lane == 0) {
        ++guard;
        w.fb_list[atomicAdd(w.fb_len, 1)] = (int32_t)job;
      }
      continue;
    }
    __syncthreads();
    for (int t = lane; t < nl; t += 64) {
      const int i = s_idx[t];
      const double thR = (i + 0.5) * (kTwoPi / a.n_sweep);
      double thI, sr, cr;
      sincos(thR, &sr, &cr);
      double2 out = make_double2(0.0, NAN);
      if (theta_imag_sc(m, mode, a.kernel, sr, cr, &thI)) {
        const double psi = ray_angle_sc(m, mode, a.kernel, sr, cr, thI);
        if (isfinite(psi)) out = make_double2(thI, psi);
        const double pe = ray_angle(energy_velocity_t(me, mode, a.kernel, Trig{sr, cr, 0.0, 1.0}));
        if (!(fabs(wrap_pi(psi - pe)) <= 0.5 * kFoldMargin)) s_bad = 1;
      }
      s_ent[t] = out;
    }
    samples += (unsigned long long)nl;
    __syncthreads();
    if (!s_bad) {
      // every bracket of every fold direction goes to the flat refinement
      // (k_warm_fold): one record per direction, its brackets contiguous in
      // scan order.  All lanes scan the table for one direction at a time.
      const WindowTable tab{s_pos, s_ent, s_idx, nl};
      for (int f = 0; f < nflag; ++f) {
        int d, col, pcol;
        const int sidx = s_flag[f];
        dir_cols(a, sidx, &d, &col, &pcol);
        const double psi_star = dir_psi(a, d, m.tilt);
        int nbr = 0;
        for (int base = 0; base < nl; base += 64)
          nbr += __popcll(__ballot(base + lane < nl &&
                                   is_bracket(tab, s_idx[base + lane], a.n_sweep, psi_star)));
        int rec = 0, first = 0;
        if (lane == 0) {
          rec = atomicAdd(w.dir_len, 1);
          first = atomicAdd(w.br_len, nbr);
        }
        rec = __shfl(rec, 0);
        first = __shfl(first, 0);
        if (rec >= w.dir_cap || (int64_t)first + nbr > w.br_cap) {
          if (lane == 0 && rec < w.dir_cap) w.dirs[rec] = make_int4(-1, 0, 0, 0);
          s_bad = 1;  // no room: the job is redone below
          break;      // wavefront-uniform
        }
        int q = first;
        for (int base = 0; base < nl; base += 64) {
          const bool br = base + lane < nl &&
                          is_bracket(tab, s_idx[base + lane], a.n_sweep, psi_star);
          const unsigned long long mask = __ballot(br);
          if (br) {
            const int jj = s_idx[base + lane];
            WinBracket b;
            b.sa = tab.at(jj);
            b.sb = tab.at(jj + 1 == a.n_sweep ? 0 : jj + 1);
            b.j = jj;
            w.brs[q + __popcll(mask & ((1ull << lane) - 1ull))] = b;
          }
          q += __popcll(mask);
        }
        if (lane == 0) w.dirs[rec] = make_int4((int)job, sidx, first, nbr);
      }
      __syncthreads();
    }
    if (s_bad && lane == 0) {  // guard failed or no room: the plain path redoes the job
      ++guard;
      w.fb_list[atomicAdd(w.fb_len, 1)] = (int32_t)job;
    }
  }
  if (lane == 0 && samples) atomicAdd(&stat_slot(w.shard)[8], samples);
  if (lane == 0 && guard) {
    atomicAdd(&stat_slot(w.shard)[9], guard);
    atomicAdd(&stat_slot(w.shard)[1], guard);
  }
}

// Fold directions across all window jobs, one lane each: refine the
// direction's brackets in scan order and keep the plain search's choice
// (the fold of refine_bracket), then store the entry and its copy.
__global__ void __launch_bounds__(64) k_warm_fold(WarmArgs w) {
  const SolveArgs& a = w.so;
  const int64_t n = *w.dir_len < w.dir_cap ? *w.dir_len : w.dir_cap;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int4 r = w.dirs[t];
    if (r.x < 0) continue;
    const int64_t job = r.x;
    const int64_t k = job % a.n_classes;
    const int mode = a.modes[job / a.n_classes];
    const chert_class c = a.classes[k];
    const int64_t row = ((int64_t)mode * a.n_classes + k) * a.n_cols;
    const Medium m = load_medium(c);
    const bool el = theta_i_zero(m, mode);
    int d, col, pcol;
    dir_cols(a, r.y, &d, &col, &pcol);
    const double psi_star = dir_psi(a, d, m.tilt);
    bool found = false, ill = false;
    Entry best{};
    for (int b = 0; b < r.w; ++b) {
      const WinBracket br = w.brs[r.z + b];
      refine_bracket_at(a, m, mode, br.j, br.sa, br.sb, psi_star, el, &found, &ill, &best);
    }
    store_pair(a, row, col, pcol, best, m.tilt, solve_status(found, ill, best));
  }
}

// ------------------------------------------- slowness-sampled caches
// Column s of (mode, class): the homogeneous solution at real slowness
// angle theta_R = s 2 pi / n_cols in the class's symmetry-axis frame (eq 26
// with the slowness angle as index): theta_I is the homogeneity root
// nearest 0 (eq 9), the ray quantities follow (eqs 10-11) and the ray
// direction is rotated to the global frame; RES is |h|.  One lane per
// (mode, class, column).
__global__ void __launch_bounds__(256) k_build_slow(SolveArgs a) {
  const int64_t total = (int64_t)a.n_modes * a.n_classes * a.n_cols;
  const int64_t stride = 3 * a.n_classes * (int64_t)a.n_cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(t % a.n_cols);
    const int64_t job = t / a.n_cols;
    const int64_t k = job % a.n_classes;
    const int mode = a.modes[job / a.n_classes];
    const chert_class c = a.classes[k];
    const int64_t idx = ((int64_t)mode * a.n_classes + k) * a.n_cols + q;
    const int32_t blocked = class_block(c, mode);
    if (blocked) {
      store_invalid(a, idx, stride, blocked);
      continue;
    }
    const Medium m = load_medium(c);
    const double thR = q * (kTwoPi / a.n_cols);
    double sr, cr, thI;
    sincos(thR, &sr, &cr);
    if (!theta_imag_sc(m, mode, a.kernel, sr, cr, &thI)) {
      store_invalid(a, idx, stride, CHERT_ST_NO_BRACKET);
      continue;
    }
    const Vel v = energy_velocity(m, mode, a.kernel, thR, thI);
    Entry e;
    ray_quantities(v, &e);
    e.thR = thR;
    e.thI = thI;
    e.res = theta_i_zero(m, mode) ? 0.0 : fabs(homog_residual(v));
    int32_t st = CHERT_ST_OK;
    if (!(e.A >= 0.0) || !isfinite(e.V) || !(e.V > 0.0)) st |= CHERT_ST_NONPHYS;
    if (!(e.res <= a.resid_tol)) st |= CHERT_ST_NOCONV;
    store_entry(a, idx, stride, e, m.tilt, st);
  }
}

// ------------------------------------------------------- 3D warm start
// Surrogate-started 3D caches: every (mode, class, Fibonacci direction) is
// polished on its own from its prediction (one lane each) under the same
// acceptance checks as in 2D; directions near a fold of the elastic map, or
// failing a check, are solved by the plain sweep-and-bracket search from
// their (mode, class) sweep table.  Jobs are (mode, class) pairs.
struct Warm3Args {
  SolveArgs so;                 // dim 3: n_solve = n_cols = n_dirs
  const void* blob;
  float2* pred;                 // [jobs][n_dirs] (theta_R - psi, theta_I)
  uint32_t* fold;               // [jobs][kFoldWords] fold bins of the elastic map
  int32_t* fb_list;             // job * n_dirs + direction, for the plain search
  int32_t* fb_len;
  unsigned long long* stats;    // CHERT_WARM_NSTATS counters (folded from shard)
  unsigned long long* shard;    // [kStatSlots][16] per-slot partial counters
  double resid_tol;
};

// target polar angle of direction s to the class's symmetry axis (eq 35)
__device__ __forceinline__ double warm3_target(const SolveArgs& a, int s, const chert_class& c) {
  return polar_to_axis(fib_dir(a, s), c);
}

__global__ void __launch_bounds__(mlp::kThreads) k_warm3_predict(Warm3Args w, int64_t n_rows) {
  __shared__ mlp::InferTile t;
  const SolveArgs& a = w.so;
  const mlp::Net n = mlp::net_of(w.blob);
  const int64_t base = (int64_t)blockIdx.x * mlp::kInferRows;
  for (int r = threadIdx.x; r < mlp::kInferRows; r += blockDim.x) {
    const int64_t e = base + r;
    float f[mlp::kIn] = {};
    if (e < n_rows) {
      const int64_t job = e / a.n_solve;
      const int s = (int)(e % a.n_solve);
      const chert_class c = a.classes[job % a.n_classes];
      mlp::features(c, a.modes[job / a.n_classes], warm3_target(a, s, c), f);
    }
    mlp::stage_row(n, t.x, r, f, e >= n_rows);
  }
  __syncthreads();
  mlp::forward_infer(n, t, [&](int r, int col, float v) {
    if (col < 2 && base + r < n_rows) (&w.pred[base + r].x)[col] = v;
  });
}

// fold bins of each job's elastic ray-angle map (all bins if the map is not
// finite everywhere); one wavefront per job
__global__ void __launch_bounds__(64) k_warm3_folds(Warm3Args w) {
  __shared__ double s_psi[kProxyN];
  __shared__ uint32_t s_fold[kFoldWords];
  __shared__ int s_all;
  const SolveArgs& a = w.so;
  const int64_t job = blockIdx.x;
  const chert_class c = a.classes[job % a.n_classes];
  const int mode = a.modes[job / a.n_classes];
  if (threadIdx.x < kFoldWords) s_fold[threadIdx.x] = 0u;
  if (threadIdx.x == 0) s_all = 0;
  __syncthreads();
  proxy_folds(elastic_of(load_medium(c)), mode, a.kernel, !class_block(c, mode), threadIdx.x, 64,
              s_psi, s_fold, &s_all);
  __syncthreads();
  if (threadIdx.x < kFoldWords)
    w.fold[job * kFoldWords + threadIdx.x] = s_all ? ~0u : s_fold[threadIdx.x];
  if (threadIdx.x == 0) atomicAdd(&stat_slot(w.shard)[0], 1ull);
}

// one lane per (job, direction): Newton polish from the prediction and the
// checks of k_warm_solve; the rest go to the plain-search list
__global__ void __launch_bounds__(64) k_warm3_solve(Warm3Args w, int64_t n_rows) {
  const SolveArgs& a = w.so;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long cnt[CHERT_WARM_NSTATS] = {};
  if (e < n_rows) {
    const int64_t job = e / a.n_solve;
    const int s = (int)(e % a.n_solve);
    const int64_t k = job % a.n_classes;
    const int mode = a.modes[job / a.n_classes];
    const chert_class c = a.classes[k];
    const int64_t idx = ((int64_t)mode * a.n_classes + k) * a.n_cols + s;
    const int64_t stride = 3 * a.n_classes * (int64_t)a.n_cols;
    const double3 f = fib_dir(a, s);
    const int32_t blocked = class_block(c, mode);
    cnt[2] = 1;
    bool plain = false;
    if (blocked) {
      Entry none{};
      none.V = NAN;
      store_single(a, idx, stride, none, f, blocked);
    } else {
      const Medium m = load_medium(c);
      const bool el = theta_i_zero(m, mode);
      const double psi_star = polar_to_axis(f, c);
      const int fb = fold_bin(psi_star);
      double x, y, slope;
      const float2 p = w.pred[e];
      if ((w.fold[job * kFoldWords + (fb >> 5)] >> (fb & 31)) & 1u) {
        cnt[3] = 1;
        plain = true;
      } else if (!warm_newton(m, mode, a.kernel, el, psi_star, psi_star + (double)p.x,
                              (double)p.y, &x, &y, &slope)) {
        cnt[4] = 1;
        plain = true;
      } else if (!(slope >= kWarmSlope)) {
        cnt[5] = 1;
        plain = true;
      } else if (!el && !thi_is_nearest(m, mode, a.kernel, x, y)) {
        cnt[6] = 1;
        plain = true;
      } else {
        x = fmod(x, kTwoPi);
        if (x < 0.0) x += kTwoPi;
        const Vel v = energy_velocity(m, mode, a.kernel, x, y);
        Entry en;
        ray_quantities(v, &en);
        en.thR = x;
        en.thI = y;
        const double h = el ? 0.0 : homog_residual(v);
        en.res = fmax(fabs(h), fabs(wrap_pi(ray_angle(v) - psi_star)));
        if (!(en.res <= w.resid_tol) || !(en.V > 0.0) || !isfinite(en.V) || !(en.A >= 0.0)) {
          cnt[7] = 1;
          plain = true;
        } else {
          store_single(a, idx, stride, en, f, CHERT_ST_OK);
        }
      }
      if (plain) {
        cnt[1] = 1;
        w.fb_list[atomicAdd(w.fb_len, 1)] = (int32_t)e;
      }
    }
  }
  for (int q = 1; q < 8; ++q) {
    unsigned long long v = cnt[q];
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    if (__lane_id() == 0 && v) atomicAdd(&stat_slot(w.shard)[q], v);
  }
}

// the plain sweep-and-bracket search for the listed directions, one lane
// each, from the job's sweep table (read through the caches); grid-strided
__global__ void __launch_bounds__(64) k_warm3_plain(Warm3Args w) {
  __shared__ int s_br[64 * kMaxBr];
  const SolveArgs& a = w.so;
  const int n = *w.fb_len;
  for (int64_t q0 = (int64_t)blockIdx.x * blockDim.x; q0 < n; q0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = q0 + threadIdx.x;
    if (q >= n) continue;
    const int64_t e = w.fb_list[q];
    const int64_t job = e / a.n_solve;
    const int s = (int)(e % a.n_solve);
    const int64_t k = job % a.n_classes;
    const int mode = a.modes[job / a.n_classes];
    const chert_class c = a.classes[k];
    const Medium m = load_medium(c);
    const double3 f = fib_dir(a, s);
    Entry best{};
    const int32_t st = solve_dir(a, m, mode, FullTable{a.table + job * a.n_sweep, a.n_sweep},
                                 polar_to_axis(f, c), s_br + threadIdx.x * kMaxBr, &best);
    store_single(a, ((int64_t)mode * a.n_classes + k) * a.n_cols + s,
                 3 * a.n_classes * (int64_t)a.n_cols, best, f, st);
  }
}

__global__ void k_warm_zero(int32_t* fb_len, int32_t* win_len, unsigned long long* shard) {
  if (threadIdx.x == 0) *fb_len = 0;
  if (threadIdx.x == 1) *win_len = 0;
  if (threadIdx.x == 2) win_len[1] = 0;  // fold directions
  if (threadIdx.x == 3) win_len[2] = 0;  // their brackets
  for (int i = threadIdx.x; i < kStatSlots * kStatSlotU64; i += blockDim.x) shard[i] = 0ull;
}

// the build's counters: the sums of their per-slot partials (the kernels
// add into the slot of their workgroup, not into one address)
__global__ void k_warm_stats_fold(const unsigned long long* shard, unsigned long long* stats) {
  const int i = threadIdx.x;
  if (i >= CHERT_WARM_NSTATS) return;
  unsigned long long v = 0;
  for (int q = 0; q < kStatSlots; ++q) v += shard[(size_t)q * kStatSlotU64 + i];
  stats[i] = v;
}

__global__ void k_write_header(uint8_t* cache, int32_t dim, int32_t n_dirs, uint32_t mask,
                               int32_t kernel, int32_t n_sweep, int32_t n_subset,
                               int64_t n_classes, int32_t sampling) {
  int t = threadIdx.x;
  uint32_t* w = reinterpret_cast<uint32_t*>(cache);
  if (t < 64) w[t] = 0u;
  __syncthreads();
  if (t == 0) {
    w[0] = kCacheMagic;
    w[1] = kCacheVersion;
    w[2] = (uint32_t)dim;
    w[3] = (uint32_t)n_dirs;
    w[4] = mask;
    w[5] = (uint32_t)kernel;
    w[6] = (uint32_t)n_sweep;
    w[7] = (uint32_t)n_subset;
    *reinterpret_cast<int64_t*>(cache + 32) = n_classes;
    w[10] = (uint32_t)sampling;
  }
}

__global__ void k_cache_stats_zero(chert_cache_stats* st) {
  if (threadIdx.x == 0) *st = chert_cache_stats{};
}

__device__ __forceinline__ long long wave_sum(long long v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}
__device__ __forceinline__ unsigned long long wave_max(unsigned long long v) {
  for (int d = 32; d >= 1; d >>= 1) {
    const unsigned long long o = __shfl_xor(v, d);
    v = o > v ? o : v;
  }
  return v;
}

// Counters of a built cache (chert_cache_stats) from its status and residual
// arrays, over the modes of the mask; fb_len (nullable) is the number of
// items the surrogate-started build re-solved with the plain solver, each
// holding fb_entries stored entries (a 2D job, or one 3D direction).
__global__ void __launch_bounds__(256) k_cache_stats(const int32_t* status, const double* res,
                                                     int64_t per_mode, uint32_t mask,
                                                     const int32_t* fb_len, int64_t fb_entries,
                                                     chert_cache_stats* st) {
  long long n = 0, conv = 0, noconv = 0, ill = 0, nob = 0, unus = 0;
  unsigned long long mr = 0ull;  // non-negative doubles order as their bits
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int m = 0; m < 3; ++m) {
    if (!(mask & (1u << m))) continue;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < per_mode; t += stride) {
      const int64_t e = m * per_mode + t;
      const int32_t sv = status[e];
      ++n;
      if ((sv & ~CHERT_ST_ILL) == 0) ++conv;
      if (sv & CHERT_ST_NOCONV) ++noconv;
      if (sv & CHERT_ST_ILL) ++ill;
      if (sv & CHERT_ST_NO_BRACKET) ++nob;
      if (sv & (CHERT_ST_FLUID | CHERT_ST_NONPHYS)) ++unus;
      if (!(sv & (CHERT_ST_NO_BRACKET | CHERT_ST_FLUID))) {
        const double r = fabs(res[e]);
        if (r >= 0.0) {  // not NaN
          const unsigned long long b = (unsigned long long)__double_as_longlong(r);
          mr = b > mr ? b : mr;
        }
      }
    }
  }
  n = wave_sum(n);
  conv = wave_sum(conv);
  noconv = wave_sum(noconv);
  ill = wave_sum(ill);
  nob = wave_sum(nob);
  unus = wave_sum(unus);
  mr = wave_max(mr);
  // one set of atomics per workgroup (each counter is one address)
  __shared__ unsigned long long s_v[4][7];
  const int wv = threadIdx.x >> 6;
  if (__lane_id() == 0) {
    s_v[wv][0] = n;
    s_v[wv][1] = conv;
    s_v[wv][2] = noconv;
    s_v[wv][3] = ill;
    s_v[wv][4] = nob;
    s_v[wv][5] = unus;
    s_v[wv][6] = mr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w2 = 1; w2 < (int)(blockDim.x >> 6); ++w2) {
      for (int i = 0; i < 6; ++i) s_v[0][i] += s_v[w2][i];
      s_v[0][6] = s_v[w2][6] > s_v[0][6] ? s_v[w2][6] : s_v[0][6];
    }
    atomicAdd((unsigned long long*)&st->n_entries, s_v[0][0]);
    atomicAdd((unsigned long long*)&st->n_converged, s_v[0][1]);
    atomicAdd((unsigned long long*)&st->n_noconv, s_v[0][2]);
    atomicAdd((unsigned long long*)&st->n_illcond, s_v[0][3]);
    atomicAdd((unsigned long long*)&st->n_nobracket, s_v[0][4]);
    atomicAdd((unsigned long long*)&st->n_unusable, s_v[0][5]);
    atomicMax((unsigned long long*)&st->max_resid, s_v[0][6]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    st->n_fallback = fb_len ? (int64_t)*fb_len * fb_entries : 0;
}

// Enqueue the counters of a build into d->stats_dev (if set).
static void enqueue_cache_stats(const chert_cache_desc* d, int64_t n_classes, uint8_t* cache,
                                const chert_cache_layout& lay, const int32_t* fb_len,
                                int64_t fb_entries, hipStream_t s) {
  if (!d->stats_dev) return;
  const int n_cols = d->n_subset ? d->n_subset : d->n_dirs;
  const int64_t per_mode = n_classes * (int64_t)n_cols;
  const int32_t* status = (const int32_t*)(cache + lay.status_offset);
  const double* res = (const double*)(cache + lay.fields_offset) + CHERT_F_RES * 3 * per_mode;
  int64_t blocks = (per_mode + 255) / 256;
  if (blocks > 512) blocks = 512;
  CHERT_LAUNCH("k_cache_stats_zero", k_cache_stats_zero, dim3(1), dim3(64), 0, s, d->stats_dev);
  CHERT_LAUNCH("k_cache_stats", k_cache_stats, dim3((unsigned)blocks), dim3(256), 0, s, status,
               res, per_mode, d->mode_mask, fb_len, fb_entries, d->stats_dev);
}

}  // namespace chert

using namespace chert;

// Jobs (mode x class) at or above this count use the fused one-launch path.
constexpr int64_t kFusedJobs = 512;

static int64_t n_jobs_of(const chert_cache_desc* d, int64_t n_classes) {
  return (int64_t)__builtin_popcount(d->mode_mask & 7u) * n_classes;
}

// Solve arguments of a build (desc already validated): modes, columns, the
// solved directions and the columns of their centrosymmetric copies.
static SolveArgs solve_args(const chert_cache_desc* d, const chert_class* classes_dev,
                            int64_t n_classes, uint8_t* cache, const chert_cache_layout& lay,
                            const void* table) {
  SolveArgs so{};
  for (int m = 0; m < 3; ++m)
    if (d->mode_mask & (1u << m)) so.modes[so.n_modes++] = m;
  so.classes = classes_dev;
  so.n_classes = n_classes;
  so.kernel = d->kernel;
  so.n_sweep = d->n_sweep;
  so.n_dirs = d->n_dirs;
  so.table = (const double2*)table;
  so.fields = cache ? (double*)(cache + lay.fields_offset) : nullptr;
  so.status = cache ? (int32_t*)(cache + lay.status_offset) : nullptr;
  const int half = d->n_dirs / 2;
  so.dim = d->dim;
  so.fib_ga = M_PI * (3.0 - sqrt(5.0));
  so.resid_tol = d->resid_tol > 0.0 ? d->resid_tol : 1e-9;
  so.newton_iters = d->max_iter > 0 ? d->max_iter : 12;
  so.bisect_iters = d->max_iter > 0 ? d->max_iter : 200;
  if (d->dim == 3) {
    so.subset = 0;
    so.n_cols = d->n_dirs;
    so.n_solve = d->n_dirs;
  } else if (d->n_subset == 0) {
    so.subset = 0;
    so.n_cols = d->n_dirs;
    so.n_solve = half;
  } else {
    so.subset = 1;
    so.n_cols = d->n_subset;
    so.n_solve = 0;
    for (int i = 0; i < d->n_subset; ++i) {
      const int b = d->subset_host[i];
      if (b >= half) continue;
      int p = 0;
      while (d->subset_host[p] != b + half) ++p;  // present: validated
      so.dir[so.n_solve] = (int16_t)b;
      so.col[so.n_solve] = (int16_t)i;
      so.pcol[so.n_solve] = (int16_t)p;
      ++so.n_solve;
    }
  }
  return so;
}

static int common_checks(const chert_cache_desc* d, const chert_class* classes_dev,
                         int64_t n_classes, const void* cache_dev, chert_cache_layout* lay) {
  int rc = chert_cache_layout_of(d, n_classes, lay);
  if (rc != CHERT_OK) return rc;
  if (!classes_dev || !cache_dev) return fail(CHERT_ERR_INVALID_ARG, "null classes or cache");
  if (d->n_sweep > kMaxSweep)
    return fail(CHERT_ERR_INVALID_ARG, "n_sweep above the LDS table limit");
  if (n_jobs_of(d, n_classes) > 0x7fffffffLL)
    return fail(CHERT_ERR_INVALID_ARG, "too many classes");
  return CHERT_OK;
}

static int launch_status() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  return CHERT_OK;
}

extern "C" size_t chert_build_cache_workspace_bytes(const chert_cache_desc* d,
                                                    int64_t n_classes) {
  if (!d || n_classes <= 0 || d->n_sweep <= 0) return 0;
  if (d->sampling == CHERT_SAMPLE_SLOWNESS) return 0;                     // no sweep table
  if (d->dim != 3 && n_jobs_of(d, n_classes) >= kFusedJobs) return 0;  // table stays in LDS
  return (size_t)n_jobs_of(d, n_classes) * (size_t)d->n_sweep * sizeof(double2);
}

static int build_cache(const chert_cache_desc* d, const chert_class* classes_dev,
                       int64_t n_classes, void* cache_dev, void* workspace_dev,
                       size_t workspace_bytes, void* stream);

extern "C" int chert_build_cache(const chert_cache_desc* d, const chert_class* classes_dev,
                                 int64_t n_classes, void* cache_dev, void* workspace_dev,
                                 size_t workspace_bytes, void* stream) {
  return build_cache(d, classes_dev, n_classes, cache_dev, workspace_dev, workspace_bytes, stream);
}

// ---------------------------------------------------- allocation-free build
// Scratch of chert_build_cache_noalloc: the theta_R sweep tables live in this
// file-scope device array (one copy per GPU, held until the process ends).
// Host code never passes the array's name to a kernel: it is a host-side
// stand-in; the device address comes from hipGetSymbolAddress, once per
// device.
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of this device's scratch array (resolved on first use).
static int scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(CHERT_ERR_UNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(CHERT_ERR_HIP, e != hipSuccess ? hipGetErrorString(e)
                                                 : "no device address for the build scratch");
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CHERT_OK;
}

extern "C" size_t chert_build_cache_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

extern "C" int chert_build_cache_noalloc(const chert_cache_desc* d,
                                         const chert_class* classes_dev, int64_t n_classes,
                                         void* cache_dev, void* stream) {
  chert_cache_layout lay;
  int rc = common_checks(d, classes_dev, n_classes, cache_dev, &lay);
  if (rc != CHERT_OK) return rc;
  const size_t need = chert_build_cache_workspace_bytes(d, n_classes);
  if (need > kNoAllocScratchBytes)
    return fail(CHERT_ERR_CAPACITY,
                "sweep tables exceed the 16 MiB build scratch (use chert_build_cache)");
  void* ws = nullptr;
  if (need > 0) {
    rc = scratch_of_current_device(&ws);
    if (rc != CHERT_OK) return rc;
  }
  return build_cache(d, classes_dev, n_classes, cache_dev, ws, need > 0 ? kNoAllocScratchBytes : 0,
                     stream);
}

static int build_cache(const chert_cache_desc* d, const chert_class* classes_dev,
                       int64_t n_classes, void* cache_dev, void* workspace_dev,
                       size_t workspace_bytes, void* stream) {
  chert_cache_layout lay;
  int rc = common_checks(d, classes_dev, n_classes, cache_dev, &lay);
  if (rc != CHERT_OK) return rc;
  const size_t need = chert_build_cache_workspace_bytes(d, n_classes);
  if (need > 0 && (!workspace_dev || workspace_bytes < need))
    return fail(CHERT_ERR_INVALID_ARG, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* cache = (uint8_t*)cache_dev;
  const SolveArgs so = solve_args(d, classes_dev, n_classes, cache, lay, workspace_dev);

  CHERT_LAUNCH("k_write_header", k_write_header, dim3(1), dim3(64), 0, s, cache, d->dim,
               d->n_dirs, d->mode_mask, d->kernel, d->n_sweep, d->n_subset, n_classes,
                 d->sampling);
  const int64_t jobs = (int64_t)so.n_modes * n_classes;
  if (d->sampling == CHERT_SAMPLE_SLOWNESS) {
    const int64_t total = jobs * so.n_cols;
    const int64_t blocks = (total + 255) / 256 > 65536 ? 65536 : (total + 255) / 256;
    if (total > 0)
      CHERT_LAUNCH("k_build_slow", k_build_slow, dim3((unsigned)blocks), dim3(256), 0, s, so);
  } else if (jobs >= kFusedJobs && d->dim != 3) {
    CHERT_LAUNCH("k_build_fused", k_build_fused, dim3((unsigned)jobs), dim3(kNodeThreads),
                 (size_t)d->n_sweep * sizeof(double2), s, so, (const int32_t*)nullptr,
                 (const int32_t*)nullptr, jobs);
  } else if (jobs > 0) {
    SweepArgs sa{};
    sa.classes = classes_dev;
    sa.n_classes = n_classes;
    sa.n_modes = so.n_modes;
    for (int i = 0; i < 3; ++i) sa.modes[i] = so.modes[i];
    sa.kernel = d->kernel;
    sa.n_sweep = d->n_sweep;
    sa.table = (double2*)workspace_dev;
    int64_t total = jobs * d->n_sweep;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    CHERT_LAUNCH("k_sweep", k_sweep, dim3((unsigned)blocks), dim3(256), 0, s, sa);
    // few directions (latency bound): 4 lanes share each direction's scan
    const bool split = jobs * ((so.n_solve + 63) / 64) < 1024;
    const int per_wg = split ? 16 : 64;
    const int64_t chunks = (so.n_solve + per_wg - 1) / per_wg;
    if (jobs * chunks > 0x7fffffffLL) return fail(CHERT_ERR_INVALID_ARG, "too many entries");
    if (split)
      CHERT_LAUNCH("k_solve", k_solve<4>, dim3((unsigned)(jobs * chunks)), dim3(64),
                   (size_t)d->n_sweep * sizeof(double2), s, so);
    else
      CHERT_LAUNCH("k_solve", k_solve<1>, dim3((unsigned)(jobs * chunks)), dim3(64),
                   (size_t)d->n_sweep * sizeof(double2), s, so);
  }
  enqueue_cache_stats(d, n_classes, cache, lay, nullptr, 0, s);
  return launch_status();
}

// workspace of the surrogate-started build: predictions, the fallback and
// fold-window job lists, their lengths and the internal counters
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// workspace of the 3D surrogate-started build: sweep tables, predictions,
// fold bins, the plain-search list, its length and the counters
static size_t warm3_bytes(const chert_cache_desc* d, int64_t n_classes) {
  const size_t jobs = (size_t)n_jobs_of(d, n_classes);
  const size_t rows = jobs * (size_t)d->n_dirs;
  return al256(jobs * d->n_sweep * sizeof(double2)) + al256(rows * sizeof(float2)) +
         al256(jobs * kFoldWords * sizeof(uint32_t)) + al256(rows * sizeof(int32_t)) + 256 +
         al256(kStatBytes);
}

extern "C" size_t chert_build_cache_surrogate_workspace_bytes(const chert_cache_desc* d,
                                                              int64_t n_classes) {
  chert_cache_layout lay;
  if (!d || n_classes <= 0 || chert_cache_layout_of(d, n_classes, &lay) != CHERT_OK) return 0;
  if (d->dim == 3) return warm3_bytes(d, n_classes);
  const SolveArgs so = solve_args(d, nullptr, n_classes, nullptr, lay, nullptr);
  const size_t jobs = (size_t)n_jobs_of(d, n_classes);
  return al256(jobs * so.n_solve * sizeof(float2)) + 2 * al256(jobs * sizeof(int32_t)) + 256 +
         al256(jobs * kDirsPerJob * sizeof(int4)) + al256(jobs * kBracketsPerJob * sizeof(WinBracket)) +
         al256(kStatBytes);
}

extern "C" int chert_build_cache_surrogate(const chert_cache_desc* d,
                                           const chert_class* classes_dev, int64_t n_classes,
                                           const void* blob_dev, double resid_tol,
                                           void* cache_dev, int64_t* stats_dev,
                                           void* workspace_dev, size_t workspace_bytes,
                                           void* stream) {
  chert_cache_layout lay;
  int rc = common_checks(d, classes_dev, n_classes, cache_dev, &lay);
  if (rc != CHERT_OK) return rc;
  if (d->sampling != CHERT_SAMPLE_RAY)
    return fail(CHERT_ERR_UNSUPPORTED, "surrogate-started builds fill ray-direction caches");
  if (!blob_dev || ((uintptr_t)blob_dev & 255u))
    return fail(CHERT_ERR_INVALID_ARG, "null or unaligned surrogate blob");
  if (!(resid_tol >= 0.0)) return fail(CHERT_ERR_INVALID_ARG, "negative residual tolerance");
  const size_t need = chert_build_cache_surrogate_workspace_bytes(d, n_classes);
  if (!workspace_dev || workspace_bytes < need)
    return fail(CHERT_ERR_INVALID_ARG, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* cache = (uint8_t*)cache_dev;
  if (d->dim == 3) {
    const int64_t jobs = n_jobs_of(d, n_classes);
    const int64_t rows = jobs * (int64_t)d->n_dirs;
    if (rows > 0x7fffffffLL) return fail(CHERT_ERR_INVALID_ARG, "too many entries");
    uint8_t* ws = (uint8_t*)workspace_dev;
    Warm3Args w{};
    double2* table = (double2*)ws;
    ws += al256((size_t)jobs * d->n_sweep * sizeof(double2));
    w.so = solve_args(d, classes_dev, n_classes, cache, lay, table);
    w.blob = blob_dev;
    w.pred = (float2*)ws;
    ws += al256((size_t)rows * sizeof(float2));
    w.fold = (uint32_t*)ws;
    ws += al256((size_t)jobs * kFoldWords * sizeof(uint32_t));
    w.fb_list = (int32_t*)ws;
    ws += al256((size_t)rows * sizeof(int32_t));
    w.fb_len = (int32_t*)ws;
    w.stats = stats_dev ? (unsigned long long*)stats_dev : (unsigned long long*)(ws + 64);
    w.shard = (unsigned long long*)(ws + 256);
    w.resid_tol = resid_tol > 0.0 ? resid_tol : 1e-11;
    CHERT_LAUNCH("k_write_header", k_write_header, dim3(1), dim3(64), 0, s, cache, d->dim,
                 d->n_dirs, d->mode_mask, d->kernel, d->n_sweep, d->n_subset, n_classes,
                 d->sampling);
    CHERT_LAUNCH("k_warm_zero", k_warm_zero, dim3(1), dim3(256), 0, s, w.fb_len, w.fb_len + 1,
                 w.shard);
    if (rows > 0) {
      SweepArgs sa{};
      sa.classes = classes_dev;
      sa.n_classes = n_classes;
      sa.n_modes = w.so.n_modes;
      for (int i = 0; i < 3; ++i) sa.modes[i] = w.so.modes[i];
      sa.kernel = d->kernel;
      sa.n_sweep = d->n_sweep;
      sa.table = table;
      const int64_t total = jobs * d->n_sweep;
      const int64_t sb = (total + 255) / 256 > 65536 ? 65536 : (total + 255) / 256;
      CHERT_LAUNCH("k_sweep", k_sweep, dim3((unsigned)sb), dim3(256), 0, s, sa);
      CHERT_LAUNCH("k_warm3_folds", k_warm3_folds, dim3((unsigned)jobs), dim3(64), 0, s, w);
      CHERT_LAUNCH("k_warm3_predict", k_warm3_predict,
                   dim3((unsigned)((rows + mlp::kInferRows - 1) / mlp::kInferRows)),
                   dim3(mlp::kThreads), 0, s, w, rows);
      CHERT_LAUNCH("k_warm3_solve", k_warm3_solve, dim3((unsigned)((rows + 63) / 64)), dim3(64), 0,
                   s, w, rows);
      const int64_t pg = (rows + 63) / 64 < 8192 ? (rows + 63) / 64 : 8192;
      CHERT_LAUNCH("k_warm3_plain", k_warm3_plain, dim3((unsigned)pg), dim3(64), 0, s, w);
    }
    CHERT_LAUNCH("k_warm_stats_fold", k_warm_stats_fold, dim3(1), dim3(64), 0, s,
                 (const unsigned long long*)w.shard, w.stats);
    enqueue_cache_stats(d, n_classes, cache, lay, w.fb_len, 1, s);  // listed: directions
    return launch_status();
  }
  WarmArgs w{};
  w.so = solve_args(d, classes_dev, n_classes, cache, lay, nullptr);
  if (w.so.n_solve > kMaxSubset / 2)
    return fail(CHERT_ERR_UNSUPPORTED, "surrogate-started builds take at most 512 directions");
  const int64_t jobs = (int64_t)w.so.n_modes * n_classes;
  const int64_t rows = jobs * w.so.n_solve;
  uint8_t* ws = (uint8_t*)workspace_dev;
  w.blob = blob_dev;
  w.pred = (float2*)ws;
  w.fb_list = (int32_t*)(ws + al256(rows * sizeof(float2)));
  w.win_list = (int32_t*)(ws + al256(rows * sizeof(float2)) + al256(jobs * sizeof(int32_t)));
  w.fb_len = (int32_t*)(ws + al256(rows * sizeof(float2)) + 2 * al256(jobs * sizeof(int32_t)));
  w.win_len = w.fb_len + 1;
  w.dir_len = w.fb_len + 2;
  w.br_len = w.fb_len + 3;
  {
    uint8_t* tail = ws + al256(rows * sizeof(float2)) + 2 * al256(jobs * sizeof(int32_t)) + 256;
    w.dir_cap = jobs * kDirsPerJob;
    w.dirs = (int4*)tail;
    w.br_cap = jobs * kBracketsPerJob;
    w.brs = (WinBracket*)(tail + al256(jobs * kDirsPerJob * sizeof(int4)));
  }
  w.stats = stats_dev ? (unsigned long long*)stats_dev : (unsigned long long*)(w.fb_len + 16);
  w.shard = (unsigned long long*)(ws + chert_build_cache_surrogate_workspace_bytes(d, n_classes) -
                                  al256(kStatBytes));
  w.resid_tol = resid_tol > 0.0 ? resid_tol : 1e-11;

  CHERT_LAUNCH("k_write_header", k_write_header, dim3(1), dim3(64), 0, s, cache, d->dim,
               d->n_dirs, d->mode_mask, d->kernel, d->n_sweep, d->n_subset, n_classes,
                 d->sampling);
  CHERT_LAUNCH("k_warm_zero", k_warm_zero, dim3(1), dim3(256), 0, s, w.fb_len, w.win_len,
               w.shard);
  if (jobs > 0 && rows > 0) {
    const int64_t blocks = (rows + mlp::kInferRows - 1) / mlp::kInferRows;
    if (blocks > 0x7fffffffLL) return fail(CHERT_ERR_INVALID_ARG, "too many entries");
    CHERT_LAUNCH("k_warm_predict", k_warm_predict, dim3((unsigned)blocks), dim3(mlp::kThreads),
                 0, s, w, rows);
    const int per = warm_jobs(w.so.n_solve);
    CHERT_LAUNCH("k_warm_solve", k_warm_solve, dim3((unsigned)((jobs + per - 1) / per)),
                 dim3(kWarmSolveThreads), 0, s, w, jobs);
    const int64_t grid = jobs < 4096 ? jobs : 4096;
    CHERT_LAUNCH("k_warm_window", k_warm_window, dim3((unsigned)grid), dim3(64),
                 kWinCap * (sizeof(double2) + sizeof(int16_t)) +
                     (size_t)d->n_sweep * sizeof(int16_t), s, w);
    const int64_t fgrid = (w.dir_cap + 63) / 64 < 8192 ? (w.dir_cap + 63) / 64 : 8192;
    CHERT_LAUNCH("k_warm_fold", k_warm_fold, dim3((unsigned)fgrid), dim3(64), 0, s, w);
    CHERT_LAUNCH("k_build_fused", k_build_fused, dim3((unsigned)grid), dim3(kNodeThreads),
                 (size_t)d->n_sweep * sizeof(double2), s, w.so, (const int32_t*)w.fb_list,
                 (const int32_t*)w.fb_len, jobs);
  }
  CHERT_LAUNCH("k_warm_stats_fold", k_warm_stats_fold, dim3(1), dim3(64), 0, s,
               (const unsigned long long*)w.shard, w.stats);
  enqueue_cache_stats(d, n_classes, cache, lay, w.fb_len, w.so.n_cols, s);  // listed: jobs
  return launch_status();
}
