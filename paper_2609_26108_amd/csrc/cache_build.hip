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
// Everything is FP64: qSV cusps and triplications need it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "chert.h"
#include "chert_internal.h"
#include "physics.h"

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
      double thI;
      if (theta_imag(m, mode, a.kernel, thR, &thI)) {
        double psi = ray_angle(energy_velocity(m, mode, a.kernel, thR, thI));
        if (isfinite(psi)) out = make_double2(thI, psi);
      }
    }
    a.table[t] = out;
  }
}

struct SolveArgs {
  const chert_class* classes;
  int64_t n_classes;
  int n_modes;
  int modes[3];
  int kernel;
  int n_sweep;
  int n_dirs;
  const double2* table;
  double* fields;   // [CHERT_NF][3][n_classes][n_cols]
  int32_t* status;  // [3][n_classes][n_cols]
  int n_cols;       // stored direction columns per (mode, class)
  int n_solve;      // directions solved per (mode, class); the rest are copies
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

// Newton on F = (h, psi - psi*) from the bracket interpolant.  Elastic modes
// keep theta_I = 0 exactly and solve the 1D direction equation.
__device__ __forceinline__ bool newton_root(const Medium& m, int mode, int kernel,
                                         double psi_star, double ta, double tb,
                                         double ya, double yb, double fa, double fb,
                                         double* xo, double* yo) {
  const bool el = theta_i_zero(m, mode);
  const double eps = 1e-7;
  const double dth = tb - ta;
  double t = fa / (fa - fb);
  double x = ta + t * dth;
  double y = el ? 0.0 : ya + t * (yb - ya);
  double last = 1.0;
  for (int it = 0; it < 12; ++it) {
    Vel v0 = energy_velocity(m, mode, kernel, x, y);
    double F2 = wrap_pi(ray_angle(v0) - psi_star);
    double dx, dy = 0.0;
    if (el) {
      Vel vx = energy_velocity(m, mode, kernel, x + eps, 0.0);
      double d = (wrap_pi(ray_angle(vx) - psi_star) - F2) / eps;
      dx = -F2 / d;
    } else {
      double F1 = homog_residual(v0);
      Vel vx = energy_velocity(m, mode, kernel, x + eps, y);
      Vel vy = energy_velocity(m, mode, kernel, x, y + eps);
      double J11 = (homog_residual(vx) - F1) / eps;
      double J12 = (homog_residual(vy) - F1) / eps;
      double J21 = (wrap_pi(ray_angle(vx) - psi_star) - F2) / eps;
      double J22 = (wrap_pi(ray_angle(vy) - psi_star) - F2) / eps;
      double det = J11 * J22 - J12 * J21;
      dx = -(J22 * F1 - J12 * F2) / det;
      dy = -(-J21 * F1 + J11 * F2) / det;
    }
    if (!isfinite(dx) || !isfinite(dy)) return false;
    x += dx;
    y += dy;
    if (x < ta - dth || x > tb + dth || fabs(y) > 30.0 * kPi / 180.0) return false;
    last = fmax(fabs(dx), fabs(dy));
    if (last < 1e-15) break;
  }
  if (!(last < 1e-12)) return false;
  *xo = x;
  *yo = y;
  return true;
}

// Fallback: nested bisection on theta_R with the inner theta_I solve at every
// trial point (slow, used only when Newton does not settle).
__device__ __forceinline__ bool bisect_root(const Medium& m, int mode, int kernel,
                                         double psi_star, double ta, double tb, double fa,
                                         double* xo, double* yo) {
  double lo = ta, hi = tb;
  bool neg_lo = fa < 0.0;
  for (int it = 0; it < 200 && hi - lo > 1e-14; ++it) {
    double mid = 0.5 * (lo + hi);
    double thI;
    if (!theta_imag(m, mode, kernel, mid, &thI)) return false;
    double fm = wrap_pi(ray_angle(energy_velocity(m, mode, kernel, mid, thI)) - psi_star);
    if ((fm < 0.0) == neg_lo) lo = mid;
    else hi = mid;
  }
  double x = 0.5 * (lo + hi);
  double y;
  if (!theta_imag(m, mode, kernel, x, &y)) return false;
  *xo = x;
  *yo = y;
  return true;
}

__device__ __forceinline__ double ang_dist(double a, double b) { return fabs(wrap_pi(a - b)); }

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

constexpr int kMaxBr = 6;  // brackets kept per lane for the lockstep refinement

// Refine the bracket starting at sweep sample j and fold the root into the
// running first-arrival choice (largest ray velocity; ties to the smaller
// |theta_R - psi*|).
__device__ __forceinline__ void refine_bracket(const SolveArgs& a, const Medium& m, int mode,
                                               const double2* tab, int j, double psi_star,
                                               bool el, bool* found, bool* ill, Entry* best) {
  const double dth = kTwoPi / a.n_sweep;
  double2 sa = tab[j];
  double2 sb = tab[j + 1 == a.n_sweep ? 0 : j + 1];
  double fa = wrap_pi(sa.y - psi_star);
  double fb = wrap_pi(sb.y - psi_star);
  double ta = (j + 0.5) * dth;
  double tb = ta + dth;
  double x, y;
  bool ok = newton_root(m, mode, a.kernel, psi_star, ta, tb, sa.x, sb.x, fa, fb, &x, &y);
  if (!ok) ok = bisect_root(m, mode, a.kernel, psi_star, ta, tb, fa, &x, &y);
  if (!ok) return;
  if (x >= kTwoPi) x -= kTwoPi;
  if (x < 0.0) x += kTwoPi;
  Vel v = energy_velocity(m, mode, a.kernel, x, y);
  Entry cand;
  ray_quantities(v, &cand);
  cand.thR = x;
  cand.thI = y;
  double h = el ? 0.0 : homog_residual(v);
  cand.res = fmax(fabs(h), fabs(wrap_pi(ray_angle(v) - psi_star)));
  bool cand_ill = fabs((fb - fa) / (tb - ta)) < kIllSlope;
  bool take;
  if (!*found) take = true;
  else if (cand.V > best->V * (1.0 + kTieRel)) take = true;
  else take = fabs(cand.V - best->V) <= kTieRel * best->V &&
              ang_dist(cand.thR, psi_star) < ang_dist(best->thR, psi_star);
  if (take) {
    *best = cand;
    *ill = cand_ill;
    *found = true;
  }
}

__device__ __forceinline__ bool is_bracket(const double2* tab, int j, int n, double psi_star) {
  double2 sa = tab[j];
  double2 sb = tab[j + 1 == n ? 0 : j + 1];
  if (isnan(sa.y) || isnan(sb.y)) return false;
  double fa = wrap_pi(sa.y - psi_star);
  double fb = wrap_pi(sb.y - psi_star);
  if (fabs(fb - fa) >= kPi) return false;  // the +-pi seam, not a crossing
  return brackets(fa, fb);
}

// Solve target direction d for one (class, mode) from its sweep table in
// LDS.  Lanes of a wavefront run it in step (brackets first, then the
// refinements together); `br` is this lane's kMaxBr bracket slots in LDS.
__device__ __forceinline__ int32_t solve_dir(const SolveArgs& a, const Medium& m, int mode,
                                             const double2* tab, int d, int* br, Entry* best) {
  const bool el = theta_i_zero(m, mode);
  const double psi_star = wrap_pi(d * (kTwoPi / a.n_dirs) - m.tilt);
  // phase 1: every sign change of the ray-direction miss over the sweep
  int nbr = 0;
  for (int j = 0; j < a.n_sweep; ++j) {
    if (!is_bracket(tab, j, a.n_sweep, psi_star)) continue;
    if (nbr < kMaxBr) br[nbr] = j;
    ++nbr;
  }
  // phase 2: refine the kept brackets with all lanes in step
  bool found = false, ill = false;
  for (int sidx = 0; sidx < kMaxBr; ++sidx) {
    if (__all(sidx >= nbr)) break;
    if (sidx < nbr) refine_bracket(a, m, mode, tab, br[sidx], psi_star, el, &found, &ill, best);
  }
  // rare: more brackets than slots; refine the rest in scan order
  if (nbr > kMaxBr) {
    int seen = 0;
    for (int j = 0; j < a.n_sweep; ++j) {
      if (!is_bracket(tab, j, a.n_sweep, psi_star)) continue;
      if (seen++ < kMaxBr) continue;
      refine_bracket(a, m, mode, tab, j, psi_star, el, &found, &ill, best);
    }
  }
  if (!found) return CHERT_ST_NO_BRACKET;
  int32_t st = ill ? CHERT_ST_ILL : CHERT_ST_OK;
  if (!(best->A >= 0.0) || !isfinite(best->V) || !(best->V > 0.0)) st |= CHERT_ST_NONPHYS;
  return st;
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
  store_entry(a, row + col, stride, best, tilt, st);
  Entry r = best;
  r.thR = best.thR + kPi;
  if (r.thR >= kTwoPi) r.thR -= kTwoPi;
  store_entry(a, row + pcol, stride, r, tilt, st);
  a.fields[CHERT_F_RX * stride + row + pcol] = -a.fields[CHERT_F_RX * stride + row + col];
  a.fields[CHERT_F_RZ * stride + row + pcol] = -a.fields[CHERT_F_RZ * stride + row + col];
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
__global__ void __launch_bounds__(64) k_solve(SolveArgs a) {
  extern __shared__ double2 tab[];
  __shared__ int s_br[64 * kMaxBr];
  const int chunks = (a.n_solve + 63) / 64;
  const int64_t job = blockIdx.x / chunks;
  const int chunk = blockIdx.x % chunks;
  const int64_t k = job % a.n_classes;
  const int mode = a.modes[job / a.n_classes];
  const double2* src = a.table + job * a.n_sweep;
  for (int j = threadIdx.x; j < a.n_sweep; j += blockDim.x) tab[j] = src[j];
  __syncthreads();

  const int sidx = chunk * 64 + threadIdx.x;
  if (sidx >= a.n_solve) return;
  int d, col, pcol;
  dir_cols(a, sidx, &d, &col, &pcol);
  const int64_t row = ((int64_t)mode * a.n_classes + k) * a.n_cols;
  const chert_class c = a.classes[k];
  Entry best{};
  best.V = NAN;
  int32_t st = class_block(c, mode);
  if (st) {
    store_pair(a, row, col, pcol, best, 0.0, st);
    return;
  }
  const Medium m = load_medium(c);
  st = solve_dir(a, m, mode, tab, d, s_br + threadIdx.x * kMaxBr, &best);
  store_pair(a, row, col, pcol, best, m.tilt, st);
}

// Fused path (many classes, e.g. one per node): one workgroup per
// (mode, class) sweeps theta_R into LDS, then solves that class's
// directions; no sweep table in HBM.
constexpr int kNodeThreads = 256;
__global__ void __launch_bounds__(kNodeThreads) k_build_fused(SolveArgs a) {
  extern __shared__ double2 tab[];
  __shared__ int s_br[kNodeThreads * kMaxBr];
  const int64_t job = blockIdx.x;
  const int64_t k = job % a.n_classes;
  const int mode = a.modes[job / a.n_classes];
  const chert_class c = a.classes[k];
  const int64_t row = ((int64_t)mode * a.n_classes + k) * a.n_cols;
  int32_t blocked = class_block(c, mode);
  if (blocked) {
    Entry none{};
    none.V = NAN;
    for (int sidx = threadIdx.x; sidx < a.n_solve; sidx += blockDim.x) {
      int d, col, pcol;
      dir_cols(a, sidx, &d, &col, &pcol);
      store_pair(a, row, col, pcol, none, 0.0, blocked);
    }
    return;  // block-uniform
  }
  const Medium m = load_medium(c);
  for (int j = threadIdx.x; j < a.n_sweep; j += blockDim.x) {
    const double thR = (j + 0.5) * (kTwoPi / a.n_sweep);
    double thI;
    double2 out = make_double2(0.0, NAN);
    if (theta_imag(m, mode, a.kernel, thR, &thI)) {
      const double psi = ray_angle(energy_velocity(m, mode, a.kernel, thR, thI));
      if (isfinite(psi)) out = make_double2(thI, psi);
    }
    tab[j] = out;
  }
  __syncthreads();
  for (int sidx = threadIdx.x; sidx < a.n_solve; sidx += blockDim.x) {
    int d, col, pcol;
    dir_cols(a, sidx, &d, &col, &pcol);
    Entry best{};
    const int32_t st = solve_dir(a, m, mode, tab, d, s_br + threadIdx.x * kMaxBr, &best);
    store_pair(a, row, col, pcol, best, m.tilt, st);
  }
}

__global__ void k_write_header(uint8_t* cache, int32_t dim, int32_t n_dirs, uint32_t mask,
                               int32_t kernel, int32_t n_sweep, int32_t n_subset,
                               int64_t n_classes) {
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
  }
}

}  // namespace chert

using namespace chert;

// Jobs (mode x class) at or above this count use the fused one-launch path.
constexpr int64_t kFusedJobs = 512;

static int64_t n_jobs_of(const chert_cache_desc* d, int64_t n_classes) {
  return (int64_t)__builtin_popcount(d->mode_mask & 7u) * n_classes;
}

extern "C" size_t chert_build_cache_workspace_bytes(const chert_cache_desc* d,
                                                    int64_t n_classes) {
  if (!d || n_classes <= 0 || d->n_sweep <= 0) return 0;
  if (n_jobs_of(d, n_classes) >= kFusedJobs) return 0;  // sweep table stays in LDS
  return (size_t)n_jobs_of(d, n_classes) * (size_t)d->n_sweep * sizeof(double2);
}

extern "C" int chert_build_cache(const chert_cache_desc* d, const chert_class* classes_dev,
                                 int64_t n_classes, void* cache_dev, void* workspace_dev,
                                 size_t workspace_bytes, void* stream) {
  chert_cache_layout lay;
  int rc = chert_cache_layout_of(d, n_classes, &lay);
  if (rc != CHERT_OK) return rc;
  if (!classes_dev || !cache_dev) return fail(CHERT_ERR_INVALID_ARG, "null classes or cache");
  if (d->n_sweep > kMaxSweep)
    return fail(CHERT_ERR_INVALID_ARG, "n_sweep above the LDS table limit");
  const size_t need = chert_build_cache_workspace_bytes(d, n_classes);
  if (need > 0 && (!workspace_dev || workspace_bytes < need))
    return fail(CHERT_ERR_INVALID_ARG, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* cache = (uint8_t*)cache_dev;

  int modes[3], n_modes = 0;
  for (int m = 0; m < 3; ++m)
    if (d->mode_mask & (1u << m)) modes[n_modes++] = m;

  SolveArgs so{};
  so.classes = classes_dev;
  so.n_classes = n_classes;
  so.n_modes = n_modes;
  for (int i = 0; i < 3; ++i) so.modes[i] = i < n_modes ? modes[i] : 0;
  so.kernel = d->kernel;
  so.n_sweep = d->n_sweep;
  so.n_dirs = d->n_dirs;
  so.table = (const double2*)workspace_dev;
  so.fields = (double*)(cache + lay.fields_offset);
  so.status = (int32_t*)(cache + lay.status_offset);
  const int half = d->n_dirs / 2;
  if (d->n_subset == 0) {
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

  CHERT_LAUNCH("k_write_header", k_write_header, dim3(1), dim3(64), 0, s, cache, d->dim,
               d->n_dirs, d->mode_mask, d->kernel, d->n_sweep, d->n_subset, n_classes);
  const int64_t jobs = (int64_t)n_modes * n_classes;
  if (jobs > 0x7fffffffLL) return fail(CHERT_ERR_INVALID_ARG, "too many classes");
  if (jobs >= kFusedJobs) {
    CHERT_LAUNCH("k_build_fused", k_build_fused, dim3((unsigned)jobs), dim3(kNodeThreads),
                 (size_t)d->n_sweep * sizeof(double2), s, so);
  } else if (jobs > 0) {
    SweepArgs sa{};
    sa.classes = classes_dev;
    sa.n_classes = n_classes;
    sa.n_modes = n_modes;
    for (int i = 0; i < 3; ++i) sa.modes[i] = so.modes[i];
    sa.kernel = d->kernel;
    sa.n_sweep = d->n_sweep;
    sa.table = (double2*)workspace_dev;
    int64_t total = jobs * d->n_sweep;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    CHERT_LAUNCH("k_sweep", k_sweep, dim3((unsigned)blocks), dim3(256), 0, s, sa);
    const int chunks = (so.n_solve + 63) / 64;
    CHERT_LAUNCH("k_solve", k_solve, dim3((unsigned)(jobs * chunks)), dim3(64),
                 (size_t)d->n_sweep * sizeof(double2), s, so);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  return CHERT_OK;
}
