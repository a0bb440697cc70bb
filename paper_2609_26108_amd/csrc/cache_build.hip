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
  double* fields;   // [CHERT_NF][3][n_classes][n_dirs]
  int32_t* status;  // [3][n_classes][n_dirs]
};

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

__global__ void __launch_bounds__(64) k_solve(SolveArgs a) {
  extern __shared__ double2 tab[];
  __shared__ int s_br[64 * kMaxBr];
  const int half = a.n_dirs / 2;
  const int chunks = (half + 63) / 64;
  const int64_t job = blockIdx.x / chunks;
  const int chunk = blockIdx.x % chunks;
  const int64_t k = job % a.n_classes;
  const int mode = a.modes[job / a.n_classes];
  const double2* src = a.table + job * a.n_sweep;
  for (int j = threadIdx.x; j < a.n_sweep; j += blockDim.x) tab[j] = src[j];
  __syncthreads();

  const int d = chunk * 64 + threadIdx.x;
  if (d >= half) return;
  const int64_t stride = 3 * a.n_classes * (int64_t)a.n_dirs;
  const int64_t base = ((int64_t)mode * a.n_classes + k) * a.n_dirs + d;
  const chert_class c = a.classes[k];
  if (class_invalid(c)) {
    store_invalid(a, base, stride, CHERT_ST_NONPHYS);
    store_invalid(a, base + half, stride, CHERT_ST_NONPHYS);
    return;
  }
  if (is_fluid_shear(c, mode)) {
    store_invalid(a, base, stride, CHERT_ST_FLUID);
    store_invalid(a, base + half, stride, CHERT_ST_FLUID);
    return;
  }
  const Medium m = load_medium(c);
  const bool el = theta_i_zero(m, mode);
  const double psi_star = wrap_pi(d * (kTwoPi / a.n_dirs) - m.tilt);

  // phase 1: every sign change of the ray-direction miss over the sweep
  int nbr = 0;
  int* my = s_br + threadIdx.x * kMaxBr;
  for (int j = 0; j < a.n_sweep; ++j) {
    if (!is_bracket(tab, j, a.n_sweep, psi_star)) continue;
    if (nbr < kMaxBr) my[nbr] = j;
    ++nbr;
  }
  // phase 2: refine the kept brackets with all lanes in step
  bool found = false, ill = false;
  Entry best{};
  for (int sidx = 0; sidx < kMaxBr; ++sidx) {
    if (__all(sidx >= nbr)) break;
    if (sidx < nbr) refine_bracket(a, m, mode, tab, my[sidx], psi_star, el, &found, &ill, &best);
  }
  // rare: more brackets than slots; refine the rest in scan order
  if (nbr > kMaxBr) {
    int seen = 0;
    for (int j = 0; j < a.n_sweep; ++j) {
      if (!is_bracket(tab, j, a.n_sweep, psi_star)) continue;
      if (seen++ < kMaxBr) continue;
      refine_bracket(a, m, mode, tab, j, psi_star, el, &found, &ill, &best);
    }
  }
  if (!found) {
    store_invalid(a, base, stride, CHERT_ST_NO_BRACKET);
    store_invalid(a, base + half, stride, CHERT_ST_NO_BRACKET);
    return;
  }
  int32_t st = ill ? CHERT_ST_ILL : CHERT_ST_OK;
  if (!(best.A >= 0.0) || !isfinite(best.V) || !(best.V > 0.0)) st |= CHERT_ST_NONPHYS;
  store_entry(a, base, stride, best, m.tilt, st);
  // centrosymmetric copy: same ray quantities, reversed direction, slowness
  // direction turned by pi
  Entry r = best;
  r.thR = best.thR + kPi;
  if (r.thR >= kTwoPi) r.thR -= kTwoPi;
  store_entry(a, base + half, stride, r, m.tilt, st);
  a.fields[CHERT_F_RX * stride + base + half] = -a.fields[CHERT_F_RX * stride + base];
  a.fields[CHERT_F_RZ * stride + base + half] = -a.fields[CHERT_F_RZ * stride + base];
}

__global__ void k_write_header(uint8_t* cache, int32_t dim, int32_t n_dirs, uint32_t mask,
                               int32_t kernel, int32_t n_sweep, int64_t n_classes) {
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
    w[7] = 0u;
    *reinterpret_cast<int64_t*>(cache + 32) = n_classes;
  }
}

}  // namespace chert

using namespace chert;

extern "C" size_t chert_build_cache_workspace_bytes(const chert_cache_desc* d,
                                                    int64_t n_classes) {
  if (!d || n_classes <= 0 || d->n_sweep <= 0) return 0;
  int nm = __builtin_popcount(d->mode_mask & 7u);
  return (size_t)nm * (size_t)n_classes * (size_t)d->n_sweep * sizeof(double2);
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
  size_t need = chert_build_cache_workspace_bytes(d, n_classes);
  if (!workspace_dev || workspace_bytes < need)
    return fail(CHERT_ERR_INVALID_ARG, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* cache = (uint8_t*)cache_dev;

  SweepArgs sa{};
  sa.classes = classes_dev;
  sa.n_classes = n_classes;
  sa.n_modes = 0;
  for (int m = 0; m < 3; ++m)
    if (d->mode_mask & (1u << m)) sa.modes[sa.n_modes++] = m;
  sa.kernel = d->kernel;
  sa.n_sweep = d->n_sweep;
  sa.table = (double2*)workspace_dev;

  CHERT_LAUNCH("k_write_header", k_write_header, dim3(1), dim3(64), 0, s, cache, d->dim, d->n_dirs,
                     d->mode_mask, d->kernel, d->n_sweep, n_classes);
  if (sa.n_modes > 0) {
    int64_t total = (int64_t)sa.n_modes * n_classes * d->n_sweep;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    CHERT_LAUNCH("k_sweep", k_sweep, dim3((unsigned)blocks), dim3(256), 0, s, sa);

    SolveArgs so{};
    so.classes = classes_dev;
    so.n_classes = n_classes;
    so.n_modes = sa.n_modes;
    for (int i = 0; i < 3; ++i) so.modes[i] = sa.modes[i];
    so.kernel = d->kernel;
    so.n_sweep = d->n_sweep;
    so.n_dirs = d->n_dirs;
    so.table = sa.table;
    so.fields = (double*)(cache + lay.fields_offset);
    so.status = (int32_t*)(cache + lay.status_offset);
    int chunks = (d->n_dirs / 2 + 63) / 64;
    int64_t grid = (int64_t)sa.n_modes * n_classes * chunks;
    if (grid > 0x7fffffff) return fail(CHERT_ERR_INVALID_ARG, "too many classes");
    CHERT_LAUNCH("k_solve", k_solve, dim3((unsigned)grid), dim3(64),
                       (size_t)d->n_sweep * sizeof(double2), s, so);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  return CHERT_OK;
}
