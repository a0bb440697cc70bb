// The local solve of one target ray direction (eqs 9-11), shared by the
// cache build's kernels and by the host-side operation count: bracket the
// target on a theta_R sweep table, refine each bracket by a 2D Newton
// iteration on (homogeneity residual, ray-direction miss) with a nested
// bisection as fallback, keep the first arrival; and the surrogate start's
// Newton polish with the check that its theta_I is the root nearest 0.
#pragma once

#include "physics.h"

namespace chert {

// What the solve steps read of a build's arguments.
struct SolveParams {
  int kernel;        // CHERT_KERNEL_MEV or _OEV
  int n_sweep;       // theta_R samples of the sweep table
  double resid_tol;  // entries whose residual is above this get CHERT_ST_NOCONV
  int newton_iters;  // Newton steps per bracket
  int bisect_iters;  // halvings of the bisection fallback
};

constexpr double kWarmWindow = 0.35;  // the polish may move theta_R this far [rad]

// Newton on F = (h, psi - psi*) from the bracket interpolant.  Elastic modes
// keep theta_I = 0 exactly and solve the 1D direction equation.
__device__ __forceinline__ bool newton_root(const Medium& m, int mode, int kernel,
                                         double psi_star, double ta, double tb,
                                         double ya, double yb, double fa, double fb,
                                         int iters, double* xo, double* yo) {
  const bool el = theta_i_zero(m, mode);
  const double eps = kFdEps;
  const double dth = tb - ta;
  double t = fa / (fa - fb);
  double x = ta + t * dth;
  double y = el ? 0.0 : ya + t * (yb - ya);
  double last = 1.0;
  for (int it = 0; it < iters; ++it) {
    const Trig t0 = trig_of(x, y);
    Vel v0 = energy_velocity_t(m, mode, kernel, t0);
    double F2 = wrap_pi(ray_angle(v0) - psi_star);
    double dx, dy = 0.0;
    if (el) {
      Vel vx = energy_velocity_t(m, mode, kernel, step_re(t0));
      double d = dangle(v0, vx) / eps;
      dx = -F2 / d;
    } else {
      double F1 = homog_residual(v0);
      Vel vx = energy_velocity_t(m, mode, kernel, step_re(t0));
      Vel vy = energy_velocity_t(m, mode, kernel, step_im(t0));
      double J11 = (homog_residual(vx) - F1) / eps;
      double J12 = (homog_residual(vy) - F1) / eps;
      double J21 = dangle(v0, vx) / eps;
      double J22 = dangle(v0, vy) / eps;
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
                                         int iters, double* xo, double* yo) {
  double lo = ta, hi = tb;
  bool neg_lo = fa < 0.0;
  for (int it = 0; it < iters && hi - lo > 1e-14; ++it) {
    double mid = 0.5 * (lo + hi);
    double thI, sr, cr;
    sincos(mid, &sr, &cr);
    if (!theta_imag_sc(m, mode, kernel, sr, cr, &thI)) return false;
    double fm = wrap_pi(ray_angle_sc(m, mode, kernel, sr, cr, thI) - psi_star);
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

constexpr int kMaxBr = 6;  // brackets kept per lane for the lockstep refinement

// Sweep tables as solve_dir reads them: (theta_I, ray angle) of sample j,
// NaN angle where the sample has no root.  A full table holds every sample;
// a windowed one holds the marked samples in ascending order (slot q is
// sample idx[q], pos[j] is the slot of sample j or -1) and reads every other
// sample as NaN.  count()/sample(q) enumerate the samples that can open a
// bracket, in ascending order.
struct FullTable {
  const double2* t;
  int n;
  __device__ __forceinline__ double2 at(int j) const { return t[j]; }
  __device__ __forceinline__ int count() const { return n; }
  __device__ __forceinline__ int sample(int q) const { return q; }
};
struct WindowTable {
  const int16_t* pos;
  const double2* ent;
  const int16_t* idx;
  int nl;
  __device__ __forceinline__ double2 at(int j) const {
    const int p = pos[j];
    return p < 0 ? make_double2(0.0, NAN) : ent[p];
  }
  __device__ __forceinline__ int count() const { return nl; }
  __device__ __forceinline__ int sample(int q) const { return idx[q]; }
};

// Refine the bracket starting at sweep sample j and fold the root into the
// running first-arrival choice (largest ray velocity; ties to the smaller
// |theta_R - psi*|).
// The root of the bracket at sweep sample j and its ray quantities; false if
// neither the Newton step nor the bisection converges.  *cand_ill: the
// bracket's ray-angle slope is below kIllSlope.
__device__ __forceinline__ bool bracket_root(const SolveParams& a, const Medium& m, int mode,
                                             int j,
                                             double2 sa, double2 sb, double psi_star, bool el,
                                             Entry* cand, bool* cand_ill) {
  const double dth = kTwoPi / a.n_sweep;
  double fa = wrap_pi(sa.y - psi_star);
  double fb = wrap_pi(sb.y - psi_star);
  double ta = (j + 0.5) * dth;
  double tb = ta + dth;
  double x, y;
  bool ok = newton_root(m, mode, a.kernel, psi_star, ta, tb, sa.x, sb.x, fa, fb, a.newton_iters,
                        &x, &y);
  // The 2D Newton iteration does not know which homogeneity root theta_I
  // must be: keep its root only if y is the root nearest 0 at the final
  // theta_R (the outward scan's answer there); otherwise -- theta_I(theta_R)
  // switching branches inside the bracket -- the nested bisection follows
  // that definition.
  // It must also lie in its own bracket (the bisection's interval), not
  // wander into a neighbouring one.
  if (ok) ok = x >= ta - 1e-12 && x <= tb + 1e-12;
  if (ok && !el) {
    double sx, cx, ys;
    sincos(x, &sx, &cx);
    ok = theta_imag_sc(m, mode, a.kernel, sx, cx, &ys) && fabs(ys - y) <= 1e-9;
  }
  if (!ok) ok = bisect_root(m, mode, a.kernel, psi_star, ta, tb, fa, a.bisect_iters, &x, &y);
  if (!ok) return false;
  if (x >= kTwoPi) x -= kTwoPi;
  if (x < 0.0) x += kTwoPi;
  Vel v = energy_velocity(m, mode, a.kernel, x, y);
  ray_quantities(v, cand);
  cand->thR = x;
  cand->thI = y;
  double h = el ? 0.0 : homog_residual(v);
  cand->res = fmax(fabs(h), fabs(wrap_pi(ray_angle(v) - psi_star)));
  *cand_ill = fabs((fb - fa) / (tb - ta)) < kIllSlope;
  return true;
}

// Fold a refined bracket into the running first-arrival choice, brackets in
// scan order: a root (residual within tol) beats a refinement that closed on
// a jump of the ray-angle map; among equals the first, then a larger ray
// velocity; ties (kTieRel) go to the smaller |theta_R - psi*|.
__device__ __forceinline__ void fold_choice(const Entry& cand, bool cand_ill, double psi_star,
                                            double tol, bool* found, bool* ill, Entry* best) {
  bool take;
  const bool cand_root = cand.res <= tol, best_root = *found && best->res <= tol;
  if (!*found) take = true;
  else if (cand_root != best_root) take = cand_root;
  else if (cand.V > best->V * (1.0 + kTieRel)) take = true;
  else take = fabs(cand.V - best->V) <= kTieRel * best->V &&
              ang_dist(cand.thR, psi_star) < ang_dist(best->thR, psi_star);
  if (take) {
    *best = cand;
    *ill = cand_ill;
    *found = true;
  }
}

__device__ __forceinline__ void refine_bracket_at(const SolveParams& a, const Medium& m,
                                                  int mode,
                                                  int j, double2 sa, double2 sb, double psi_star,
                                                  bool el, bool* found, bool* ill, Entry* best) {
  Entry cand;
  bool cand_ill;
  if (bracket_root(a, m, mode, j, sa, sb, psi_star, el, &cand, &cand_ill))
    fold_choice(cand, cand_ill, psi_star, a.resid_tol, found, ill, best);
}

template <class T>
__device__ __forceinline__ void refine_bracket(const SolveParams& a, const Medium& m,
                                               int mode,
                                               const T& tab, int j, double psi_star, bool el,
                                               bool* found, bool* ill, Entry* best) {
  refine_bracket_at(a, m, mode, j, tab.at(j), tab.at(j + 1 == a.n_sweep ? 0 : j + 1), psi_star,
                    el, found, ill, best);
}

// status of a solved direction from the folded choice (as the plain search)
__device__ __forceinline__ int32_t solve_status(bool found, bool ill, const Entry& best) {
  if (!found) return CHERT_ST_NO_BRACKET;
  int32_t st = ill ? CHERT_ST_ILL : CHERT_ST_OK;
  if (!(best.A >= 0.0) || !isfinite(best.V) || !(best.V > 0.0)) st |= CHERT_ST_NONPHYS;
  return st;
}

template <class T>
__device__ __forceinline__ bool is_bracket(const T& tab, int j, int n, double psi_star) {
  double2 sa = tab.at(j);
  double2 sb = tab.at(j + 1 == n ? 0 : j + 1);
  if (isnan(sa.y) || isnan(sb.y)) return false;
  double fa = wrap_pi(sa.y - psi_star);
  double fb = wrap_pi(sb.y - psi_star);
  if (fabs(fb - fa) >= kPi) return false;  // the +-pi seam, not a crossing
  return brackets(fa, fb);
}

// Solve target direction d for one (class, mode) from its sweep table in
// LDS.  Lanes of a wavefront run it in step (brackets first, then the
// refinements together); `br` is this lane's kMaxBr bracket slots in LDS.
template <class T>
__device__ __forceinline__ int32_t solve_dir(const SolveParams& a, const Medium& m,
                                             int mode,
                                             const T& tab, double psi_star, int* br,
                                             Entry* best) {
  const bool el = theta_i_zero(m, mode);
  // phase 1: every sign change of the ray-direction miss over the sweep
  int nbr = 0;
  for (int q = 0; q < tab.count(); ++q) {
    const int j = tab.sample(q);
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
    for (int q = 0; q < tab.count(); ++q) {
      const int j = tab.sample(q);
      if (!is_bracket(tab, j, a.n_sweep, psi_star)) continue;
      if (seen++ < kMaxBr) continue;
      refine_bracket(a, m, mode, tab, j, psi_star, el, &found, &ill, best);
    }
  }
  return solve_status(found, ill, *best);
}

// Newton on F = (h, psi - psi*) from (x0, y0), as newton_root but started
// from a prediction and kept within kWarmWindow of it; *slope is
// d psi / d theta_R along the homogeneous curve h = 0 at the last iterate.
__device__ __forceinline__ bool warm_newton(const Medium& m, int mode, int kernel, bool el,
                                         double psi_star, double x0, double y0, double* xo,
                                         double* yo, double* slope) {
  const double eps = kFdEps;
  double x = x0, y = el ? 0.0 : y0, last = 1.0, sl = NAN;
  for (int it = 0; it < 16; ++it) {
    const Trig t0 = trig_of(x, y);
    Vel v0 = energy_velocity_t(m, mode, kernel, t0);
    double F2 = wrap_pi(ray_angle(v0) - psi_star);
    double dx, dy = 0.0;
    if (el) {
      Vel vx = energy_velocity_t(m, mode, kernel, step_re(t0));
      double dd = dangle(v0, vx) / eps;
      dx = -F2 / dd;
      sl = dd;
    } else {
      double F1 = homog_residual(v0);
      Vel vx = energy_velocity_t(m, mode, kernel, step_re(t0));
      Vel vy = energy_velocity_t(m, mode, kernel, step_im(t0));
      double J11 = (homog_residual(vx) - F1) / eps;
      double J12 = (homog_residual(vy) - F1) / eps;
      double J21 = dangle(v0, vx) / eps;
      double J22 = dangle(v0, vy) / eps;
      double det = J11 * J22 - J12 * J21;
      dx = -(J22 * F1 - J12 * F2) / det;
      dy = -(-J21 * F1 + J11 * F2) / det;
      sl = -det / J12;
    }
    if (!isfinite(dx) || !isfinite(dy)) return false;
    x += dx;
    y += dy;
    if (fabs(x - x0) > kWarmWindow || fabs(y) > 30.0 * kPi / 180.0) return false;
    last = fmax(fabs(dx), fabs(dy));
    if (last < 1e-15) break;
  }
  if (!(last < 1e-12)) return false;
  *xo = x;
  *yo = y;
  *slope = sl;
  return true;
}

// Is y the theta_I that theta_imag's outward scan returns at theta_R = x?
// No bracket of the residual closer to 0 on either side, the bracket
// holding y on its side, none in the same step on the other side.
__device__ __forceinline__ bool thi_is_nearest(const Medium& m, int mode, int kernel, double x,
                                               double y) {
  const int kr = (int)floor(fabs(y) / kThiStep);
  if (kr >= kThiSteps || y == 0.0) return false;
  double sr, cr;
  sincos(x, &sr, &cr);
  const double h0 = h_t(m, mode, kernel, sr, cr, 0.0, 1.0);
  if (h0 == 0.0) return false;
  double hp_lo = h0, hn_hi = h0;
  for (int k = 0; k <= kr; ++k) {
    double hp_hi, hn_lo;  // the same evaluations as theta_imag's scan
    h_scan_pair(m, mode, kernel, sr, cr, k, &hp_hi, &hn_lo);
    const bool bp = brackets(hp_lo, hp_hi);
    const bool bn = brackets(hn_lo, hn_hi);
    if (k < kr) {
      if (bp || bn) return false;
    } else {
      const bool mine = y > 0.0 ? bp : bn;
      const bool other = y > 0.0 ? bn : bp;
      if (!mine || other) return false;
    }
    hp_lo = hp_hi;
    hn_hi = hn_lo;
  }
  return true;
}

}  // namespace chert
