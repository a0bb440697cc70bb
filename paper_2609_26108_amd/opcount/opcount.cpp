// FP64 operation count of the local physics (physics.h, solve.h) on the host.
//
// The headers are compiled with `double` replaced by F, a scalar that counts
// every add, subtract, multiply, divide and square root (one flop each; a
// fused multiply-add in the device code is the same two source operations)
// and, separately, every transcendental call (sincos, expm1, atan2).
// Comparisons, fabs, fmin/fmax and copysign are not counted.  The program
// runs, on the classes given on stdin, the primitives the cache build is
// made of and the build's own per-class steps (the theta_R sweep, the
// solve of every direction of an n_dirs cache, the surrogate start's
// polish of every direction from a perturbed root) and prints the mean
// counts as JSON.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <type_traits>
#include <vector>

#include "chert.h"

namespace opc {
struct Counts {
  long long flops = 0, trans = 0;
};
Counts g;
}  // namespace opc

struct F {
  double v;
  constexpr F() : v(0.0) {}
  constexpr F(double x) : v(x) {}
  constexpr F(int x) : v((double)x) {}
  constexpr F(long x) : v((double)x) {}
  constexpr F(long long x) : v((double)x) {}
  explicit operator int() const { return (int)v; }
  explicit operator long() const { return (long)v; }
  explicit operator long long() const { return (long long)v; }
  F& operator+=(F b) { ++opc::g.flops; v += b.v; return *this; }
  F& operator-=(F b) { ++opc::g.flops; v -= b.v; return *this; }
  F& operator*=(F b) { ++opc::g.flops; v *= b.v; return *this; }
  F& operator/=(F b) { ++opc::g.flops; v /= b.v; return *this; }
};
// constant expressions (the header's constants) are not counted
constexpr void tick() {
  if (!std::is_constant_evaluated()) ++opc::g.flops;
}
constexpr F operator+(F a, F b) { tick(); return F(a.v + b.v); }
constexpr F operator-(F a, F b) { tick(); return F(a.v - b.v); }
constexpr F operator*(F a, F b) { tick(); return F(a.v * b.v); }
constexpr F operator/(F a, F b) { tick(); return F(a.v / b.v); }
constexpr F operator-(F a) { return F(-a.v); }
inline bool operator<(F a, F b) { return a.v < b.v; }
inline bool operator>(F a, F b) { return a.v > b.v; }
inline bool operator<=(F a, F b) { return a.v <= b.v; }
inline bool operator>=(F a, F b) { return a.v >= b.v; }
inline bool operator==(F a, F b) { return a.v == b.v; }
inline bool operator!=(F a, F b) { return a.v != b.v; }
inline F sqrt(F a) { ++opc::g.flops; return F(::sqrt(a.v)); }
inline F fabs(F a) { return F(::fabs(a.v)); }
inline F fmin(F a, F b) { return F(::fmin(a.v, b.v)); }
inline F fmax(F a, F b) { return F(::fmax(a.v, b.v)); }
inline F copysign(F a, F b) { return F(::copysign(a.v, b.v)); }
inline F floor(F a) { return F(::floor(a.v)); }
inline F expm1(F a) { ++opc::g.trans; return F(::expm1(a.v)); }
inline F atan2(F a, F b) { ++opc::g.trans; return F(::atan2(a.v, b.v)); }
inline void sincos(F a, F* s, F* c) {
  ++opc::g.trans;
  s->v = ::sin(a.v);
  c->v = ::cos(a.v);
}
inline bool isnan(F a) { return ::isnan(a.v); }
inline bool isinf(F a) { return ::isinf(a.v); }
inline bool isfinite(F a) { return ::isfinite(a.v); }

#define double F
#include "physics.h"
#include "solve.h"
#undef double

using namespace chert;

static opc::Counts take() {
  opc::Counts c = opc::g;
  opc::g = opc::Counts{};
  return c;
}

int main() {
  // classes on stdin: 13 numbers per line (the chert_class fields)
  std::vector<chert_class> cls;
  double v[13];
  while (true) {
    int got = 0;
    for (int i = 0; i < 13; ++i) got += scanf("%lf", &v[i]) == 1;
    if (got < 13) break;
    cls.push_back(chert_class{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9],
                              v[10], v[11], v[12]});
  }
  int n_dirs = 360, n_sweep = 1440, mode_sel = 1, kernel_sel = 0;
  double dx0 = 1e-3, dy0 = 2e-4;
  const char* env = getenv("OPCOUNT_ARGS");  // "n_dirs n_sweep mode kernel dx dy"
  if (env) sscanf(env, "%d %d %d %d %lf %lf", &n_dirs, &n_sweep, &mode_sel, &kernel_sel, &dx0, &dy0);
  const int kSamples = 90;
  printf("{");
  const char* sep = "";
  for (int kernel = 0; kernel < 2; ++kernel)
    for (int mode = 0; mode < 3; ++mode) {
      long long e_fl = 0, e_tr = 0, n_e = 0, t_fl = 0, t_tr = 0, n_t = 0, t_ok = 0;
      long long r_fl = 0, n_r = 0;
      for (const chert_class& c : cls) {
        const Medium m = load_medium(c);
        for (int s = 0; s < kSamples; ++s) {
          const double thR = (s + 0.5) * (3.141592653589793 / kSamples);
          take();
          Trig t = trig_of(thR, 0.01);
          Vel ve = energy_velocity_t(m, mode, kernel, t);
          opc::Counts c1 = take();
          e_fl += c1.flops;
          e_tr += c1.trans;
          ++n_e;
          F th;
          F sr, cr;
          sincos(F(thR), &sr, &cr);
          take();
          const bool ok = theta_imag_sc(m, mode, kernel, sr, cr, &th);
          opc::Counts c2 = take();
          t_fl += c2.flops;
          t_tr += c2.trans;
          ++n_t;
          t_ok += ok;
          Entry en;
          ray_quantities(ve, &en);
          F h = homog_residual(ve);
          (void)h;
          opc::Counts c3 = take();
          r_fl += c3.flops;
          ++n_r;
        }
      }
      printf("%s\"%s_%s\": {\"energy_eval_flops\": %.2f, \"energy_eval_trans\": %.2f, "
             "\"theta_i_solve_flops\": %.1f, \"theta_i_solve_trans\": %.1f, "
             "\"theta_i_found\": %.3f, \"ray_quantities_and_residual_flops\": %.1f}",
             sep, kernel ? "OEV" : "MEV", mode == 0 ? "qP" : (mode == 1 ? "qSV" : "qSH"),
             (double)e_fl / n_e, (double)e_tr / n_e, (double)t_fl / n_t, (double)t_tr / n_t,
             (double)t_ok / n_t, (double)r_fl / n_r);
      sep = ", ";
    }
  // the build's per-class steps for one (mode, kernel)
  {
    SolveParams sp{};
    sp.kernel = kernel_sel;
    sp.n_sweep = n_sweep;
    sp.resid_tol = 1e-9;
    sp.newton_iters = 12;
    sp.bisect_iters = 200;
    std::vector<double2> tab((size_t)n_sweep);
    long long sw_fl = 0, sw_tr = 0, so_fl = 0, so_tr = 0, n_dir = 0, wa_fl = 0, wa_tr = 0;
    long long n_warm = 0, n_warm_ok = 0;
    for (const chert_class& c : cls) {
      const Medium m = load_medium(c);
      const int mode = mode_sel;
      take();
      for (int j = 0; j < n_sweep; ++j) {  // as k_sweep / k_build_fused
        const F thR = (j + 0.5) * (kTwoPi / n_sweep);
        F thI, sr, cr;
        sincos(thR, &sr, &cr);
        double2 out = make_double2(0.0, NAN);
        if (theta_imag_sc(m, mode, sp.kernel, sr, cr, &thI)) {
          const F ps = ray_angle_sc(m, mode, sp.kernel, sr, cr, thI);
          if (isfinite(ps)) out = make_double2(thI, ps);
        }
        tab[j] = out;
      }
      opc::Counts cs = take();
      sw_fl += cs.flops;
      sw_tr += cs.trans;
      const bool el = theta_i_zero(m, mode);
      for (int d = 0; d < n_dirs / 2; ++d) {  // as k_solve: one solve per direction
        int br[kMaxBr];
        Entry best{};
        take();
        const F psi = wrap_pi(d * (kTwoPi / n_dirs) - m.tilt);
        const int32_t st = solve_dir(sp, m, mode, FullTable{tab.data(), n_sweep}, psi, br, &best);
        opc::Counts c1 = take();
        so_fl += c1.flops;
        so_tr += c1.trans;
        ++n_dir;
        if (st & (CHERT_ST_NO_BRACKET | CHERT_ST_NONPHYS)) continue;
        // as k_warm_solve from a prediction off the root by (dx0, dy0)
        F x, y, slope;
        take();
        bool ok = warm_newton(m, mode, sp.kernel, el, psi, best.thR + dx0, best.thI + dy0, &x,
                              &y, &slope);
        if (ok && !el) ok = thi_is_nearest(m, mode, sp.kernel, x, y);
        if (ok) {
          const Vel v = energy_velocity(m, mode, sp.kernel, x, y);
          Entry e;
          ray_quantities(v, &e);
          const F h = el ? F(0.0) : homog_residual(v);
          e.res = fmax(fabs(h), fabs(wrap_pi(ray_angle(v) - psi)));
        }
        opc::Counts c2 = take();
        wa_fl += c2.flops;
        wa_tr += c2.trans;
        ++n_warm;
        n_warm_ok += ok;
      }
    }
    const double nc = cls.empty() ? 1.0 : (double)cls.size();
    printf("%s\"build\": {\"mode\": %d, \"kernel\": %d, \"n_sweep\": %d, \"n_dirs\": %d, "
           "\"sweep_flops_per_class\": %.1f, \"sweep_trans_per_class\": %.1f, "
           "\"solve_flops_per_direction\": %.1f, \"solve_trans_per_direction\": %.1f, "
           "\"warm_flops_per_direction\": %.1f, \"warm_trans_per_direction\": %.1f, "
           "\"warm_accepted\": %.3f, \"warm_start_offset\": [%g, %g]}",
           sep, mode_sel, kernel_sel, n_sweep, n_dirs, sw_fl / nc, sw_tr / nc,
           (double)so_fl / (n_dir ? n_dir : 1), (double)so_tr / (n_dir ? n_dir : 1),
           (double)wa_fl / (n_warm ? n_warm : 1), (double)wa_tr / (n_warm ? n_warm : 1),
           (double)n_warm_ok / (n_warm ? n_warm : 1), dx0, dy0);
  }
  printf("}\n");
  return 0;
}
