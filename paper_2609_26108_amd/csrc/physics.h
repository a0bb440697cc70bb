// Device-side local physics of the CHERT cache builder (gfx950, FP64).
//
// Complex energy velocity of a transversely isotropic viscoelastic medium at
// a complex slowness angle theta_R + i theta_I in the sagittal plane of the
// local symmetry-axis frame:
//   complex moduli a = a^R (1 - i/Q)                         (eq 2)
//   n = (sin z, 0, cos z), z = theta_R + i theta_I           (eq 7)
//   Christoffel matrix Gamma_jk = a_ijkl n_i n_l, eigenpair (eq 4)
//   c = sqrt(G), p = n / c                                   (eq 5)
//   MEV: v_m = a_mjkl p_l Re(g_j conj g_k) / (g^H g)          (eqs 13-14)
//   OEV: v_m = a_mjkl p_l g_j g_k / (g^T g)                   (eq 12)
// plus the homogeneity residual (eq 9) and the ray quantities (eqs 10-11).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "chert.h"

namespace chert {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kThiStep = 0.25 * kPi / 180.0;  // outward scan step for theta_I
constexpr int kThiSteps = 120;                    // 120 * 0.25 deg = 30 deg
constexpr double kThiTol = 1e-15;
constexpr double kIllSlope = 1e-2;
constexpr double kTieRel = 1e-12;

struct cd {
  double re, im;
};

__device__ __forceinline__ cd mk(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd operator+(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd operator*(cd a, cd b) {
  return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cd operator*(double s, cd a) { return cd{s * a.re, s * a.im}; }
__device__ __forceinline__ double norm2(cd a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ cd conjg(cd a) { return cd{a.re, -a.im}; }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
  double d = norm2(b);
  return cd{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
// a / b and c / b with one reciprocal of |b|^2 (one division instead of four)
__device__ __forceinline__ void cdiv2(cd a, cd c, cd b, cd* qa, cd* qc) {
  const double inv = 1.0 / norm2(b);
  *qa = cd{(a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv};
  *qc = cd{(c.re * b.re + c.im * b.im) * inv, (c.im * b.re - c.re * b.im) * inv};
}
// sinh x and cosh x from one expm1 (half the instructions of the two
// library calls): e^x - e^-x = m + m / (1 + m) with m = e^x - 1, no
// cancellation for either sign; exact at x = 0
__device__ __forceinline__ void sinh_cosh(double x, double* sh, double* ch) {
  const double m = expm1(x);
  const double e = 1.0 + m;
  const double ie = 1.0 / e;
  *sh = 0.5 * (m + m * ie);
  *ch = 0.5 * (e + ie);
}
// principal square root (Re >= 0), cancellation-free form
__device__ __forceinline__ cd csqrt_p(cd z) {
  double ax = fabs(z.re);
  double r = sqrt(z.re * z.re + z.im * z.im);
  if (r == 0.0) return cd{0.0, 0.0};
  double t = sqrt(0.5 * (ax + r));
  if (z.re >= 0.0) return cd{t, z.im / (2.0 * t)};
  return cd{fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

// complex moduli of one class
struct Medium {
  cd a11, a13, a33, a44, a66;
  bool elastic_ps, elastic_sh;
  bool fluid;  // no shear stiffness and a11 = a13 = a33: isotropic fluid
  double tilt;
};

__device__ __forceinline__ cd complex_modulus(double aR, double q) {
  double aI = isinf(q) ? 0.0 : aR / q;
  return cd{aR, -aI};
}

__device__ __forceinline__ Medium load_medium(const chert_class& c) {
  Medium m;
  m.a11 = complex_modulus(c.a11, c.q11);
  m.a13 = complex_modulus(c.a13, c.q13);
  m.a33 = complex_modulus(c.a33, c.q33);
  m.a44 = complex_modulus(c.a44, c.q44);
  m.a66 = complex_modulus(c.a66, c.q66);
  m.elastic_ps = m.a11.im == 0.0 && m.a13.im == 0.0 && m.a33.im == 0.0 && m.a44.im == 0.0;
  m.elastic_sh = m.a44.im == 0.0 && m.a66.im == 0.0;
  m.fluid = m.a44.re == 0.0 && m.a44.im == 0.0 && m.a66.re == 0.0 && m.a66.im == 0.0 &&
            m.a11.re == m.a13.re && m.a11.im == m.a13.im && m.a11.re == m.a33.re &&
            m.a11.im == m.a33.im;
  m.tilt = c.tilt;
  return m;
}

__device__ __forceinline__ bool mode_elastic(const Medium& m, int mode) {
  return mode == CHERT_QSH ? m.elastic_sh : m.elastic_ps;
}

// Modes whose homogeneous solution is theta_I = 0 exactly: elastic modes and
// qP of an isotropic fluid (its residual is cubic in theta_I, so a numerical
// root would only be determined to ~1e-6 rad).
__device__ __forceinline__ bool theta_i_zero(const Medium& m, int mode) {
  return mode_elastic(m, mode) || (mode == CHERT_QP && m.fluid);
}

// complex energy velocity (local frame): v = (v1, v3)
struct Vel {
  cd v1, v3;
};

// sin, cos of theta_R and sinh, cosh of theta_I: the only transcendental
// inputs of the evaluation, so loops that hold theta_R (the theta_I scan)
// or step it by a fixed amount (difference quotients) compute them once
struct Trig {
  double sr, cr, sh, ch;
};

__device__ __forceinline__ Trig trig_of(double thR, double thI) {
  Trig t;
  sincos(thR, &t.sr, &t.cr);
  sinh_cosh(thI, &t.sh, &t.ch);
  return t;
}

// difference-quotient step kFdEps in theta_R or theta_I by the addition
// formulas (sine, cosine, sinh, cosh of the double nearest 1e-7)
constexpr double kFdEps = 1e-7;
constexpr double kSinEps = 9.999999999999982e-08, kCosEps = 0.999999999999995;
constexpr double kSinhEps = 1.0000000000000015e-07, kCoshEps = 1.000000000000005;
__device__ __forceinline__ Trig step_re(const Trig& t) {
  return Trig{t.sr * kCosEps + t.cr * kSinEps, t.cr * kCosEps - t.sr * kSinEps, t.sh, t.ch};
}
__device__ __forceinline__ Trig step_im(const Trig& t) {
  return Trig{t.sr, t.cr, t.sh * kCoshEps + t.ch * kSinhEps, t.ch * kCoshEps + t.sh * kSinhEps};
}

__device__ __forceinline__ Vel energy_velocity_t(const Medium& m, int mode, int kernel,
                                                 const Trig& t) {
  const double sr = t.sr, cr = t.cr, sh = t.sh, ch = t.ch;
  cd n1 = cd{sr * ch, cr * sh};   // sin(z)
  cd n3 = cd{cr * ch, -sr * sh};  // cos(z)
  cd n11 = n1 * n1, n33 = n3 * n3;
  Vel out;
  if (mode == CHERT_QSH) {
    cd G = m.a66 * n11 + m.a44 * n33;
    cd c = csqrt_p(G);
    cd p1, p3;
    cdiv2(n1, n3, c, &p1, &p3);
    out.v1 = m.a66 * p1;
    out.v3 = m.a44 * p3;
    return out;
  }
  cd G11 = m.a11 * n11 + m.a44 * n33;
  cd G33 = m.a44 * n11 + m.a33 * n33;
  cd a1344 = m.a13 + m.a44;
  cd G13 = a1344 * (n1 * n3);
  cd mean = 0.5 * (G11 + G33);
  cd half = 0.5 * (G11 - G33);
  cd root = csqrt_p(half * half + G13 * G13);
  cd G = (mode == CHERT_QP) ? mean + root : mean - root;
  cd ua = G13, ub = G - G11;
  cd wa = G - G33, wb = G13;
  double nu = norm2(ua) + norm2(ub);
  double nw = norm2(wa) + norm2(wb);
  cd g1 = (nu >= nw) ? ua : wa;
  cd g3 = (nu >= nw) ? ub : wb;
  cd c = csqrt_p(G);
  cd p1, p3;
  cdiv2(n1, n3, c, &p1, &p3);
  if (kernel == CHERT_KERNEL_OEV) {
    cd N = g1 * g1 + g3 * g3;
    cd S11 = cdiv(g1 * g1, N);
    cd S33 = cdiv(g3 * g3, N);
    cd S13 = cdiv(g1 * g3, N);
    out.v1 = p1 * (m.a11 * S11 + m.a44 * S33) + p3 * (a1344 * S13);
    out.v3 = p3 * (m.a33 * S33 + m.a44 * S11) + p1 * (a1344 * S13);
    return out;
  }
  // MEV: S = Re(g g^H) / (g^H g) is real, so moduli scale by reals
  double q1 = norm2(g1), q3 = norm2(g3);
  const double invN = 1.0 / (q1 + q3);
  const double S11 = q1 * invN, S33 = q3 * invN;
  const double S13 = (g1.re * g3.re + g1.im * g3.im) * invN;
  const cd B = S13 * a1344;
  out.v1 = p1 * (S11 * m.a11 + S33 * m.a44) + p3 * B;
  out.v3 = p3 * (S33 * m.a33 + S11 * m.a44) + p1 * B;
  return out;
}

__device__ __forceinline__ Vel energy_velocity(const Medium& m, int mode, int kernel,
                                               double thR, double thI) {
  return energy_velocity_t(m, mode, kernel, trig_of(thR, thI));
}

// sine of the angle between v^R and v^I (eq 9): zero when collinear
__device__ __forceinline__ double homog_residual(const Vel& v) {
  double r1 = v.v1.re, r3 = v.v3.re, i1 = v.v1.im, i3 = v.v3.im;
  return (r1 * i3 - r3 * i1) / sqrt((r1 * r1 + r3 * r3) * (i1 * i1 + i3 * i3));
}

__device__ __forceinline__ double ray_angle(const Vel& v) { return atan2(v.v1.re, v.v3.re); }

// angle of w minus angle of v for nearly parallel v, w (difference
// quotients): the tangent of the difference, exact to third order
__device__ __forceinline__ double dangle(const Vel& v, const Vel& w) {
  return (v.v3.re * w.v1.re - v.v1.re * w.v3.re) / (v.v1.re * w.v1.re + v.v3.re * w.v3.re);
}

// into (-pi, pi]
__device__ __forceinline__ double wrap_pi(double a) {
  if (a > kPi) a -= kTwoPi;
  else if (a <= -kPi) a += kTwoPi;
  return a;
}

__device__ __forceinline__ double h_at(const Medium& m, int mode, int kernel, double thR,
                                       double thI) {
  return homog_residual(energy_velocity(m, mode, kernel, thR, thI));
}

// residual at theta_R with sine/cosine (sr, cr) and theta_I with (sh, ch)
__device__ __forceinline__ double h_t(const Medium& m, int mode, int kernel, double sr, double cr,
                                      double sh, double ch) {
  return homog_residual(energy_velocity_t(m, mode, kernel, Trig{sr, cr, sh, ch}));
}

// the outward scan's residuals at +-(k + 1) kThiStep (sinh is odd, cosh
// even: one sinh_cosh for both sides)
__device__ __forceinline__ void h_scan_pair(const Medium& m, int mode, int kernel, double sr,
                                            double cr, int k, double* hp, double* hn) {
  double sb, cb;
  sinh_cosh((k + 1) * kThiStep, &sb, &cb);
  *hp = h_t(m, mode, kernel, sr, cr, sb, cb);
  *hn = h_t(m, mode, kernel, sr, cr, -sb, cb);
}

__device__ __forceinline__ bool brackets(double fa, double fb) {
  if (isnan(fa) || isnan(fb)) return false;
  return (fa < 0.0) != (fb < 0.0);
}

// Illinois (modified regula falsi) on a bracket [a, b] of h(thR, .);
// (sr, cr) = sine and cosine of thR
__device__ __forceinline__ double refine_thi(const Medium& m, int mode, int kernel, double sr,
                                             double cr, double a, double b, double fa,
                                             double fb) {
  int side = 0;
  double c = 0.5 * (a + b);
  for (int it = 0; it < 80; ++it) {
    double cn = (a * fb - b * fa) / (fb - fa);
    if (!(cn > fmin(a, b) && cn < fmax(a, b))) cn = 0.5 * (a + b);
    double shc, chc;
    sinh_cosh(cn, &shc, &chc);
    double fc = h_t(m, mode, kernel, sr, cr, shc, chc);
    double step = fabs(cn - c);
    c = cn;
    if (fc == 0.0) break;
    if ((fc < 0.0) == (fa < 0.0)) {
      a = c;
      fa = fc;
      if (side == -1) fb *= 0.5;
      side = -1;
    } else {
      b = c;
      fb = fc;
      if (side == 1) fa *= 0.5;
      side = 1;
    }
    if (fabs(b - a) <= kThiTol || step <= 1e-17) break;
  }
  return c;
}

// theta_I(theta_R): root of the homogeneity residual nearest 0 in [-30, 30]
// deg, found by an outward 0.25-degree scan.  Returns false if none.
// Written for wavefront lockstep: every lane first scans until the whole
// wavefront has its bracket, then all lanes refine together.  (sr, cr) =
// sine and cosine of thR.
__device__ __forceinline__ bool theta_imag_sc(const Medium& m, int mode, int kernel, double sr,
                                              double cr, double* thI) {
  if (theta_i_zero(m, mode)) {
    *thI = 0.0;
    return true;
  }
  double h0 = h_t(m, mode, kernel, sr, cr, 0.0, 1.0);
  bool done = (h0 == 0.0);
  bool bp = false, bn = false;
  double pa = 0.0, pb = 0.0, fpa = 0.0, fpb = 0.0;  // positive-side bracket
  double na = 0.0, nb = 0.0, fna = 0.0, fnb = 0.0;  // negative-side bracket
  double hp_lo = h0, hn_hi = h0;
  for (int k = 0; k < kThiSteps; ++k) {
    if (!done) {
      double a = k * kThiStep, b = (k + 1) * kThiStep;
      double hp_hi, hn_lo;
      h_scan_pair(m, mode, kernel, sr, cr, k, &hp_hi, &hn_lo);
      bp = brackets(hp_lo, hp_hi);
      bn = brackets(hn_lo, hn_hi);
      if (bp) { pa = a; pb = b; fpa = hp_lo; fpb = hp_hi; }
      if (bn) { na = -b; nb = -a; fna = hn_lo; fnb = hn_hi; }
      done = bp || bn;
      hp_lo = hp_hi;
      hn_hi = hn_lo;
    }
    if (__all(done)) break;
  }
  if (h0 == 0.0) {
    *thI = 0.0;
    return true;
  }
  if (!bp && !bn) return false;
  double rp = bp ? refine_thi(m, mode, kernel, sr, cr, pa, pb, fpa, fpb) : 0.0;
  double rn = bn ? refine_thi(m, mode, kernel, sr, cr, na, nb, fna, fnb) : 0.0;
  if (bp && bn) *thI = (fabs(rn) < fabs(rp)) ? rn : rp;
  else *thI = bp ? rp : rn;
  return true;
}

__device__ __forceinline__ bool theta_imag(const Medium& m, int mode, int kernel, double thR,
                                           double* thI) {
  double sr, cr;
  sincos(thR, &sr, &cr);
  return theta_imag_sc(m, mode, kernel, sr, cr, thI);
}

// ray angle at (thR, thI) given sin, cos of thR
__device__ __forceinline__ double ray_angle_sc(const Medium& m, int mode, int kernel, double sr,
                                               double cr, double thI) {
  double sh, ch;
  sinh_cosh(thI, &sh, &ch);
  return ray_angle(energy_velocity_t(m, mode, kernel, Trig{sr, cr, sh, ch}));
}

struct Entry {
  double V, A, Q, r1, r3, thR, thI, res;
};

// ray quantities from a homogeneous complex energy velocity (eqs 10-11)
__device__ __forceinline__ void ray_quantities(const Vel& v, Entry* e) {
  double r1 = v.v1.re, r3 = v.v3.re, i1 = v.v1.im, i3 = v.v3.im;
  double vr = sqrt(r1 * r1 + r3 * r3);
  double u1 = r1 / vr, u3 = r3 / vr;
  double vi = i1 * u1 + i3 * u3;
  double s = vr * vr + vi * vi;
  e->V = s / vr;
  e->A = -vi / s;
  e->Q = (vi == 0.0) ? INFINITY : -(vr * vr - vi * vi) / (2.0 * vr * vi);
  e->r1 = u1;
  e->r3 = u3;
}

}  // namespace chert
