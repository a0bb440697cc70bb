/*
 * CHERT CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 implementation of what the CHERT hot
 * path computes (Darwis, Bouchaala, Waheed, Riahi: "CHERT: Cached
 * Hamiltonian-Enhanced Ray Tracing in Viscoelastic Anisotropic Media").
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no source, header, table or helper with the HIP
 * library, and the library never calls it.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fPIC -shared -lm
 *
 * Conventions (all SI; angles in radians):
 *   - 2D frame: x to the right, z down; angles are measured from +z towards +x,
 *     so the unit vector at angle a is (sin a, cos a) in (x, z).
 *   - Symmetry axis of a tilted class: e_z' = (sin t0, cos t0) (eq 36), so a
 *     global angle a is the local angle a - t0.
 *   - Node index = ix + nx*iz.
 *   - A class is 13 doubles: a11 a13 a33 a44 a66 (real density-normalised
 *     moduli, m^2/s^2), q11 q13 q33 q44 q66 (quality factors, INFINITY =
 *     elastic), rho (kept, unused by kinematics), tilt, azimuth.
 *
 * Readings of the paper that this file takes (the paper leaves them open):
 *   - MEV (eq 14): the gradient of eq 13 with the eigenvector g and its
 *     conjugate held fixed, symmetrised:  v_m = a_mjkl p_l Re(g_j g_k^*)/(g^H g).
 *     OEV (eq 12): v_m = a_mjkl p_l g_j g_k/(g^T g).
 *   - Per-component Q: a_pq = a_pq^R (1 - i/Q_pq) (eq 2).
 *   - The imaginary slowness angle is the root of the homogeneity residual
 *     nearest zero inside [-30 deg, 30 deg] (the search bracket of the local
 *     benchmark section).  A mode whose moduli are all real is elastic:
 *     theta_I = 0 exactly.
 *   - The cache is indexed by ray direction: entry d holds the solution whose
 *     ray direction is exactly d * 360/n_dirs degrees (global frame).  Where
 *     several slowness angles give that ray direction (qSV triplication) the
 *     one with the largest ray velocity (first arrival) is kept.
 *   - Entries d >= n_dirs/2 are the centrosymmetric copies of d - n_dirs/2.
 *   - Edge weights: endpoint-averaged velocity and attenuation (eqs 28-30) at
 *     the bin of the edge direction; propagation and attenuation are two
 *     independent shortest-path problems (eqs 24, 31).
 *   - Predecessors: the tight neighbour with the fewest BFS hops over tight
 *     edges, then the lowest offset index (forward star) or node index (cell
 *     network); t* folds the attenuation weights along that tree.
 *   - Cell network (O-18): nodes on cell edges, every boundary pair of a cell
 *     a segment; the block marching is re-entrant (a cell returns to the heap
 *     whenever one of its nodes improves).  In 3D (O-20) the cells are blocks
 *     and the nodes lie on their faces.
 *   - MSPM (O-19): corner quantities solved at the segment's exact
 *     direction; nodes between two corners interpolate them linearly.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_PI 3.14159265358979323846

enum { ORC_QP = 0, ORC_QSV = 1, ORC_QSH = 2 };
enum { ORC_MEV = 0, ORC_OEV = 1 };

/* entry status bits */
enum {
  ORC_ST_OK = 0,
  ORC_ST_NO_BRACKET = 1,  /* no slowness angle reaches the target ray direction */
  ORC_ST_ILL = 2,         /* chosen root sits where d(psi)/d(theta_R) is tiny  */
  ORC_ST_FLUID = 4,       /* shear mode in a medium without shear stiffness     */
  ORC_ST_NONPHYS = 8,     /* negative attenuation or non-finite ray quantities  */
  ORC_ST_NOCONV = 16      /* the root's residual is above ORC_RESID_TOL          */
};

/* output fields of one cache entry */
enum { F_V = 0, F_A, F_Q, F_RX, F_RZ, F_THR, F_THI, F_RES, ORC_NF };

#define ORC_THI_STEP (0.25 * ORC_PI / 180.0) /* outward scan step for theta_I */
#define ORC_THI_MAX_STEPS 120                /* 120 * 0.25 deg = 30 deg      */
#define ORC_THI_TOL 1e-15                    /* bisection width for theta_I  */
#define ORC_THR_TOL 1e-14                    /* bisection width for theta_R  */
#define ORC_ILL_SLOPE 1e-2                   /* |dpsi/dtheta_R| flag level   */
#define ORC_TIE_REL 1e-12                    /* equal ray velocities         */
#define ORC_RESID_TOL 1e-9                   /* converged-root residual cap  */

/* ------------------------------------------------------------------------ */
/* O-1  constitutive step (eq 2; Thomsen 1986 for the real part)           */
/* ------------------------------------------------------------------------ */

/* Thomsen (vp0, vs0, eps, delta, gamma) -> a11 a13 a33 a44 a66.
 * Returns 0, or 1 when the a13 radicand is negative. */
int orc_thomsen(double vp0, double vs0, double eps, double delta, double gamma,
                double *a5) {
  double a33 = vp0 * vp0;
  double a44 = vs0 * vs0;
  double rad = 2.0 * delta * a33 * (a33 - a44) + (a33 - a44) * (a33 - a44);
  if (!(rad >= 0.0)) return 1;
  a5[0] = a33 * (1.0 + 2.0 * eps);  /* a11 */
  a5[1] = sqrt(rad) - a44;          /* a13 */
  a5[2] = a33;                      /* a33 */
  a5[3] = a44;                      /* a44 */
  a5[4] = a44 * (1.0 + 2.0 * gamma);/* a66 */
  return 0;
}

typedef struct {
  cplx a11, a13, a33, a44, a66;
  int elastic_ps; /* qP/qSV see only real moduli  */
  int elastic_sh; /* qSH sees only real moduli    */
  int fluid;      /* ideal (visco-)fluid: no shear, a11 = a13 = a33 */
  double tilt;
} medium_t;

static cplx complex_modulus(double aR, double q) {
  /* eq 2: a = a^R - i a^I with a^I = a^R / Q;  Q = inf gives a real modulus */
  double aI = isinf(q) ? 0.0 : aR / q;
  return aR - I * aI;
}

static void load_medium(const double *c, medium_t *m) {
  m->a11 = complex_modulus(c[0], c[5]);
  m->a13 = complex_modulus(c[1], c[6]);
  m->a33 = complex_modulus(c[2], c[7]);
  m->a44 = complex_modulus(c[3], c[8]);
  m->a66 = complex_modulus(c[4], c[9]);
  m->elastic_ps = cimag(m->a11) == 0.0 && cimag(m->a13) == 0.0 &&
                  cimag(m->a33) == 0.0 && cimag(m->a44) == 0.0;
  m->elastic_sh = cimag(m->a44) == 0.0 && cimag(m->a66) == 0.0;
  m->fluid = m->a44 == 0.0 && m->a66 == 0.0 && m->a11 == m->a13 && m->a11 == m->a33;
  m->tilt = c[11];
}

static int mode_elastic(const medium_t *m, int mode) {
  return mode == ORC_QSH ? m->elastic_sh : m->elastic_ps;
}

/* Modes whose homogeneous solution is theta_I = 0 exactly: elastic modes
 * (the residual is 0/0 there) and qP in an ideal fluid, which is isotropic
 * (the visco-isotropic simplification of the cache-construction section);
 * its residual is cubic in theta_I, so a numerical root would only be good
 * to ~1e-6 rad. */
static int theta_i_zero(const medium_t *m, int mode) {
  return mode_elastic(m, mode) || (mode == ORC_QP && m->fluid);
}

/* ------------------------------------------------------------------------ */
/* O-3  complex energy velocity at a trial slowness-angle pair              */
/*      (eqs 4, 5, 7, 12, 14), in the local symmetry-axis frame             */
/* ------------------------------------------------------------------------ */

typedef struct {
  cplx v1, v3;  /* complex energy velocity (x', z') */
  cplx c;       /* complex phase velocity, Re c > 0 */
  cplx g1, g3;  /* eigenvector (unnormalised)        */
  cplx p1, p3;  /* complex slowness                   */
} eval_t;

static void energy_velocity(const medium_t *m, int mode, int reading,
                            double thR, double thI, eval_t *e) {
  cplx z = thR + I * thI;
  cplx n1 = csin(z), n3 = ccos(z); /* eq 7 */
  if (mode == ORC_QSH) {
    /* SH polarisation is e_y: Gamma_22 = a66 n1^2 + a44 n3^2 */
    cplx G = m->a66 * n1 * n1 + m->a44 * n3 * n3;
    cplx c = csqrt(G);
    cplx p1 = n1 / c, p3 = n3 / c; /* eq 5 */
    e->c = c;
    e->g1 = 0.0;
    e->g3 = 0.0;
    e->p1 = p1;
    e->p3 = p3;
    e->v1 = m->a66 * p1; /* a_1221 p_1 */
    e->v3 = m->a44 * p3; /* a_3223 p_3 */
    return;
  }
  /* Christoffel matrix of the sagittal plane for the unit direction n (eq 4) */
  cplx G11 = m->a11 * n1 * n1 + m->a44 * n3 * n3;
  cplx G33 = m->a44 * n1 * n1 + m->a33 * n3 * n3;
  cplx G13 = (m->a13 + m->a44) * n1 * n3;
  cplx mean = 0.5 * (G11 + G33);
  cplx half = 0.5 * (G11 - G33);
  cplx root = csqrt(half * half + G13 * G13);
  cplx G = (mode == ORC_QP) ? mean + root : mean - root; /* qP: larger Re */
  /* eigenvector: the better-conditioned of the two null-space forms */
  cplx ua = G13, ub = G - G11;   /* from row 1 */
  cplx wa = G - G33, wb = G13;   /* from row 2 */
  double nu = creal(ua * conj(ua)) + creal(ub * conj(ub));
  double nw = creal(wa * conj(wa)) + creal(wb * conj(wb));
  cplx g1, g3;
  if (nu >= nw) {
    g1 = ua;
    g3 = ub;
  } else {
    g1 = wa;
    g3 = wb;
  }
  cplx c = csqrt(G);               /* G = c^2; principal root has Re c > 0 */
  cplx p1 = n1 / c, p3 = n3 / c;   /* eq 5 */
  cplx S11, S33, S13;
  if (reading == ORC_OEV) {
    cplx N = g1 * g1 + g3 * g3;    /* g^T g */
    S11 = g1 * g1 / N;
    S33 = g3 * g3 / N;
    S13 = g1 * g3 / N;
  } else {
    double N = creal(g1 * conj(g1)) + creal(g3 * conj(g3)); /* g^H g */
    S11 = creal(g1 * conj(g1)) / N;
    S33 = creal(g3 * conj(g3)) / N;
    S13 = creal(g1 * conj(g3)) / N;
  }
  /* v_m = a_mjkl p_l S_jk with the TI tensor (a_1111=a11, a_3333=a33,
   * a_1133=a13, a_1313=a44) */
  e->v1 = p1 * (m->a11 * S11 + m->a44 * S33) + p3 * (m->a13 + m->a44) * S13;
  e->v3 = p3 * (m->a33 * S33 + m->a44 * S11) + p1 * (m->a13 + m->a44) * S13;
  e->c = c;
  e->g1 = g1;
  e->g3 = g3;
  e->p1 = p1;
  e->p3 = p3;
}

/* Exported for tests: out = vR1 vR3 vI1 vI3 cR cI g1R g1I g3R g3I p1R p1I p3R p3I */
int orc_velocity(const double *cls, int mode, int reading, double thR,
                 double thI, double *out) {
  medium_t m;
  eval_t e;
  load_medium(cls, &m);
  energy_velocity(&m, mode, reading, thR, thI, &e);
  out[0] = creal(e.v1);
  out[1] = creal(e.v3);
  out[2] = cimag(e.v1);
  out[3] = cimag(e.v3);
  out[4] = creal(e.c);
  out[5] = cimag(e.c);
  out[6] = creal(e.g1);
  out[7] = cimag(e.g1);
  out[8] = creal(e.g3);
  out[9] = cimag(e.g3);
  out[10] = creal(e.p1);
  out[11] = cimag(e.p1);
  out[12] = creal(e.p3);
  out[13] = cimag(e.p3);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O-4  homogeneity residual (eq 9) and local ray angle                     */
/* ------------------------------------------------------------------------ */

/* sine of the angle between v^R and v^I: zero when they are collinear */
static double homog_residual(const eval_t *e) {
  double r1 = creal(e->v1), r3 = creal(e->v3);
  double i1 = cimag(e->v1), i3 = cimag(e->v3);
  double nr = sqrt(r1 * r1 + r3 * r3), ni = sqrt(i1 * i1 + i3 * i3);
  return (r1 * i3 - r3 * i1) / (nr * ni);
}

static double ray_angle_local(const eval_t *e) {
  return atan2(creal(e->v1), creal(e->v3));
}

double orc_residual(const double *cls, int mode, int reading, double thR,
                    double thI) {
  medium_t m;
  eval_t e;
  load_medium(cls, &m);
  energy_velocity(&m, mode, reading, thR, thI, &e);
  return homog_residual(&e);
}

/* ------------------------------------------------------------------------ */
/* O-5  root searches                                                       */
/* ------------------------------------------------------------------------ */

static double h_at(const medium_t *m, int mode, int reading, double thR,
                   double thI) {
  eval_t e;
  energy_velocity(m, mode, reading, thR, thI, &e);
  return homog_residual(&e);
}

/* plain bisection of h(thR, .) on [lo, hi] with h(lo), h(hi) of opposite
 * sign classes (negative / non-negative) */
static double bisect_thi(const medium_t *m, int mode, int reading, double thR,
                         double lo, double hi, double hlo) {
  int neg_lo = hlo < 0.0;
  for (int it = 0; it < 200 && hi - lo > ORC_THI_TOL; ++it) {
    double mid = 0.5 * (lo + hi);
    double hm = h_at(m, mode, reading, thR, mid);
    if ((hm < 0.0) == neg_lo) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* does [a, b] with residuals ha, hb bracket a root?  (zero counts as
 * non-negative, so a root exactly on a sample is bracketed exactly once) */
static int brackets(double ha, double hb) {
  if (isnan(ha) || isnan(hb)) return 0;
  return (ha < 0.0) != (hb < 0.0);
}

/* theta_I(theta_R): the root of the homogeneity residual nearest zero in
 * [-30 deg, 30 deg], found by scanning outwards from 0 in 0.25 deg steps.
 * Returns 0 on success, 1 when there is no root in the bracket. */
static int theta_imag(const medium_t *m, int mode, int reading, double thR,
                      double *thI) {
  if (theta_i_zero(m, mode)) {
    *thI = 0.0;
    return 0;
  }
  double h0 = h_at(m, mode, reading, thR, 0.0);
  if (h0 == 0.0) {
    *thI = 0.0;
    return 0;
  }
  double hp_lo = h0, hn_hi = h0; /* residuals at +k*step and -k*step */
  for (int k = 0; k < ORC_THI_MAX_STEPS; ++k) {
    double a = k * ORC_THI_STEP, b = (k + 1) * ORC_THI_STEP;
    double hp_hi = h_at(m, mode, reading, thR, b);
    double hn_lo = h_at(m, mode, reading, thR, -b);
    int bp = brackets(hp_lo, hp_hi);
    int bn = brackets(hn_lo, hn_hi);
    double rp = 0.0, rn = 0.0;
    if (bp) rp = bisect_thi(m, mode, reading, thR, a, b, hp_lo);
    if (bn) rn = bisect_thi(m, mode, reading, thR, -b, -a, hn_lo);
    if (bp && bn) {
      *thI = (fabs(rn) < fabs(rp)) ? rn : rp;
      return 0;
    }
    if (bp) { *thI = rp; return 0; }
    if (bn) { *thI = rn; return 0; }
    hp_lo = hp_hi;
    hn_hi = hn_lo;
  }
  return 1;
}

int orc_theta_imag(const double *cls, int mode, int reading, double thR,
                   double *thI) {
  medium_t m;
  load_medium(cls, &m);
  return theta_imag(&m, mode, reading, thR, thI);
}

static double wrap_pi(double a) {
  /* into (-pi, pi] */
  while (a > ORC_PI) a -= 2.0 * ORC_PI;
  while (a <= -ORC_PI) a += 2.0 * ORC_PI;
  return a;
}

typedef struct {
  double thR, thI, psi;
  int ok;
} sample_t;

/* the theta_R sweep: M samples at (j + 1/2) * 2 pi / M */
static void sweep(const medium_t *m, int mode, int reading, int M,
                  sample_t *tab) {
  for (int j = 0; j < M; ++j) {
    double thR = (j + 0.5) * (2.0 * ORC_PI / M);
    double thI = 0.0;
    tab[j].thR = thR;
    tab[j].ok = 0;
    if (theta_imag(m, mode, reading, thR, &thI) != 0) continue;
    eval_t e;
    energy_velocity(m, mode, reading, thR, thI, &e);
    double psi = ray_angle_local(&e);
    if (!isfinite(psi)) continue;
    tab[j].thI = thI;
    tab[j].psi = psi;
    tab[j].ok = 1;
  }
}

typedef struct {
  double thR, thI, V, A, Q, r1, r3, res;
} entry_t;

/* O-6: ray quantities from the homogeneous complex energy velocity (eqs 10-11) */
static void ray_quantities(const eval_t *e, entry_t *out) {
  double r1 = creal(e->v1), r3 = creal(e->v3);
  double i1 = cimag(e->v1), i3 = cimag(e->v3);
  double vr = sqrt(r1 * r1 + r3 * r3);
  double u1 = r1 / vr, u3 = r3 / vr;   /* ray direction */
  double vi = i1 * u1 + i3 * u3;       /* signed v^I along the ray */
  double s = vr * vr + vi * vi;
  out->V = s / vr;
  out->A = -vi / s;
  out->Q = (vi == 0.0) ? INFINITY : -(vr * vr - vi * vi) / (2.0 * vr * vi);
  out->r1 = u1;
  out->r3 = u3;
}

/* evaluate the full solution at theta_R: inner root, velocity, quantities */
static int solution_at(const medium_t *m, int mode, int reading, double thR,
                       double psi_star, entry_t *out) {
  double thI;
  if (theta_imag(m, mode, reading, thR, &thI) != 0) return 1;
  eval_t e;
  energy_velocity(m, mode, reading, thR, thI, &e);
  ray_quantities(&e, out);
  out->thR = thR;
  out->thI = thI;
  double h = theta_i_zero(m, mode) ? 0.0 : homog_residual(&e);
  double dpsi = wrap_pi(ray_angle_local(&e) - psi_star);
  out->res = fmax(fabs(h), fabs(dpsi));
  return 0;
}

static double ang_dist(double a, double b) { return fabs(wrap_pi(a - b)); }

/* solve one target local ray angle psi_star from a sweep table */
static int solve_direction(const medium_t *m, int mode, int reading, int M,
                           const sample_t *tab, double psi_star,
                           entry_t *best) {
  int found = 0, ill = 0;
  for (int j = 0; j < M; ++j) {
    const sample_t *sa = &tab[j];
    const sample_t *sb = &tab[(j + 1) % M];
    if (!sa->ok || !sb->ok) continue;
    double ta = sa->thR;
    double tb = sb->thR + (j == M - 1 ? 2.0 * ORC_PI : 0.0);
    double fa = wrap_pi(sa->psi - psi_star);
    double fb = wrap_pi(sb->psi - psi_star);
    if (fabs(fb - fa) >= ORC_PI) continue; /* the +-pi seam, not a crossing */
    if (!brackets(fa, fb)) continue;
    /* bisection on theta_R; every trial re-solves theta_I */
    double lo = ta, hi = tb;
    int neg_lo = fa < 0.0, failed = 0;
    for (int it = 0; it < 200 && hi - lo > ORC_THR_TOL; ++it) {
      double mid = 0.5 * (lo + hi);
      double thI;
      if (theta_imag(m, mode, reading, mid, &thI) != 0) { failed = 1; break; }
      eval_t e;
      energy_velocity(m, mode, reading, mid, thI, &e);
      double fm = wrap_pi(ray_angle_local(&e) - psi_star);
      if ((fm < 0.0) == neg_lo) lo = mid; else hi = mid;
    }
    if (failed) continue;
    double thR = 0.5 * (lo + hi);
    if (thR >= 2.0 * ORC_PI) thR -= 2.0 * ORC_PI;
    entry_t cand;
    if (solution_at(m, mode, reading, thR, psi_star, &cand) != 0) continue;
    double slope = (fb - fa) / (tb - ta);
    int cand_ill = fabs(slope) < ORC_ILL_SLOPE;
    /* Only a root competes as a root: a bisection that closed on a jump of
     * the ray-angle map (theta_I(theta_R) changing branch inside the
     * bracket) leaves a residual far above ORC_RESID_TOL, and any genuine
     * root is preferred to it.  Among roots, the first arrival (largest
     * V^Ray) wins, equal velocities going to the smaller |theta_R - psi*|. */
    int cand_root = cand.res <= ORC_RESID_TOL;
    int best_root = found && best->res <= ORC_RESID_TOL;
    int take = 0;
    if (!found) {
      take = 1;
    } else if (cand_root != best_root) {
      take = cand_root;
    } else if (cand.V > best->V * (1.0 + ORC_TIE_REL)) {
      take = 1;
    } else if (fabs(cand.V - best->V) <= ORC_TIE_REL * best->V &&
               ang_dist(cand.thR, psi_star) < ang_dist(best->thR, psi_star)) {
      take = 1;
    }
    if (take) {
      *best = cand;
      ill = cand_ill;
      found = 1;
    }
  }
  if (!found) return ORC_ST_NO_BRACKET;
  return ill ? ORC_ST_ILL : ORC_ST_OK;
}

static void rotate_to_global(double tilt, double l1, double l3, double *gx,
                             double *gz) {
  /* x = x' cos t0 + z' sin t0 ;  z = -x' sin t0 + z' cos t0  (eq 36) */
  *gx = l1 * cos(tilt) + l3 * sin(tilt);
  *gz = -l1 * sin(tilt) + l3 * cos(tilt);
}

static void write_entry(double *fields, long stride, long idx,
                        const entry_t *e, double tilt) {
  double gx, gz;
  rotate_to_global(tilt, e->r1, e->r3, &gx, &gz);
  fields[F_V * stride + idx] = e->V;
  fields[F_A * stride + idx] = e->A;
  fields[F_Q * stride + idx] = e->Q;
  fields[F_RX * stride + idx] = gx;
  fields[F_RZ * stride + idx] = gz;
  fields[F_THR * stride + idx] = e->thR;
  fields[F_THI * stride + idx] = e->thI;
  fields[F_RES * stride + idx] = e->res;
}

static void write_invalid(double *fields, long stride, long idx) {
  for (int f = 0; f < ORC_NF; ++f) fields[f * stride + idx] = NAN;
}

/* Solve a single target local ray angle (test helper).  out = 8 fields in
 * the F_* order with the direction left in the local frame; returns status. */
int orc_solve(const double *cls, int mode, int reading, int n_sweep,
              double psi_star_local, double *out) {
  medium_t m;
  load_medium(cls, &m);
  sample_t *tab = (sample_t *)malloc(sizeof(sample_t) * (size_t)n_sweep);
  if (!tab) return -1;
  sweep(&m, mode, reading, n_sweep, tab);
  entry_t e;
  int st = solve_direction(&m, mode, reading, n_sweep, tab, psi_star_local, &e);
  free(tab);
  if (st & ORC_ST_NO_BRACKET) {
    for (int f = 0; f < ORC_NF; ++f) out[f] = NAN;
    return st;
  }
  out[F_V] = e.V;
  out[F_A] = e.A;
  out[F_Q] = e.Q;
  out[F_RX] = e.r1;
  out[F_RZ] = e.r3;
  out[F_THR] = e.thR;
  out[F_THI] = e.thI;
  out[F_RES] = e.res;
  return st;
}

/* Sweep table export for tests: thR, thI, psi, ok per sample. */
int orc_sweep(const double *cls, int mode, int reading, int n_sweep,
              double *thR, double *thI, double *psi, int *ok) {
  medium_t m;
  load_medium(cls, &m);
  sample_t *tab = (sample_t *)malloc(sizeof(sample_t) * (size_t)n_sweep);
  if (!tab) return -1;
  sweep(&m, mode, reading, n_sweep, tab);
  for (int j = 0; j < n_sweep; ++j) {
    thR[j] = tab[j].thR;
    thI[j] = tab[j].ok ? tab[j].thI : NAN;
    psi[j] = tab[j].ok ? tab[j].psi : NAN;
    ok[j] = tab[j].ok;
  }
  free(tab);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O-7  the directional cache C(m, k, theta) (eq 26)                        */
/* ------------------------------------------------------------------------ */

/* fields: [ORC_NF][3 modes][n_classes][n_cols]; status: [3][n_classes][n_cols].
 * subset (ascending directions, closed under d -> d + n_dirs/2) selects the
 * stored columns; NULL means every direction (n_cols = n_dirs).  Modes
 * outside mode_mask are left untouched. */
int orc_build_cache_2d_cols(const double *classes, long n_classes, int n_dirs,
                            const int32_t *subset, int n_subset,
                            unsigned mode_mask, int reading, int n_sweep,
                            double *fields, int32_t *status) {
  if (n_dirs <= 0 || (n_dirs & 1) || n_sweep < 8) return 1;
  int n_cols = subset ? n_subset : n_dirs;
  int half = n_dirs / 2;
  /* columns of each direction (-1: not stored) */
  int *col = (int *)malloc(sizeof(int) * (size_t)n_dirs);
  if (!col) return 2;
  for (int d = 0; d < n_dirs; ++d) col[d] = subset ? -1 : d;
  if (subset)
    for (int q = 0; q < n_subset; ++q) col[subset[q]] = q;
  for (int d = 0; d < half; ++d)
    if ((col[d] < 0) != (col[d + half] < 0)) { free(col); return 3; }
  long stride = 3L * n_classes * n_cols;
  sample_t *tab = (sample_t *)malloc(sizeof(sample_t) * (size_t)n_sweep);
  if (!tab) { free(col); return 2; }
  for (int mode = 0; mode < 3; ++mode) {
    if (!(mode_mask & (1u << mode))) continue;
    for (long k = 0; k < n_classes; ++k) {
      const double *cls = classes + 13 * k;
      medium_t m;
      load_medium(cls, &m);
      long base = ((long)mode * n_classes + k) * n_cols;
      int fluid = (mode != ORC_QP) && (cls[3] == 0.0 || (mode == ORC_QSH && cls[4] == 0.0));
      if (fluid) {
        for (int c = 0; c < n_cols; ++c) {
          write_invalid(fields, stride, base + c);
          status[base + c] = ORC_ST_FLUID;
        }
        continue;
      }
      sweep(&m, mode, reading, n_sweep, tab);
      for (int d = 0; d < half; ++d) {
        if (col[d] < 0) continue;
        long e0 = base + col[d], e1 = base + col[d + half];
        double psi_global = d * (2.0 * ORC_PI / n_dirs);
        double psi_star = wrap_pi(psi_global - m.tilt);
        entry_t e;
        int st = solve_direction(&m, mode, reading, n_sweep, tab, psi_star, &e);
        if (st & ORC_ST_NO_BRACKET) {
          write_invalid(fields, stride, e0);
          write_invalid(fields, stride, e1);
          status[e0] = st;
          status[e1] = st;
          continue;
        }
        if (!(e.A >= 0.0) || !isfinite(e.V) || !(e.V > 0.0)) st |= ORC_ST_NONPHYS;
        if (!(e.res <= ORC_RESID_TOL)) st |= ORC_ST_NOCONV;
        write_entry(fields, stride, e0, &e, m.tilt);
        status[e0] = st;
        /* centrosymmetric copy: the reversed ray direction has the same
         * ray quantities; the slowness direction turns by pi */
        entry_t r = e;
        r.thR = e.thR + ORC_PI;
        if (r.thR >= 2.0 * ORC_PI) r.thR -= 2.0 * ORC_PI;
        write_entry(fields, stride, e1, &r, m.tilt);
        /* exact negation of the already-rotated direction */
        fields[F_RX * stride + e1] = -fields[F_RX * stride + e0];
        fields[F_RZ * stride + e1] = -fields[F_RZ * stride + e0];
        status[e1] = st;
      }
    }
  }
  free(tab);
  free(col);
  return 0;
}

int orc_build_cache_2d(const double *classes, long n_classes, int n_dirs,
                       unsigned mode_mask, int reading, int n_sweep,
                       double *fields, int32_t *status) {
  return orc_build_cache_2d_cols(classes, n_classes, n_dirs, NULL, 0, mode_mask,
                                 reading, n_sweep, fields, status);
}

/* ------------------------------------------------------------------------ */
/* O-8  forward star, edge lengths and direction bins (eq 27)               */
/* ------------------------------------------------------------------------ */

static int gcd_int(int a, int b) {
  a = abs(a);
  b = abs(b);
  while (b) {
    int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

/* Offsets o with max(|ox|,|oz|) <= R and gcd(|ox|,|oz|) = 1, ordered by
 * (oz, ox) ascending.  Returns the count (arrays may be NULL to count).
 * bin(o) is the tabulated direction nearest to the edge (eq 27 and the
 * cache lookup after it).  An edge exactly half-way between two tabulated
 * directions is decided on the half-plane of angles [0, pi) -- rounding
 * half away from zero there -- and an offset in the other half-plane takes
 * the direction opposite to its reverse's, so that an edge and its reverse
 * always read diametrically opposite directions. */
static int32_t bin_2d(int x, int z, double hx, double hz, int n_dirs) {
  double dx = x * hx, dz = z * hz;
  int upper = (x > 0) || (x == 0 && z > 0); /* angle in [0, pi) */
  double ang = upper ? atan2(dx, dz) : atan2(-dx, -dz); /* from +z to +x */
  long b = lround(ang * n_dirs / (2.0 * ORC_PI));
  if (!upper) b = b + n_dirs / 2;
  b = ((b % n_dirs) + n_dirs) % n_dirs;
  return (int32_t)b;
}

int orc_star_2d(int R, double hx, double hz, int n_dirs, int32_t *ox,
                int32_t *oz, double *L, int32_t *bin) {
  int n = 0;
  for (int z = -R; z <= R; ++z) {
    for (int x = -R; x <= R; ++x) {
      if (x == 0 && z == 0) continue;
      if (gcd_int(x, z) != 1) continue;
      if (ox) {
        double dx = x * hx, dz = z * hz;
        ox[n] = x;
        oz[n] = z;
        L[n] = sqrt(dx * dx + dz * dz);
        bin[n] = bin_2d(x, z, hx, hz, n_dirs);
      }
      ++n;
    }
  }
  return n;
}

/* ------------------------------------------------------------------------ */
/* O-9 .. O-12  edge weights, Dijkstra, predecessors, t*                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  double key;
  long node;
} heap_item;

typedef struct {
  heap_item *a;
  long n, cap;
} heap_t;

static int heap_push(heap_t *h, double key, long node) {
  if (h->n == h->cap) {
    long nc = h->cap ? 2 * h->cap : 1024;
    heap_item *na = (heap_item *)realloc(h->a, sizeof(heap_item) * (size_t)nc);
    if (!na) return 1;
    h->a = na;
    h->cap = nc;
  }
  long i = h->n++;
  h->a[i].key = key;
  h->a[i].node = node;
  while (i > 0) {
    long p = (i - 1) / 2;
    if (h->a[p].key <= h->a[i].key) break;
    heap_item t = h->a[p];
    h->a[p] = h->a[i];
    h->a[i] = t;
    i = p;
  }
  return 0;
}

static heap_item heap_pop(heap_t *h) {
  heap_item top = h->a[0];
  h->a[0] = h->a[--h->n];
  long i = 0;
  for (;;) {
    long l = 2 * i + 1, r = l + 1, s = i;
    if (l < h->n && h->a[l].key < h->a[s].key) s = l;
    if (r < h->n && h->a[r].key < h->a[s].key) s = r;
    if (s == i) break;
    heap_item t = h->a[s];
    h->a[s] = h->a[i];
    h->a[i] = t;
    i = s;
  }
  return top;
}

typedef struct {
  long nx, nz;
  int n_off;
  const int32_t *ox, *oz, *bin;
  long ny;              /* 1 in 2D */
  const int32_t *oy;    /* NULL in 2D */
  const double *L;
  const int32_t *cls;   /* node -> class; NULL: the class is the node */
  int n_cols;           /* cache columns */
  const int32_t *col;   /* direction -> column */
  const double *V, *A;  /* [class][column] for one mode */
  const int32_t *st;    /* [class][column] */
  const int32_t *best;  /* slowness-sampled caches: [class][offset] column of
                           the closest stored ray direction (-1: none);
                           NULL for ray-direction caches */
} graph_t;

static long class_of(const graph_t *g, long node) {
  return g->cls ? g->cls[node] : node;
}

static int entry_usable(const graph_t *g, long k, int c) {
  int32_t s = g->st[k * g->n_cols + c];
  return !(s & (ORC_ST_NO_BRACKET | ORC_ST_FLUID | ORC_ST_NONPHYS | ORC_ST_NOCONV));
}

/* eq 29 / eq 30 with endpoint averages (eq 28); field 0 = propagation,
 * field 1 = attenuation.  Not usable -> +inf. */
static double edge_weight(const graph_t *g, int field, long i, long j, int o) {
  long ki = class_of(g, i), kj = class_of(g, j);
  int ci, cj;
  if (g->best) { /* each endpoint its own closest stored direction */
    ci = g->best[ki * g->n_off + o];
    cj = g->best[kj * g->n_off + o];
    if (ci < 0 || cj < 0) return INFINITY;
  } else {
    ci = cj = g->col[g->bin[o]];
  }
  if (!entry_usable(g, ki, ci) || !entry_usable(g, kj, cj)) return INFINITY;
  if (field == 0) {
    double vbar = 0.5 * (g->V[ki * g->n_cols + ci] + g->V[kj * g->n_cols + cj]);
    return g->L[o] / vbar;
  }
  double abar = 0.5 * (g->A[ki * g->n_cols + ci] + g->A[kj * g->n_cols + cj]);
  return g->L[o] * abar;
}

/* node index ix + nx (iy + ny iz): x fastest, then y, then z (2D: ny = 1) */
static long node_at(const graph_t *g, long x, long y, long z) {
  if (x < 0 || x >= g->nx || y < 0 || y >= g->ny || z < 0 || z >= g->nz) return -1;
  return x + g->nx * (y + g->ny * z);
}

/* neighbour j = i + s o (s = +1 forward, -1 backward; in-grid) or -1 */
static long step_dir(const graph_t *g, long i, int o, int s) {
  long ix = i % g->nx, r = i / g->nx, iy = r % g->ny, iz = r / g->ny;
  long dy = g->oy ? g->oy[o] : 0;
  return node_at(g, ix + s * g->ox[o], iy + s * dy, iz + s * g->oz[o]);
}

static long step(const graph_t *g, long i, int o) { return step_dir(g, i, o, 1); }

/* textbook Dijkstra with a binary heap and lazy deletion */
static int dijkstra(const graph_t *g, int field, long src, double *tau) {
  long n = g->nx * g->ny * g->nz;
  for (long i = 0; i < n; ++i) tau[i] = INFINITY;
  char *done = (char *)calloc((size_t)n, 1);
  heap_t h = {0, 0, 0};
  if (!done) return 1;
  tau[src] = 0.0;
  if (heap_push(&h, 0.0, src)) { free(done); return 1; }
  while (h.n > 0) {
    heap_item it = heap_pop(&h);
    long u = it.node;
    if (done[u] || it.key != tau[u]) continue;
    done[u] = 1;
    for (int o = 0; o < g->n_off; ++o) {
      long v = step(g, u, o);
      if (v < 0 || done[v]) continue;
      double w = edge_weight(g, field, u, v, o);
      double cand = tau[u] + w;
      if (cand < tau[v]) {
        tau[v] = cand;
        if (heap_push(&h, cand, v)) { free(done); free(h.a); return 1; }
      }
    }
  }
  free(done);
  free(h.a);
  return 0;
}

/* Deterministic predecessors: BFS hop counts over tight edges
 * (tau_i + w_ij == tau_j), then pred_j = the tight i with the smallest
 * (hop, offset index).  order[] receives the BFS order (n_reached entries). */
static int predecessors(const graph_t *g, int field, long src,
                        const double *tau, int32_t *pred, int32_t *hop,
                        long *order, long *n_reached) {
  long n = g->nx * g->ny * g->nz;
  for (long i = 0; i < n; ++i) {
    pred[i] = -1;
    hop[i] = -1;
  }
  long head = 0, tail = 0;
  hop[src] = 0;
  order[tail++] = src;
  while (head < tail) {
    long i = order[head++];
    for (int o = 0; o < g->n_off; ++o) {
      long j = step(g, i, o);
      if (j < 0 || hop[j] >= 0 || !isfinite(tau[j])) continue;
      double w = edge_weight(g, field, i, j, o);
      if (tau[i] + w == tau[j]) {
        hop[j] = hop[i] + 1;
        order[tail++] = j;
      }
    }
  }
  *n_reached = tail;
  /* pull over in-edges i = j - o, i.e. j = i + o */
  for (long t = 1; t < tail; ++t) {
    long j = order[t];
    int best_o = -1;
    long best_i = -1;
    for (int o = 0; o < g->n_off; ++o) {
      long i = step_dir(g, j, o, -1); /* i = j - o */
      if (i < 0) continue;
      if (hop[i] < 0) continue;
      double w = edge_weight(g, field, i, j, o);
      if (!(tau[i] + w == tau[j])) continue;
      if (best_i < 0 || hop[i] < hop[best_i]) {
        best_i = i;
        best_o = o;
      }
      /* equal hop: the lower offset index wins, which the ascending loop
       * already guarantees */
    }
    (void)best_o;
    pred[j] = (int32_t)best_i;
  }
  return 0;
}

/* Trace one source for one mode on a 2D grid with a class cache.
 * V, A, st: [n_classes][n_dirs] slices of the chosen mode.
 * Any output pointer may be NULL.  tstar needs tauR's tree (pred_p). */
int orc_trace_2d_cols(long nx, long nz, double hx, double hz,
                      const int32_t *class_id, int R, int n_dirs,
                      const int32_t *subset, int n_subset,
                      const double *V, const double *A, const int32_t *st,
                      long src, double *tauR, double *tauI, int32_t *predP,
                      int32_t *predA, double *tstar, int32_t *hopP,
                      int32_t *hopA) {
  long n = nx * nz;
  if (src < 0 || src >= n || R < 1) return 1;
  int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_dirs);
  if (!col) return 2;
  for (int d = 0; d < n_dirs; ++d) col[d] = subset ? -1 : d;
  if (subset)
    for (int q = 0; q < n_subset; ++q) col[subset[q]] = q;
  int n_off = orc_star_2d(R, hx, hz, n_dirs, NULL, NULL, NULL, NULL);
  int32_t *ox = (int32_t *)malloc(sizeof(int32_t) * n_off);
  int32_t *oz = (int32_t *)malloc(sizeof(int32_t) * n_off);
  int32_t *bin = (int32_t *)malloc(sizeof(int32_t) * n_off);
  double *L = (double *)malloc(sizeof(double) * n_off);
  double *tR = (double *)malloc(sizeof(double) * (size_t)n);
  double *tI = (double *)malloc(sizeof(double) * (size_t)n);
  int32_t *pP = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *pA = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *hP = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *hA = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  long *ordP = (long *)malloc(sizeof(long) * (size_t)n);
  long *ordA = (long *)malloc(sizeof(long) * (size_t)n);
  int rc = 0;
  if (!ox || !oz || !bin || !L || !tR || !tI || !pP || !pA || !hP || !hA ||
      !ordP || !ordA) {
    rc = 2;
    goto out;
  }
  orc_star_2d(R, hx, hz, n_dirs, ox, oz, L, bin);
  for (int o = 0; o < n_off; ++o)
    if (col[bin[o]] < 0) { rc = 3; goto out; } /* cache lacks a star direction */
  graph_t g = {.nx = nx, .nz = nz, .n_off = n_off, .ox = ox, .oz = oz, .bin = bin,
               .ny = 1, .oy = NULL, .L = L, .cls = class_id,
               .n_cols = subset ? n_subset : n_dirs, .col = col, .V = V, .A = A, .st = st};
  long nrP = 0, nrA = 0;
  /* the attenuation field is solved only when one of its outputs is asked for */
  int want_att = tauI || predA || hopA;
  if (dijkstra(&g, 0, src, tR) || (want_att && dijkstra(&g, 1, src, tI))) { rc = 2; goto out; }
  predecessors(&g, 0, src, tR, pP, hP, ordP, &nrP);
  if (want_att) predecessors(&g, 1, src, tI, pA, hA, ordA, &nrA);
  if (tstar) {
    /* t*: attenuation folded along the propagation raypath tree, source
     * outwards in BFS order so each parent is final first */
    for (long i = 0; i < n; ++i) tstar[i] = INFINITY;
    tstar[src] = 0.0;
    for (long t = 1; t < nrP; ++t) {
      long j = ordP[t];
      long i = pP[j];
      /* offset index of j - i */
      long dx = (j % nx) - (i % nx), dz = (j / nx) - (i / nx);
      int oo = -1;
      for (int o = 0; o < n_off; ++o)
        if (ox[o] == dx && oz[o] == dz) { oo = o; break; }
      tstar[j] = tstar[i] + edge_weight(&g, 1, i, j, oo);
    }
  }
  if (tauR) memcpy(tauR, tR, sizeof(double) * (size_t)n);
  if (tauI) memcpy(tauI, tI, sizeof(double) * (size_t)n);
  if (predP) memcpy(predP, pP, sizeof(int32_t) * (size_t)n);
  if (predA) memcpy(predA, pA, sizeof(int32_t) * (size_t)n);
  if (hopP) memcpy(hopP, hP, sizeof(int32_t) * (size_t)n);
  if (hopA) memcpy(hopA, hA, sizeof(int32_t) * (size_t)n);
out:
  free(ox); free(oz); free(bin); free(L); free(tR); free(tI);
  free(pP); free(pA); free(hP); free(hA); free(ordP); free(ordA); free(col);
  return rc;
}

int orc_trace_2d(long nx, long nz, double hx, double hz,
                 const int32_t *class_id, int R, int n_dirs,
                 const double *V, const double *A, const int32_t *st,
                 long src, double *tauR, double *tauI, int32_t *predP,
                 int32_t *predA, double *tstar, int32_t *hopP,
                 int32_t *hopA) {
  return orc_trace_2d_cols(nx, nz, hx, hz, class_id, R, n_dirs, NULL, 0, V, A,
                           st, src, tauR, tauI, predP, predA, tstar, hopP, hopA);
}

/* ------------------------------------------------------------------------ */
/* O-16  the slowness-sampled cache (eq 26 read literally) and its lookup   */
/* ------------------------------------------------------------------------ */

/* Entry s of class k holds the homogeneous solution whose real slowness
 * angle, in the class's symmetry-axis frame (eq 36), is theta_R = s 2pi/n:
 * theta_I is the homogeneity root nearest 0 in [-30, 30] deg (eq 9), the ray
 * quantities follow (eqs 10-11) with the ray direction rotated to the
 * global frame, and the residual field is |h| (no target direction).  No
 * root: NO_BRACKET.  fields: [ORC_NF][3][n_classes][n]; status [3][K][n]. */
int orc_build_cache_slow_2d(const double *classes, long n_classes, int n,
                            unsigned mode_mask, int reading, double *fields,
                            int32_t *status) {
  if (n < 4) return 1;
  long stride = 3L * n_classes * n;
  for (int mode = 0; mode < 3; ++mode) {
    if (!(mode_mask & (1u << mode))) continue;
    for (long k = 0; k < n_classes; ++k) {
      const double *cls = classes + 13 * k;
      medium_t m;
      load_medium(cls, &m);
      long base = ((long)mode * n_classes + k) * n;
      int fluid = (mode != ORC_QP) && (cls[3] == 0.0 || (mode == ORC_QSH && cls[4] == 0.0));
      for (int q = 0; q < n; ++q) {
        if (fluid) {
          write_invalid(fields, stride, base + q);
          status[base + q] = ORC_ST_FLUID;
          continue;
        }
        double thR = q * (2.0 * ORC_PI / n);
        double thI;
        if (theta_imag(&m, mode, reading, thR, &thI) != 0) {
          write_invalid(fields, stride, base + q);
          status[base + q] = ORC_ST_NO_BRACKET;
          continue;
        }
        eval_t e;
        energy_velocity(&m, mode, reading, thR, thI, &e);
        entry_t en;
        ray_quantities(&e, &en);
        en.thR = thR;
        en.thI = thI;
        en.res = theta_i_zero(&m, mode) ? 0.0 : fabs(homog_residual(&e));
        int st = ORC_ST_OK;
        if (!(en.A >= 0.0) || !isfinite(en.V) || !(en.V > 0.0)) st |= ORC_ST_NONPHYS;
        if (!(en.res <= ORC_RESID_TOL)) st |= ORC_ST_NOCONV;
        write_entry(fields, stride, base + q, &en, m.tilt);
        status[base + q] = st;
      }
    }
  }
  return 0;
}

/* The closest stored ray direction of every class to every star offset
 * (text after eq 27: the normalised dot product): best[k][o] = the sample
 * whose r-hat (global frame) has the largest dot product with the edge's
 * unit vector, the lowest index on ties, among samples that hold a ray
 * direction (no NO_BRACKET, no FLUID); -1 if none does. */
int orc_slow_lookup(long n_classes, int n, const double *RX, const double *RZ,
                    const int32_t *st, int n_off, const int32_t *ox,
                    const int32_t *oz, double hx, double hz, int32_t *best) {
  for (int o = 0; o < n_off; ++o) {
    double ex = ox[o] * hx, ez = oz[o] * hz;
    double len = sqrt(ex * ex + ez * ez);
    double dx = ex / len, dz = ez / len;
    for (long k = 0; k < n_classes; ++k) {
      int b = -1;
      double bd = 0.0;
      for (int q = 0; q < n; ++q) {
        if (st[k * n + q] & (ORC_ST_NO_BRACKET | ORC_ST_FLUID)) continue;
        double dd = RX[k * n + q] * dx + RZ[k * n + q] * dz;
        if (b < 0 || dd > bd) {
          b = q;
          bd = dd;
        }
      }
      best[k * n_off + o] = b;
    }
  }
  return 0;
}

/* Dijkstra (O-10..O-12) for one mode of a slowness-sampled cache: slice
 * V, A, RX, RZ, status [K][n]; class map required. */
int orc_trace_2d_slow(long nx, long nz, double hx, double hz, const int32_t *class_id,
                      long n_classes, int R, int n, const double *V, const double *A,
                      const double *RX, const double *RZ, const int32_t *st, long src,
                      double *tauR, double *tauI, int32_t *predP, int32_t *predA,
                      double *tstar) {
  long nn = nx * nz;
  if (src < 0 || src >= nn || R < 1 || !class_id) return 1;
  int n_off = orc_star_2d(R, hx, hz, 4, NULL, NULL, NULL, NULL);
  int32_t *ox = (int32_t *)malloc(sizeof(int32_t) * n_off);
  int32_t *oz = (int32_t *)malloc(sizeof(int32_t) * n_off);
  int32_t *bin = (int32_t *)malloc(sizeof(int32_t) * n_off);
  double *L = (double *)malloc(sizeof(double) * n_off);
  int32_t *best = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_classes * n_off);
  double *t = (double *)malloc(sizeof(double) * (size_t)nn);
  int32_t *pr = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  int32_t *hp = (int32_t *)malloc(sizeof(int32_t) * (size_t)nn);
  long *ord = (long *)malloc(sizeof(long) * (size_t)nn);
  int rc = 0;
  if (!ox || !oz || !bin || !L || !best || !t || !pr || !hp || !ord) { rc = 2; goto out; }
  orc_star_2d(R, hx, hz, 4, ox, oz, L, bin);
  orc_slow_lookup(n_classes, n, RX, RZ, st, n_off, ox, oz, hx, hz, best);
  graph_t g = {.nx = nx, .nz = nz, .n_off = n_off, .ox = ox, .oz = oz, .bin = bin,
               .ny = 1, .oy = NULL, .L = L, .cls = class_id, .n_cols = n, .col = NULL,
               .V = V, .A = A, .st = st, .best = best};
  for (int field = 0; field < 2; ++field) {
    double *out_t = field ? tauI : tauR;
    int32_t *out_p = field ? predA : predP;
    int want_ts = (field == 0 && tstar != NULL);
    if (!out_t && !out_p && !want_ts) continue;
    if (dijkstra(&g, field, src, t)) { rc = 2; goto out; }
    long nr = 0;
    predecessors(&g, field, src, t, pr, hp, ord, &nr);
    if (out_p) memcpy(out_p, pr, sizeof(int32_t) * (size_t)nn);
    if (want_ts) {
      for (long i = 0; i < nn; ++i) tstar[i] = INFINITY;
      tstar[src] = 0.0;
      for (long q = 1; q < nr; ++q) {
        long j = ord[q], i = pr[j];
        long dx = (j % nx) - (i % nx), dz = (j / nx) - (i / nx);
        int oo = -1;
        for (int o = 0; o < n_off; ++o)
          if (ox[o] == dx && oz[o] == dz) { oo = o; break; }
        tstar[j] = tstar[i] + edge_weight(&g, 1, i, j, oo);
      }
    }
    if (out_t) memcpy(out_t, t, sizeof(double) * (size_t)nn);
  }
out:
  free(ox); free(oz); free(bin); free(L); free(best); free(t); free(pr); free(hp); free(ord);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* O-14  uncached (MSPM-style) form: every relaxation re-solves the local   */
/*       problem at both endpoints for the edge's bin (no cache, no memo)   */
/* ------------------------------------------------------------------------ */

static int solve_bin_fresh(const double *cls, int mode, int reading,
                           int n_sweep, int n_dirs, int b, double *V,
                           double *A) {
  medium_t m;
  load_medium(cls, &m);
  int fluid = (mode != ORC_QP) && (cls[3] == 0.0 || (mode == ORC_QSH && cls[4] == 0.0));
  if (fluid) return ORC_ST_FLUID;
  int half = n_dirs / 2;
  int d = b % half; /* the solved half; b >= half is its centrosymmetric copy */
  sample_t *tab = (sample_t *)malloc(sizeof(sample_t) * (size_t)n_sweep);
  if (!tab) return ORC_ST_NO_BRACKET;
  sweep(&m, mode, reading, n_sweep, tab);
  double psi_star = wrap_pi(d * (2.0 * ORC_PI / n_dirs) - m.tilt);
  entry_t e;
  int st = solve_direction(&m, mode, reading, n_sweep, tab, psi_star, &e);
  free(tab);
  if (st & ORC_ST_NO_BRACKET) return st;
  if (!(e.A >= 0.0) || !isfinite(e.V) || !(e.V > 0.0)) st |= ORC_ST_NONPHYS;
  if (!(e.res <= ORC_RESID_TOL)) st |= ORC_ST_NOCONV;
  *V = e.V;
  *A = e.A;
  return st;
}

/* Dijkstra for one field where each edge weight comes from fresh solves. */
int orc_trace_uncached_2d(long nx, long nz, double hx, double hz,
                          const int32_t *class_id, const double *classes,
                          int R, int n_dirs, int mode, int reading,
                          int n_sweep, int field, long src, double *tau,
                          long *n_solves) {
  long n = nx * nz;
  if (src < 0 || src >= n) return 1;
  int n_off = orc_star_2d(R, hx, hz, n_dirs, NULL, NULL, NULL, NULL);
  int32_t ox[4 * 121], oz[4 * 121], bin[4 * 121];
  double L[4 * 121];
  if (n_off > 4 * 121) return 1;
  orc_star_2d(R, hx, hz, n_dirs, ox, oz, L, bin);
  for (long i = 0; i < n; ++i) tau[i] = INFINITY;
  char *done = (char *)calloc((size_t)n, 1);
  heap_t h = {0, 0, 0};
  long solves = 0;
  tau[src] = 0.0;
  heap_push(&h, 0.0, src);
  while (h.n > 0) {
    heap_item it = heap_pop(&h);
    long u = it.node;
    if (done[u] || it.key != tau[u]) continue;
    done[u] = 1;
    for (int o = 0; o < n_off; ++o) {
      long ux = u % nx, uz = u / nx;
      long vx = ux + ox[o], vz = uz + oz[o];
      if (vx < 0 || vx >= nx || vz < 0 || vz >= nz) continue;
      long v = vx + nx * vz;
      if (done[v]) continue;
      double Vu, Au, Vv, Av;
      int su = solve_bin_fresh(classes + 13 * class_id[u], mode, reading,
                               n_sweep, n_dirs, bin[o], &Vu, &Au);
      int sv = solve_bin_fresh(classes + 13 * class_id[v], mode, reading,
                               n_sweep, n_dirs, bin[o], &Vv, &Av);
      solves += 2;
      int bad = ORC_ST_NO_BRACKET | ORC_ST_FLUID | ORC_ST_NONPHYS | ORC_ST_NOCONV;
      double w;
      if ((su & bad) || (sv & bad)) w = INFINITY;
      else if (field == 0) w = L[o] / (0.5 * (Vu + Vv));
      else w = L[o] * (0.5 * (Au + Av));
      double cand = tau[u] + w;
      if (cand < tau[v]) {
        tau[v] = cand;
        heap_push(&h, cand, v);
      }
    }
  }
  free(done);
  free(h.a);
  if (n_solves) *n_solves = solves;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O-13  raypath extraction (eqs 33-34), source -> receiver order           */
/* ------------------------------------------------------------------------ */

/* returns 0 ok, 6 unreachable, 7 cycle, 5 capacity (len set to required) */
int orc_raypath(const int32_t *pred, long n_nodes, long src, long rcv,
                int64_t *path, long capacity, long *len) {
  if (src < 0 || src >= n_nodes || rcv < 0 || rcv >= n_nodes) return 1;
  long count = 1;
  long cur = rcv;
  while (cur != src) {
    long p = pred[cur];
    if (p < 0) return 6;
    if (++count > n_nodes) return 7;
    cur = p;
  }
  *len = count;
  if (count > capacity) return 5;
  cur = rcv;
  for (long q = count - 1; q >= 0; --q) {
    path[q] = cur;
    if (q > 0) cur = pred[cur];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* 3D: Fibonacci ray directions, sagittal-plane cache (eqs 6, 35), 3D star  */
/* ------------------------------------------------------------------------ */

/* Readings for 3D (the paper gives the basis of eq 35 and the complex
 * slowness direction of eq 6, not a 3D direction set):
 *   - ray directions: the Fibonacci set f_i = (r cos phi_i, r sin phi_i, z_i),
 *     z_i = 1 - (2i+1)/N, r = sqrt(1 - z_i^2), phi_i = i pi (3 - sqrt 5),
 *     in global (x, y, z), z down; N = 41253 gives about one per square
 *     degree;
 *   - a TI class's axis is e_z' of eq 35; the solution whose ray direction is
 *     f_i has its slowness in the plane of e_z' and f_i with zero imaginary
 *     azimuth (the medium is symmetric about that plane), so entry i is the
 *     2D sagittal solve (eq 7) at the local polar angle
 *     alpha_i = arccos(f_i . e_z');
 *   - entry i stores RX, RZ = the x and z components of f_i (its y component
 *     is f_i's); there is no centrosymmetric copy (the set is not symmetric).
 *   - node index ix + nx (iy + ny iz); star offsets with max norm <= R and
 *     gcd(|ox|, |oy|, |oz|) = 1 ordered by (oy, oz, ox) ascending; length
 *     sqrt((ox hx)^2 + (oz hz)^2 + (oy hy)^2) summed in that order; bin = the
 *     i maximising f_i . o_hat (x, y, z order), ties to the lowest i. */

void orc_fibonacci(int N, double *f) {
  const double ga = ORC_PI * (3.0 - sqrt(5.0));
  for (int i = 0; i < N; ++i) {
    double z = 1.0 - (2.0 * i + 1.0) / N;
    double r = sqrt(1.0 - z * z);
    double ph = i * ga;
    f[3 * i] = r * cos(ph);
    f[3 * i + 1] = r * sin(ph);
    f[3 * i + 2] = z;
  }
}

/* symmetry axis e_z' of eq 35 */
static void axis_3d(double tilt, double azimuth, double e[3]) {
  e[0] = sin(tilt) * cos(azimuth);
  e[1] = sin(tilt) * sin(azimuth);
  e[2] = cos(tilt);
}

/* fields [ORC_NF][3][n_classes][N], status [3][n_classes][N] */
int orc_build_cache_3d(const double *classes, long n_classes, int N,
                       unsigned mode_mask, int reading, int n_sweep,
                       double *fields, int32_t *status) {
  if (N < 2 || n_sweep < 8) return 1;
  double *f = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  sample_t *tab = (sample_t *)malloc(sizeof(sample_t) * (size_t)n_sweep);
  if (!f || !tab) { free(f); free(tab); return 2; }
  orc_fibonacci(N, f);
  long stride = 3L * n_classes * N;
  for (int mode = 0; mode < 3; ++mode) {
    if (!(mode_mask & (1u << mode))) continue;
    for (long k = 0; k < n_classes; ++k) {
      const double *cls = classes + 13 * k;
      medium_t m;
      load_medium(cls, &m);
      long base = ((long)mode * n_classes + k) * N;
      int fluid = (mode != ORC_QP) && (cls[3] == 0.0 || (mode == ORC_QSH && cls[4] == 0.0));
      if (fluid) {
        for (int i = 0; i < N; ++i) {
          write_invalid(fields, stride, base + i);
          status[base + i] = ORC_ST_FLUID;
        }
        continue;
      }
      double ax[3];
      axis_3d(cls[11], cls[12], ax);
      sweep(&m, mode, reading, n_sweep, tab);
      for (int i = 0; i < N; ++i) {
        double c = f[3 * i] * ax[0] + f[3 * i + 1] * ax[1] + f[3 * i + 2] * ax[2];
        if (c > 1.0) c = 1.0;
        if (c < -1.0) c = -1.0;
        double alpha = acos(c);
        entry_t e;
        int st = solve_direction(&m, mode, reading, n_sweep, tab, alpha, &e);
        long idx = base + i;
        if (st & ORC_ST_NO_BRACKET) {
          write_invalid(fields, stride, idx);
          status[idx] = st;
          continue;
        }
        if (!(e.A >= 0.0) || !isfinite(e.V) || !(e.V > 0.0)) st |= ORC_ST_NONPHYS;
        if (!(e.res <= ORC_RESID_TOL)) st |= ORC_ST_NOCONV;
        fields[F_V * stride + idx] = e.V;
        fields[F_A * stride + idx] = e.A;
        fields[F_Q * stride + idx] = e.Q;
        fields[F_RX * stride + idx] = f[3 * i];
        fields[F_RZ * stride + idx] = f[3 * i + 2];
        fields[F_THR * stride + idx] = e.thR;
        fields[F_THI * stride + idx] = e.thI;
        fields[F_RES * stride + idx] = e.res;
        status[idx] = st;
      }
    }
  }
  free(f);
  free(tab);
  return 0;
}

static int gcd3(int a, int b, int c) { return gcd_int(gcd_int(a, b), c); }

/* 3D star (see the readings above).  Returns the count; arrays may be NULL. */
int orc_star_3d(int R, double hx, double hy, double hz, int N, int32_t *ox,
                int32_t *oy, int32_t *oz, double *L, int32_t *bin) {
  double *f = NULL;
  if (ox) {
    f = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    if (!f) return -1;
    orc_fibonacci(N, f);
  }
  int n = 0;
  for (int y = -R; y <= R; ++y)
    for (int z = -R; z <= R; ++z)
      for (int x = -R; x <= R; ++x) {
        if (x == 0 && y == 0 && z == 0) continue;
        if (gcd3(x, y, z) != 1) continue;
        if (ox) {
          double dx = x * hx, dy = y * hy, dz = z * hz;
          double len = sqrt(dx * dx + dz * dz + dy * dy);
          double u0 = dx / len, u1 = dy / len, u2 = dz / len;
          int best = 0;
          double bd = -2.0;
          for (int i = 0; i < N; ++i) {
            double d = f[3 * i] * u0 + f[3 * i + 1] * u1 + f[3 * i + 2] * u2;
            if (d > bd) { bd = d; best = i; }
          }
          ox[n] = x;
          oy[n] = y;
          oz[n] = z;
          L[n] = len;
          bin[n] = best;
        }
        ++n;
      }
  free(f);
  return n;
}

/* Dijkstra traveltimes and predecessors on a 3D grid with a class cache
 * on the Fibonacci directions (V, A, st: [n_classes][N] of one mode). */
int orc_trace_3d(long nx, long ny, long nz, double hx, double hy, double hz,
                 const int32_t *class_id, int R, int N, const double *V,
                 const double *A, const int32_t *st, long src, double *tauR,
                 double *tauI, int32_t *predP, int32_t *predA, double *tstar) {
  long n = nx * ny * nz;
  if (src < 0 || src >= n || R < 1) return 1;
  int n_off = orc_star_3d(R, hx, hy, hz, N, NULL, NULL, NULL, NULL, NULL);
  int32_t *ox = (int32_t *)malloc(sizeof(int32_t) * n_off);
  int32_t *oy = (int32_t *)malloc(sizeof(int32_t) * n_off);
  int32_t *oz = (int32_t *)malloc(sizeof(int32_t) * n_off);
  int32_t *bin = (int32_t *)malloc(sizeof(int32_t) * n_off);
  double *L = (double *)malloc(sizeof(double) * n_off);
  int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  double *t = (double *)malloc(sizeof(double) * (size_t)n);
  int32_t *pr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *hp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  long *ord = (long *)malloc(sizeof(long) * (size_t)n);
  int rc = 0;
  if (!ox || !oy || !oz || !bin || !L || !col || !t || !pr || !hp || !ord) { rc = 2; goto out; }
  orc_star_3d(R, hx, hy, hz, N, ox, oy, oz, L, bin);
  for (int i = 0; i < N; ++i) col[i] = i;
  graph_t g = {.nx = nx, .nz = nz, .n_off = n_off, .ox = ox, .oz = oz, .bin = bin,
               .ny = ny, .oy = oy, .L = L, .cls = class_id, .n_cols = N, .col = col,
               .V = V, .A = A, .st = st};
  for (int field = 0; field < 2; ++field) {
    double *out_t = field ? tauI : tauR;
    int32_t *out_p = field ? predA : predP;
    int want_ts = (field == 0 && tstar != NULL);
    if (!out_t && !out_p && !want_ts) continue;
    if (dijkstra(&g, field, src, t)) { rc = 2; goto out; }
    if (out_p || want_ts) {
      long nr = 0;
      predecessors(&g, field, src, t, pr, hp, ord, &nr);
      if (out_p) memcpy(out_p, pr, sizeof(int32_t) * (size_t)n);
      if (want_ts) {
        /* t*: attenuation folded along the propagation tree in BFS order */
        for (long i = 0; i < n; ++i) tstar[i] = INFINITY;
        tstar[src] = 0.0;
        for (long q = 1; q < nr; ++q) {
          long j = ord[q], i = pr[j];
          long dx = (j % nx) - (i % nx), dy = (j / nx) % ny - (i / nx) % ny,
               dz = j / (nx * ny) - i / (nx * ny);
          int oo = -1;
          for (int o = 0; o < n_off; ++o)
            if (ox[o] == dx && oy[o] == dy && oz[o] == dz) { oo = o; break; }
          tstar[j] = tstar[i] + edge_weight(&g, 1, i, j, oo);
        }
      }
    }
    if (out_t) memcpy(out_t, t, sizeof(double) * (size_t)n);
  }
out:
  free(ox); free(oy); free(oz); free(bin); free(L); free(col);
  free(t); free(pr); free(hp); free(ord);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* O-18  the cell network (grid and nodal ray-network section, eqs 23-24,   */
/*       27-32): nodes on cell edges, every node pair of a cell an edge,    */
/*       optionally marched block by block from a heap of cells             */
/* ------------------------------------------------------------------------ */

/* The network: ncx x ncz rectangular cells, each side divided into cn
 * intervals of hx (along x) or hz (along z).  Its nodes are the points of
 * the (ncx cn + 1) x (ncz cn + 1) lattice that lie on a cell edge
 * (ix % cn == 0 or iz % cn == 0), indexed ix + NX iz like the lattice; the
 * points inside a cell are not nodes.  Two nodes are joined when both lie on
 * the boundary of one cell (eq 27: the straight segment between them).  Its
 * weight follows eqs 28-30 with the classes of its two end nodes: with a
 * ray-direction cache both ends read the tabulated direction nearest to the
 * segment (the same rule as for forward-star offsets); with a
 * slowness-sampled cache each end reads its class's sample whose stored ray
 * direction has the largest normalised dot product with the segment. */
typedef struct {
  long ncx, ncz, NX, NZ;
  int cn, side;          /* side = 2 cn + 1: offsets (dx, dz) in [-cn, cn]^2 */
  int dim;               /* 2, or 3 for blocks (O-20) */
  long ncy, NY;          /* 3D: blocks and lattice points along y (2D: 1, 1) */
  const int32_t *cls;    /* lattice -> class */
  long K;
  int n_cols;
  const double *V, *A;   /* [K][n_cols] of one mode */
  const int32_t *st;
  double *L;             /* [side^2] segment length per offset */
  int32_t *colR;         /* ray-direction cache: [side^2] column; NULL otherwise */
  int32_t *best;         /* slowness-sampled cache: [K][side^2]; NULL otherwise */
  /* MSPM (O-19): no cache; corner solves at the segment's exact direction */
  int mspm;
  const double *classes; /* [K][13] */
  int mode, reading, n_sweep;
  double hx, hz;
  double *mV, *mA;       /* [K][side^2] memo of the fresh solves (canonical offsets) */
  int32_t *mst;          /* status; -1: not solved yet */
} cellnet_t;

static int cell_is_node(const cellnet_t *g, long ix, long iz) {
  return ix % g->cn == 0 || iz % g->cn == 0;
}

static int cell_off(const cellnet_t *g, long dx, long dz) {
  return (int)((dz + g->cn) * g->side + (dx + g->cn));
}

/* lattice node index ix + NX (iy + NY iz) and back (2D: iy = 0, NY = 1) */
static long cell_n_nodes(const cellnet_t *g) { return g->NX * g->NY * g->NZ; }
static void cell_xyz(const cellnet_t *g, long u, long *x, long *y, long *z) {
  *x = u % g->NX;
  *y = (u / g->NX) % g->NY;
  *z = u / (g->NX * g->NY);
}
/* offset index: 2D (dz, dx), 3D (dz, dy, dx), each in [-cn, cn] */
static int cell_off3(const cellnet_t *g, long dx, long dy, long dz) {
  if (g->dim == 2) return cell_off(g, dx, dz);
  return (int)(((dz + g->cn) * g->side + (dy + g->cn)) * g->side + (dx + g->cn));
}

static double mspm_weight(cellnet_t *g, int field, long c, long i, long j);

/* Weight of segment i -> j of cell c (the cell matters only to MSPM). */
static double cell_weight(cellnet_t *g, int field, long c, long i, long j) {
  if (g->mspm) return mspm_weight(g, field, c, i, j);
  long xi, yi, zi, xj, yj, zj;
  cell_xyz(g, i, &xi, &yi, &zi);
  cell_xyz(g, j, &xj, &yj, &zj);
  int o = cell_off3(g, xj - xi, yj - yi, zj - zi);
  long ki = g->cls[i], kj = g->cls[j];
  int ci, cj;
  if (g->best) {
    ci = g->best[ki * g->side * g->side + o];
    cj = g->best[kj * g->side * g->side + o];
    if (ci < 0 || cj < 0) return INFINITY;
  } else {
    ci = cj = g->colR[o];
  }
  const int bad = ORC_ST_NO_BRACKET | ORC_ST_FLUID | ORC_ST_NONPHYS | ORC_ST_NOCONV;
  if ((g->st[ki * g->n_cols + ci] & bad) || (g->st[kj * g->n_cols + cj] & bad)) return INFINITY;
  if (field == 0)
    return g->L[o] / (0.5 * (g->V[ki * g->n_cols + ci] + g->V[kj * g->n_cols + cj]));
  return g->L[o] * (0.5 * (g->A[ki * g->n_cols + ci] + g->A[kj * g->n_cols + cj]));
}

/* the cell indices along one axis whose closed range holds coordinate q */
static int cells_along(long q, int cn, long ncells, long *out) {
  int n = 0;
  if (q % cn == 0) {
    if (q / cn - 1 >= 0) out[n++] = q / cn - 1;
    if (q / cn < ncells) out[n++] = q / cn;
  } else {
    out[n++] = q / cn;
  }
  return n;
}

/* The cells (blocks) whose boundary holds lattice node u: up to two per
 * axis.  Writes cell indices cx + ncx (cy + ncy cz) into c[] (at most 4 in
 * 2D, 8 in 3D), returns the count. */
static int cells_of(const cellnet_t *g, long u, long *c) {
  long ix, iy, iz;
  cell_xyz(g, u, &ix, &iy, &iz);
  long xs[2], ys[2] = {0, 0}, zs[2];
  int nxs = cells_along(ix, g->cn, g->ncx, xs);
  int nys = g->dim == 3 ? cells_along(iy, g->cn, g->ncy, ys) : 1;
  int nzs = cells_along(iz, g->cn, g->ncz, zs);
  int n = 0;
  for (int a = 0; a < nxs; ++a)
    for (int d = 0; d < nys; ++d)
      for (int b = 0; b < nzs; ++b) c[n++] = xs[a] + g->ncx * (ys[d] + g->ncy * zs[b]);
  return n;
}

/* The boundary nodes of cell c (each once), in any order: 4 cn in 2D, the
 * (cn + 1)^3 - (cn - 1)^3 face points of a block in 3D. */
static int cell_nodes(const cellnet_t *g, long c, long *v) {
  long x0 = (c % g->ncx) * g->cn, y0 = ((c / g->ncx) % g->ncy) * g->cn,
       z0 = (c / (g->ncx * g->ncy)) * g->cn;
  long ny = g->dim == 3 ? g->cn : 0;
  int n = 0;
  for (long dz = 0; dz <= g->cn; ++dz)
    for (long dy = 0; dy <= ny; ++dy)
      for (long dx = 0; dx <= g->cn; ++dx) {
        int on = dx == 0 || dz == 0 || dx == g->cn || dz == g->cn;
        if (g->dim == 3) on = on || dy == 0 || dy == g->cn;
        if (on) v[n++] = (x0 + dx) + g->NX * ((y0 + dy) + g->NY * (z0 + dz));
      }
  return n;
}

/* Neighbours of u: the other boundary nodes of every cell holding u, with
 * that cell in nbc (a node shared by two cells along their common edge is
 * listed twice; the two copies are the same segment and carry the same
 * weight). */
static int cell_neighbours(const cellnet_t *g, long u, long *nb, long *nbc) {
  long cs[8], v[64 * 4];
  int nc = cells_of(g, u, cs), n = 0;
  for (int a = 0; a < nc; ++a) {
    int m = cell_nodes(g, cs[a], v);
    for (int b = 0; b < m; ++b)
      if (v[b] != u) {
        nbc[n] = cs[a];
        nb[n++] = v[b];
      }
  }
  return n;
}

/* A cell whose boundary holds both nodes i and j. */
static long common_cell(const cellnet_t *g, long i, long j) {
  long cs[8];
  int nc = cells_of(g, j, cs);
  long ix, iy, iz;
  cell_xyz(g, i, &ix, &iy, &iz);
  for (int a = 0; a < nc; ++a) {
    long x0 = (cs[a] % g->ncx) * g->cn, y0 = ((cs[a] / g->ncx) % g->ncy) * g->cn,
         z0 = (cs[a] / (g->ncx * g->ncy)) * g->cn;
    if (ix >= x0 && ix <= x0 + g->cn && iz >= z0 && iz <= z0 + g->cn &&
        (g->dim == 2 || (iy >= y0 && iy <= y0 + g->cn)))
      return cs[a];
  }
  return -1;
}

static int cell_dijkstra(cellnet_t *g, int field, long src, double *tau) {
  long n = cell_n_nodes(g);
  for (long i = 0; i < n; ++i) tau[i] = INFINITY;
  char *done = (char *)calloc((size_t)n, 1);
  long *nb = (long *)malloc(sizeof(long) * 16 * 64);
  long *nbc = (long *)malloc(sizeof(long) * 16 * 64);
  heap_t h = {0, 0, 0};
  int rc = 0;
  if (!done || !nb || !nbc) { rc = 1; goto out; }
  tau[src] = 0.0;
  if (heap_push(&h, 0.0, src)) { rc = 1; goto out; }
  while (h.n > 0) {
    heap_item it = heap_pop(&h);
    long u = it.node;
    if (done[u] || it.key != tau[u]) continue;
    done[u] = 1;
    int m = cell_neighbours(g, u, nb, nbc);
    for (int b = 0; b < m; ++b) {
      long v = nb[b];
      if (done[v]) continue;
      double cand = tau[u] + cell_weight(g, field, nbc[b], u, v);
      if (cand < tau[v]) {
        tau[v] = cand;
        if (heap_push(&h, cand, v)) { rc = 1; goto out; }
      }
    }
  }
out:
  free(done);
  free(nb);
  free(nbc);
  free(h.a);
  return rc;
}

/* The paper's block marching (eqs 23-24, 31-32): a heap of cells keyed by
 * their block traveltime T_b = the smallest node traveltime in the cell
 * (eq 24).  The cell with the smallest key is taken; every ordered pair of
 * its boundary nodes is relaxed (eq 31 applies both directions of each
 * segment) until a full pass changes nothing; each neighbouring cell that
 * shares an improved node is pushed again with its new T_b.  A cell re-enters
 * the heap whenever one of its nodes improves, so the marching ends at the
 * network's shortest-path traveltimes (the same fixed point as node
 * Dijkstra) whatever the order. */
static int cell_block_march(cellnet_t *g, int field, long src, double *tau) {
  long n = cell_n_nodes(g), nc = g->ncx * g->ncy * g->ncz;
  for (long i = 0; i < n; ++i) tau[i] = INFINITY;
  double *key = (double *)malloc(sizeof(double) * (size_t)nc);
  long *v = (long *)malloc(sizeof(long) * 64 * 4);
  long cs[8];
  heap_t h = {0, 0, 0};
  int rc = 0;
  if (!key || !v) { rc = 1; goto out; }
  for (long c = 0; c < nc; ++c) key[c] = INFINITY;
  tau[src] = 0.0;
  {
    int k = cells_of(g, src, cs);
    for (int a = 0; a < k; ++a) {
      key[cs[a]] = 0.0;
      if (heap_push(&h, 0.0, cs[a])) { rc = 1; goto out; }
    }
  }
  while (h.n > 0) {
    heap_item it = heap_pop(&h);
    long c = it.node;
    if (it.key != key[c]) continue; /* stale entry */
    key[c] = INFINITY;              /* taken: re-enters only on a new improvement */
    int m = cell_nodes(g, c, v);
    char improved[256] = {0};
    int changed = 1;
    while (changed) {
      changed = 0;
      for (int a = 0; a < m; ++a) {
        if (!isfinite(tau[v[a]])) continue;
        for (int b = 0; b < m; ++b) {
          if (a == b) continue;
          double cand = tau[v[a]] + cell_weight(g, field, c, v[a], v[b]);
          if (cand < tau[v[b]]) {
            tau[v[b]] = cand;
            improved[b] = 1;
            changed = 1;
          }
        }
      }
    }
    for (int b = 0; b < m; ++b) {
      if (!improved[b]) continue;
      int k = cells_of(g, v[b], cs);
      for (int a = 0; a < k; ++a) {
        long c2 = cs[a];
        if (c2 == c) continue;
        /* T_b of the neighbour (eq 24) over its nodes */
        int m2 = cell_nodes(g, c2, v + 64 * 2);
        double tb = INFINITY;
        for (int q = 0; q < m2; ++q)
          if (tau[v[64 * 2 + q]] < tb) tb = tau[v[64 * 2 + q]];
        key[c2] = tb;
        if (heap_push(&h, tb, c2)) { rc = 1; goto out; }
      }
    }
  }
out:
  free(key);
  free(v);
  free(h.a);
  return rc;
}

/* Deterministic predecessors: BFS hop counts over tight segments
 * (tau_i + w_ij == tau_j), pred_j = the tight neighbour i with the smallest
 * (hop, node index); t* (field 0 only) folds the attenuation weights along
 * that tree from the source outwards. */
static int cell_predecessors(cellnet_t *g, int field, long src, const double *tau,
                             int32_t *pred, double *tstar) {
  long n = cell_n_nodes(g);
  int32_t *hop = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  long *order = (long *)malloc(sizeof(long) * (size_t)n);
  long *nb = (long *)malloc(sizeof(long) * 16 * 64);
  long *nbc = (long *)malloc(sizeof(long) * 16 * 64);
  if (!hop || !order || !nb || !nbc) { free(hop); free(order); free(nb); free(nbc); return 1; }
  for (long i = 0; i < n; ++i) {
    pred[i] = -1;
    hop[i] = -1;
  }
  long head = 0, tail = 0;
  hop[src] = 0;
  order[tail++] = src;
  while (head < tail) {
    long i = order[head++];
    int m = cell_neighbours(g, i, nb, nbc);
    for (int b = 0; b < m; ++b) {
      long j = nb[b];
      if (hop[j] >= 0 || !isfinite(tau[j])) continue;
      if (tau[i] + cell_weight(g, field, nbc[b], i, j) == tau[j]) {
        hop[j] = hop[i] + 1;
        order[tail++] = j;
      }
    }
  }
  for (long t = 1; t < tail; ++t) {
    long j = order[t], bi = -1;
    int m = cell_neighbours(g, j, nb, nbc);
    for (int b = 0; b < m; ++b) {
      long i = nb[b];
      if (hop[i] < 0) continue;
      if (!(tau[i] + cell_weight(g, field, nbc[b], i, j) == tau[j])) continue;
      if (bi < 0 || hop[i] < hop[bi] || (hop[i] == hop[bi] && i < bi)) bi = i;
    }
    pred[j] = (int32_t)bi;
  }
  if (tstar) {
    for (long i = 0; i < n; ++i) tstar[i] = INFINITY;
    tstar[src] = 0.0;
    for (long t = 1; t < tail; ++t) {
      long j = order[t];
      tstar[j] = tstar[pred[j]] + cell_weight(g, 1, common_cell(g, pred[j], j), pred[j], j);
    }
  }
  free(hop);
  free(order);
  free(nb);
  free(nbc);
  return 0;
}

/* Both fields of one source on a network (outputs NULL to skip); t and p
 * are lattice-sized scratch. */
static int cell_fields(cellnet_t *g, long src, int block, double *t, int32_t *p,
                       double *tauR, double *tauI, int32_t *predP, int32_t *predA,
                       double *tstar) {
  long n = cell_n_nodes(g);
  for (int field = 0; field < 2; ++field) {
    double *out_t = field ? tauI : tauR;
    int32_t *out_p = field ? predA : predP;
    double *ts = field ? NULL : tstar;
    if (!out_t && !out_p && !ts) continue;
    if (block ? cell_block_march(g, field, src, t) : cell_dijkstra(g, field, src, t)) return 2;
    if (out_p || ts) {
      if (cell_predecessors(g, field, src, t, p, ts)) return 2;
      if (out_p) memcpy(out_p, p, sizeof(int32_t) * (size_t)n);
    }
    if (out_t) memcpy(out_t, t, sizeof(double) * (size_t)n);
  }
  return 0;
}

/* Trace one source on the cell network for one mode.  sampling 0: a
 * ray-direction cache of n_cols = n_dirs columns; 1: a slowness-sampled cache
 * of n_cols samples (RX, RZ: stored ray directions).  V, A, RX, RZ, st:
 * [K][n_cols] slices of the mode.  block != 0 computes the traveltimes with
 * the block marching instead of node Dijkstra.  Outputs (NULL to skip) are
 * lattice-sized; points inside cells stay +inf / -1. */
int orc_trace_cells_2d(long ncx, long ncz, int cn, double hx, double hz,
                       const int32_t *class_id, long K, int sampling, int n_cols,
                       const double *V, const double *A, const double *RX, const double *RZ,
                       const int32_t *st, long src, int block, double *tauR, double *tauI,
                       int32_t *predP, int32_t *predA, double *tstar) {
  if (ncx < 1 || ncz < 1 || cn < 1 || cn > 16 || !class_id) return 1;
  cellnet_t g = {.ncx = ncx, .ncz = ncz, .NX = ncx * cn + 1, .NZ = ncz * cn + 1, .cn = cn,
                 .side = 2 * cn + 1, .dim = 2, .ncy = 1, .NY = 1, .cls = class_id, .K = K,
                 .n_cols = n_cols, .V = V, .A = A, .st = st};
  long n = g.NX * g.NZ;
  if (src < 0 || src >= n || !cell_is_node(&g, src % g.NX, src / g.NX)) return 1;
  int n_o = g.side * g.side;
  int32_t *ox = (int32_t *)malloc(sizeof(int32_t) * n_o);
  int32_t *oz = (int32_t *)malloc(sizeof(int32_t) * n_o);
  double *t = (double *)malloc(sizeof(double) * (size_t)n);
  int32_t *p = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  g.L = (double *)malloc(sizeof(double) * n_o);
  int rc = 0;
  if (!ox || !oz || !t || !p || !g.L) { rc = 2; goto out; }
  for (int dz = -cn; dz <= cn; ++dz)
    for (int dx = -cn; dx <= cn; ++dx) {
      int o = cell_off(&g, dx, dz);
      ox[o] = (dx == 0 && dz == 0) ? 1 : dx; /* the centre is never a segment */
      oz[o] = dz;
      double ex = ox[o] * hx, ez = oz[o] * hz;
      g.L[o] = sqrt(ex * ex + ez * ez);
    }
  if (sampling == 0) {
    g.colR = (int32_t *)malloc(sizeof(int32_t) * n_o);
    if (!g.colR) { rc = 2; goto out; }
    /* nearest tabulated direction: the forward-star rule applied to the
     * segment (non-primitive offsets included) */
    for (int o = 0; o < n_o; ++o) g.colR[o] = bin_2d(ox[o], oz[o], hx, hz, n_cols);
  } else {
    g.best = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * n_o);
    if (!g.best) { rc = 2; goto out; }
    orc_slow_lookup(K, n_cols, RX, RZ, st, n_o, ox, oz, hx, hz, g.best);
  }
  rc = cell_fields(&g, src, block, t, p, tauR, tauI, predP, predA, tstar);
out:
  free(ox); free(oz); free(t); free(p); free(g.L); free(g.colR); free(g.best);
  return rc;
}


/* ------------------------------------------------------------------------ */
/* O-19  MSPM (Algorithm 1) on the cell network: no cache.  A segment's     */
/*       ray quantities at a cell corner come from a fresh solve at the     */
/*       segment's exact direction with the corner's class; at a node       */
/*       between two corners they are reconstructed from those corners      */
/* ------------------------------------------------------------------------ */

/* One fresh solve at global ray angle psi (eqs 9-11 through the sweep and
 * bisection of O-5): V, A and the status rules of cache entries. */
static int solve_angle_fresh(const double *cls, int mode, int reading, int n_sweep,
                             double psi, double *V, double *A) {
  medium_t m;
  load_medium(cls, &m);
  int fluid = (mode != ORC_QP) && (cls[3] == 0.0 || (mode == ORC_QSH && cls[4] == 0.0));
  if (fluid) return ORC_ST_FLUID;
  sample_t *tab = (sample_t *)malloc(sizeof(sample_t) * (size_t)n_sweep);
  if (!tab) return ORC_ST_NO_BRACKET;
  sweep(&m, mode, reading, n_sweep, tab);
  entry_t e;
  int st = solve_direction(&m, mode, reading, n_sweep, tab, wrap_pi(psi - m.tilt), &e);
  free(tab);
  if (st & ORC_ST_NO_BRACKET) return st;
  if (!(e.A >= 0.0) || !isfinite(e.V) || !(e.V > 0.0)) st |= ORC_ST_NONPHYS;
  if (!(e.res <= ORC_RESID_TOL)) st |= ORC_ST_NOCONV;
  *V = e.V;
  *A = e.A;
  return st;
}

/* The canonical one of offsets o and -o: direction angle in [0, pi). */
static int mspm_canon(const cellnet_t *g, long dx, long dz) {
  if (!(dx > 0 || (dx == 0 && dz > 0))) {
    dx = -dx;
    dz = -dz;
  }
  return cell_off(g, dx, dz);
}

/* Corner quantities of class k along canonical offset o (a reversed
 * segment has the same ray quantities).  Each (class, offset) pair is
 * solved once and reused: the solve is a pure function of them, so this
 * changes no value, only the oracle's run time. */
static int mspm_corner(cellnet_t *g, long k, int o, double *V, double *A) {
  long idx = k * g->side * g->side + o;
  if (g->mst[idx] < 0) {
    int dx = o % g->side - g->cn, dz = o / g->side - g->cn;
    double v = NAN, a = NAN;
    g->mst[idx] = solve_angle_fresh(g->classes + 13 * k, g->mode, g->reading, g->n_sweep,
                                    atan2(dx * g->hx, dz * g->hz), &v, &a);
    g->mV[idx] = v;
    g->mA[idx] = a;
  }
  *V = g->mV[idx];
  *A = g->mA[idx];
  return g->mst[idx];
}

/* Quantities of a node of cell c along canonical offset o: its own at a
 * corner; between corners c1 and c2 of its edge, at fraction t of the edge
 * from c1, q = q1 + t (q2 - q1) for V and A (linear reconstruction). */
static int mspm_node(cellnet_t *g, long c, long node, int o, double *V, double *A) {
  long x0 = (c % g->ncx) * g->cn, z0 = (c / g->ncx) * g->cn;
  long lx = node % g->NX - x0, lz = node / g->NX - z0;
  int cx = (lx == 0 || lx == g->cn), cz = (lz == 0 || lz == g->cn);
  if (cx && cz) return mspm_corner(g, g->cls[node], o, V, A);
  long c1, c2;
  double t;
  if (cz) { /* on a horizontal edge */
    c1 = x0 + g->NX * (z0 + lz);
    c2 = x0 + g->cn + g->NX * (z0 + lz);
    t = (double)lx / (double)g->cn;
  } else { /* on a vertical edge */
    c1 = x0 + lx + g->NX * z0;
    c2 = x0 + lx + g->NX * (z0 + g->cn);
    t = (double)lz / (double)g->cn;
  }
  double V1, A1, V2, A2;
  int s1 = mspm_corner(g, g->cls[c1], o, &V1, &A1);
  int s2 = mspm_corner(g, g->cls[c2], o, &V2, &A2);
  *V = V1 + t * (V2 - V1);
  *A = A1 + t * (A2 - A1);
  return s1 | s2;
}

static double mspm_weight(cellnet_t *g, int field, long c, long i, long j) {
  long dx = (j % g->NX) - (i % g->NX), dz = (j / g->NX) - (i / g->NX);
  int o = mspm_canon(g, dx, dz);
  double Vi, Ai, Vj, Aj;
  int si = mspm_node(g, c, i, o, &Vi, &Ai);
  int sj = mspm_node(g, c, j, o, &Vj, &Aj);
  const int bad = ORC_ST_NO_BRACKET | ORC_ST_FLUID | ORC_ST_NONPHYS | ORC_ST_NOCONV;
  if ((si & bad) || (sj & bad)) return INFINITY;
  double L = g->L[cell_off(g, dx, dz)];
  if (field == 0) return L / (0.5 * (Vi + Vj));
  return L * (0.5 * (Ai + Aj));
}

/* MSPM trace of one source for one mode on the cell network of the class
 * map (classes [K][13], reading MEV/OEV, n_sweep samples per solve); the
 * same outputs and predecessor rule as orc_trace_cells_2d.  *n_solves
 * (nullable) receives the number of distinct (class, direction) solves. */
int orc_trace_mspm_2d(long ncx, long ncz, int cn, double hx, double hz,
                      const int32_t *class_id, const double *classes, long K, int mode,
                      int reading, int n_sweep, long src, int block, double *tauR,
                      double *tauI, int32_t *predP, int32_t *predA, double *tstar,
                      long *n_solves) {
  if (ncx < 1 || ncz < 1 || cn < 1 || cn > 16 || !class_id || n_sweep < 8) return 1;
  cellnet_t g = {.ncx = ncx, .ncz = ncz, .NX = ncx * cn + 1, .NZ = ncz * cn + 1, .cn = cn,
                 .side = 2 * cn + 1, .dim = 2, .ncy = 1, .NY = 1, .cls = class_id, .K = K,
                 .mspm = 1, .classes = classes,
                 .mode = mode, .reading = reading, .n_sweep = n_sweep, .hx = hx, .hz = hz};
  long n = g.NX * g.NZ;
  if (src < 0 || src >= n || !cell_is_node(&g, src % g.NX, src / g.NX)) return 1;
  int n_o = g.side * g.side;
  double *t = (double *)malloc(sizeof(double) * (size_t)n);
  int32_t *p = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  g.L = (double *)malloc(sizeof(double) * n_o);
  g.mV = (double *)malloc(sizeof(double) * (size_t)K * n_o);
  g.mA = (double *)malloc(sizeof(double) * (size_t)K * n_o);
  g.mst = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * n_o);
  int rc = 0;
  if (!t || !p || !g.L || !g.mV || !g.mA || !g.mst) { rc = 2; goto out; }
  for (int dz = -cn; dz <= cn; ++dz)
    for (int dx = -cn; dx <= cn; ++dx) {
      double ex = dx * hx, ez = dz * hz;
      g.L[cell_off(&g, dx, dz)] = sqrt(ex * ex + ez * ez);
    }
  for (long q = 0; q < K * n_o; ++q) g.mst[q] = -1;
  rc = cell_fields(&g, src, block, t, p, tauR, tauI, predP, predA, tstar);
  if (n_solves) {
    long c = 0;
    for (long q = 0; q < K * n_o; ++q) c += g.mst[q] >= 0;
    *n_solves = c;
  }
out:
  free(t); free(p); free(g.L); free(g.mV); free(g.mA); free(g.mst);
  return rc;
}


/* ------------------------------------------------------------------------ */
/* O-20  the cell network in 3D: blocks (section on 3D extension, eq 35)    */
/* ------------------------------------------------------------------------ */

/* ncx x ncy x ncz blocks of cn intervals per side (hx, hy, hz).  Nodes are
 * the lattice points on a block face (any coordinate a multiple of cn),
 * indexed ix + NX (iy + NY iz); two nodes are joined when both lie on the
 * boundary of one block.  Weights follow eqs 28-30 with both ends reading the
 * Fibonacci direction closest to the segment (largest dot product with its
 * unit vector; the lowest index among equals, the 3D forward-star rule).
 * V, A, st: [K][N] slices of one mode of a 3D cache; outputs as for
 * orc_trace_cells_2d, lattice-sized, interior points +inf / -1. */
int orc_trace_blocks_3d(long ncx, long ncy, long ncz, int cn, double hx, double hy,
                        double hz, const int32_t *class_id, long K, int N, const double *V,
                        const double *A, const int32_t *st, long src, int block, double *tauR,
                        double *tauI, int32_t *predP, int32_t *predA, double *tstar) {
  if (ncx < 1 || ncy < 1 || ncz < 1 || cn < 1 || cn > 4 || !class_id || N < 2) return 1;
  cellnet_t g = {.ncx = ncx, .ncz = ncz, .NX = ncx * cn + 1, .NZ = ncz * cn + 1, .cn = cn,
                 .side = 2 * cn + 1, .dim = 3, .ncy = ncy, .NY = ncy * cn + 1,
                 .cls = class_id, .K = K, .n_cols = N, .V = V, .A = A, .st = st};
  long n = cell_n_nodes(&g);
  if (src < 0 || src >= n) return 1;
  {
    long x, y, z;
    cell_xyz(&g, src, &x, &y, &z);
    if (!(x % cn == 0 || y % cn == 0 || z % cn == 0)) return 1;
  }
  int n_o = g.side * g.side * g.side;
  double *t = (double *)malloc(sizeof(double) * (size_t)n);
  int32_t *p = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  double *f = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  g.L = (double *)malloc(sizeof(double) * n_o);
  g.colR = (int32_t *)malloc(sizeof(int32_t) * n_o);
  int rc = 0;
  if (!t || !p || !f || !g.L || !g.colR) { rc = 2; goto out; }
  orc_fibonacci(N, f);
  for (int z = -cn; z <= cn; ++z)
    for (int y = -cn; y <= cn; ++y)
      for (int x = -cn; x <= cn; ++x) {
        int o = cell_off3(&g, x, y, z);
        if (x == 0 && y == 0 && z == 0) { /* the centre is never a segment */
          g.L[o] = 0.0;
          g.colR[o] = 0;
          continue;
        }
        double dx = x * hx, dy = y * hy, dz = z * hz;
        double len = sqrt(dx * dx + dz * dz + dy * dy);
        double u0 = dx / len, u1 = dy / len, u2 = dz / len;
        int best = 0;
        double bd = -2.0;
        for (int i = 0; i < N; ++i) {
          double d = f[3 * i] * u0 + f[3 * i + 1] * u1 + f[3 * i + 2] * u2;
          if (d > bd) { bd = d; best = i; }
        }
        g.L[o] = len;
        g.colR[o] = best;
      }
  rc = cell_fields(&g, src, block, t, p, tauR, tauI, predP, predA, tstar);
out:
  free(t); free(p); free(f); free(g.L); free(g.colR);
  return rc;
}
