// Host-only entry points of the C ABI: error reporting, the constitutive
// step, cache layout, forward-star geometry and raypath extraction.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "chert.h"
#include "chert_internal.h"

#pragma clang fp contract(off)

namespace chert {

static thread_local char g_err[512] = "";

int fail(int code, const char* msg) {
  snprintf(g_err, sizeof(g_err), "%s", msg ? msg : "");
  return code;
}

static int gcd_i(int a, int b) {
  a = abs(a);
  b = abs(b);
  while (b) {
    int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Nearest tabulated direction of an edge (the cached direction closest to
// the edge vector).  The bin is rounded on the half of the star with
// direction angle in [0, pi) (ox > 0, or ox == 0 and oz > 0); the reversed
// offset takes the diametrically opposite bin, so bin(-o) = bin(o) + n_dirs/2
// also where the angle falls exactly between two tabulated directions.
int32_t star_bin_2d(int x, int z, double hx, double hz, int n_dirs) {
  const bool canon = x > 0 || (x == 0 && z > 0);
  const double dx = (canon ? x : -x) * hx, dz = (canon ? z : -z) * hz;
  long b = lround(atan2(dx, dz) * n_dirs / (2.0 * M_PI));
  if (!canon) b += n_dirs / 2;
  b %= n_dirs;
  if (b < 0) b += n_dirs;
  return (int32_t)b;
}

int star_2d(int R, double hx, double hz, int n_dirs, int32_t* ox, int32_t* oz, double* L,
            int32_t* bin) {
  int n = 0;
  for (int z = -R; z <= R; ++z) {
    for (int x = -R; x <= R; ++x) {
      if ((x == 0 && z == 0) || gcd_i(x, z) != 1) continue;
      if (ox) {
        double dx = x * hx, dz = z * hz;
        ox[n] = x;
        oz[n] = z;
        L[n] = sqrt(dx * dx + dz * dz);  // eq 27, IEEE sqrt
        bin[n] = star_bin_2d(x, z, hx, hz, n_dirs);
      }
      ++n;
    }
  }
  return n;
}

int star_columns(const chert_cache_desc* d, const int32_t* bin, int n_off, int32_t* col) {
  for (int o = 0; o < n_off; ++o) {
    int c = bin[o];
    if (d->n_subset) {
      c = -1;
      for (int q = 0; q < d->n_subset; ++q)
        if (d->subset_host[q] == bin[o]) c = q;
    }
    if (c < 0) return fail(CHERT_ERR_INVALID_ARG, "the cache lacks a direction of the star");
    col[o] = c;
  }
  return CHERT_OK;
}

void fibonacci(int N, double* f) {
  const double ga = M_PI * (3.0 - sqrt(5.0));
  for (int i = 0; i < N; ++i) {
    const double z = 1.0 - (2.0 * i + 1.0) / N;
    const double r = sqrt(1.0 - z * z);
    const double ph = i * ga;
    f[3 * i] = r * cos(ph);
    f[3 * i + 1] = r * sin(ph);
    f[3 * i + 2] = z;
  }
}

int star_3d(int R, double hx, double hy, double hz, int N, int32_t* ox, int32_t* oy, int32_t* oz,
            double* L, int32_t* bin) {
  std::vector<double> f;
  if (ox) {
    f.resize(3 * (size_t)N);
    fibonacci(N, f.data());
  }
  int n = 0;
  for (int y = -R; y <= R; ++y)
    for (int z = -R; z <= R; ++z)
      for (int x = -R; x <= R; ++x) {
        if ((x == 0 && y == 0 && z == 0) || gcd_i(gcd_i(x, y), z) != 1) continue;
        if (ox) {
          const double dx = x * hx, dy = y * hy, dz = z * hz;
          const double len = sqrt(dx * dx + dz * dz + dy * dy);  // eq 27 in 3D
          const double u0 = dx / len, u1 = dy / len, u2 = dz / len;
          int best = 0;
          double bd = -2.0;
          for (int i = 0; i < N; ++i) {  // nearest tabulated direction
            const double dd = f[3 * i] * u0 + f[3 * i + 1] * u1 + f[3 * i + 2] * u2;
            if (dd > bd) {
              bd = dd;
              best = i;
            }
          }
          ox[n] = x;
          oy[n] = y;
          oz[n] = z;
          L[n] = len;
          bin[n] = best;
        }
        ++n;
      }
  return n;
}

// ------------------------------------------------------------ profiling --

struct ProfRec {
  std::string name;
  hipEvent_t start, stop;
};
static bool g_prof_on = false;
static std::string g_prof_only;           // empty: every kernel
static std::vector<ProfRec> g_prof;       // records of this profiling window
static std::vector<hipEvent_t> g_pool;    // reusable events

static hipEvent_t pool_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int prof_begin(const char* name, hipStream_t s) {
  if (!g_prof_on) return -1;
  if (!g_prof_only.empty() && g_prof_only != name) return -1;
  ProfRec r;
  r.name = name;
  r.start = pool_event();
  r.stop = pool_event();
  if (!r.start || !r.stop) return -1;
  hipEventRecord(r.start, s);
  g_prof.push_back(r);
  return (int)g_prof.size() - 1;
}

void prof_end(int slot, hipStream_t s) {
  if (slot < 0 || slot >= (int)g_prof.size()) return;
  hipEventRecord(g_prof[slot].stop, s);
}

bool prof_suspend() {
  const bool was = g_prof_on;
  g_prof_on = false;
  return was;
}

void prof_resume(bool was) { g_prof_on = was; }

static void prof_recycle() {
  for (auto& r : g_prof) {
    g_pool.push_back(r.start);
    g_pool.push_back(r.stop);
  }
  g_prof.clear();
}

}  // namespace chert

using namespace chert;

extern "C" int chert_prof_enable(int32_t on, const char* only) {
  if (on) prof_recycle();
  g_prof_only = only ? only : "";
  g_prof_on = on != 0;
  return CHERT_OK;
}

extern "C" int chert_prof_read(chert_prof_entry* out, int32_t capacity, int32_t* n_out) {
  if (!n_out) return fail(CHERT_ERR_INVALID_ARG, "null count");
  std::vector<chert_prof_entry> acc;
  for (auto& r : g_prof) {
    hipError_t e = hipEventSynchronize(r.stop);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
    if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
    size_t k = 0;
    for (; k < acc.size(); ++k)
      if (r.name == acc[k].name) break;
    if (k == acc.size()) {
      chert_prof_entry z{};
      snprintf(z.name, sizeof(z.name), "%s", r.name.c_str());
      acc.push_back(z);
    }
    acc[k].launches += 1;
    acc[k].total_ms += ms;
  }
  *n_out = (int32_t)acc.size();
  if (out)
    for (int32_t i = 0; i < capacity && i < (int32_t)acc.size(); ++i) out[i] = acc[i];
  return CHERT_OK;
}

extern "C" const char* chert_last_error(void) { return g_err; }

extern "C" int chert_class_from_thomsen(double vp0, double vs0, double rho, double eps,
                                        double delta, double gamma, double tilt,
                                        double azimuth, double qp, double qs,
                                        chert_class* out) {
  if (!out) return fail(CHERT_ERR_INVALID_ARG, "null output");
  double v[] = {vp0, vs0, rho, eps, delta, gamma, tilt, azimuth, qp, qs};
  for (double x : v)
    if (isnan(x)) return fail(CHERT_ERR_INVALID_ARG, "NaN Thomsen parameter");
  if (!(vp0 > 0.0) || vs0 < 0.0 || !(vs0 < vp0))
    return fail(CHERT_ERR_INVALID_ARG, "need vp0 > vs0 >= 0");
  if (!(qp > 0.0) || !(qs > 0.0)) return fail(CHERT_ERR_INVALID_ARG, "Q must be positive");
  // exact Thomsen (1986) relations for the real moduli
  double a33 = vp0 * vp0;
  double a44 = vs0 * vs0;
  double rad = 2.0 * delta * a33 * (a33 - a44) + (a33 - a44) * (a33 - a44);
  if (!(rad >= 0.0)) return fail(CHERT_ERR_INVALID_ARG, "negative a13 radicand");
  out->a11 = a33 * (1.0 + 2.0 * eps);
  out->a13 = sqrt(rad) - a44;
  out->a33 = a33;
  out->a44 = a44;
  out->a66 = a44 * (1.0 + 2.0 * gamma);
  out->q11 = out->q13 = out->q33 = qp;
  out->q44 = out->q66 = qs;
  out->rho = rho;
  out->tilt = tilt;
  out->azimuth = azimuth;
  return CHERT_OK;
}

// Device batch of the constitutive step for per-node media.  Same relations
// and operation order as chert_class_from_thomsen (this file is built
// without floating-point contraction, so both agree bitwise).
__global__ void k_classes_from_thomsen(const double* p, int64_t n, chert_class* out) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double* r = p + 10 * t;
    const double vp0 = r[0], vs0 = r[1], rho = r[2], eps = r[3], delta = r[4], gamma = r[5];
    const double tilt = r[6], azimuth = r[7], qp = r[8], qs = r[9];
    bool ok = true;
    for (int i = 0; i < 10; ++i) ok = ok && !isnan(r[i]);
    ok = ok && vp0 > 0.0 && vs0 >= 0.0 && vs0 < vp0 && qp > 0.0 && qs > 0.0;
    const double a33 = vp0 * vp0;
    const double a44 = vs0 * vs0;
    const double rad = 2.0 * delta * a33 * (a33 - a44) + (a33 - a44) * (a33 - a44);
    ok = ok && rad >= 0.0;
    chert_class c;
    c.a11 = ok ? a33 * (1.0 + 2.0 * eps) : NAN;
    c.a13 = ok ? sqrt(rad) - a44 : NAN;
    c.a33 = ok ? a33 : NAN;
    c.a44 = ok ? a44 : NAN;
    c.a66 = ok ? a44 * (1.0 + 2.0 * gamma) : NAN;
    c.q11 = c.q13 = c.q33 = qp;
    c.q44 = c.q66 = qs;
    c.rho = rho;
    c.tilt = tilt;
    c.azimuth = azimuth;
    out[t] = c;
  }
}

extern "C" int chert_classes_from_thomsen(const double* params_dev, int64_t n,
                                          chert_class* out_dev, void* stream) {
  if (!params_dev || !out_dev || n <= 0) return fail(CHERT_ERR_INVALID_ARG, "bad arguments");
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  CHERT_LAUNCH("k_classes_from_thomsen", k_classes_from_thomsen, dim3((unsigned)blocks),
               dim3(256), 0, (hipStream_t)stream, params_dev, n, out_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  return CHERT_OK;
}

extern "C" int chert_cache_layout_of(const chert_cache_desc* d, int64_t n_classes,
                                     chert_cache_layout* out) {
  if (!d || !out) return fail(CHERT_ERR_INVALID_ARG, "null desc or output");
  if (d->dim != 2 && d->dim != 3) return fail(CHERT_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (d->dim == 3) {
    if (d->n_dirs < 2 || d->n_dirs > kMaxFibonacci)
      return fail(CHERT_ERR_INVALID_ARG, "3D n_dirs (Fibonacci directions) must be 2..1048576");
    if (d->n_subset != 0)
      return fail(CHERT_ERR_UNSUPPORTED, "3D caches hold every direction (no subset)");
  } else if (d->n_dirs < 4 || (d->n_dirs & 1)) {
    return fail(CHERT_ERR_INVALID_ARG, "n_dirs must be even, >= 4");
  }
  if ((d->mode_mask & ~7u) != 0) return fail(CHERT_ERR_INVALID_ARG, "bad mode mask");
  if (d->kernel != CHERT_KERNEL_MEV && d->kernel != CHERT_KERNEL_OEV)
    return fail(CHERT_ERR_INVALID_ARG, "bad kernel");
  if (d->n_sweep < 16) return fail(CHERT_ERR_INVALID_ARG, "n_sweep must be >= 16");
  if (n_classes <= 0) return fail(CHERT_ERR_INVALID_ARG, "n_classes must be positive");
  if (!(d->resid_tol >= 0.0) || !isfinite(d->resid_tol))
    return fail(CHERT_ERR_INVALID_ARG, "resid_tol must be finite and >= 0");
  if (d->max_iter < 0) return fail(CHERT_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (d->sampling != CHERT_SAMPLE_RAY && d->sampling != CHERT_SAMPLE_SLOWNESS)
    return fail(CHERT_ERR_INVALID_ARG, "sampling must be CHERT_SAMPLE_RAY or _SLOWNESS");
  if (d->sampling == CHERT_SAMPLE_SLOWNESS && (d->dim != 2 || d->n_subset != 0))
    return fail(CHERT_ERR_UNSUPPORTED, "slowness-sampled caches are 2D, without subsets");
  if (d->n_subset != 0) {
    if (d->n_subset < 0 || d->n_subset > kMaxSubset || !d->subset_host || (d->n_subset & 1))
      return fail(CHERT_ERR_INVALID_ARG, "subset needs 2..512 (even) directions");
    const int half = d->n_dirs / 2;
    for (int i = 0; i < d->n_subset; ++i) {
      int b = d->subset_host[i];
      if (b < 0 || b >= d->n_dirs || (i > 0 && b <= d->subset_host[i - 1]))
        return fail(CHERT_ERR_INVALID_ARG, "subset must be ascending directions in range");
      // partner b + half (mod n_dirs) must be present
      int pb = (b + half) % d->n_dirs, lo = 0, hi = d->n_subset - 1;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (d->subset_host[mid] < pb) lo = mid + 1;
        else hi = mid;
      }
      if (d->subset_host[lo] != pb)
        return fail(CHERT_ERR_INVALID_ARG, "subset not closed under reversal");
    }
  }
  const int n_cols = d->n_subset ? d->n_subset : d->n_dirs;
  size_t entries = (size_t)3 * (size_t)n_classes * (size_t)n_cols;
  out->fields_offset = kHeaderBytes;
  out->status_offset = kHeaderBytes + entries * CHERT_NF * sizeof(double);
  size_t end = out->status_offset + entries * sizeof(int32_t);
  out->total_bytes = (end + 255) & ~(size_t)255;
  return CHERT_OK;
}

extern "C" int chert_star_3d(int32_t radius, double hx, double hy, double hz, int32_t n_dirs,
                             int32_t* ox, int32_t* oy, int32_t* oz, double* len, int32_t* bin) {
  if (radius < 1 || radius > kMaxRadius3 || !(hx > 0.0) || !(hy > 0.0) || !(hz > 0.0) ||
      n_dirs < 2 || n_dirs > kMaxFibonacci) {
    fail(CHERT_ERR_INVALID_ARG, "bad star arguments");
    return -1;
  }
  if (ox && (!oy || !oz || !len || !bin)) {
    fail(CHERT_ERR_INVALID_ARG, "star arrays must all be given");
    return -1;
  }
  return star_3d(radius, hx, hy, hz, n_dirs, ox, oy, oz, len, bin);
}

extern "C" int chert_star_2d(int32_t radius, double hx, double hz, int32_t n_dirs,
                             int32_t* ox, int32_t* oz, double* len, int32_t* bin) {
  if (radius < 1 || radius > kMaxRadius || !(hx > 0.0) || !(hz > 0.0) || n_dirs < 4) {
    fail(CHERT_ERR_INVALID_ARG, "bad star arguments");
    return -1;
  }
  if (ox && (!oz || !len || !bin)) {
    fail(CHERT_ERR_INVALID_ARG, "star arrays must all be given");
    return -1;
  }
  return star_2d(radius, hx, hz, n_dirs, ox, oz, len, bin);
}

extern "C" int chert_extract_raypath(const int32_t* pred_host, int64_t n_nodes, int64_t src,
                                     int64_t rcv, int64_t* path_out, int64_t capacity,
                                     int64_t* path_len) {
  if (!pred_host || !path_len || n_nodes <= 0)
    return fail(CHERT_ERR_INVALID_ARG, "null pred/path_len or empty grid");
  if (src < 0 || src >= n_nodes || rcv < 0 || rcv >= n_nodes)
    return fail(CHERT_ERR_INVALID_ARG, "source or receiver out of range");
  // eq 33: walk the parent pointers from the receiver back to the source
  int64_t count = 1;
  int64_t cur = rcv;
  while (cur != src) {
    int64_t p = pred_host[cur];
    if (p < 0) return fail(CHERT_ERR_UNREACHABLE, "receiver not reachable from source");
    if (p >= n_nodes) return fail(CHERT_ERR_INVALID_ARG, "predecessor out of range");
    if (++count > n_nodes) return fail(CHERT_ERR_CYCLE, "predecessor chain has a cycle");
    cur = p;
  }
  *path_len = count;
  if (count > capacity || !path_out) return fail(CHERT_ERR_CAPACITY, "path buffer too small");
  // eq 34: list the nodes from the source to the receiver
  cur = rcv;
  for (int64_t q = count - 1; q >= 0; --q) {
    path_out[q] = cur;
    if (q > 0) cur = pred_host[cur];
  }
  return CHERT_OK;
}
