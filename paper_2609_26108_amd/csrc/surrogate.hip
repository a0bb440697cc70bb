// Training and inference of the cache-solve surrogate (see mlp.h) on the
// gfx950 matrix cores.
//   k_sg_init      header, master weights from the caller, zero moments,
//                  identity standardisation, BF16 copies
//   k_sg_dataset   (features, targets, usable) of every entry of a cache
//   k_sg_norm      per-column mean and standard deviation of the usable
//                  samples (FP64 sums, one workgroup, fixed order)
//   k_sg_grad      one workgroup per 32 samples: forward with activations
//                  kept in LDS, MSE error, backward; writes that tile's
//                  gradient and loss partial
//   k_sg_reduce    sums the partials in workgroup order (deterministic)
//   k_sg_adam      Adam on the FP32 master weights, refreshes BF16 copies
//   k_sg_infer     forward of 64 samples per workgroup
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "chert.h"
#include "chert_internal.h"
#include "mlp.h"

namespace chert {
using namespace mlp;

namespace {

// BF16 operand slots of master parameter p (fwd index, bwd index or -1)
__device__ __forceinline__ void bf16_slots(int p, int* fi, int* bi) {
  *fi = -1;
  *bi = -1;
  if (p < oB1) {  // W1[i][j]
    int i = p / kHid, j = p % kHid;
    *fi = fW1 + j * kIn + i;
  } else if (p >= oW2 && p < oB2) {
    int q = p - oW2, i = q / kHid, j = q % kHid;
    *fi = fW2 + j * kHid + i;
    *bi = bW2 + i * kHid + j;
  } else if (p >= oW3 && p < oB3) {
    int q = p - oW3, i = q / kHid, j = q % kHid;
    *fi = fW3 + j * kHid + i;
    *bi = bW3 + i * kHid + j;
  } else if (p >= oW4 && p < oB4) {
    int q = p - oW4, i = q / kOut, j = q % kOut;
    *fi = fW4 + j * kHid + i;
    *bi = bW4 + i * kOutPad + j;
  }
}

__global__ void __launch_bounds__(256) k_sg_init(uint8_t* blob, const float* params) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  float* master = (float*)(blob + kOffMaster);
  float* m = (float*)(blob + kOffM);
  float* v = (float*)(blob + kOffV);
  uint16_t* fwd = (uint16_t*)(blob + kOffFwd);
  uint16_t* bwd = (uint16_t*)(blob + kOffBwd);
  if (p < kFwdN) fwd[p] = 0;  // padding rows stay zero
  if (p < kBwdN) bwd[p] = 0;
  if (blockIdx.x == 0) {
    uint32_t* h = (uint32_t*)blob;
    if (threadIdx.x < 64) h[threadIdx.x] = 0u;
    // identity standardisation: means 0, inverse input scales 1, output scales 1
    float* nrm = (float*)(blob + kOffNorm);
    const int i = threadIdx.x;
    if (i < 40) nrm[i] = ((i >= 16 && i < 32) || i >= 36) ? 1.f : 0.f;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    uint32_t* h = (uint32_t*)blob;
    h[0] = kMagic;
    h[1] = kVersion;
    h[2] = kIn;
    h[3] = kHid;
    h[4] = kOut;
    h[5] = kParams;
  }
  if (p >= kParams) return;
  const float w = params[p];
  master[p] = w;
  m[p] = 0.f;
  v[p] = 0.f;
}

// second pass: BF16 copies (after the zero fill of the first launch)
__global__ void __launch_bounds__(256) k_sg_copies(uint8_t* blob) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float w = ((const float*)(blob + kOffMaster))[p];
  int fi, bi;
  bf16_slots(p, &fi, &bi);
  const uint16_t h = to_bf16(w);
  if (fi >= 0) ((uint16_t*)(blob + kOffFwd))[fi] = h;
  if (bi >= 0) ((uint16_t*)(blob + kOffBwd))[bi] = h;
}

struct DatasetArgs {
  const chert_class* classes;
  int64_t n_classes;
  const double* fields;    // cache fields [NF][3][K][n_cols]
  const int32_t* status;   // [3][K][n_cols]
  int n_modes;
  int modes[3];
  int n_cols;
  int n_dirs;
  int16_t dir[kMaxSubset];  // direction of each column
  float* x;
  float* y;
  int32_t* ok;
};

__global__ void __launch_bounds__(256) k_sg_dataset(DatasetArgs a) {
  const int64_t total = (int64_t)a.n_modes * a.n_classes * a.n_cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(e % a.n_cols);
    const int64_t job = e / a.n_cols;
    const int64_t k = job % a.n_classes;
    const int mode = a.modes[job / a.n_classes];
    const chert_class c = a.classes[k];
    double psi = a.dir[col] * (6.28318530717958647692 / a.n_dirs) - c.tilt;
    if (psi > 3.14159265358979323846) psi -= 6.28318530717958647692;
    else if (psi <= -3.14159265358979323846) psi += 6.28318530717958647692;
    float f[kIn];
    features(c, mode, psi, f);
    for (int i = 0; i < kIn; ++i) a.x[e * kIn + i] = f[i];
    const int64_t stride = 3 * a.n_classes * (int64_t)a.n_cols;
    const int64_t slot = ((int64_t)mode * a.n_classes + k) * a.n_cols + col;
    const double V = a.fields[CHERT_F_V * stride + slot];
    const double A = a.fields[CHERT_F_A * stride + slot];
    const double thR = a.fields[CHERT_F_THR * stride + slot];
    const double thI = a.fields[CHERT_F_THI * stride + slot];
    const double s = sqrt(c.a33);
    double dth = thR - psi;
    if (dth > 3.14159265358979323846) dth -= 6.28318530717958647692;
    else if (dth <= -3.14159265358979323846) dth += 6.28318530717958647692;
    const int32_t st = a.status[slot];
    a.y[e * kOut + 0] = (float)dth;
    a.y[e * kOut + 1] = (float)thI;
    a.y[e * kOut + 2] = (float)log(V / s);
    a.y[e * kOut + 3] = (float)(A * s);
    a.ok[e] = (st == CHERT_ST_OK) ? 1 : 0;
  }
}

// mean and standard deviation of every input and target column over the
// usable samples; one workgroup, two passes, FP64 sums in a fixed order
__global__ void __launch_bounds__(1024) k_sg_norm(uint8_t* blob, const float* x, const float* y,
                                                  const int32_t* ok, int64_t n) {
  constexpr int kC = kIn + kOut;
  __shared__ double red[1024];
  __shared__ double mean[kC];
  __shared__ double cnt;
  float* nrm = (float*)(blob + kOffNorm);
  for (int pass = 0; pass < 2; ++pass) {
    double acc[kC];
    double c = 0.0;
#pragma unroll
    for (int i = 0; i < kC; ++i) acc[i] = 0.0;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
      if (!ok[e]) continue;
      c += 1.0;
#pragma unroll
      for (int i = 0; i < kC; ++i) {
        const double v = i < kIn ? x[e * kIn + i] : y[e * kOut + (i - kIn)];
        if (pass == 0) acc[i] += v;
        else {
          const double dv = v - mean[i];
          acc[i] += dv * dv;
        }
      }
    }
#pragma unroll
    for (int i = -1; i < kC; ++i) {
      red[threadIdx.x] = i < 0 ? c : acc[i];
      __syncthreads();
      for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        if (i < 0) cnt = red[0];
        else if (pass == 0) mean[i] = cnt > 0.0 ? red[0] / cnt : 0.0;
        else {
          double sd = cnt > 0.0 ? sqrt(red[0] / cnt) : 0.0;
          if (!(sd > 0.0)) sd = 1.0;
          if (i < kIn) {
            nrm[i] = (float)mean[i];
            nrm[16 + i] = (float)(1.0 / sd);
          } else {
            nrm[32 + (i - kIn)] = (float)mean[i];
            nrm[36 + (i - kIn)] = (float)sd;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_sg_infer(const uint8_t* blob, const float* x,
                                                       int64_t n_rows, float* y) {
  __shared__ InferTile t;
  const Net n = net_of(blob);
  const int64_t base = (int64_t)blockIdx.x * kInferRows;
  stage_x<false, kInferRows>(n, t.x, nullptr, [&](int r, int i) -> float {
    return base + r < n_rows ? x[(base + r) * kIn + i] : NAN;
  });
  __syncthreads();
  forward_infer(n, t, [&](int r, int c, float v) {
    if (base + r < n_rows) y[(base + r) * kOut + c] = v;
  });
}

// backward through one hidden layer's output error already in t.d / t.dt
// (BF16, rows = samples): weight and bias gradients of that layer into `part`
template <int KIN, int NOUT>
__device__ __forceinline__ void layer_grads(const uint16_t* at, const uint16_t* dt, float* part,
                                            int oW, int oB, int nvalid_out, int wave, int lane) {
  // dW[i][j] = sum_s a[s][i] d[s][j]: tiles (ib, jb), K = 32 samples
  constexpr int nib = KIN / 16, njb = NOUT / 16;
  for (int tix = wave; tix < nib * njb; tix += kThreads / 64) {
    const int ib = tix / njb, jb = tix % njb;
    const f32x4 acc = mma_k32(at + ib * 16 * kPT, kPT, dt + jb * 16 * kPT, kPT, kRows, lane);
    const int j = jb * 16 + acc_col(lane);
    if (j < nvalid_out)
      for (int t = 0; t < 4; ++t) {
        const int i = ib * 16 + acc_row(lane, t);
        part[oW + i * nvalid_out + j] = acc[t];
      }
  }
  for (int j = threadIdx.x; j < nvalid_out; j += blockDim.x) {
    float s = 0.f;
    for (int r = 0; r < kRows; ++r) s += from_bf16(dt[j * kPT + r]);
    part[oB + j] = s;
  }
}

// propagate the error through W (Bt = W [in=128][out=K]) and the tanh of
// the layer below (activations h): t.d <- (d W^T) * (1 - h^2)
template <int K>
__device__ __forceinline__ void back_error(TrainTile& t, const uint16_t* Wb, const uint16_t* h,
                                           int wave, int lane) {
  f32x4 acc[2][2];
  for (int rb = 0; rb < 2; ++rb)
    for (int q = 0; q < 2; ++q) {
      const int cb = 2 * wave + q;
      if constexpr (K == 16)
        acc[rb][q] = mma_k16(t.d + rb * 16 * kPH, kPH, Wb + cb * 16 * K, K, lane);
      else
        acc[rb][q] = mma_k32(t.d + rb * 16 * kPH, kPH, Wb + cb * 16 * K, K, K, lane);
    }
  __syncthreads();  // every wave has read t.d
  for (int rb = 0; rb < 2; ++rb)
    for (int q = 0; q < 2; ++q) {
      const int col = (2 * wave + q) * 16 + acc_col(lane);
      for (int tt = 0; tt < 4; ++tt) {
        const int row = rb * 16 + acc_row(lane, tt);
        const float hv = from_bf16(h[row * kPH + col]);
        const uint16_t v = to_bf16(acc[rb][q][tt] * (1.f - hv * hv));
        t.d[row * kPH + col] = v;
        t.dt[col * kPT + row] = v;
      }
    }
  __syncthreads();
}

__global__ void __launch_bounds__(kThreads) k_sg_grad(const uint8_t* blob, const float* x,
                                                      const float* y, const int32_t* idx,
                                                      int32_t batch, float* partials) {
  __shared__ TrainTile t;
  const Net n = net_of(blob);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int base = blockIdx.x * kRows;
  float* part = partials + (size_t)blockIdx.x * kPartStride;
  stage_x<true>(n, t.x, t.xt, [&](int r, int i) -> float {
    return base + r < batch ? x[(int64_t)idx[base + r] * kIn + i] : NAN;
  });
  __syncthreads();
  hidden_layer<kIn>(t.x, kPX, n.fwd + fW1, n.master + oB1, t.h[0], t.ht[0], wave, lane);
  __syncthreads();
  hidden_layer<kHid>(t.h[0], kPH, n.fwd + fW2, n.master + oB2, t.h[1], t.ht[1], wave, lane);
  __syncthreads();
  hidden_layer<kHid>(t.h[1], kPH, n.fwd + fW3, n.master + oB3, t.h[2], t.ht[2], wave, lane);
  // output layer and its error: d = 2 (out - y) / (batch * 4), zero on
  // padded rows and columns
  for (int q = threadIdx.x; q < kRows * kPH; q += blockDim.x) t.d[q] = 0;
  for (int q = threadIdx.x; q < kHid * kPT; q += blockDim.x) t.dt[q] = 0;
  __syncthreads();
  float lsum = 0.f;
  if (wave < 2) {
    const f32x4 acc = mma_k32(t.h[2] + wave * 16 * kPH, kPH, n.fwd + fW4, kHid, kHid, lane);
    const int col = acc_col(lane);
    const float scale = 2.f / ((float)batch * (float)kOut);
    if (col < kOut)
      for (int tt = 0; tt < 4; ++tt) {
        const int row = wave * 16 + acc_row(lane, tt);
        if (base + row >= batch) continue;
        const float ys = (y[(int64_t)idx[base + row] * kOut + col] - n.norm[32 + col]) /
                         n.norm[36 + col];
        const float e = acc[tt] + n.master[oB4 + col] - ys;
        lsum += e * e;
        const uint16_t v = to_bf16(scale * e);
        t.d[row * kPH + col] = v;
        t.dt[col * kPT + row] = v;
      }
  }
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
  if (lane == 0) t.loss[wave] = lsum;
  __syncthreads();
  layer_grads<kHid, kOutPad>(t.ht[2], t.dt, part, oW4, oB4, kOut, wave, lane);
  back_error<kOutPad>(t, n.bwd + bW4, t.h[2], wave, lane);
  layer_grads<kHid, kHid>(t.ht[1], t.dt, part, oW3, oB3, kHid, wave, lane);
  back_error<kHid>(t, n.bwd + bW3, t.h[1], wave, lane);
  layer_grads<kHid, kHid>(t.ht[0], t.dt, part, oW2, oB2, kHid, wave, lane);
  back_error<kHid>(t, n.bwd + bW2, t.h[0], wave, lane);
  layer_grads<kIn, kHid>(t.xt, t.dt, part, oW1, oB1, kHid, wave, lane);
  if (threadIdx.x == 0) part[kParams] = t.loss[0] + t.loss[1] + t.loss[2] + t.loss[3];
}

__global__ void __launch_bounds__(256) k_sg_reduce(const float* partials, int n_parts,
                                                   int32_t batch, float* grad, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kParams) return;
  float s = 0.f;
  for (int w = 0; w < n_parts; ++w) s += partials[(size_t)w * kPartStride + p];
  if (p < kParams) grad[p] = s;
  else if (loss) *loss = s / ((float)batch * (float)kOut);
}

// bc1, bc2: the bias corrections 1 - beta^step, formed in FP64 on the host
__global__ void __launch_bounds__(256) k_sg_adam(uint8_t* blob, const float* grad, int32_t step,
                                                 float lr, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) ((int32_t*)blob)[6] = step;
  if (p >= kParams) return;
  float* master = (float*)(blob + kOffMaster);
  float* m = (float*)(blob + kOffM);
  float* v = (float*)(blob + kOffV);
  const float g = grad[p];
  const float mn = kBeta1 * m[p] + kOneMinusBeta1 * g;
  const float vn = kBeta2 * v[p] + kOneMinusBeta2 * g * g;
  const float mh = mn / bc1;
  const float vh = vn / bc2;
  const float w = master[p] - lr * mh / (sqrtf(vh) + kAdamEps);
  m[p] = mn;
  v[p] = vn;
  master[p] = w;
  int fi, bi;
  bf16_slots(p, &fi, &bi);
  const uint16_t h = to_bf16(w);
  if (fi >= 0) ((uint16_t*)(blob + kOffFwd))[fi] = h;
  if (bi >= 0) ((uint16_t*)(blob + kOffBwd))[bi] = h;
}

int check_blob(const void* blob) {
  if (!blob) return fail(CHERT_ERR_INVALID_ARG, "null surrogate blob");
  if (((uintptr_t)blob & 255u) != 0)
    return fail(CHERT_ERR_INVALID_ARG, "surrogate blob not 256-byte aligned");
  return CHERT_OK;
}

int launch_status() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CHERT_ERR_HIP, hipGetErrorString(e));
  return CHERT_OK;
}

}  // namespace
}  // namespace chert

using namespace chert;
using namespace chert::mlp;

extern "C" int chert_surrogate_layout_of(chert_surrogate_layout* out) {
  if (!out) return fail(CHERT_ERR_INVALID_ARG, "null layout");
  out->total_bytes = kBlobBytes;
  out->norm_offset = kOffNorm;
  out->params_offset = kOffMaster;
  out->adam_m_offset = kOffM;
  out->adam_v_offset = kOffV;
  out->n_params = kParams;
  out->n_in = kIn;
  out->n_hidden = kHid;
  out->n_out = kOut;
  return CHERT_OK;
}

extern "C" int chert_surrogate_init(void* blob_dev, const float* params_dev, void* stream) {
  int rc = check_blob(blob_dev);
  if (rc) return rc;
  if (!params_dev) return fail(CHERT_ERR_INVALID_ARG, "null initial parameters");
  hipStream_t s = (hipStream_t)stream;
  const int blocks = (kFwdN + 255) / 256;  // kFwdN > kBwdN > kParams
  CHERT_LAUNCH("k_sg_init", k_sg_init, dim3(blocks), dim3(256), 0, s, (uint8_t*)blob_dev,
               params_dev);
  CHERT_LAUNCH("k_sg_copies", k_sg_copies, dim3((kParams + 255) / 256), dim3(256), 0, s,
               (uint8_t*)blob_dev);
  return launch_status();
}

extern "C" int chert_surrogate_dataset(const chert_cache_desc* d, const void* cache_dev,
                                       const chert_class* classes_dev, int64_t n_classes,
                                       float* x_dev, float* y_dev, int32_t* ok_dev,
                                       void* stream) {
  chert_cache_layout lay;
  int rc = chert_cache_layout_of(d, n_classes, &lay);
  if (rc) return rc;
  if (!cache_dev || !classes_dev || !x_dev || !y_dev || !ok_dev)
    return fail(CHERT_ERR_INVALID_ARG, "null pointer");
  if (d->dim != 2) return fail(CHERT_ERR_UNSUPPORTED, "training samples come from 2D caches");
  DatasetArgs a{};
  a.classes = classes_dev;
  a.n_classes = n_classes;
  a.fields = (const double*)((const uint8_t*)cache_dev + lay.fields_offset);
  a.status = (const int32_t*)((const uint8_t*)cache_dev + lay.status_offset);
  for (int m = 0; m < 3; ++m)
    if (d->mode_mask & (1u << m)) a.modes[a.n_modes++] = m;
  a.n_dirs = d->n_dirs;
  a.n_cols = d->n_subset ? d->n_subset : d->n_dirs;
  if (a.n_cols > kMaxSubset) return fail(CHERT_ERR_INVALID_ARG, "too many directions");
  for (int c = 0; c < a.n_cols; ++c) a.dir[c] = (int16_t)(d->n_subset ? d->subset_host[c] : c);
  a.x = x_dev;
  a.y = y_dev;
  a.ok = ok_dev;
  const int64_t total = (int64_t)a.n_modes * n_classes * a.n_cols;
  if (total == 0) return CHERT_OK;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  CHERT_LAUNCH("k_sg_dataset", k_sg_dataset, dim3((unsigned)blocks), dim3(256), 0,
               (hipStream_t)stream, a);
  return launch_status();
}

extern "C" int chert_surrogate_fit_norm(void* blob_dev, const float* x_dev, const float* y_dev,
                                        const int32_t* ok_dev, int64_t n, void* stream) {
  int rc = check_blob(blob_dev);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!x_dev || !y_dev || !ok_dev)))
    return fail(CHERT_ERR_INVALID_ARG, "bad samples");
  CHERT_LAUNCH("k_sg_norm", k_sg_norm, dim3(1), dim3(1024), 0, (hipStream_t)stream,
               (uint8_t*)blob_dev, x_dev, y_dev, ok_dev, n);
  return launch_status();
}

extern "C" size_t chert_surrogate_grad_workspace_bytes(int32_t batch) {
  if (batch <= 0) return 0;
  return (size_t)((batch + kRows - 1) / kRows) * kPartStride * sizeof(float);
}

extern "C" int chert_surrogate_grad(const void* blob_dev, const float* x_dev, const float* y_dev,
                                    const int32_t* idx_dev, int32_t batch, float* grad_dev,
                                    float* loss_dev, void* workspace_dev, size_t workspace_bytes,
                                    void* stream) {
  int rc = check_blob(blob_dev);
  if (rc) return rc;
  if (batch <= 0 || !x_dev || !y_dev || !idx_dev || !grad_dev)
    return fail(CHERT_ERR_INVALID_ARG, "bad batch or null pointer");
  if (!workspace_dev || workspace_bytes < chert_surrogate_grad_workspace_bytes(batch))
    return fail(CHERT_ERR_INVALID_ARG, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const int parts = (batch + kRows - 1) / kRows;
  float* partials = (float*)workspace_dev;
  CHERT_LAUNCH("k_sg_grad", k_sg_grad, dim3(parts), dim3(kThreads), 0, s,
               (const uint8_t*)blob_dev, x_dev, y_dev, idx_dev, batch, partials);
  CHERT_LAUNCH("k_sg_reduce", k_sg_reduce, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s,
               partials, parts, batch, grad_dev, loss_dev);
  return launch_status();
}

extern "C" int chert_surrogate_adam(void* blob_dev, const float* grad_dev, int32_t step,
                                    float lr, void* stream) {
  int rc = check_blob(blob_dev);
  if (rc) return rc;
  if (!grad_dev || step < 1 || !(lr >= 0.f))
    return fail(CHERT_ERR_INVALID_ARG, "bad gradient, step or learning rate");
  const float bc1 = (float)(1.0 - pow(0.9, step));
  const float bc2 = (float)(1.0 - pow(0.999, step));
  CHERT_LAUNCH("k_sg_adam", k_sg_adam, dim3((kParams + 255) / 256), dim3(256), 0,
               (hipStream_t)stream, (uint8_t*)blob_dev, grad_dev, step, lr, bc1, bc2);
  return launch_status();
}

extern "C" int chert_surrogate_infer(const void* blob_dev, const float* x_dev, int64_t n,
                                     float* y_dev, void* stream) {
  int rc = check_blob(blob_dev);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!x_dev || !y_dev))) return fail(CHERT_ERR_INVALID_ARG, "bad samples");
  if (n == 0) return CHERT_OK;
  const int64_t blocks = (n + kInferRows - 1) / kInferRows;
  if (blocks > 0x7fffffffLL) return fail(CHERT_ERR_INVALID_ARG, "too many samples");
  CHERT_LAUNCH("k_sg_infer", k_sg_infer, dim3((unsigned)blocks), dim3(kThreads), 0,
               (hipStream_t)stream, (const uint8_t*)blob_dev, x_dev, n, y_dev);
  return launch_status();
}
