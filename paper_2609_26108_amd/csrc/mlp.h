// Learned surrogate of the cache solve: a 16 -> 128 -> 128 -> 128 -> 4 MLP
// with tanh hidden layers, BF16 weights and activations on the matrix cores
// (v_mfma_f32_16x16x{16,32}_bf16, FP32 accumulation), FP32 master weights
// and Adam moments.  It maps a class's moduli ratios, inverse quality factors
// (eq 2), the mode and the target ray angle to (theta_R - psi, theta_I,
// log V / sqrt(a33), A sqrt(a33)) (eqs 9-11); the cache builder uses the
// first two as the starting point of its Newton polish.
//
// Every product here is C[i][j] = sum_k A[i][k] Bt[j][k] with both operands
// stored k-contiguous (BF16, 16-byte aligned rows), computed per 16 x 16
// tile by one wavefront.  MFMA lane layout (gfx950): lane l holds
// A[l % 16][K0 + kk], Bt[l % 16][K0 + kk] for kk in [w (l / 16), w (l / 16) + w)
// with w = 8 (16x16x32) or 4 (16x16x16), and returns C[4 (l / 16) + t][l % 16]
// for t = 0..3.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "chert.h"

namespace chert {
namespace mlp {

constexpr int kIn = 16, kHid = 128, kOut = 4, kOutPad = 16;
// master parameter vector: W1[16][128] b1 W2[128][128] b2 W3[128][128] b3
// W4[128][4] b4; a layer maps x -> x W + b
constexpr int oW1 = 0;
constexpr int oB1 = oW1 + kIn * kHid;
constexpr int oW2 = oB1 + kHid;
constexpr int oB2 = oW2 + kHid * kHid;
constexpr int oW3 = oB2 + kHid;
constexpr int oB3 = oW3 + kHid * kHid;
constexpr int oW4 = oB3 + kHid;
constexpr int oB4 = oW4 + kHid * kOut;
constexpr int kParams = oB4 + kOut;  // 35716

// BF16 copies: forward operands Bt = W^T ([out][in]); backward operands
// Bt = W ([in][out]); the output layer padded to 16 columns with zeros.
constexpr int fW1 = 0;                      // [128][16]
constexpr int fW2 = fW1 + kHid * kIn;       // [128][128]
constexpr int fW3 = fW2 + kHid * kHid;      // [128][128]
constexpr int fW4 = fW3 + kHid * kHid;      // [16][128]
constexpr int kFwdN = fW4 + kOutPad * kHid;
constexpr int bW2 = 0;                      // [128][128]
constexpr int bW3 = bW2 + kHid * kHid;      // [128][128]
constexpr int bW4 = bW3 + kHid * kHid;      // [128][16]
constexpr int kBwdN = bW4 + kHid * kOutPad;

constexpr size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr uint32_t kMagic = 0x47534843u;  // 'CHSG'
constexpr uint32_t kVersion = 1;
constexpr size_t kOffNorm = 256;    // float in_mean[16], in_inv_std[16], out_mean[4], out_std[4]
constexpr size_t kOffMaster = 512;
constexpr size_t kOffM = kOffMaster + al256(kParams * 4);
constexpr size_t kOffV = kOffM + al256(kParams * 4);
constexpr size_t kOffFwd = kOffV + al256(kParams * 4);
constexpr size_t kOffBwd = kOffFwd + al256(kFwdN * 2);
constexpr size_t kBlobBytes = kOffBwd + al256(kBwdN * 2);

// Adam constants; 1 - beta is given rounded once (1.f - 0.999f would carry
// the 3e-8 rounding of 0.999f as a 3e-5 relative error)
constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kAdamEps = 1e-8f;
constexpr float kOneMinusBeta1 = 0.1f, kOneMinusBeta2 = 0.001f;

// per-workgroup gradient partial: kParams floats, then the loss sum
constexpr int kPartStride = 35776;  // >= kParams + 1, multiple of 64
constexpr int kRows = 32;           // samples per workgroup tile
constexpr int kThreads = 256;       // 4 wavefronts

struct Net {
  const float* norm;      // in_mean[16], in_inv[16], out_mean[4], out_std[4]
  const float* master;    // FP32 weights (biases read from here)
  const uint16_t* fwd;    // BF16 forward operands
  const uint16_t* bwd;    // BF16 backward operands
};

__host__ __device__ inline Net net_of(const void* blob) {
  const uint8_t* b = (const uint8_t*)blob;
  Net n;
  n.norm = (const float*)(b + kOffNorm);
  n.master = (const float*)(b + kOffMaster);
  n.fwd = (const uint16_t*)(b + kOffFwd);
  n.bwd = (const uint16_t*)(b + kOffBwd);
  return n;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest, ties to even (NaN stays NaN):
// gfx950's conversion instruction
__device__ __forceinline__ uint16_t to_bf16(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}

// tanh of a hidden pre-activation whose result is rounded to BF16 next:
// within 1e-6 relative (BF16's step is 4e-3).  Below |x| = 1/2 the odd
// Taylor series through x^11; above, 1 - 2 / (1 + e^{2|x|}) with the
// hardware exp2 and reciprocal.  Half the instructions of tanhf.
__device__ __forceinline__ float tanh_act(float x) {
  const float a = fabsf(x);
  const float s = a * a;
  float p = -0.008863235f;  // -1382/155925
  p = p * s + 0.021869489f;  // 62/2835
  p = p * s - 0.053968254f;  // -17/315
  p = p * s + 0.13333334f;   // 2/15
  p = p * s - 0.33333334f;   // -1/3
  const float small = a + a * s * p;
  const float e = __builtin_amdgcn_exp2f(a * 2.88539008f);  // e^{2a}
  const float big = 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
  return copysignf(a < 0.5f ? small : big, x);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// 16 x 16 tile of A Bt^T over K (multiple of 32); A, Bt point at the tile's
// first row; pa, pb are row pitches in elements
__device__ __forceinline__ f32x4 mma_k32(const uint16_t* A, int pa, const uint16_t* Bt, int pb,
                                         int K, int lane) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const uint16_t* a = A + (lane & 15) * pa + 8 * (lane >> 4);
  const uint16_t* b = Bt + (lane & 15) * pb + 8 * (lane >> 4);
  for (int k = 0; k < K; k += 32) {
    bf16x8 av = *reinterpret_cast<const bf16x8*>(a + k);
    bf16x8 bv = *reinterpret_cast<const bf16x8*>(b + k);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

// same for K = 16
__device__ __forceinline__ f32x4 mma_k16(const uint16_t* A, int pa, const uint16_t* Bt, int pb,
                                         int lane) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  s16x4 av = *reinterpret_cast<const s16x4*>(A + (lane & 15) * pa + 4 * (lane >> 4));
  s16x4 bv = *reinterpret_cast<const s16x4*>(Bt + (lane & 15) * pb + 4 * (lane >> 4));
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
}

// LDS row pitches (elements): +8 BF16 per row keeps 16-byte reads of 16
// consecutive rows on distinct banks
constexpr int kPX = kIn + 8;     // x  [32][16]
constexpr int kPH = kHid + 8;    // h, d [32][128]
constexpr int kPT = kRows + 8;   // transposed tiles [k][32]

// inference: kInferRows samples per workgroup (each wavefront loads a weight
// column block once and sweeps it over all row blocks); the hidden layers
// are computed in place (every product is held in registers until the whole
// tile has read its input)
constexpr int kInferRows = 64;
struct __align__(16) InferTile {
  uint16_t x[kInferRows * kPX];
  uint16_t h[kInferRows * kPH];
};

// training tile: activations in both orientations and one error buffer
struct __align__(16) TrainTile {
  uint16_t x[kRows * kPX];
  uint16_t xt[kIn * kPT];
  uint16_t h[3][kRows * kPH];
  uint16_t ht[3][kHid * kPT];
  uint16_t d[kRows * kPH];
  uint16_t dt[kHid * kPT];
  float loss[kThreads / 64];
};

// rows (4 (lane/16) + t) and column (lane % 16) of a tile's accumulator
__device__ __forceinline__ int acc_row(int lane, int t) { return 4 * (lane >> 4) + t; }
__device__ __forceinline__ int acc_col(int lane) { return lane & 15; }

// hidden layer: out = tanh(in W + b), tiles (rb in {0,1}) x (cb in {2w, 2w+1})
// of wavefront w; writes the BF16 activations row-major and, if ht != null,
// transposed
template <int K>
__device__ __forceinline__ void hidden_layer(const uint16_t* in, int pin, const uint16_t* Wt,
                                             const float* bias, uint16_t* out, uint16_t* ht,
                                             int wave, int lane) {
  for (int rb = 0; rb < 2; ++rb)
    for (int q = 0; q < 2; ++q) {
      const int cb = 2 * wave + q;
      f32x4 acc;
      if constexpr (K == 16)
        acc = mma_k16(in + rb * 16 * pin, pin, Wt + cb * 16 * K, K, lane);
      else
        acc = mma_k32(in + rb * 16 * pin, pin, Wt + cb * 16 * K, K, K, lane);
      const int col = cb * 16 + acc_col(lane);
      const float b = bias[col];
      for (int t = 0; t < 4; ++t) {
        const int row = rb * 16 + acc_row(lane, t);
        const uint16_t v = to_bf16(tanhf(acc[t] + b));
        out[row * kPH + col] = v;
        if (ht) ht[col * kPT + row] = v;
      }
    }
}

// stage R standardised input rows (BF16) into the tile; src(r, i) is the
// raw input i of row r, NaN for a padding row (staged as zero)
template <bool kTrans, int R = kRows, typename Src>
__device__ __forceinline__ void stage_x(const Net& n, uint16_t* tx, uint16_t* txt, Src src) {
  for (int q = threadIdx.x; q < R * kIn; q += blockDim.x) {
    const int r = q / kIn, i = q % kIn;
    const float v = src(r, i);
    const uint16_t h = isnan(v) ? (uint16_t)0 : to_bf16((v - n.norm[i]) * n.norm[16 + i]);
    tx[r * kPX + i] = h;
    if (kTrans) txt[i * kPT + r] = h;
  }
}

// inference layer over kInferRows rows: out = tanh(in W + b); wavefront w
// owns column blocks 2w and 2w + 1, keeps each one's weight fragments in
// registers and runs it over every row block (same products, in the same
// k order, as hidden_layer).  out may alias in: all threads pass a barrier
// between the last read of in and the first write of out.
template <int K>
__device__ __forceinline__ void infer_layer(const uint16_t* in, int pin, const uint16_t* Wt,
                                            const float* bias, uint16_t* out, int wave, int lane) {
  constexpr int RB = kInferRows / 16;
  f32x4 acc[2][RB];
  for (int q = 0; q < 2; ++q) {
    const int cb = 2 * wave + q;
    if constexpr (K == 16) {
      const s16x4 bv =
          *reinterpret_cast<const s16x4*>(Wt + (cb * 16 + (lane & 15)) * K + 4 * (lane >> 4));
      for (int rb = 0; rb < RB; ++rb) {
        const s16x4 av = *reinterpret_cast<const s16x4*>(in + (rb * 16 + (lane & 15)) * pin +
                                                         4 * (lane >> 4));
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
        acc[q][rb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, z, 0, 0, 0);
      }
    } else {
      bf16x8 bv[K / 32];
      const uint16_t* wb = Wt + (cb * 16 + (lane & 15)) * K + 8 * (lane >> 4);
      for (int kk = 0; kk < K / 32; ++kk) bv[kk] = *reinterpret_cast<const bf16x8*>(wb + 32 * kk);
      for (int rb = 0; rb < RB; ++rb) {
        const uint16_t* a = in + (rb * 16 + (lane & 15)) * pin + 8 * (lane >> 4);
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        for (int kk = 0; kk < K / 32; ++kk)
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(a + 32 * kk),
                                                      bv[kk], c, 0, 0, 0);
        acc[q][rb] = c;
      }
    }
  }
  __syncthreads();
  for (int q = 0; q < 2; ++q) {
    const int col = (2 * wave + q) * 16 + acc_col(lane);
    const float b = bias[col];
    for (int rb = 0; rb < RB; ++rb)
      for (int t = 0; t < 4; ++t)
        out[(rb * 16 + acc_row(lane, t)) * kPH + col] = to_bf16(tanh_act(acc[q][rb][t] + b));
  }
}

// forward pass of a staged tile (all kThreads threads); store(r, c, v)
// receives the de-standardised output c of row r
template <typename Store>
__device__ __forceinline__ void forward_infer(const Net& n, InferTile& t, Store store) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  infer_layer<kIn>(t.x, kPX, n.fwd + fW1, n.master + oB1, t.h, wave, lane);
  __syncthreads();
  infer_layer<kHid>(t.h, kPH, n.fwd + fW2, n.master + oB2, t.h, wave, lane);
  __syncthreads();
  infer_layer<kHid>(t.h, kPH, n.fwd + fW3, n.master + oB3, t.h, wave, lane);
  __syncthreads();
  // output layer: one (padded) column block, row blocks spread over the waves
  const int col = acc_col(lane);
  bf16x8 bv[kHid / 32];
  const uint16_t* wb = n.fwd + fW4 + (lane & 15) * kHid + 8 * (lane >> 4);
  for (int kk = 0; kk < kHid / 32; ++kk) bv[kk] = *reinterpret_cast<const bf16x8*>(wb + 32 * kk);
  for (int rb = wave; rb < kInferRows / 16; rb += kThreads / 64) {
    const uint16_t* a = t.h + (rb * 16 + (lane & 15)) * kPH + 8 * (lane >> 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < kHid / 32; ++kk)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(a + 32 * kk),
                                                    bv[kk], acc, 0, 0, 0);
    if (col < kOut)
      for (int tt = 0; tt < 4; ++tt)
        store(rb * 16 + acc_row(lane, tt), col,
              (acc[tt] + n.master[oB4 + col]) * n.norm[36 + col] + n.norm[32 + col]);
  }
}

// standardised BF16 input row r of an inference tile from its 16 raw inputs
// (a padding row or a NaN input is staged as zero, as in stage_x)
__device__ __forceinline__ void stage_row(const Net& n, uint16_t* tx, int r, const float* f,
                                          bool pad) {
  for (int i = 0; i < kIn; ++i)
    tx[r * kPX + i] =
        (pad || isnan(f[i])) ? (uint16_t)0 : to_bf16((f[i] - n.norm[i]) * n.norm[16 + i]);
}

// the 16 network inputs of (class, mode, local target ray angle)
__device__ __forceinline__ void features(const chert_class& c, int mode, double psi,
                                         float* f) {
  const double inv33 = 1.0 / c.a33;
  f[0] = (float)(c.a11 * inv33 - 1.0);
  f[1] = (float)(c.a13 * inv33);
  f[2] = (float)(c.a44 * inv33);
  f[3] = (float)(c.a66 * inv33);
  const double* q = &c.q11;
  for (int i = 0; i < 5; ++i) f[4 + i] = isinf(q[i]) ? 0.f : (float)(1.0 / q[i]);
  for (int m = 0; m < 3; ++m) f[9 + m] = (mode == m) ? 1.f : 0.f;
  double s, co, s2, c2;
  sincos(psi, &s, &co);
  sincos(2.0 * psi, &s2, &c2);
  f[12] = (float)co;
  f[13] = (float)s;
  f[14] = (float)c2;
  f[15] = (float)s2;
}

}  // namespace mlp
}  // namespace chert
