// Learned collision surrogate: 12 -> 64 -> 64 -> 9 network on bfloat16 matrix cores.
//
// All three layers are evaluated in transposed form, Z^T = W H^T, one wavefront per 64 samples,
// with v_mfma_f32_16x16x16_bf16 (D = A B + C, A 16x16 rows = output features, B 16x16 columns
// = samples, float32 accumulation). Register layout of the 64 lanes l (j = 0..3):
//   A (M x K):  A[l % 16][4 (l / 16) + j]
//   B (K x N):  B[4 (l / 16) + j][l % 16]
//   C/D (M x N): D[4 (l / 16) + j][l % 16]
// so the output tile (m, n) of one layer is already the B operand tile (k = m, n) of the next:
// activations never leave registers between layers. Weights (bfloat16) and biases (float32)
// live in LDS; features, outputs and the transposed copies needed by the weight gradients go
// through small per-wave LDS tiles.
#pragma once

#include "device_common.h"

namespace lbm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 12, kHid = 64, kOut = 9;
constexpr int kNParam = 5577;
// float32 parameter blob offsets: W1[64][12], b1[64], W2[64][64], b2[64], W3[9][64], b3[9]
constexpr int oW1 = 0, oB1 = 768, oW2 = 832, oB2 = 4928, oW3 = 4992, oB3 = 5568;
// input encoding scales (powers of two)
constexpr float kSNeq = 1024.0f, kSU = 16.0f;

// float32 -> bfloat16, round to nearest even (lowered to v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ short f2bf(float f) { return __builtin_bit_cast(short, (__bf16)f); }
__device__ __forceinline__ float bf2f(short h) {
  return __uint_as_float(((uint32_t)(uint16_t)h) << 16);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// CDNA4 double-K tile v_mfma_f32_16x16x32_bf16: A 16 x 32, B 32 x 16, C/D 16 x 16 as above.
// Lane l supplies 8 K-slots of row (A) or column (B) l % 16; the slot assignment depends only
// on (l / 16, element) and is the same for A and B, so any pairing of logical K indices with
// those slots gives the full sum as long as A and B use the same pairing (cat8 below).
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16v8, a),
                                                 __builtin_bit_cast(bf16v8, b), c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 cat8(bf16x4 lo, bf16x4 hi) {
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// GELU, tanh form (Hendrycks and Gimpel 2016), and its derivative, in float32;
// tanh(t) = 1 - 2 / (1 + exp(2 t)).
__device__ __forceinline__ void gelu_and_grad(float z, float& g, float& dg) {
  const float k = 0.7978845608028654f, a = 0.044715f;
  const float t = k * (z + a * z * z * z);
  const float e = __expf(2.0f * t);
  const float th = 1.0f - 2.0f / (1.0f + e);
  g = 0.5f * z * (1.0f + th);
  dg = 0.5f * (1.0f + th) + 0.5f * z * (1.0f - th * th) * k * (1.0f + 3.0f * a * z * z);
}
// Forward-only form: (1 + tanh t)/2 = 1/(1 + exp(-2t)), so gelu(z) = z / (1 + 2^(z (c0 + c1 z^2)))
// with c0 = -2 k log2(e), c1 = -2 k a log2(e): five VALU operations, one hardware 2^x and one
// hardware reciprocal (exp2 -> inf for very negative z gives 0, -> 0 for large z gives z).
__device__ __forceinline__ float gelu(float z) {
  const float c0 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;
  const float c1 = c0 * 0.044715f;
  const float t = z * __builtin_fmaf(z * z, c1, c0);
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
}

// Shared weights of one workgroup (bfloat16, zero padded) and biases (float32).
struct __attribute__((aligned(16))) MlpLds {
  short w1[kHid][16];    // W1 padded to 16 inputs
  short w2[kHid][kHid];
  short w3[16][kHid];    // W3 padded to 16 outputs
  float b1[kHid], b2[kHid], b3[16];
};

// The same weights for the inference tiles, rows padded (W1 to 20, W2 and W3 to 68 bfloat16)
// so that the 16 rows one operand read touches start on distinct LDS banks.
constexpr int kW1S = 20, kW2S = 68;
struct __attribute__((aligned(16))) MlpLdsP {
  short w1[kHid][kW1S];
  short w2[kHid][kW2S];
  short w3[16][kW2S];
  float b1[kHid], b2[kHid], b3[16];
};

// Cooperative load of the float32 blob (16-byte aligned) into the padded inference layout:
// every thread issues all its 16-byte loads first (kBlock threads, trip counts known at
// compile time), then rounds and writes, so the workgroup waits for memory about once.
__device__ __forceinline__ void mlp_load_lds_vec(const float* __restrict__ w, MlpLdsP& s) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int t = threadIdx.x;
  const f4* w4 = reinterpret_cast<const f4*>(w);
  constexpr int n1 = kHid * kIn / 4, n2 = kHid * kHid / 4, n3 = kOut * kHid / 4;  // 192, 1024, 144
  static_assert(n1 <= kBlock && n3 <= kBlock && n2 == 4 * kBlock, "one pass per thread");
  f4 a1 = {0.0f, 0.0f, 0.0f, 0.0f}, a3 = a1, a2[4];
  if (t < n1) a1 = w4[oW1 / 4 + t];
#pragma unroll
  for (int k = 0; k < 4; ++k) a2[k] = w4[oW2 / 4 + t + k * kBlock];
  if (t < n3) a3 = w4[oW3 / 4 + t];
  float b = 0.0f;
  if (t < 2 * kHid + kOut) b = w[t < kHid ? oB1 + t : (t < 2 * kHid ? oB2 + t - kHid : oB3 + t - 2 * kHid)];
  if (t < n1) {  // W1 rows of 12 = 3 quads
    const int o = t / 3, i = 4 * (t % 3);
#pragma unroll
    for (int j = 0; j < 4; ++j) s.w1[o][i + j] = f2bf(a1[j]);
  }
  if (t < kHid)
#pragma unroll
    for (int i = kIn; i < kW1S; ++i) s.w1[t][i] = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = 4 * (t + k * kBlock);
#pragma unroll
    for (int j = 0; j < 4; ++j) s.w2[e / kHid][e % kHid + j] = f2bf(a2[k][j]);
  }
  if (t < n3) {
    const int e = 4 * t;
#pragma unroll
    for (int j = 0; j < 4; ++j) s.w3[e / kHid][e % kHid + j] = f2bf(a3[j]);
  }
  for (int k = t; k < (16 - kOut) * kHid; k += kBlock) s.w3[kOut + k / kHid][k % kHid] = 0;
  if (t < kHid) s.b1[t] = b;
  else if (t < 2 * kHid) s.b2[t - kHid] = b;
  else if (t < 2 * kHid + kOut) s.b3[t - 2 * kHid] = b;
  else if (t < 2 * kHid + 16) s.b3[t - 2 * kHid] = 0.0f;
}

// Cooperative load of the float32 blob into LDS (rounded to bfloat16); either weight layout.
template <class Lds>
__device__ __forceinline__ void mlp_load_lds(const float* __restrict__ w, Lds& s) {
  for (int k = threadIdx.x; k < kHid * 16; k += blockDim.x) {
    const int o = k / 16, i = k % 16;
    s.w1[o][i] = i < kIn ? f2bf(w[oW1 + o * kIn + i]) : (short)0;
  }
  for (int k = threadIdx.x; k < kHid * kHid; k += blockDim.x)
    s.w2[k / kHid][k % kHid] = f2bf(w[oW2 + k]);
  for (int k = threadIdx.x; k < 16 * kHid; k += blockDim.x) {
    const int o = k / kHid, i = k % kHid;
    s.w3[o][i] = o < kOut ? f2bf(w[oW3 + o * kHid + i]) : (short)0;
  }
  for (int k = threadIdx.x; k < kHid; k += blockDim.x) {
    s.b1[k] = w[oB1 + k];
    s.b2[k] = w[oB2 + k];
  }
  for (int k = threadIdx.x; k < 16; k += blockDim.x) s.b3[k] = k < kOut ? w[oB3 + k] : 0.0f;
}

// Four consecutive bfloat16 values from LDS; p is 8-byte aligned at every call site (rows of
// 16, 20, 24, 64 or 68 elements, column offsets multiples of 4, arrays 16-byte aligned), which lets the
// compiler emit one ds_read_b64 with an immediate offset instead of a per-load address register.
__device__ __forceinline__ bf16x4 ld4(const short* p) {
  return *reinterpret_cast<const bf16x4*>(__builtin_assume_aligned(p, 8));
}

// b: 16-byte aligned; one 16-byte read (its 16-bit immediate offset reaches every bias array,
// where two-word reads would need an address add each)
__device__ __forceinline__ f32x4 bias4(const float* b, int lane) {
  return *reinterpret_cast<const f32x4*>(b + 4 * (lane >> 4));
}

// Forward pass of one wavefront: 64 samples, sample s = 16 n + (l % 16) in tile column n.
// xs: [64][16] bfloat16 inputs (row = sample). On return z1, z2 hold the pre-activations and
// h1, h2 the bfloat16 activations in the C layout, y the outputs (C layout, rows 0..8 valid).
struct MlpAct {
  f32x4 z1[4][4], z2[4][4];  // [m][n]
  bf16x4 h1[4][4], h2[4][4];
  f32x4 y[4];                // [n]
};

__device__ __forceinline__ void mlp_forward_wave(const MlpLds& s, const short (*xs)[16],
                                                 MlpAct& a, bool keep_z) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  // layer 1: K = 16 (12 inputs + zero padding)
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const bf16x4 xb = ld4(&xs[16 * n + r][4 * q]);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      f32x4 acc = bias4(s.b1 + 16 * m, lane);
      acc = mfma16(ld4(&s.w1[16 * m + r][4 * q]), xb, acc);
      if (keep_z) a.z1[m][n] = acc;
#pragma unroll
      for (int j = 0; j < 4; ++j) a.h1[m][n][j] = f2bf(gelu(acc[j]));
    }
  }
  // layer 2: K = 64
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    bf16x4 wa[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) wa[k] = ld4(&s.w2[16 * m + r][16 * k + 4 * q]);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      f32x4 acc = bias4(s.b2 + 16 * m, lane);
#pragma unroll
      for (int k = 0; k < 4; ++k) acc = mfma16(wa[k], a.h1[k][n], acc);
      if (keep_z) a.z2[m][n] = acc;
#pragma unroll
      for (int j = 0; j < 4; ++j) a.h2[m][n][j] = f2bf(gelu(acc[j]));
    }
  }
  // layer 3: 9 outputs padded to 16
  bf16x4 w3a[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) w3a[k] = ld4(&s.w3[r][16 * k + 4 * q]);
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    f32x4 acc = bias4(s.b3, lane);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc = mfma16(w3a[k], a.h2[k][n], acc);
    a.y[n] = acc;
  }
}

// Forward pass of node tile n (16 samples) only: the activations of one tile stay in
// registers (8 VGPRs per layer), which keeps the inference kernel's register count low.
// Returns the output tile (C layout, rows 0..8 valid).
__device__ __forceinline__ f32x4 mlp_forward_tile(const MlpLds& s, const short (*xs)[16], int n) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  const bf16x4 xb = ld4(&xs[16 * n + r][4 * q]);
  bf16x4 h1[4], h2[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 acc = bias4(s.b1 + 16 * m, lane);
    acc = mfma16(ld4(&s.w1[16 * m + r][4 * q]), xb, acc);
#pragma unroll
    for (int j = 0; j < 4; ++j) h1[m][j] = f2bf(gelu(acc[j]));
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 acc = bias4(s.b2 + 16 * m, lane);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc = mfma16(ld4(&s.w2[16 * m + r][16 * k + 4 * q]), h1[k], acc);
#pragma unroll
    for (int j = 0; j < 4; ++j) h2[m][j] = f2bf(gelu(acc[j]));
  }
  f32x4 acc = bias4(s.b3, lane);
#pragma unroll
  for (int k = 0; k < 4; ++k) acc = mfma16(ld4(&s.w3[r][16 * k + 4 * q]), h2[k], acc);
  return acc;
}

// Inference tile (16 samples, tile column n) on the CDNA4 double-K matrix tiles: layer 1 is one
// 16x16x16 tile per 16 outputs (K = 12 inputs + 4 zeros); layers 2 and 3 (K = 64) take two
// 16x16x32 tiles per 16 outputs, block p pairing the C-layout output tiles 2p and 2p + 1 of
// the previous layer: lane (q, r) supplies hidden units 32p + 4q + j and 32p + 16 + 4q + j
// (j = 0..3) of sample r, and the weights are read with the same pairing, so the activations
// still go from one layer to the next in registers. 4 + 8 + 2 = 14 matrix instructions per 16
// samples. xs: [64][xstride] bfloat16 inputs (row = sample). Returns the output tile (C
// layout, rows 0..8 valid).
template <int XS>
__device__ __forceinline__ f32x4 mlp_forward_tile32(const MlpLdsP& s, const short (*xs)[XS],
                                                    int n) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  const int rz = r;
  const bf16x4 xb = ld4(&xs[16 * n + r][4 * q]);
  bf16x4 h1[4], h2[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 acc = bias4(s.b1 + 16 * m, lane);
    acc = mfma16(ld4(&s.w1[16 * m + rz][4 * q]), xb, acc);
#pragma unroll
    for (int j = 0; j < 4; ++j) h1[m][j] = f2bf(gelu(acc[j]));
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 acc = bias4(s.b2 + 16 * m, lane);
#pragma unroll
    for (int p = 0; p < 2; ++p)
      acc = mfma32(cat8(ld4(&s.w2[16 * m + rz][32 * p + 4 * q]),
                        ld4(&s.w2[16 * m + rz][32 * p + 16 + 4 * q])),
                   cat8(h1[2 * p], h1[2 * p + 1]), acc);
#pragma unroll
    for (int j = 0; j < 4; ++j) h2[m][j] = f2bf(gelu(acc[j]));
  }
  f32x4 acc = bias4(s.b3, lane);
#pragma unroll
  for (int p = 0; p < 2; ++p)
    acc = mfma32(cat8(ld4(&s.w3[rz][32 * p + 4 * q]), ld4(&s.w3[rz][32 * p + 16 + 4 * q])),
                 cat8(h2[2 * p], h2[2 * p + 1]), acc);
  return acc;
}

// Orthogonal projection of 9 outputs onto zero mass and zero momentum (D2Q9 order
// i = (c_x+1) + 3 (c_y+1)): y -= sum(y)/9 + c_x sum(c_x y)/6 + c_y sum(c_y y)/6.
__device__ __forceinline__ void project9(float (&y)[9]) {
  float s = 0.0f, sx = 0.0f, sy = 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    s += y[i];
    sx += (float)(i % 3 - 1) * y[i];
    sy += (float)(i / 3 - 1) * y[i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i)
    y[i] -= s * (1.0f / 9.0f) + (float)(i % 3 - 1) * sx * (1.0f / 6.0f) +
            (float)(i / 3 - 1) * sy * (1.0f / 6.0f);
}

// Network inputs of one node from pre-collision f and its moments (theta = 1/3 equilibrium).
__device__ __forceinline__ void mlp_features(const double (&f)[9], double rho, double ux,
                                             double uy, double omega, float (&x)[12]) {
  const double u2x = ux * ux, u2y = uy * uy;
  const double px[3] = {1.0 / 6.0 + 0.5 * (u2x - ux), 2.0 / 3.0 - u2x, 1.0 / 6.0 + 0.5 * (u2x + ux)};
  const double py[3] = {1.0 / 6.0 + 0.5 * (u2y - uy), 2.0 / 3.0 - u2y, 1.0 / 6.0 + 0.5 * (u2y + uy)};
  const double inv = 1.0 / rho;
#pragma unroll
  for (int i = 0; i < 9; ++i) x[i] = (float)(kSNeq * (f[i] - rho * px[i % 3] * py[i / 3]) * inv);
  x[9] = (float)(kSU * ux);
  x[10] = (float)(kSU * uy);
  x[11] = (float)omega;
}

}  // namespace lbm
