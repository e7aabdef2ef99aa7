// Learned collision surrogate: training (forward, backward, Adam) and inference fused into the
// D2Q9 stream-collide step, on bfloat16 matrix cores with float32 accumulation. See
// mlp_common.h for the network, the transposed GEMM formulation and the register layouts.
//
// Training of one batch is two launches: k_mlp_grad (forward and backward, one wavefront per
// 64 samples, per-wavefront partial gradients: the weight gradients are split along the
// sample dimension, K) and k_mlp_reduce_adam (deterministic sum of the partials in a fixed
// order, then the Adam update of the float32 master weights).
#include "mlp_common.h"

#include <algorithm>
#include <cfloat>
#include <cstdlib>
#include <mutex>

#include "lbm.h"

namespace lbm {

constexpr int kPart = kNParam + 1;  // parameters + loss

// ---- forward and backward of one batch -----------------------------------------------------
// Samples (start + i) mod n for i in [0, B); wavefront w of the grid takes i in [64 w, 64 w + 64).
__global__ void __launch_bounds__(kBlock)
k_mlp_grad(const float* __restrict__ X, const float* __restrict__ T, int64_t n, int64_t start,
           int B, const float* __restrict__ w, float* __restrict__ partials) {
  __shared__ MlpLds s;
  __shared__ __attribute__((aligned(16))) short xs[4][64][16];
  __shared__ float ys[4][64][16];
  __shared__ __attribute__((aligned(16))) short tA[4][64][64];
  __shared__ __attribute__((aligned(16))) short tB[4][64][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int gw = blockIdx.x * 4 + wv;  // global wavefront
  const int i_loc = gw * 64 + lane;
  const bool valid = i_loc < B;
  const int64_t idx = (start + (int64_t)(valid ? i_loc : 0)) % n;

  mlp_load_lds(w, s);
  // inputs (bfloat16, zero padded); invalid samples have zero input and zero gradient
#pragma unroll
  for (int k = 0; k < 16; ++k)
    xs[wv][lane][k] = (valid && k < kIn) ? f2bf(X[idx * kIn + k]) : (short)0;
  __syncthreads();

  MlpAct a;
  mlp_forward_wave(s, xs[wv], a, true);
  // outputs to per-sample rows
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int j = 0; j < 4; ++j) ys[wv][16 * nt + r][4 * q + j] = a.y[nt][j];
  // H2^T rows [hidden][sample] for dW3
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j) tB[wv][16 * m + 4 * q + j][16 * nt + r] = a.h2[m][nt][j];
  __syncthreads();

  // ---- loss and output gradient (lane = sample) ----------------------------------------
  float y[9], dy[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) y[i] = ys[wv][lane][i];
  project9(y);
  float loss = 0.0f;
  const float scale = 2.0f / ((float)B * 9.0f);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float d = valid ? y[i] - T[idx * kOut + i] : 0.0f;
    loss += d * d;
    dy[i] = scale * d;
  }
  project9(dy);  // the projection is symmetric: dL/dy = P dL/dyhat
#pragma unroll
  for (int o = 0; o < 16; ++o) tA[wv][o][lane] = o < 9 ? f2bf(dy[o]) : (short)0;
  __syncthreads();

  float* out = partials + (int64_t)gw * kPart;
  // db3 and the loss: wavefront sums (fixed shuffle tree)
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float v = (float)wave_sum((double)dy[i]);
    if (lane == 0) out[oB3 + i] = v;
  }
  {
    const float v = (float)wave_sum((double)loss);
    if (lane == 0) out[kNParam] = v / ((float)B * 9.0f);
  }
  // dW3[o][h] = sum_s dy[s][o] h2[s][h]: A = dY^T (rows o), B = H2 (cols h), K = samples
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      acc = mfma16(ld4(&tA[wv][r][16 * kt + 4 * q]), ld4(&tB[wv][16 * nt + r][16 * kt + 4 * q]), acc);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * q + j < kOut) out[oW3 + (4 * q + j) * kHid + 16 * nt + r] = acc[j];
  }
  // dH2^T = W3^T dY^T, then dZ2 = dH2 gelu'(Z2)
  bf16x4 dz2[4][4];
  float db2[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    bf16x4 wa;
#pragma unroll
    for (int j = 0; j < 4; ++j) wa[j] = s.w3[4 * q + j][16 * m + r];
#pragma unroll
    for (int j = 0; j < 4; ++j) db2[m][j] = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      bf16x4 bb;
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = tA[wv][4 * q + j][16 * nt + r];
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      acc = mfma16(wa, bb, acc);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float g, dg;
        gelu_and_grad(a.z2[m][nt][j], g, dg);
        const float d = acc[j] * dg;
        db2[m][j] += d;
        dz2[m][nt][j] = f2bf(d);
      }
    }
  }
  __syncthreads();  // tA (dY^T) and tB (H2^T) are free again
  // dZ2 rows [out][sample] into tA, H1^T rows [hidden][sample] into tB
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        tA[wv][16 * m + 4 * q + j][16 * nt + r] = dz2[m][nt][j];
        tB[wv][16 * m + 4 * q + j][16 * nt + r] = a.h1[m][nt][j];
      }
  // db2: sum over the 16 lanes that share q (samples r)
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float v = db2[m][j];
      v += __shfl_xor(v, 8, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 1, 64);
      if (r == 0) out[oB2 + 16 * m + 4 * q + j] = v;
    }
  __syncthreads();
  // dW2 = dZ2^T H1
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt)
        acc = mfma16(ld4(&tA[wv][16 * m + r][16 * kt + 4 * q]), ld4(&tB[wv][16 * nt + r][16 * kt + 4 * q]), acc);
#pragma unroll
      for (int j = 0; j < 4; ++j) out[oW2 + (16 * m + 4 * q + j) * kHid + 16 * nt + r] = acc[j];
    }
  // dH1^T = W2^T dZ2^T, dZ1 = dH1 gelu'(Z1)
  bf16x4 dz1[4][4];
  float db1[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    bf16x4 wa[4];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
      for (int j = 0; j < 4; ++j) wa[kt][j] = s.w2[16 * kt + 4 * q + j][16 * m + r];
#pragma unroll
    for (int j = 0; j < 4; ++j) db1[m][j] = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) acc = mfma16(wa[kt], dz2[kt][nt], acc);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float g, dg;
        gelu_and_grad(a.z1[m][nt][j], g, dg);
        const float d = acc[j] * dg;
        db1[m][j] += d;
        dz1[m][nt][j] = f2bf(d);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float v = db1[m][j];
      v += __shfl_xor(v, 8, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 1, 64);
      if (r == 0) out[oB1 + 16 * m + 4 * q + j] = v;
    }
  __syncthreads();  // tA, tB free
  // dZ1 rows [out][sample] into tA, X^T rows [feature][sample] into tB
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j) tA[wv][16 * m + 4 * q + j][16 * nt + r] = dz1[m][nt][j];
#pragma unroll
  for (int k = 0; k < 16; ++k) tB[wv][k][lane] = xs[wv][lane][k];
  __syncthreads();
  // dW1 = dZ1^T X (features 0..11 of 16)
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
      acc = mfma16(ld4(&tA[wv][16 * m + r][16 * kt + 4 * q]), ld4(&tB[wv][r][16 * kt + 4 * q]), acc);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (r < kIn) out[oW1 + (16 * m + 4 * q + j) * kIn + r] = acc[j];
  }
}

// Sum of the per-wavefront partials in wavefront order; optional gradient output and Adam step.
__global__ void k_mlp_reduce_adam(const float* __restrict__ partials, int nw, float* __restrict__ grad,
                                  float* __restrict__ loss, float* __restrict__ w, float* __restrict__ m,
                                  float* __restrict__ v, int adam, float lr, float b1, float b2,
                                  float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kNParam) return;
  float g = 0.0f;
  for (int k = 0; k < nw; ++k) g += partials[(int64_t)k * kPart + p];
  if (p == kNParam) {
    if (loss) *loss = g;
    return;
  }
  if (grad) grad[p] = g;
  if (adam) {
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    // bias-corrected moments: c1 = 1 - b1^t, c2 = 1 - b2^t
    w[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// Per-wave LDS rows of the inference kernels: a sample's 12 bfloat16 inputs (zero padded to
// 24) and, once its tile has been evaluated, the same row's 12 float32 outputs (9 used). The
// outputs of tile n overwrite the inputs of tile n only, which that tile has already read.
constexpr int kIoS = 12;  // floats per row (48 bytes)

// Orders this wave's LDS writes before other lanes of the same wave read them: LDS operations
// of one wave execute in order, so only the compiler has to be kept from moving memory
// operations across this point (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Network of the four tiles of one wave: inputs in io rows (bfloat16), outputs back into the
// same rows (float32, C layout scattered to rows).
__device__ __forceinline__ void mlp_wave_tiles(const MlpLdsP& s, float (*io)[kIoS]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  const short(*xs)[2 * kIoS] = reinterpret_cast<const short(*)[2 * kIoS]>(io);
#pragma unroll 1
  for (int nt = 0; nt < 4; ++nt) {
    // The weights are re-read from LDS for every tile instead of being hoisted into registers
    // across the tiles (fewer registers, more wavefronts in flight): the byte offset z is 0,
    // but the compiler cannot see it, so the reads stay in the loop. Offsetting the LDS object
    // (rather than laundering the pointer itself) keeps them LDS reads, and every read is the
    // offset base plus an immediate.
    int z = 0;
    asm volatile("" : "+v"(z));
    const MlpLdsP& sz = *reinterpret_cast<const MlpLdsP*>(reinterpret_cast<const char*>(&s) + z);
    const f32x4 yt = mlp_forward_tile32<2 * kIoS>(sz, xs, nt);
    if (q < 3) {  // output rows 0..11 (9 used)
#pragma unroll
      for (int j = 0; j < 4; ++j) io[16 * nt + r][4 * q + j] = yt[j];
    }
  }
}

// A sample's 12 inputs as bfloat16 pairs in the first 6 words of its row, zeros in the next 2
// (the layer-1 tile reads 16 inputs); written as two 16-byte stores (rows are 48-byte aligned).
__device__ __forceinline__ void put_inputs(float* row, const float (&xf)[kIn], bool valid) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  unsigned w[6];
#pragma unroll
  for (int k = 0; k < 6; ++k)
    w[k] = valid ? ((unsigned)(uint16_t)f2bf(xf[2 * k]) | ((unsigned)(uint16_t)f2bf(xf[2 * k + 1]) << 16))
                 : 0u;
  u32x4* r = reinterpret_cast<u32x4*>(__builtin_assume_aligned(row, 16));
  r[0] = u32x4{w[0], w[1], w[2], w[3]};
  r[1] = u32x4{w[4], w[5], 0u, 0u};
}

// Forward pass for n samples (projected outputs), on the inference tiles.
__global__ void __launch_bounds__(kBlock)
k_mlp_forward(const float* __restrict__ X, int64_t n, const float* __restrict__ w, float* __restrict__ Y) {
  __shared__ MlpLdsP s;
  __shared__ __attribute__((aligned(16))) float io[4][64][kIoS];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i = ((int64_t)blockIdx.x * 4 + wv) * 64 + lane;
  const bool valid = i < n;
  mlp_load_lds_vec(w, s);
  float xf[kIn];
#pragma unroll
  for (int k = 0; k < kIn; ++k) xf[k] = valid ? X[i * kIn + k] : 0.0f;
  put_inputs(io[wv][lane], xf, valid);
  __syncthreads();  // the weights
  mlp_wave_tiles(s, io[wv]);
  wave_lds_sync();
  float y[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) y[k] = io[wv][lane][k];
  project9(y);
  if (valid)
#pragma unroll
    for (int k = 0; k < 9; ++k) Y[i * kOut + k] = y[k];
}

// ---- lattice side: harvest and surrogate step ------------------------------------------------
__device__ __forceinline__ double wrest(int i) {
  return (i % 3 == 1 ? 2.0 / 3.0 : 1.0 / 6.0) * (i / 3 == 1 ? 2.0 / 3.0 : 1.0 / 6.0);
}

// Pre-collision shifted values h_i = f_i - w_i at node (x, y) pulled from the state A.
// ROW_UNIFORM: every lane of the wavefront pulls for the same row y (the surrogate step), so
// the source rows are addressed from scalar bases with 32-bit lane offsets; otherwise (the
// harvest, one sampled node per lane) each lane forms its own addresses.
template <bool WALLS, bool ROW_UNIFORM>
__device__ __forceinline__ void pull9h(const float* __restrict__ A, int nx, int ny, int64_t pitch,
                                       int64_t plane, int x, int y, float (&h)[9]) {
  const int xc[3] = {x == nx - 1 ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};
  const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
  if constexpr (ROW_UNIFORM) {
    // byte offsets of the source columns
    const uint32_t xs[3] = {fresh(4u * xc[0]), fresh(4u * xc[1]), fresh(4u * xc[2])};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int ka = i % 3, kb = i / 3;
      const bool bounce = WALLS && ((kb == 2 && y == 0) || (kb == 0 && y == ny - 1));
      const float* row = bounce ? A + (8 - i) * plane + (int64_t)y * pitch
                                : A + i * plane + (int64_t)ys[kb] * pitch;
      h[i] = gload_nt(at_byte(sbase(row), bounce ? xs[1] : xs[ka]));
    }
  } else {
    const int64_t self = (int64_t)y * pitch + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int ka = i % 3, kb = i / 3;
      const bool bounce = WALLS && ((kb == 2 && y == 0) || (kb == 0 && y == ny - 1));
      h[i] = bounce ? A[(8 - i) * plane + self] : A[i * plane + (int64_t)ys[kb] * pitch + xc[ka]];
    }
  }
}

// Pre-collision populations at node (x, y) pulled from the shifted float32 state A.
template <bool WALLS>
__device__ __forceinline__ void pull9(const float* __restrict__ A, int nx, int ny, int64_t pitch,
                                      int64_t plane, int x, int y, double (&f)[9]) {
  float h[9];
  pull9h<WALLS, false>(A, nx, ny, pitch, plane, x, y, h);
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = (double)h[i] + wrest(i);
}

// Pre-collision populations of the next step at node (x, y) from a stored state of either
// layout: view -1 two-buffer (pull of slot i from x - c_i), 0 single-buffer after an even step
// count (slot 8-i of x - c_i; slot i of x where x - c_i lies beyond a wall), 1 single-buffer
// after an odd step count (slot i of x, already streamed).
template <bool WALLS>
__device__ __forceinline__ void next_input9(const float* __restrict__ A, int nx, int ny,
                                            int64_t pitch, int64_t plane, int view, int x, int y,
                                            double (&f)[9]) {
  if (view < 0) {
    pull9<WALLS>(A, nx, ny, pitch, plane, x, y, f);
    return;
  }
  const int xs[3] = {x == nx - 1 ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};
  const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
  const int64_t self = (int64_t)y * pitch + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int ka = i % 3, kb = i / 3;
    const bool wall = WALLS && ((kb == 2 && y == 0) || (kb == 0 && y == ny - 1));
    float h;
    if (view == 1 || wall)
      h = A[i * plane + self];
    else
      h = A[(8 - i) * plane + (int64_t)ys[kb] * pitch + xs[ka]];
    f[i] = (double)h + wrest(i);
  }
}

template <bool WALLS>
__global__ void k_harvest(const float* __restrict__ A, int nx, int ny, int64_t pitch, int64_t plane,
                          int view, double omega, const int64_t* __restrict__ nodes, int64_t n,
                          float* __restrict__ X, float* __restrict__ Y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t node = nodes[k];
  const int x = (int)(node % nx), y = (int)(node / nx);
  double f[9];
  next_input9<WALLS>(A, nx, ny, pitch, plane, view, x, y, f);
  const double rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const double ux = ((f[2] + f[5] + f[8]) - (f[0] + f[3] + f[6])) / rho;
  const double uy = ((f[6] + f[7] + f[8]) - (f[0] + f[1] + f[2])) / rho;
  float xf[12];
  mlp_features(f, rho, ux, uy, omega, xf);
#pragma unroll
  for (int i = 0; i < 12; ++i) X[k * kIn + i] = xf[i];
  // plain-collision target S (f~ - f^eq)/rho = (1 - omega) S (f - f^eq)/rho
#pragma unroll
  for (int i = 0; i < 9; ++i) Y[k * kOut + i] = (float)((1.0 - omega) * (double)xf[i]);
}

// One D2Q9 step with the surrogate collision and the per-node plain-collision judge, in float32
// on the shifted values h = f - w (w the rest weights). With theta = 1/3 the per-axis factors
// are psi_c = W_c + d_c, W = (1/6, 2/3, 1/6), d_0 = -u^2, d_+- = (u^2 +- u)/2, and
//   h^eq_i = f^eq_i - w_i = (rho - 1) psi_a psi_b + W_a d_b + d_a W_b + d_a d_b,
// with float32 constants whose sum is exactly one (W_+- = 2796203 2^-24, W_0 = 1 - 2 W_+-:
// with the nearest float32 values of 1/6 and 2/3 the sum of the factors misses one by 3e-8 and
// every collision rescales mass and momentum by that amount).
//   features  x = [1024 (h_i - h^eq_i)/rho, 16 u_x, 16 u_y, omega]
//   network   y (projected), surrogate f~ = f^eq + rho y / 1024
//   judge     |f~_mlp - f~_plain| <= tol |f~_plain - f^eq| with f~_plain - f^eq = (1 - omega)(f - f^eq),
//             i.e. |y - (1 - omega) x_neq| <= tol |1 - omega| |x_neq| (the factor rho / 1024 cancels)
//   fallback  h~ = h + omega (h^eq - h)
// One wavefront evaluates the network for its 64 nodes of a row; only the weights are shared by
// the workgroup (one barrier after their load), the rest of a row is synchronised per wave.
template <bool WALLS, bool DIAG>
__global__ void __launch_bounds__(kBlock)
k_bgk_d2q9_mlp(const float* __restrict__ A, float* __restrict__ B, int nx, int ny, int64_t pitch,
               int64_t plane, float omega, int rows, const float* __restrict__ wblob, float tol2,
               unsigned long long* __restrict__ counters, double* __restrict__ partials) {
  __shared__ MlpLdsP s;
  __shared__ __attribute__((aligned(16))) float io[4][64][kIoS];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nbx = gridDim.x;
  const int tile = xcd_tile(blockIdx.x + nbx * blockIdx.y, nbx * gridDim.y);
  const int bx = tile % nbx, by = tile / nbx;
  const int x = bx * blockDim.x + threadIdx.x;
  const bool valid = x < nx;
  const int y0 = by * rows, yend = min(y0 + rows, ny);
  const float W1 = 2796203.0f / 16777216.0f, W0 = 1.0f - 2.0f * W1;  // exact in float32
  const float keep = 1.0f - omega;
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};
  unsigned fallbacks = 0;
  mlp_load_lds_vec(wblob, s);
  // One row: features, network, judge and store from the pulled populations h of row y.
  // Lanes past the right edge work on the last column's values (pulled from a valid column,
  // so finite) and store nothing: no separate zero-filled path.
  auto row = [&](const float (&h)[9], int y) {
    float heq[9], xf[kIn];
    float drho, ux, uy;
    {
      drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
      const float jx = (h[2] + h[5] + h[8]) - (h[0] + h[3] + h[6]);
      const float jy = (h[6] + h[7] + h[8]) - (h[0] + h[1] + h[2]);
      const float inv = __builtin_amdgcn_rcpf(1.0f + drho);
      // u = j / rho with one residual correction of the hardware reciprocal (unbiased: a
      // one-sided velocity error would shift every node's momentum the same way each step)
      ux = jx * inv;
      uy = jy * inv;
      ux = __builtin_fmaf(__builtin_fmaf(-(1.0f + drho), ux, jx), inv, ux);
      uy = __builtin_fmaf(__builtin_fmaf(-(1.0f + drho), uy, jy), inv, uy);
      const float u2x = ux * ux, u2y = uy * uy;
      const float dx[3] = {0.5f * (u2x - ux), -u2x, 0.5f * (u2x + ux)};
      const float dy[3] = {0.5f * (u2y - uy), -u2y, 0.5f * (u2y + uy)};
      const float Wk[3] = {W1, W0, W1};
      const float sx = kSNeq * inv;
      // the same sum regrouped: h^eq_i = psi_b (drho psi_a + d_a) + W_a d_b (psi = W + d)
      float A[3], P[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        A[k] = __builtin_fmaf(drho, Wk[k] + dx[k], dx[k]);
        P[k] = Wk[k] + dy[k];
      }
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int ia = i % 3, ib = i / 3;
        heq[i] = __builtin_fmaf(P[ib], A[ia], Wk[ia] * dy[ib]);
        xf[i] = (h[i] - heq[i]) * sx;
      }
      xf[9] = kSU * ux;
      xf[10] = kSU * uy;
      xf[11] = omega;
    }
    wave_lds_sync();  // the previous row's outputs have been read
    put_inputs(io[wv][lane], xf, true);
    wave_lds_sync();
    mlp_wave_tiles(s, io[wv]);
    wave_lds_sync();
    if (valid) {
      float yv[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) yv[i] = io[wv][lane][i];
      project9(yv);
      float err = 0.0f, ref = 0.0f;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const float d = yv[i] - keep * xf[i];
        err += d * d;
        ref += xf[i] * xf[i];
      }
      const bool fb = !(err <= tol2 * (keep * keep) * ref);
      fallbacks += fb ? 1u : 0u;
      const float rs = (1.0f + drho) * (1.0f / kSNeq);
      const uint32_t xo = fresh(4u * x);
#pragma unroll
      for (int i = 0; i < 9; ++i)
        gstore_nt(at_byte(sbase(B + i * plane + (int64_t)y * pitch), xo),
                  fb ? h[i] + omega * (heq[i] - h[i]) : heq[i] + rs * yv[i]);
      if (DIAG) {
        const double rho = 1.0 + (double)drho;
        acc[0] += rho;
        acc[1] += rho * (double)ux;
        acc[2] += rho * (double)uy;
        acc[4] += 0.5 * rho * ((double)ux * ux + (double)uy * uy);
      }
    }
  };
  // Rows in pairs with two pull buffers: the populations of the next row are loaded while the
  // network of the current one runs (software pipelining without register copies).
  // The loads are unconditional (lanes past the edge read the last column, a pull past the
  // last row re-reads it), so that the compiler's wait for one buffer never includes the other.
  float ha[9], hb[9];
  const int xl = valid ? x : nx - 1;
  const int ylast = yend - 1;
  if (y0 < yend) pull9h<WALLS, true>(A, nx, ny, pitch, plane, xl, y0, ha);
  __syncthreads();
  for (int y = y0; y < yend; y += 2) {
    pull9h<WALLS, true>(A, nx, ny, pitch, plane, xl, min(y + 1, ylast), hb);
    row(ha, y);
    if (y + 1 >= yend) break;
    pull9h<WALLS, true>(A, nx, ny, pitch, plane, xl, min(y + 2, ylast), ha);
    row(hb, y + 1);
  }
  // integer fallback counts: order-independent, so atomics stay deterministic
  unsigned long long fb = (unsigned long long)fallbacks;
  unsigned long long upd = (unsigned long long)(valid ? yend - y0 : 0);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    fb += __shfl_xor(fb, off, 64);
    upd += __shfl_xor(upd, off, 64);
  }
  if (lane == 0) {
    atomicAdd(counters, fb);
    atomicAdd(counters + 1, upd);
  }
  if (DIAG) block_sum_store<kDiagValues>(acc, partials + (int64_t)tile * kDiagValues);
}

// ---- launchers ---------------------------------------------------------------------------------
hipError_t launch_mlp_grad(const float* X, const float* T, int64_t n, int64_t start, int B,
                           const float* w, float* partials, hipStream_t s) {
  const int nw = (B + 63) / 64;
  k_mlp_grad<<<(nw + 3) / 4, kBlock, 0, s>>>(X, T, n, start, B, w, partials);
  return hipGetLastError();
}

int mlp_partial_count(int B) { return (((B + 63) / 64) + 3) / 4 * 4; }

hipError_t launch_mlp_reduce_adam(const float* partials, int nw, float* grad, float* loss, float* w,
                                  float* m, float* v, bool adam, float lr, int64_t t, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)t));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)t));
  k_mlp_reduce_adam<<<(kNParam + 1 + kBlock - 1) / kBlock, kBlock, 0, s>>>(
      partials, nw, grad, loss, w, m, v, adam ? 1 : 0, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* X, int64_t n, const float* w, float* Y, hipStream_t s) {
  const int64_t nw = (n + 63) / 64;
  k_mlp_forward<<<(unsigned)((nw + 3) / 4), kBlock, 0, s>>>(X, n, w, Y);
  return hipGetLastError();
}

hipError_t launch_harvest(const void* A, const Layout& L, bool walls, int view, double omega,
                          const int64_t* nodes, int64_t n, float* X, float* Y, hipStream_t s) {
  const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
  if (walls)
    k_harvest<true><<<nb, kBlock, 0, s>>>(static_cast<const float*>(A), L.nx, L.ny, L.pitch, L.plane, view, omega, nodes, n, X, Y);
  else
    k_harvest<false><<<nb, kBlock, 0, s>>>(static_cast<const float*>(A), L.nx, L.ny, L.pitch, L.plane, view, omega, nodes, n, X, Y);
  return hipGetLastError();
}

// Workgroups of the surrogate step that the current device holds at once (compute units times
// the workgroups one compute unit holds with this kernel's registers and LDS), or 0 if the
// device cannot be queried.
static int mlp_resident_workgroups() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_bgk_d2q9_mlp<false, false>, kBlock, 0) !=
      hipSuccess)
    return 0;
  return cus * per;
}

// Rows per workgroup: as few as keep every workgroup resident at once (one round over the
// chip, so no tail of late workgroups), which also spreads the per-workgroup weight load over
// as many rows as possible. 2048^2 on MI355X: 13 rows, 1264 workgroups for 256 x 5 resident.
Grid make_grid_mlp(const Layout& L) {
  Grid G;
  G.bx = kBlock;
  G.nbx = (L.nx + kBlock - 1) / kBlock;
  G.rows = 8;
  const int64_t resident = mlp_resident_workgroups();
  if (resident > 0) {
    const int64_t units = (int64_t)L.ny * G.nbx;
    G.rows = (int)std::max<int64_t>(1, (units + resident - 1) / resident);
  }
#ifdef LBM_TUNING_ENV
  if (const char* v = getenv("LBM_MLP_ROWS")) G.rows = atoi(v);
#endif
  fit_rows(G, L.ny);
  return G;
}

hipError_t launch_bgk_d2q9_mlp(const void* A, void* B, const Layout& L, const Grid& G, double omega_d,
                               bool walls, const float* wblob, double tol_d,
                               unsigned long long* counters, double* partials, hipStream_t s) {
  dim3 grid(G.nbx, G.nby), block(kBlock);
  auto a = static_cast<const float*>(A);
  auto b = static_cast<float*>(B);
  const float omega = (float)omega_d;
  // tol^2 as a finite float32 (a huge tolerance then still gives 0 * tol^2 = 0 where the
  // non-equilibrium part vanishes, as the float64 comparison does)
  const float tol2 = (float)std::min(tol_d * tol_d, (double)FLT_MAX);
  if (walls) {
    if (partials) k_bgk_d2q9_mlp<true, true><<<grid, block, 0, s>>>(a, b, L.nx, L.ny, L.pitch, L.plane, omega, G.rows, wblob, tol2, counters, partials);
    else k_bgk_d2q9_mlp<true, false><<<grid, block, 0, s>>>(a, b, L.nx, L.ny, L.pitch, L.plane, omega, G.rows, wblob, tol2, counters, nullptr);
  } else {
    if (partials) k_bgk_d2q9_mlp<false, true><<<grid, block, 0, s>>>(a, b, L.nx, L.ny, L.pitch, L.plane, omega, G.rows, wblob, tol2, counters, partials);
    else k_bgk_d2q9_mlp<false, false><<<grid, block, 0, s>>>(a, b, L.nx, L.ny, L.pitch, L.plane, omega, G.rows, wblob, tol2, counters, nullptr);
  }
  return hipGetLastError();
}

// ---- gradient without allocation ---------------------------------------------------------------
// For callers that cannot call hipMalloc (graph capture, serving loops): the per-wavefront
// partial gradients of k_mlp_grad go to a fixed device array instead of a trainer buffer. Each
// GPU the library runs on holds its own copy of the array until the process ends; its device
// address is looked up once per device (with that device current) and kept. k_mlp_grad writes
// every entry of the rows it uses, so nothing has to be cleared between calls; calls that
// overlap on one GPU race on the array.
namespace {
constexpr int kStaticMaxSamples = LBM_MLP_STATIC_MAX_SAMPLES;
constexpr int kStaticRows = ((kStaticMaxSamples + 63) / 64 + 3) / 4 * 4;
static __device__ __align__(256) float scratch[(size_t)kStaticRows * kPart];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call per device).
hipError_t scratch_on_current_device(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

}  // namespace lbm

extern "C" int lbm_mlp_grad_static(const float* dev_weights, const float* dev_x,
                                   const float* dev_t, int64_t n, float* dev_grad,
                                   float* dev_loss, void* stream) {
  using namespace lbm;
  if (n <= 0 || n > kStaticMaxSamples) return LBM_EINVAL;
  if (!dev_weights || !dev_x || !dev_t || !dev_grad) return LBM_EINVAL;
  static_assert((size_t)kStaticRows * kPart * sizeof(float) <= ((size_t)8 << 20),
                "the fixed partials array stays below 8 MiB");
  float* part = nullptr;
  if (scratch_on_current_device(&part) != hipSuccess) return LBM_EDEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int B = (int)n;
  hipError_t e = launch_mlp_grad(dev_x, dev_t, n, 0, B, dev_weights, part, s);
  // adam = false: the kernel reads the partials and writes grad (and loss); w, m, v untouched
  if (e == hipSuccess)
    e = launch_mlp_reduce_adam(part, mlp_partial_count(B), dev_grad, dev_loss,
                               const_cast<float*>(dev_weights), nullptr, nullptr, false, 0.0f, 1, s);
  return e == hipSuccess ? LBM_OK : LBM_EDEVICE;
}
