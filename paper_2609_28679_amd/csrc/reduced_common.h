// Reduced-precision storage of the populations: float32 moments + 16-bit non-equilibrium part.
//
// State per node (post-collision, time t): moments m = (rho - 1, u_x, u_y [, T - 1]) in float32
// planes and the non-equilibrium part n_i = f~_i - f_i^eq(m) (and g~_i - g_i^eq(m)) in 16-bit
// planes. The post-collision populations keep the node's rho and rho u (and rho E), so n obeys
// sum_i n_i = 0 and sum_i c_i n_i = 0 (and sum_i n^g_i = 0): only the Q - (D + 1) = 6
// independent f values and the Q - 1 = 8 independent g values are stored, the others are
// rebuilt from these identities when read, which keeps mass, momentum and energy of the
// decoded state equal to the stored moments exactly.
//   f: stored i in {0, 1, 2, 3, 6, 8}; rebuilt  n_5 = n_0 - n_2 + n_3 + n_6 - n_8   (x momentum)
//                                               n_7 = n_0 + n_1 + n_2 - n_6 - n_8   (y momentum)
//                                               n_4 = -sum_{i != 4} n_i            (mass)
//   g: stored i != 4; rebuilt n_4 = -sum_{i != 4} n_i                               (energy)
// Codecs (encode from float32): bfloat16 (round to nearest even, upper 16 bits) or float16 of
// n * 2^S (round to nearest even, subnormals kept; S lifts |n| ~ 1e-8 .. 1e-3 into the normal
// range). Values computed in float64 are rounded to float32 first.
#pragma once

#include "device_common.h"

namespace lbm {

struct CodecBF16 {
  __device__ static __forceinline__ uint16_t enc(float f, float) {
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
  }
  __device__ static __forceinline__ float dec(uint16_t h, float) {
    return __uint_as_float((uint32_t)h << 16);
  }
  // Two codes in one 32-bit word (first value in the low half, the lower address): one
  // hardware conversion, round to nearest even as enc.
  __device__ static __forceinline__ uint32_t enc2(float a, float b, float) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
  }
  __device__ static __forceinline__ float dec_lo(uint32_t w, float) { return __uint_as_float(w << 16); }
  __device__ static __forceinline__ float dec_hi(uint32_t w, float) {
    return __uint_as_float(w & 0xFFFF0000u);
  }
};

struct CodecFP16 {
  // scale = 2^S on encode, 2^-S on decode (exact powers of two)
  __device__ static __forceinline__ uint16_t enc(float v, float scale) {
    const _Float16 h = (_Float16)(v * scale);
    return __builtin_bit_cast(uint16_t, h);
  }
  __device__ static __forceinline__ float dec(uint16_t h, float inv_scale) {
    return (float)__builtin_bit_cast(_Float16, h) * inv_scale;
  }
  __device__ static __forceinline__ uint32_t enc2(float a, float b, float scale) {
    return (uint32_t)enc(a, scale) | ((uint32_t)enc(b, scale) << 16);
  }
  __device__ static __forceinline__ float dec_lo(uint32_t w, float inv_scale) {
    return dec((uint16_t)(w & 0xFFFFu), inv_scale);
  }
  __device__ static __forceinline__ float dec_hi(uint32_t w, float inv_scale) {
    return dec((uint16_t)(w >> 16), inv_scale);
  }
};

// stored-plane slot of f population i (-1: rebuilt)
__host__ __device__ constexpr int f_slot(int i) {
  return i == 0 ? 0 : i == 1 ? 1 : i == 2 ? 2 : i == 3 ? 3 : i == 6 ? 4 : i == 8 ? 5 : -1;
}
// stored-plane slot of g population i (-1: rebuilt)
__host__ __device__ constexpr int g_slot(int i) { return i < 4 ? i : (i == 4 ? -1 : i - 1); }

constexpr int kRedF = 6;  // stored f planes
constexpr int kRedG = 8;  // stored g planes

// Decoded non-equilibrium part of f population i at element offset `off`.
template <typename Codec>
__device__ __forceinline__ double neq_f(const uint16_t* __restrict__ N, int64_t plane, int64_t off,
                                        int i, float s) {
  auto d = [&](int slot) { return (double)Codec::dec(N[slot * plane + off], s); };
  switch (i) {
    case 5: return d(0) - d(2) + d(3) + d(4) - d(5);
    case 7: return d(0) + d(1) + d(2) - d(4) - d(5);
    case 4: {
      const double n0 = d(0), n1 = d(1), n2 = d(2), n3 = d(3), n6 = d(4), n8 = d(5);
      const double n5 = n0 - n2 + n3 + n6 - n8;
      const double n7 = n0 + n1 + n2 - n6 - n8;
      return -(((n0 + n1) + (n2 + n3)) + ((n5 + n6) + (n7 + n8)));
    }
    default: return d(f_slot(i));
  }
}

template <typename Codec>
__device__ __forceinline__ double neq_g(const uint16_t* __restrict__ N, int64_t plane, int64_t off,
                                        int i, float s) {
  if (i != 4) return (double)Codec::dec(N[g_slot(i) * plane + off], s);
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < kRedG; ++k) t += (double)Codec::dec(N[k * plane + off], s);
  return -t;
}

}  // namespace lbm
