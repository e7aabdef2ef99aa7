// Device-side helpers shared by the HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm_internal.h"

namespace lbm {

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on XCD b % 8). Remap
// the hardware order so that each XCD owns one contiguous range of tiles: neighbouring tiles
// then share the XCD's L2 for their halo rows.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
#if defined(LBM_NO_XCD_REMAP)
  return b;
#endif
  const int per = nblocks / kNumXcd;
  const int rem = nblocks % kNumXcd;
  const int xcd = b % kNumXcd;
  const int k = b / kNumXcd;
  return xcd < rem ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic workgroup sum of N doubles per thread; thread 0 writes out[0..N).
template <int N>
__device__ __forceinline__ void block_sum_store(double (&v)[N], double* out) {
  __shared__ double red[kBlock / 64][N];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) red[wid][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[w][k];
      out[k] = s;
    }
  }
}

// Streaming load for kernels that read every stored value once per step (the plain BGK pulls:
// a neighbour in the same cache line aside, nothing is read twice), so the line need not stay
// cached. Measured on MI355X: D2Q9 float32 5.58 -> 5.95 TB/s at 2048^2, 5.58 -> 5.77 TB/s at
// 4096^2, D3Q27 5.43 -> 5.53 TB/s. Kernels that re-read rows (the Phi stencil window, the
// staged reduced-storage rows shared by neighbouring workgroups) keep cached loads: streaming
// loads cost them 7-22%.
template <typename T>
__device__ __forceinline__ T load_nt(const T* p) {
#if defined(LBM_CACHED_LOADS)
  return *p;
#else
  return __builtin_nontemporal_load(p);
#endif
}

template <typename T>
__device__ __forceinline__ void store_nt(T* p, T v) {
#if defined(LBM_PLAIN_STORES)
  *p = v;
#else
  __builtin_nontemporal_store(v, p);
#endif
}


// ---- scalar-base addressing ------------------------------------------------------------------
// A row of a plane is wave-uniform in the streaming kernels; with its address in scalar
// registers and a 32-bit lane offset, a load or store needs one vector register for the
// address instead of a 64-bit address computed per lane.
// Global-memory (address space 1) accesses, the form the scalar-base addressing takes.
#define LBM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T gload_nt(const LBM_GLOBAL T* p) {
#if defined(LBM_CACHED_LOADS)
  return *p;
#else
  return __builtin_nontemporal_load(p);
#endif
}
template <typename T>
__device__ __forceinline__ void gstore_nt(LBM_GLOBAL T* p, T v) {
#if defined(LBM_PLAIN_STORES)
  *p = v;
#else
  __builtin_nontemporal_store(v, p);
#endif
}
// A wave-uniform pointer held in scalar registers, so that an access p[i] with a 32-bit lane
// index i takes the scalar-base form (one vector offset register, no 64-bit address per lane).
template <typename T>
__device__ __forceinline__ LBM_GLOBAL T* sbase(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<LBM_GLOBAL T*>(((uint64_t)hi << 32) | lo);
}
// A 32-bit lane offset re-declared at its use (an empty asm), so that the compiler does not
// hoist its 64-bit extension out of a loop, which loses the scalar-base form of the access.
__device__ __forceinline__ uint32_t fresh(uint32_t o) {
  asm volatile("" : "+v"(o));
  return o;
}
// base + a 32-bit byte offset (a zero-extended 32-bit offset is what the scalar-base form takes)
template <typename T>
__device__ __forceinline__ LBM_GLOBAL T* at_byte(LBM_GLOBAL T* base, uint32_t off) {
  typedef LBM_GLOBAL char* cp;
  typedef LBM_GLOBAL T* tp;
  return (tp)((cp)(base) + off);
}

}  // namespace lbm
