// Isothermal fused pull stream-collide kernels (D2Q9 and D3Q27), float32 or float64 storage.
//
// One launch advances one time step of Eq. (LBM_f) of Sec. II C at
// theta = varsigma^2 = 1/3 (isothermal), with an optional uniform body force F:
//   buffer A holds the post-collision populations f~(t-1), stored shifted by the rest
//   equilibrium, h_i = f_i - w_i with w_i = f_i^eq(rho = 1, u = 0): h is O(Mach), so float32
//   storage keeps ~7 significant digits of the part that carries the flow instead of the
//   part that is constant;
//   pull:     f_i(x, t) = f~_i(x - c_i, t-1)  (periodic wrap, or half-way bounce-back
//             f_i(x, t) = f~_ibar(x, t-1) where x - c_i lies beyond a y wall);
//   moments:  rho = sum f_i, rho u = sum c_i f_i + F/2;
//   equilibrium: f_i^eq = rho prod_a Psi_ia(u_a, theta + u_a^2) (Sec. II C);
//   relax:    f~_i = f_i + omega (f_i^eq - f_i) + (1 - omega/2)(f_i^* - f_i^eq), omega = 2 beta
//             (Sec. II B), f^* the equilibrium at u + F/rho (f^* = f^eq without a force);
//   store f~(t) into buffer B (non-temporal: it is not read again by this launch).
// All arithmetic is float64 whatever the storage type: on this chip double-precision vector
// FMA runs at the same rate as unpacked single precision, and float64 arithmetic removes the
// coherent rounding drift that float32 arithmetic adds to every collision (the division
// u = j / rho and the linear-in-u equilibrium terms round with a bias that accumulates in
// the decay of a Taylor-Green mode at ~1.6e-8 per step).
// Optional float64 conservation totals per workgroup (mass, momentum, kinetic energy of the
// moments at time t) for the diagnostics.
#include "device_common.h"

#include <cstdlib>
#include <type_traits>

namespace lbm {

// Psi(c; u, theta + u^2) for c = -1, 0, +1 at theta = 1/3 (Sec. II C).
__device__ __forceinline__ void psi3(double u, double (&p)[3]) {
  const double u2 = u * u;
  p[1] = (2.0 / 3.0) - u2;               // c = 0:  1 - theta - u^2
  p[2] = (1.0 / 6.0) + 0.5 * (u2 + u);   // c = +1: (theta + u^2 + u) / 2
  p[0] = (1.0 / 6.0) + 0.5 * (u2 - u);   // c = -1: (theta + u^2 - u) / 2
}

// Rest weights w_i = prod_a Psi(c_ia; 0, 1/3) as a function of the per-axis index k = c + 1.
__device__ __forceinline__ double w1(int k) { return k == 1 ? 2.0 / 3.0 : 1.0 / 6.0; }

// Moments of one node for the diagnostics: rho, rho u (with the half-step force term) and u.
struct NodeMoments {
  double rho, j[3], u[3];
};

// Collision of one node held shifted (h = f - w), Eq. (LBM_f) at theta = 1/3 (Phi = 0):
//   rho = sum f, rho u = sum c f + F/2,
//   f~ = f + omega (f^eq - f) + (1 - omega/2)(f^* - f^eq),
// where f^* is the equilibrium at u* = u + F/rho (Sec. II C; no heat source, theta* = theta).
// Without a force (FORCE = false) f^* = f^eq. `sink(i, h~_i)` receives the post-collision
// values in storage precision. D2Q9 and D3Q27 (D = 2, 3; i = (cx+1) + 3(cy+1) + 9(cz+1)).
template <int D, bool FORCE, typename S, typename Sink>
__device__ __forceinline__ void collide_bgk(const S (&hs)[D == 2 ? 9 : 27], double omega,
                                            const Force& F, NodeMoments& m, Sink&& sink) {
  constexpr int Q = D == 2 ? 9 : 27;
  double rho, j[3] = {0.0, 0.0, 0.0};
  if (D == 2) {
    double h[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = (double)hs[i];
    // sum w_i = 1 and sum c_i w_i = 0, so rho = 1 + sum h and rho u = sum c h
    rho = 1.0 + (((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8]);
    j[0] = (h[2] + h[5] + h[8]) - (h[0] + h[3] + h[6]);
    j[1] = (h[6] + h[7] + h[8]) - (h[0] + h[1] + h[2]);
  } else {
    double drho = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
      const double v = (double)hs[i];
      drho += v;
      if (cx) j[0] += cx > 0 ? v : -v;
      if (cy) j[1] += cy > 0 ? v : -v;
      if (cz) j[2] += cz > 0 ? v : -v;
    }
    rho = 1.0 + drho;
  }
  if (FORCE) {
    j[0] += 0.5 * F.x;
    j[1] += 0.5 * F.y;
    if (D == 3) j[2] += 0.5 * F.z;
  }
  double p[3][3], ps[3][3];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    m.u[a] = j[a] / rho;
    psi3(m.u[a], p[a]);
  }
  if (FORCE) {
    const double fa[3] = {F.x, F.y, F.z};
#pragma unroll
    for (int a = 0; a < D; ++a) psi3(m.u[a] + fa[a] / rho, ps[a]);
  }
  const double keep = 1.0 - 0.5 * omega;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int a = i % 3, b = (i / 3) % 3, c = i / 9;
    // rho p_a p_b (p_c), multiplied left to right so that rho p_a is shared between directions
    double feq = rho * p[0][a] * p[1][b];
    double ww = w1(a) * w1(b);
    if (D == 3) {
      feq *= p[2][c];
      ww *= w1(c);
    }
    const double heq = feq - ww;
    const double v = (double)hs[i];
    double out = v + omega * (heq - v);
    if (FORCE) {
      double fs = rho * ps[0][a] * ps[1][b];
      if (D == 3) fs *= ps[2][c];
      out += keep * (fs - feq);
    }
    sink(i, (S)out);
  }
  m.rho = rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) m.j[a] = a < D ? j[a] : 0.0;
}

template <int D>
__device__ __forceinline__ void add_diag(double (&acc)[kDiagValues], const NodeMoments& m) {
  acc[0] += m.rho;
  acc[1] += m.j[0];
  acc[2] += m.j[1];
  if (D == 3) acc[3] += m.j[2];
  double u2 = m.u[0] * m.u[0] + m.u[1] * m.u[1];
  if (D == 3) u2 += m.u[2] * m.u[2];
  acc[4] += 0.5 * m.rho * u2;
}

// ---- D2Q9 ---------------------------------------------------------------------------------
template <typename S, bool WALLS, bool DIAG, bool FORCE>
__global__ void __launch_bounds__(kBlock)
k_bgk_d2q9(const S* __restrict__ A, S* __restrict__ B, int nx, int ny, int64_t pitch,
           int64_t plane, double omega, Force F, int rows, double* __restrict__ partials) {
  const int nbx = gridDim.x;
  const int tile = xcd_tile(blockIdx.x + nbx * blockIdx.y, nbx * gridDim.y);
  const int bx = tile % nbx;
  const int by = tile / nbx;
  const int x = bx * blockDim.x + threadIdx.x;
  const int y0 = by * rows;
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};

  if (x < nx) {
    const int xm = x == 0 ? nx - 1 : x - 1;
    const int xp = x == nx - 1 ? 0 : x + 1;
    const int yend = min(y0 + rows, ny);
    for (int y = y0; y < yend; ++y) {
      const int ym = y == 0 ? ny - 1 : y - 1;
      const int yp = y == ny - 1 ? 0 : y + 1;
      const int64_t r0 = (int64_t)y * pitch;
      const int64_t rm = (int64_t)ym * pitch;
      const int64_t rp = (int64_t)yp * pitch;
      S hs[9];
      // i = (cx+1) + 3(cy+1); source node x - c_i
      hs[3] = load_nt(A + 3 * plane + r0 + xp);
      hs[4] = load_nt(A + 4 * plane + r0 + x);
      hs[5] = load_nt(A + 5 * plane + r0 + xm);
      if (WALLS && y == ny - 1) {  // c_y = -1 would come from beyond the top wall
        hs[0] = load_nt(A + 8 * plane + r0 + x);
        hs[1] = load_nt(A + 7 * plane + r0 + x);
        hs[2] = load_nt(A + 6 * plane + r0 + x);
      } else {
        hs[0] = load_nt(A + 0 * plane + rp + xp);
        hs[1] = load_nt(A + 1 * plane + rp + x);
        hs[2] = load_nt(A + 2 * plane + rp + xm);
      }
      if (WALLS && y == 0) {  // c_y = +1 would come from below the bottom wall
        hs[6] = load_nt(A + 2 * plane + r0 + x);
        hs[7] = load_nt(A + 1 * plane + r0 + x);
        hs[8] = load_nt(A + 0 * plane + r0 + x);
      } else {
        hs[6] = load_nt(A + 6 * plane + rm + xp);
        hs[7] = load_nt(A + 7 * plane + rm + x);
        hs[8] = load_nt(A + 8 * plane + rm + xm);
      }
      S* out = B + r0 + x;
      NodeMoments m;
      collide_bgk<2, FORCE>(hs, omega, F, m, [&](int i, S v) { store_nt(out + i * plane, v); });
      if (DIAG) add_diag<2>(acc, m);
    }
  }
  if (DIAG) block_sum_store<kDiagValues>(acc, partials + (int64_t)tile * kDiagValues);
}

// ---- D2Q9, single buffer ------------------------------------------------------------------
// Two-step in-place streaming on one population buffer (the "AA" access pattern of Bailey et
// al., 2009): every node reads and writes the same nine locations, so no second buffer is
// needed and the state of a lattice is half the size. With t the number of steps taken:
//   t even: slot Q-1-i of node x holds the post-collision h~_i(x, t) (stored "swapped");
//   t odd:  slot i of node x holds h~_i(x - c_i, t) = h_i(x, t + 1), already streamed; where
//           x - c_i lies beyond a y wall it holds the bounce-back value h~_ibar(x, t).
// Step from an even state (ODD = false): pull h_i(x) = slot Q-1-i of x - c_i (slot i of x at a
// wall), collide, push h~_i(x) into slot i of x + c_i (slot Q-1-i of x at a wall).
// Step from an odd state (ODD = true): read slot i of x, collide, write h~_i into slot Q-1-i
// of x. The read and write sets of a node coincide and are disjoint from every other node's,
// so the update is race-free without barriers. The state that fits the 256 MB last-level
// cache at 2048^2 (151 MB in float32) stays resident there: measured 11% faster than the
// two-buffer kernel at 2048^2, 12% slower at 4096^2, so the context picks it by size.
// The state is read again by the next step, so loads and stores keep the default cache policy
// (non-temporal hints measured slower here).
template <typename T>
__device__ __forceinline__ T aa_load(const T* p) {
#if defined(LBM_AA_NT_LOADS)
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}
template <typename T>
__device__ __forceinline__ void aa_store(T* p, T v) {
#if defined(LBM_AA_NT_STORES)
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

template <typename S, bool WALLS, bool DIAG, bool ODD, bool FORCE>
__global__ void __launch_bounds__(kBlock)
k_bgk_d2q9_aa(S* __restrict__ A, int nx, int ny, int64_t pitch, int64_t plane, double omega,
              Force F, int rows, double* __restrict__ partials) {
  const int nbx = gridDim.x;
  const int tile = xcd_tile(blockIdx.x + nbx * blockIdx.y, nbx * gridDim.y);
  const int bx = tile % nbx;
  const int by = tile / nbx;
  const int x = bx * blockDim.x + threadIdx.x;
  const int y0 = by * rows;
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};

  if (x < nx) {
    const int xm = x == 0 ? nx - 1 : x - 1;
    const int xp = x == nx - 1 ? 0 : x + 1;
    const int yend = min(y0 + rows, ny);
    for (int y = y0; y < yend; ++y) {
      const int ym = y == 0 ? ny - 1 : y - 1;
      const int yp = y == ny - 1 ? 0 : y + 1;
      const int64_t r0 = (int64_t)y * pitch;
      // src[i]: element offset of the node x - c_i, i = (cx+1) + 3(cy+1); the same offset is
      // the destination x + c_(8-i) of the opposite direction
      const bool top = WALLS && y == ny - 1;  // sources above (c_y = -1) lie beyond the wall
      const bool bot = WALLS && y == 0;       // sources below (c_y = +1) lie beyond the wall
      const int64_t rowm = (int64_t)ym * pitch, rowp = (int64_t)yp * pitch;
      const int64_t xo[3] = {xp, x, xm};  // x - c_x for c_x = -1, 0, +1
      const int64_t yo[3] = {rowp, r0, rowm};  // row of y - c_y
      int64_t src[9];
      bool wall_in[9];  // x - c_i beyond a wall
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int ka = i % 3, kb = i / 3;
        src[i] = yo[kb] + xo[ka];
        wall_in[i] = (kb == 0 && top) || (kb == 2 && bot);
      }
      S hs[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        if (ODD)
          hs[i] = aa_load(A + i * plane + r0 + x);
        else
          hs[i] = aa_load(wall_in[i] ? A + i * plane + r0 + x : A + (8 - i) * plane + src[i]);
      }
      NodeMoments m;
      collide_bgk<2, FORCE>(hs, omega, F, m, [&](int i, S v) {
        if (ODD) {
          aa_store(A + (8 - i) * plane + r0 + x, v);
        } else {
          // destination x + c_i is the source of the opposite direction, x - c_(8-i)
          aa_store(A + (wall_in[8 - i] ? (8 - i) * plane + r0 + x : i * plane + src[8 - i]), v);
        }
      });
      if (DIAG) add_diag<2>(acc, m);
    }
  }
  if (DIAG) block_sum_store<kDiagValues>(acc, partials + (int64_t)tile * kDiagValues);
}

// ---- D3Q27 --------------------------------------------------------------------------------
// 3 waves per SIMD lets the compiler keep all 27 loads of a node in flight without spilling
#ifndef LBM_D3Q27_WAVES
#define LBM_D3Q27_WAVES 3
#endif
template <typename S, bool WALLS, bool DIAG, bool FORCE>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(LBM_D3Q27_WAVES)))
k_bgk_d3q27(const S* __restrict__ A, S* __restrict__ B, int nx, int ny, int nz, int64_t pitch,
            int64_t plane, double omega, Force F, int rows, double* __restrict__ partials) {
  const int nbx = gridDim.x;
  // hardware workgroup order (consecutive rows on different XCDs): measured 6% faster than the
  // per-XCD contiguous ranges for D3Q27 at 256^3, whose 27 streams then stay close in memory
  const int tile = blockIdx.x + nbx * blockIdx.y;
  const int bx = tile % nbx;
  const int by = tile / nbx;
  const int x = bx * blockDim.x + threadIdx.x;
  const int r_begin = by * rows;
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};

  if (x < nx) {
    int xs[3];
    xs[0] = x == nx - 1 ? 0 : x + 1;  // c_x = -1: source x + 1
    xs[1] = x;
    xs[2] = x == 0 ? nx - 1 : x - 1;  // c_x = +1: source x - 1
    const int r_end = min(r_begin + rows, ny * nz);
    for (int r = r_begin; r < r_end; ++r) {
      const int y = r % ny;
      const int z = r / ny;
      const int ysrc[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
      const int zsrc[3] = {z == nz - 1 ? 0 : z + 1, z, z == 0 ? nz - 1 : z - 1};
      const int64_t self = ((int64_t)z * ny + y) * pitch + x;
      // populations stay in storage precision in registers (27 values); the arithmetic
      // converts each one to float64 where it is used
      S h[27];
#pragma unroll
      for (int i = 0; i < 27; ++i) {
        const int cx = i % 3, cy = (i / 3) % 3, cz = i / 9;  // component + 1
        const bool bounce = WALLS && ((cy == 2 && y == 0) || (cy == 0 && y == ny - 1));
        if (bounce) {
          h[i] = load_nt(A + (26 - i) * plane + self);
        } else {
          h[i] = load_nt(A + i * plane + ((int64_t)zsrc[cz] * ny + ysrc[cy]) * pitch + xs[cx]);
        }
      }
      S* out = B + self;
      NodeMoments m;
      collide_bgk<3, FORCE>(h, omega, F, m, [&](int i, S v) { store_nt(out + i * plane, v); });
      if (DIAG) add_diag<3>(acc, m);
    }
  }
  if (DIAG) block_sum_store<kDiagValues>(acc, partials + (int64_t)tile * kDiagValues);
}

// ---- D3Q27, single buffer ----------------------------------------------------------------
// The in-place two-step layout of k_bgk_d2q9_aa with 27 directions (slot Q-1-i = 26-i).
template <typename S, bool WALLS, bool DIAG, bool ODD, bool FORCE>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ODD ? 3 : 2)))
k_bgk_d3q27_aa(S* __restrict__ A, int nx, int ny, int nz, int64_t pitch, int64_t plane,
               double omega, Force F, int rows, double* __restrict__ partials) {
  const int nbx = gridDim.x;
  const int tile = blockIdx.x + nbx * blockIdx.y;  // hardware order, as k_bgk_d3q27
  const int bx = tile % nbx;
  const int by = tile / nbx;
  const int x = bx * blockDim.x + threadIdx.x;
  const int r_begin = by * rows;
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};

  if (x < nx) {
    int xs[3];
    xs[0] = x == nx - 1 ? 0 : x + 1;  // c_x = -1: node x - c_x = x + 1
    xs[1] = x;
    xs[2] = x == 0 ? nx - 1 : x - 1;  // c_x = +1: node x - 1
    const int r_end = min(r_begin + rows, ny * nz);
    for (int r = r_begin; r < r_end; ++r) {
      const int y = r % ny;
      const int z = r / ny;
      const int ysrc[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
      const int zsrc[3] = {z == nz - 1 ? 0 : z + 1, z, z == 0 ? nz - 1 : z - 1};
      const int64_t self = ((int64_t)z * ny + y) * pitch + x;
      // element offset of the node x - c_i, which is also the destination x + c_(26-i)
      auto src = [&](int i) {
        return ((int64_t)zsrc[i / 9] * ny + ysrc[(i / 3) % 3]) * pitch + xs[i % 3];
      };
      // x - c_i lies beyond a y wall
      auto wall_in = [&](int i) {
        const int cy = (i / 3) % 3;
        return WALLS && ((cy == 2 && y == 0) || (cy == 0 && y == ny - 1));
      };
      S h[27];
#pragma unroll
      for (int i = 0; i < 27; ++i) {
        if (ODD)
          h[i] = aa_load(A + i * plane + self);
        else
          h[i] = aa_load(wall_in(i) ? A + i * plane + self : A + (26 - i) * plane + src(i));
      }
      NodeMoments m;
      collide_bgk<3, FORCE>(h, omega, F, m, [&](int i, S o) {
        if (ODD)
          aa_store(A + (26 - i) * plane + self, o);
        else
          aa_store(wall_in(26 - i) ? A + (26 - i) * plane + self : A + i * plane + src(26 - i), o);
      });
      if (DIAG) add_diag<3>(acc, m);
    }
  }
  if (DIAG) block_sum_store<kDiagValues>(acc, partials + (int64_t)tile * kDiagValues);
}

// ---- initialisation and read-out -----------------------------------------------------------
// f_i <- f_i^eq(rho, u) with theta = 1/3 (Fig. 1 initialisation), stored as h = f - w; swap = 1
// stores population i in slot Q-1-i (the single-buffer state at an even step count). The
// stored state is post-collision: without a force the collision leaves an equilibrium as it
// is; with a force (FORCE) the equilibrium is collided once, in float64, before it is stored.
template <typename S, bool FORCE>
__global__ void k_init_bgk(int D, const double* __restrict__ rho, const double* __restrict__ u,
                           S* __restrict__ A, int nx, int ny, int nz, int64_t pitch,
                           int64_t plane, int swap, double omega, Force F) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nodes = (int64_t)nx * ny * nz;
  if (n >= nodes) return;
  const int x = (int)(n % nx);
  const int64_t row = n / nx;
  const int64_t off = row * pitch + x;
  double p[3][3];
  for (int a = 0; a < D; ++a) psi3(u[a * nodes + n], p[a]);
  const int Q = D == 2 ? 9 : 27;
  double h[27];
  for (int i = 0; i < Q; ++i) {
    const int ka = i % 3, kb = (i / 3) % 3, kc = i / 9;
    double v = rho[n] * p[0][ka] * p[1][kb];
    double w = w1(ka) * w1(kb);
    if (D == 3) {
      v *= p[2][kc];
      w *= w1(kc);
    }
    h[i] = v - w;
  }
  auto put = [&](int i, double v) { A[(swap ? Q - 1 - i : i) * plane + off] = (S)v; };
  if (!FORCE) {
    for (int i = 0; i < Q; ++i) put(i, h[i]);
    return;
  }
  NodeMoments m;
  if (D == 2) {
    double h9[9];
    for (int i = 0; i < 9; ++i) h9[i] = h[i];
    collide_bgk<2, true>(h9, omega, F, m, put);
  } else {
    collide_bgk<3, true>(h, omega, F, m, put);
  }
}

// Element index of the post-collision population i of node (x, y, z) in the stored state
// (z = 0 and nz = 1 for D2Q9):
//   view -1: two-buffer state, slot i of the node;
//   view  0: single-buffer state after an even step count, slot Q-1-i of the node;
//   view  1: single-buffer state after an odd step count, slot i of the node x + c_i, or
//            slot Q-1-i of the node itself where x + c_i lies beyond a y wall.
__device__ __forceinline__ int64_t post_index(int view, int walls, int D, int nx, int ny, int nz,
                                              int64_t pitch, int64_t plane, int x, int y, int z,
                                              int i) {
  const int Q = D == 2 ? 9 : 27;
  const int64_t self = ((int64_t)z * ny + y) * pitch + x;
  if (view < 0) return i * plane + self;
  if (view == 0) return (Q - 1 - i) * plane + self;
  const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = D == 3 ? i / 9 - 1 : 0;
  const int yd = y + cy;
  if (walls && (yd < 0 || yd >= ny)) return (Q - 1 - i) * plane + self;
  const int xd = (x + cx + nx) % nx, yw = (yd + ny) % ny, zd = (z + cz + nz) % nz;
  return i * plane + ((int64_t)zd * ny + yw) * pitch + xd;
}

// Moments of the stored post-collision state: the collision conserves rho and, without a force,
// rho u, so these equal the moments of the pre-collision populations at the same time. With a
// force the collision adds F to sum c f, and rho u = sum c f + F/2 before it, so
// rho u = sum c f~ - F/2.
template <typename S>
__global__ void k_moments_bgk(int D, const S* __restrict__ A, int nx, int ny, int nz,
                              int64_t pitch, int64_t plane, int view, int walls, Force F,
                              double* __restrict__ rho, double* __restrict__ u) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nodes = (int64_t)nx * ny * nz;
  if (n >= nodes) return;
  const int x = (int)(n % nx);
  const int y = (int)((n / nx) % ny);
  const int z = (int)(n / ((int64_t)nx * ny));
  const int Q = D == 2 ? 9 : 27;
  double s = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    const double v = (double)A[post_index(view, walls, D, nx, ny, nz, pitch, plane, x, y, z, i)];
    s += v;
    const int c[3] = {i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1};
    for (int a = 0; a < D; ++a) j[a] += c[a] * v;
  }
  j[0] -= 0.5 * F.x;
  j[1] -= 0.5 * F.y;
  j[2] -= 0.5 * F.z;
  const double r = 1.0 + s;
  rho[n] = r;
  for (int a = 0; a < D; ++a) u[a * nodes + n] = j[a] / r;
}

// Population plane i decoded to float64 f_i = h_i + w_i.
template <typename S>
__global__ void k_decode_f(int D, int i, const S* __restrict__ A, int nx, int ny, int nz,
                           int64_t pitch, int64_t plane, int view, int walls,
                           double* __restrict__ f) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nodes = (int64_t)nx * ny * nz;
  if (n >= nodes) return;
  const int x = (int)(n % nx);
  const int y = (int)((n / nx) % ny);
  const int z = (int)(n / ((int64_t)nx * ny));
  double w = w1(i % 3) * w1((i / 3) % 3);
  if (D == 3) w *= w1(i / 9);
  f[n] = (double)A[post_index(view, walls, D, nx, ny, nz, pitch, plane, x, y, z, i)] + w;
}

// ---- diagnostics ---------------------------------------------------------------------------
__global__ void k_diag_finalize(const double* __restrict__ partials, int nblocks, double t,
                                double* __restrict__ out) {
  double v[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < kDiagValues; ++k) v[k] += partials[(int64_t)b * kDiagValues + k];
  __shared__ double tot[kDiagValues];
  block_sum_store<kDiagValues>(v, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = t;
#pragma unroll
    for (int k = 0; k < kDiagValues; ++k) out[1 + k] = tot[k];
  }
}

__global__ void k_field_totals(int D, const double* __restrict__ rho, const double* __restrict__ u,
                               const double* __restrict__ edens, int64_t nodes, int kinetic,
                               double* __restrict__ partials) {
  double v[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nodes;
       n += (int64_t)gridDim.x * blockDim.x) {
    const double r = rho[n];
    double u2 = 0.0;
    v[0] += r;
    for (int a = 0; a < D; ++a) {
      const double ua = u[a * nodes + n];
      v[1 + a] += r * ua;
      u2 += ua * ua;
    }
    v[4] += kinetic ? 0.5 * r * u2 : edens[n];
  }
  block_sum_store<kDiagValues>(v, partials + (int64_t)blockIdx.x * kDiagValues);
}

// ---- launchers -----------------------------------------------------------------------------
Layout make_layout(int nx, int ny, int nz, int elem) {
  // Rows start on 256-byte boundaries. Population planes are padded to a 4 KiB multiple plus
  // 17 KiB so that the Q concurrent read and write streams of a workgroup, which sit whole
  // planes apart, start on different HBM channels; the padding was chosen by a sweep of row
  // and plane padding on MI355X (D2Q9 at 2048^2 and 4096^2, D3Q27 at 256^3).
  Layout L;
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  const int64_t row_align = 256 / elem;
  int64_t pitch = ((int64_t)nx + row_align - 1) / row_align * row_align;
  int64_t plane_pad = 17 * 1024 / elem;
#ifdef LBM_TUNING_ENV
  if (const char* v = getenv("LBM_PITCH_PAD")) pitch += atoll(v);
  if (const char* v = getenv("LBM_PLANE_PAD")) plane_pad = atoll(v);
#endif
  L.pitch = pitch;
  const int64_t raw = pitch * ny * nz;
  const int64_t epk = 4096 / elem;
  L.plane = (raw + epk - 1) / epk * epk + plane_pad;
  return L;
}

Grid make_grid(const Layout& L) {
  // One row per workgroup measured best for the streaming kernels on MI355X (more
  // workgroups in flight); the row count only grows for very large lattices.
  int bx_max = kBlock, max_rows = 16;
  int64_t target = 1 << 20;
#ifdef LBM_TUNING_ENV
  if (const char* v = getenv("LBM_BX")) bx_max = atoi(v);
  if (const char* v = getenv("LBM_ROWS")) max_rows = atoi(v);
  if (const char* v = getenv("LBM_TARGET")) target = atoll(v);
#endif
  Grid G;
  G.bx = L.nx >= bx_max ? bx_max : ((L.nx + 63) / 64) * 64;
  G.nbx = (L.nx + G.bx - 1) / G.bx;
  const int64_t nrows = (int64_t)L.ny * L.nz;
  // aim for >= `target` workgroups (8 per compute unit) with at most max_rows rows each
  int64_t rows = (nrows * G.nbx + target - 1) / target;
  rows = rows < 1 ? 1 : (rows > max_rows ? max_rows : rows);
  G.rows = (int)rows;
  fit_rows(G, nrows);
  return G;
}

// Calls fn(std::integral_constant<bool, b>{}): turns a run-time flag into a template argument.
template <typename Fn>
static void with_flag(bool b, Fn&& fn) {
  if (b)
    fn(std::true_type{});
  else
    fn(std::false_type{});
}

template <typename R>
static hipError_t bgk2_(const void* A, void* B, const Layout& L, const Grid& G, double omega,
                        const Force& F, bool walls, double* partials, hipStream_t s) {
  dim3 grid(G.nbx, G.nby), block(G.bx);
  auto a = static_cast<const R*>(A);
  auto b = static_cast<R*>(B);
  with_flag(walls, [&](auto W) {
    with_flag(partials != nullptr, [&](auto Dg) {
      with_flag(F.on(), [&](auto Fo) {
        k_bgk_d2q9<R, decltype(W)::value, decltype(Dg)::value, decltype(Fo)::value>
            <<<grid, block, 0, s>>>(a, b, L.nx, L.ny, L.pitch, L.plane, omega, F, G.rows, partials);
      });
    });
  });
  return hipGetLastError();
}

template <typename R>
static hipError_t bgk3(const void* A, void* B, const Layout& L, const Grid& G, double omega,
                       const Force& F, bool walls, double* partials, hipStream_t s) {
  dim3 grid(G.nbx, G.nby), block(G.bx);
  auto a = static_cast<const R*>(A);
  auto b = static_cast<R*>(B);
  with_flag(walls, [&](auto W) {
    with_flag(partials != nullptr, [&](auto Dg) {
      with_flag(F.on(), [&](auto Fo) {
        k_bgk_d3q27<R, decltype(W)::value, decltype(Dg)::value, decltype(Fo)::value>
            <<<grid, block, 0, s>>>(a, b, L.nx, L.ny, L.nz, L.pitch, L.plane, omega, F, G.rows,
                                    partials);
      });
    });
  });
  return hipGetLastError();
}

hipError_t launch_bgk_d2q9(int kind, const void* A, void* B, const Layout& L, const Grid& G,
                           double omega, const Force& F, bool walls, double* partials,
                           hipStream_t s) {
  return kind == 0 ? bgk2_<float>(A, B, L, G, omega, F, walls, partials, s)
                   : bgk2_<double>(A, B, L, G, omega, F, walls, partials, s);
}

hipError_t launch_bgk_d3q27(int kind, const void* A, void* B, const Layout& L, const Grid& G,
                            double omega, const Force& F, bool walls, double* partials,
                            hipStream_t s) {
  return kind == 0 ? bgk3<float>(A, B, L, G, omega, F, walls, partials, s)
                   : bgk3<double>(A, B, L, G, omega, F, walls, partials, s);
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename R>
static hipError_t bgk2_aa(void* A, const Layout& L, const Grid& G, double omega, const Force& F,
                          bool walls, bool odd, double* partials, hipStream_t s) {
  dim3 grid(G.nbx, G.nby), block(G.bx);
  auto a = static_cast<R*>(A);
  with_flag(walls, [&](auto W) {
    with_flag(partials != nullptr, [&](auto Dg) {
      with_flag(odd, [&](auto O) {
        with_flag(F.on(), [&](auto Fo) {
          k_bgk_d2q9_aa<R, decltype(W)::value, decltype(Dg)::value, decltype(O)::value,
                        decltype(Fo)::value>
              <<<grid, block, 0, s>>>(a, L.nx, L.ny, L.pitch, L.plane, omega, F, G.rows, partials);
        });
      });
    });
  });
  return hipGetLastError();
}

hipError_t launch_bgk_d2q9_aa(int kind, bool odd, void* A, const Layout& L, const Grid& G,
                              double omega, const Force& F, bool walls, double* partials,
                              hipStream_t s) {
  return kind == 0 ? bgk2_aa<float>(A, L, G, omega, F, walls, odd, partials, s)
                   : bgk2_aa<double>(A, L, G, omega, F, walls, odd, partials, s);
}

template <typename R>
static hipError_t bgk3_aa(void* A, const Layout& L, const Grid& G, double omega, const Force& F,
                          bool walls, bool odd, double* partials, hipStream_t s) {
  dim3 grid(G.nbx, G.nby), block(G.bx);
  auto a = static_cast<R*>(A);
  with_flag(walls, [&](auto W) {
    with_flag(partials != nullptr, [&](auto Dg) {
      with_flag(odd, [&](auto O) {
        with_flag(F.on(), [&](auto Fo) {
          k_bgk_d3q27_aa<R, decltype(W)::value, decltype(Dg)::value, decltype(O)::value,
                         decltype(Fo)::value><<<grid, block, 0, s>>>(
              a, L.nx, L.ny, L.nz, L.pitch, L.plane, omega, F, G.rows, partials);
        });
      });
    });
  });
  return hipGetLastError();
}

hipError_t launch_bgk_d3q27_aa(int kind, bool odd, void* A, const Layout& L, const Grid& G,
                               double omega, const Force& F, bool walls, double* partials,
                               hipStream_t s) {
  return kind == 0 ? bgk3_aa<float>(A, L, G, omega, F, walls, odd, partials, s)
                   : bgk3_aa<double>(A, L, G, omega, F, walls, odd, partials, s);
}

hipError_t launch_init_bgk(int kind, int D, const double* rho, const double* u, void* A,
                           const Layout& L, bool swap, double omega, const Force& F,
                           hipStream_t s) {
  const int sw = swap ? 1 : 0;
  with_flag(F.on(), [&](auto Fo) {
    constexpr bool FO = decltype(Fo)::value;
    if (kind == 0)
      k_init_bgk<float, FO><<<nblk(L.nodes()), kBlock, 0, s>>>(
          D, rho, u, static_cast<float*>(A), L.nx, L.ny, L.nz, L.pitch, L.plane, sw, omega, F);
    else
      k_init_bgk<double, FO><<<nblk(L.nodes()), kBlock, 0, s>>>(
          D, rho, u, static_cast<double*>(A), L.nx, L.ny, L.nz, L.pitch, L.plane, sw, omega, F);
  });
  return hipGetLastError();
}

hipError_t launch_moments_bgk(int kind, int D, const void* A, const Layout& L, int view,
                              bool walls, const Force& F, double* rho, double* u, hipStream_t s) {
  if (kind == 0)
    k_moments_bgk<float><<<nblk(L.nodes()), kBlock, 0, s>>>(D, static_cast<const float*>(A), L.nx, L.ny, L.nz, L.pitch, L.plane, view, walls ? 1 : 0, F, rho, u);
  else
    k_moments_bgk<double><<<nblk(L.nodes()), kBlock, 0, s>>>(D, static_cast<const double*>(A), L.nx, L.ny, L.nz, L.pitch, L.plane, view, walls ? 1 : 0, F, rho, u);
  return hipGetLastError();
}

hipError_t launch_decode_f(int kind, int D, int i, const void* A, const Layout& L, int view,
                           bool walls, double* f, hipStream_t s) {
  if (kind == 0)
    k_decode_f<float><<<nblk(L.nodes()), kBlock, 0, s>>>(D, i, static_cast<const float*>(A), L.nx, L.ny, L.nz, L.pitch, L.plane, view, walls ? 1 : 0, f);
  else
    k_decode_f<double><<<nblk(L.nodes()), kBlock, 0, s>>>(D, i, static_cast<const double*>(A), L.nx, L.ny, L.nz, L.pitch, L.plane, view, walls ? 1 : 0, f);
  return hipGetLastError();
}

hipError_t launch_diag_finalize(const double* partials, int nblocks, double t, double* out,
                                hipStream_t s) {
  k_diag_finalize<<<1, kBlock, 0, s>>>(partials, nblocks, t, out);
  return hipGetLastError();
}

hipError_t launch_field_totals(int D, const double* rho, const double* u, const double* edens,
                               int64_t nodes, bool kinetic, double* partials, int nparts,
                               double* out, hipStream_t s) {
  k_field_totals<<<nparts, kBlock, 0, s>>>(D, rho, u, edens, nodes, kinetic ? 1 : 0, partials);
  k_diag_finalize<<<1, kBlock, 0, s>>>(partials, nparts, 0.0, out);
  return hipGetLastError();
}

}  // namespace lbm
