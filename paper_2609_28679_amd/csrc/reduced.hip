// Isothermal D2Q9 fused pull stream-collide on reduced-precision storage (float32 moments +
// 16-bit non-equilibrium part, see reduced_common.h).
//
// Pull: the pre-collision population i at x is the post-collision population i of the source
// node s = x - c_i, rebuilt from that node's stored moments and non-equilibrium part,
//   f_i(x, t) = f_i^eq(m(s)) + n_i(s)       (f_ibar(x) at a half-way bounce-back wall),
// with the product-form equilibrium of Sec. II C at theta = 1/3. The collision is the plain
// BGK relaxation of Eq. (LBM_f) with f* = f^eq; the new state is written back as
// m(x) = (rho - 1, u) and n(x) = f~(x) - f^eq(m(x)).
#include "reduced_common.h"

#include <cstdlib>

namespace lbm {

// Arithmetic is float32 on shifted values h_i = f_i - w_i (w the rest weights). With
// theta = 1/3 the per-axis factors are psi_c = W_c + d_c, W = (1/6, 2/3, 1/6), d_0 = -u^2,
// d_+- = (u^2 +- u)/2, and
//   f_i^eq - w_i = (rho - 1) psi_a psi_b + (W_a d_b + d_a W_b + d_a d_b).
// The float32 constants are W_+- = 2796203 2^-24 and W_0 = 1 - 2 W_+- (exact), so the factors
// sum to one exactly; with the nearest float32 values of 1/6 and 2/3 they miss it by 3e-8 and
// every rebuild shifts a node's mass by that fraction, the same way at every step.
//
// Rebuild of a stored node (moments m, six codes): h_i = h^eq_i(m) + n_i for the six stored
// directions, then the remaining three from the node's own conserved sums, which the state
// holds exactly as stored moments:
//   h_5 = j_x - (h_2 + h_8) + (h_0 + h_3 + h_6),  h_7 = j_y - (h_6 + h_8) + (h_0 + h_1 + h_2),
//   h_4 = (rho - 1) - sum_{i != 4} h_i,  j = rho u.
// (In exact arithmetic this equals h^eq + n with n_5, n_7, n_4 from the zero sums of the
// non-equilibrium part; in float32 it keeps the rounding of the equilibrium out of the rebuilt
// mass and momentum, which otherwise repeats at a node from step to step: a float32 rebuild
// h^eq + n drifted to a velocity rel-L2 of 6e-5 against the float64 scheme after 10^4 steps of
// 256^2 turbulence at tau 0.51 with float32 non-equilibrium values.)
// u = j / rho to within half an ulp or so, unbiased: the hardware reciprocal alone (1 ulp)
// errs to one side for a given rho, and a stored velocity that is always slightly small or
// large rebuilds a momentum that shrinks or grows the same way at every step (a velocity
// drift of 1e-4 after 10^4 steps); one residual correction r = j - rho q (exact with fma)
// removes that bias.
__device__ __forceinline__ float quotient(float j, float rho) {
  const float inv = __builtin_amdgcn_rcpf(rho);
  const float q = j * inv;
  return __builtin_fmaf(__builtin_fmaf(-rho, q, j), inv, q);
}

constexpr float kW1 = 2796203.0f / 16777216.0f;
constexpr float kW0 = 1.0f - 2.0f * kW1;

__device__ __forceinline__ float wk(int k) { return k == 1 ? kW0 : kW1; }

__device__ __forceinline__ void dpsi3(float u, float (&d)[3]) {
  const float u2 = u * u;
  d[0] = 0.5f * (u2 - u);
  d[1] = -u2;
  d[2] = 0.5f * (u2 + u);
}

// f_i^eq - w_i of the six stored directions from drho = rho - 1 and the per-axis deviations,
// factored as psi_b (drho psi_a + d_a) + W_a d_b (psi = W + d, the same sum regrouped): six
// per-axis values, then one fma per direction.
__device__ __forceinline__ void heq_stored(float drho, const float (&dx)[3], const float (&dy)[3],
                                           float (&e)[9]) {
  float A[3], P[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    A[k] = __builtin_fmaf(drho, wk(k) + dx[k], dx[k]);
    P[k] = wk(k) + dy[k];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i)
    if (f_slot(i) >= 0) e[i] = __builtin_fmaf(P[i / 3], A[i % 3], wk(i % 3) * dy[i / 3]);
}

// Post-collision populations (shifted, h = f~ - w) of a stored node from its moments and its
// six decoded non-equilibrium values, rebuilt as described above.
__device__ __forceinline__ void rebuild(float drho, float ux, float uy, const float (&n)[kRedF],
                                        float (&h)[9]) {
  float dx[3], dy[3], e[9];
  dpsi3(ux, dx);
  dpsi3(uy, dy);
  heq_stored(drho, dx, dy, e);
#pragma unroll
  for (int i = 0; i < 9; ++i)
    if (f_slot(i) >= 0) h[i] = e[i] + n[f_slot(i)];
  const float rho = 1.0f + drho;
  h[5] = rho * ux - (h[2] + h[8]) + (h[0] + h[3] + h[6]);
  h[7] = rho * uy - (h[6] + h[8]) + (h[0] + h[1] + h[2]);
  h[4] = drho - (((h[0] + h[1]) + (h[2] + h[3])) + ((h[5] + h[6]) + (h[7] + h[8])));
}

// Stored values of one node: moments (rho - 1, u_x, u_y) and the six codes.
struct RawNode {
  float m[3];
  uint16_t n[kRedF];
};

template <typename Codec>
__device__ __forceinline__ void rebuild_node(const RawNode& v, float s_dec, float (&h)[9]) {
  float n[kRedF];
#pragma unroll
  for (int k = 0; k < kRedF; ++k) n[k] = Codec::dec(v.n[k], s_dec);
  rebuild(v.m[0], v.m[1], v.m[2], n, h);
}

// Wavefront-strip kernel. A wavefront owns 128 consecutive columns (x0 = 128 k), two per lane
// (columns x0 + 2 l and x0 + 2 l + 1, so every load and store moves a pair: 8 bytes of a moment
// plane, 4 bytes of a code plane), and `rows` rows, which it walks bottom to top; nothing is
// shared between wavefronts, so there is no barrier. Each lane rebuilds the post-collision
// populations of its two columns once per row and keeps the last three rows in registers. A
// pull from column x - c_x takes the value from the lane's other column or, across a pair
// boundary, from the neighbouring lane with one wave-wide DPP shift. The two columns beyond the
// strip (x0 - 1 and the one after the strip's last column, periodic) are rebuilt once per
// launch for all rows of the strip from the edge records below, one node per lane (lanes 0-31
// the left column, 32-63 the right one, row y0 - 1 + lane mod 32), and read with readlane. The
// stored values of a row are loaded three rows ahead of its turn. The collision is the plain BGK
// relaxation of Eq. (LBM_f) with f* = f^eq; the new state is written as m = (rho - 1, u) and
// the six codes of (1 - omega)(f - f^eq(m)).
constexpr int kRedMaxRows = 30;              // rows + 2 halo rows per half wavefront
constexpr int kRedBlockCols = 2 * kBlock;    // columns of one workgroup
constexpr int kRedStrip = 128;               // columns of one wavefront strip

// Edge records: the stored values (moments and codes, the same bits as in the planes) of the
// first and last column of every 128-column strip, contiguous in y, written by the step that
// produces them. A strip's neighbour columns are the last column of the strip to its left and
// the first column of the strip to its right (periodic), so the halo table of a wavefront reads
// a few cache lines instead of one line per value: read from the planes, the halo of a strip of
// 12 rows pulled 64 lines per load instruction through the L1 for 256 useful bytes, which
// delayed the start of every wavefront (49 vs 43 us at 2048^2).
struct __attribute__((aligned(16))) EdgeRec {
  float m[4];        // rho - 1, u_x, u_y, unused
  uint16_t n[8];     // the six codes, two unused
};
static_assert(sizeof(EdgeRec) == 32, "edge records are two 16-byte words");
// record of strip s, side e (0 first column, 1 last column), row y
__host__ __device__ inline int64_t edge_index(int s, int e, int y, int ny) {
  return ((int64_t)s * 2 + e) * ny + y;
}

typedef float f2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float shift_from_left(float v) {  // lane l receives lane l - 1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float shift_from_right(float v) {  // lane l receives lane l + 1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Pre-collision moments and the scaled non-equilibrium part (1 - omega)(f - f^eq) of the six
// stored directions of one column.
struct Collided {
  float drho, ux, uy, jx, jy;
  float q[kRedF];
};

__device__ __forceinline__ Collided collide_column(const float (&h)[9], float keep) {
  Collided c;
  c.drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
  c.jx = (h[2] + h[5] + h[8]) - (h[0] + h[3] + h[6]);
  c.jy = (h[6] + h[7] + h[8]) - (h[0] + h[1] + h[2]);
  const float rho = 1.0f + c.drho;
  c.ux = quotient(c.jx, rho);
  c.uy = quotient(c.jy, rho);
  float dx[3], dy[3], e[9];
  dpsi3(c.ux, dx);
  dpsi3(c.uy, dy);
  heq_stored(c.drho, dx, dy, e);
#pragma unroll
  for (int i = 0; i < 9; ++i)
    if (f_slot(i) >= 0) c.q[f_slot(i)] = keep * (h[i] - e[i]);
  return c;
}

template <typename Codec, bool WALLS, bool DIAG>
__global__ void __launch_bounds__(kBlock)
k_bgk_d2q9_red(const float* __restrict__ M, const uint16_t* __restrict__ N,
               const EdgeRec* __restrict__ E, float* __restrict__ Mo, uint16_t* __restrict__ No,
               EdgeRec* __restrict__ Eo, int nx, int ny, int64_t pitch, int64_t plane,
               float omega, float s_enc, float s_dec, int rows, double* __restrict__ partials) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nbx = (nx + kRedBlockCols - 1) / kRedBlockCols;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bx = tile % nbx, by = tile / nbx;
  const int x0 = bx * kRedBlockCols + wv * 128;  // first column of this wave's strip
  const int y0 = by * rows;
  const int yend = min(y0 + rows, ny);
  const float keep = 1.0f - omega;
  const int64_t hp = plane >> 1;                 // plane stride in pairs (planes are even)
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (x0 < nx) {  // strips past the right edge only join the diagnostics reduction
  const int ncol = min(128, nx - x0);
  const int ll = (ncol - 1) >> 1;                // lane holding the strip's last column
  const bool last_even = ((ncol - 1) & 1) == 0;  // ... in its first slot
  // column pair of this lane; pairs past the row's end load the last pair (the odd column of
  // an odd-width row lies in the row padding) and store nothing
  const int pmax = (nx + 1) / 2 - 1;
  const int p = x0 / 2 + lane;
  const uint32_t pc = (uint32_t)min(p, pmax);
  const bool own0 = p <= pmax, own1 = 2 * p + 1 < nx;
  const uint32_t pc8 = pc * 8u, pc4 = pc * 4u;  // byte offsets in a row (rows are < 4 GiB)
  // a row beyond a wall reads the nearest real row (its values are then not used)
  auto src_row = [&](int r) {
    return WALLS ? min(max(r, 0), ny - 1) : (r < 0 ? r + ny : (r >= ny ? r - ny : r));
  };

  // ---- halo columns, one node per lane, from the edge records --------------------------------
  // lanes 0-31: the column left of the strip (last column of strip s - 1), keeping populations
  // 2, 5, 8 (moving +x); lanes 32-63: the column right of it (first column of strip s + 1),
  // keeping 0, 3, 6 (moving -x); row y0 - 1 + lane mod 32
  float hv[3];
  {
    const int ns = (nx + kRedStrip - 1) / kRedStrip, s = x0 / kRedStrip;
    const int side = lane >> 5;
    const int hr = min(lane & 31, yend - y0 + 1);
    const int64_t rec = side ? edge_index(s + 1 == ns ? 0 : s + 1, 0, src_row(y0 - 1 + hr), ny)
                             : edge_index(s == 0 ? ns - 1 : s - 1, 1, src_row(y0 - 1 + hr), ny);
    typedef float f4v __attribute__((ext_vector_type(4)));
    typedef uint32_t u4v __attribute__((ext_vector_type(4)));
    const f4v em = *reinterpret_cast<const f4v*>(&E[rec].m[0]);
    const u4v en = *reinterpret_cast<const u4v*>(&E[rec].n[0]);
    RawNode v;
    v.m[0] = em.x; v.m[1] = em.y; v.m[2] = em.z;
    v.n[0] = (uint16_t)(en.x & 0xFFFFu); v.n[1] = (uint16_t)(en.x >> 16);
    v.n[2] = (uint16_t)(en.y & 0xFFFFu); v.n[3] = (uint16_t)(en.y >> 16);
    v.n[4] = (uint16_t)(en.z & 0xFFFFu); v.n[5] = (uint16_t)(en.z >> 16);
    float h[9];
    rebuild_node<Codec>(v, s_dec, h);
#pragma unroll
    for (int k = 0; k < 3; ++k) hv[k] = side ? h[3 * k] : h[3 * k + 2];
  }

  // ---- own columns: rows y0 - 1 and y0 rebuilt, y0 + 1 and y0 + 2 loading -------------------
  // Slot of row r in both rings: (r - y0 + 1) mod 3, a compile-time constant in the unrolled
  // loop body. The stored values of a row are loaded three rows before its turn (two rows in
  // flight per wavefront while one collides), rebuilt one row before.
  float R0[3][9], R1[3][9];  // rebuilt rows of the even / odd column
  f2v rm[3][3];              // raw moments of the rows in flight
  uint32_t rn[3][kRedF];     // raw code pairs of the rows in flight
  // The loads are unconditional: a load issued only on some paths would make the compiler wait
  // for every outstanding memory operation, the previous row's stores included.
  // The 32-bit lane offsets are re-declared where they are used (an empty asm), so that the
  // compiler does not hoist their 64-bit extension out of the loop, which loses the scalar-base
  // form of the accesses.
  auto fetch = [&](int r, f2v (&m)[3], uint32_t (&n)[kRedF]) {
    uint32_t o8 = pc8, o4 = pc4;
    asm volatile("" : "+v"(o8), "+v"(o4));
    const int64_t base = (int64_t)src_row(r) * pitch;
    const f2v* mrow = reinterpret_cast<const f2v*>(M + base);
    const uint32_t* nrow = reinterpret_cast<const uint32_t*>(N + base);
#pragma unroll
    for (int k = 0; k < 3; ++k) m[k] = gload_nt(at_byte(sbase(mrow + k * hp), o8));
#pragma unroll
    for (int k = 0; k < kRedF; ++k) n[k] = gload_nt(at_byte(sbase(nrow + k * hp), o4));
  };
  auto put = [&](const f2v (&m)[3], const uint32_t (&n)[kRedF], float (&d0)[9], float (&d1)[9]) {
    float n0[kRedF], n1[kRedF];
#pragma unroll
    for (int k = 0; k < kRedF; ++k) {
      n0[k] = Codec::dec_lo(n[k], s_dec);
      n1[k] = Codec::dec_hi(n[k], s_dec);
    }
    rebuild(m[0].x, m[1].x, m[2].x, n0, d0);
    rebuild(m[0].y, m[1].y, m[2].y, n1, d1);
  };
  fetch(y0 - 1, rm[0], rn[0]);
  put(rm[0], rn[0], R0[0], R1[0]);
  fetch(y0, rm[1], rn[1]);
  put(rm[1], rn[1], R0[1], R1[1]);
  fetch(y0 + 1, rm[2], rn[2]);
  fetch(min(y0 + 2, yend), rm[0], rn[0]);
  // a per-lane copy of yend: the store conditions below are then lane masks, whose skip paths
  // the compiler's wait counting handles without draining every outstanding load and store at
  // the top of the loop (a uniform branch around the stores made it wait for everything)
  int yend_v = yend;
  asm volatile("" : "+v"(yend_v));

  // the body always runs all three rows (rows past yend compute on re-read data and store
  // nothing), so the loop has no early exit and no loop-carried register copies, which would
  // make the compiler wait for every outstanding store at the back edge
  for (int yb = y0; yb < yend; yb += 3) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int y = yb + j;
    const bool live = y < yend_v;
    // rebuild row y + 1, load row y + 3 (into the slot row y held)
    put(rm[(j + 2) % 3], rn[(j + 2) % 3], R0[(j + 2) % 3], R1[(j + 2) % 3]);
    fetch(min(y + 3, yend), rm[(j + 1) % 3], rn[(j + 1) % 3]);  // past yend: a harmless re-read
    const int hr = min(y, yend - 1) - y0 + 1;  // halo row of y (rows past yend: the last)
    // pull: f_i(x) = f~_i(x - c_i); i = (c_x + 1) + 3 (c_y + 1); rows beyond a wall bounce back
    float a[9], b[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int ka = i % 3, kb = i / 3;  // c_x = ka - 1, c_y = kb - 1
      const int cur = (j + 1) % 3;
      const bool bounce = WALLS && ((kb == 2 && y == 0) || (kb == 0 && y == ny - 1));
      if (bounce) {
        a[i] = R0[cur][8 - i];
        b[i] = R1[cur][8 - i];
        continue;
      }
      const int sr = kb == 0 ? (j + 2) % 3 : (kb == 1 ? cur : j);  // ring slot of row y - c_y
      const int hrow = hr - (kb - 1);
      if (ka == 1) {
        a[i] = R0[sr][i];
        b[i] = R1[sr][i];
      } else if (ka == 2) {  // from column x - 1
        b[i] = R0[sr][i];
        const float v = shift_from_left(R1[sr][i]);
        const float edge = read_lane(hv[kb], hrow);
        a[i] = lane == 0 ? edge : v;
      } else {               // from column x + 1
        const float edge = read_lane(hv[kb], 32 + hrow);
        a[i] = (lane == ll && last_even) ? edge : R1[sr][i];
        const float v = shift_from_right(R0[sr][i]);
        b[i] = lane == ll ? edge : v;
      }
    }
    const Collided c0 = collide_column(a, keep);
    const Collided c1 = collide_column(b, keep);
    {
      // a pair store also for the last column of an odd-width row: its second column is the
      // row's padding (pitch > nx), which nothing reads
      const int64_t self = (int64_t)y * pitch;
      if (own0 && live) {
        uint32_t o8 = pc8, o4 = pc4;
        asm volatile("" : "+v"(o8), "+v"(o4));
        f2v* mrow = reinterpret_cast<f2v*>(Mo + self);
        uint32_t* nrow = reinterpret_cast<uint32_t*>(No + self);
        gstore_nt(at_byte(sbase(mrow), o8), f2v{c0.drho, c1.drho});
        gstore_nt(at_byte(sbase(mrow + hp), o8), f2v{c0.ux, c1.ux});
        gstore_nt(at_byte(sbase(mrow + 2 * hp), o8), f2v{c0.uy, c1.uy});
        uint32_t w[kRedF];
#pragma unroll
        for (int k = 0; k < kRedF; ++k) w[k] = Codec::enc2(c0.q[k], c1.q[k], s_enc);
#pragma unroll
        for (int k = 0; k < kRedF; ++k) gstore_nt(at_byte(sbase(nrow + k * hp), o4), w[k]);
        // edge records of the strip's first column (lane 0, even slot) and last column
        typedef float f4v __attribute__((ext_vector_type(4)));
        typedef uint32_t u4v __attribute__((ext_vector_type(4)));
        const int s = x0 / kRedStrip;
        if (lane == 0) {
          EdgeRec* r = Eo + edge_index(s, 0, y, ny);
          *reinterpret_cast<f4v*>(&r->m[0]) = f4v{c0.drho, c0.ux, c0.uy, 0.0f};
          *reinterpret_cast<u4v*>(&r->n[0]) = u4v{(w[0] & 0xFFFFu) | (w[1] << 16),
                                                  (w[2] & 0xFFFFu) | (w[3] << 16),
                                                  (w[4] & 0xFFFFu) | (w[5] << 16), 0u};
        }
        if (lane == ll) {
          EdgeRec* r = Eo + edge_index(s, 1, y, ny);
          if (last_even) {
            *reinterpret_cast<f4v*>(&r->m[0]) = f4v{c0.drho, c0.ux, c0.uy, 0.0f};
            *reinterpret_cast<u4v*>(&r->n[0]) = u4v{(w[0] & 0xFFFFu) | (w[1] << 16),
                                                    (w[2] & 0xFFFFu) | (w[3] << 16),
                                                    (w[4] & 0xFFFFu) | (w[5] << 16), 0u};
          } else {
            *reinterpret_cast<f4v*>(&r->m[0]) = f4v{c1.drho, c1.ux, c1.uy, 0.0f};
            *reinterpret_cast<u4v*>(&r->n[0]) = u4v{(w[0] >> 16) | (w[1] & 0xFFFF0000u),
                                                    (w[2] >> 16) | (w[3] & 0xFFFF0000u),
                                                    (w[4] >> 16) | (w[5] & 0xFFFF0000u), 0u};
          }
        }
      }
      if (DIAG) {
        if (own0 && live) {
          const double rho = 1.0 + (double)c0.drho;
          acc[0] += rho;
          acc[1] += (double)c0.jx;
          acc[2] += (double)c0.jy;
          acc[4] += 0.5 * rho * ((double)c0.ux * c0.ux + (double)c0.uy * c0.uy);
        }
        if (own1 && live) {
          const double rho = 1.0 + (double)c1.drho;
          acc[0] += rho;
          acc[1] += (double)c1.jx;
          acc[2] += (double)c1.jy;
          acc[4] += 0.5 * rho * ((double)c1.ux * c1.ux + (double)c1.uy * c1.uy);
        }
      }
    }
  }
  }
  }
  if (DIAG) block_sum_store<kDiagValues>(acc, partials + (int64_t)tile * kDiagValues);
}

// Initial state f = f^eq(rho0, u0): moments stored, non-equilibrium part zero.
__global__ void k_init_bgk_red(const double* __restrict__ rho, const double* __restrict__ u,
                               float* __restrict__ M, uint16_t* __restrict__ N,
                               EdgeRec* __restrict__ E, int nx, int ny, int64_t nodes,
                               int64_t pitch, int64_t plane) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int x = (int)(n % nx), y = (int)(n / nx);
  const int64_t off = (int64_t)y * pitch + x;
  const float m[3] = {(float)(rho[n] - 1.0), (float)u[n], (float)u[nodes + n]};
  M[off] = m[0];
  M[plane + off] = m[1];
  M[2 * plane + off] = m[2];
  for (int k = 0; k < kRedF; ++k) N[k * plane + off] = 0;  // +0 in both codecs
  // the same values in the edge records of the strip's first and last column
  const int s = x / kRedStrip;
  for (int e = 0; e < 2; ++e) {
    if (e == 0 ? x % kRedStrip != 0 : (x % kRedStrip != kRedStrip - 1 && x != nx - 1)) continue;
    EdgeRec& r = E[edge_index(s, e, y, ny)];
    r.m[0] = m[0];
    r.m[1] = m[1];
    r.m[2] = m[2];
    r.m[3] = 0.0f;
    for (int k = 0; k < 8; ++k) r.n[k] = 0;
  }
}

__global__ void k_moments_bgk_red(const float* __restrict__ M, int nx, int64_t nodes,
                                  int64_t pitch, int64_t plane, double* __restrict__ rho,
                                  double* __restrict__ u) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  rho[n] = 1.0 + (double)M[off];
  u[n] = (double)M[plane + off];
  u[nodes + n] = (double)M[2 * plane + off];
}

template <typename Codec>
__global__ void k_decode_bgk_red(int i, const float* __restrict__ M, const uint16_t* __restrict__ N,
                                 int nx, int64_t nodes, int64_t pitch, int64_t plane, float s_dec,
                                 double* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  RawNode v;
#pragma unroll
  for (int k = 0; k < 3; ++k) v.m[k] = M[k * plane + off];
#pragma unroll
  for (int k = 0; k < kRedF; ++k) v.n[k] = N[k * plane + off];
  float h[9];
  rebuild_node<Codec>(v, s_dec, h);
  // f = h + w with the rest weights of the float32 constants (products exact in float64)
  out[n] = (double)h[i] + (double)wk(i % 3) * (double)wk(i / 3);
}

// ---- launchers -----------------------------------------------------------------------------
// Tiles of 512 columns (four 128-column wavefront strips) by `rows` rows, launched as a
// one-dimensional grid (tile = bx + nbx by), so tall lattices need no more rows per tile; the
// halo rows of a strip (rows + 2) fit one half wavefront. 18 rows measured best on MI355X
// (bf16, 2048^2 / 4096^2: 44.6 / 178 us at 18 rows; 45.4 / 185 at 12; 48.7 / 196 at 6;
// 54.4 / 185 at 30).
Grid make_grid_red(const Layout& L) {
  Grid G;
  G.bx = kBlock;
  G.nbx = (L.nx + kRedBlockCols - 1) / kRedBlockCols;
  G.rows = 18;
#ifdef LBM_TUNING_ENV
  if (const char* v = getenv("LBM_RED_ROWS")) G.rows = atoi(v);
#endif
  if (G.rows > kRedMaxRows) G.rows = kRedMaxRows;
  if (G.rows < 1) G.rows = 1;
  G.nby = (L.ny + G.rows - 1) / G.rows;
  return G;
}

template <typename Codec, bool WALLS>
static void red_launch(const float* M, const uint16_t* N, const EdgeRec* E, float* Mo,
                       uint16_t* No, EdgeRec* Eo, const Layout& L, const Grid& G, double omega,
                       float se, float sd, double* partials, hipStream_t s) {
  dim3 grid((unsigned)G.blocks()), block(kBlock);
  const float om = (float)omega;
  if (partials)
    k_bgk_d2q9_red<Codec, WALLS, true><<<grid, block, 0, s>>>(M, N, E, Mo, No, Eo, L.nx, L.ny, L.pitch, L.plane, om, se, sd, G.rows, partials);
  else
    k_bgk_d2q9_red<Codec, WALLS, false><<<grid, block, 0, s>>>(M, N, E, Mo, No, Eo, L.nx, L.ny, L.pitch, L.plane, om, se, sd, G.rows, nullptr);
}

// Buffer layout: 3 float moment planes, then kRedF uint16 planes (plane elements each), then
// (256-byte aligned) the edge records of every strip, side and row.
static inline const uint16_t* neq_of(const void* buf, const Layout& L, int nm) {
  return reinterpret_cast<const uint16_t*>(static_cast<const float*>(buf) + nm * L.plane);
}
static inline size_t red_edge_offset(const Layout& L) {
  return ((size_t)L.plane * (3 * 4 + kRedF * 2) + 255) / 256 * 256;
}
static inline EdgeRec* edges_of(const void* buf, const Layout& L) {
  return reinterpret_cast<EdgeRec*>(const_cast<char*>(static_cast<const char*>(buf)) +
                                    red_edge_offset(L));
}
size_t red_state_bytes(const Layout& L) {
  const size_t strips = ((size_t)L.nx + kRedStrip - 1) / kRedStrip;
  return red_edge_offset(L) + strips * 2 * (size_t)L.ny * sizeof(EdgeRec);
}

hipError_t launch_bgk_d2q9_red(int codec, const void* A, void* B, const Layout& L, const Grid& G,
                               double omega, bool walls, float s_enc, float s_dec,
                               double* partials, hipStream_t s) {
  // the step moves column pairs: 8-byte moment pairs and 4-byte code pairs
  if ((L.pitch | L.plane) & 1) return hipErrorInvalidValue;
  if (G.rows < 1 || G.rows > kRedMaxRows) return hipErrorInvalidValue;
  const float* M = static_cast<const float*>(A);
  const uint16_t* N = neq_of(A, L, 3);
  float* Mo = static_cast<float*>(B);
  uint16_t* No = const_cast<uint16_t*>(neq_of(B, L, 3));
  const EdgeRec* E = edges_of(A, L);
  EdgeRec* Eo = edges_of(B, L);
  if (codec == 0) {
    if (walls) red_launch<CodecBF16, true>(M, N, E, Mo, No, Eo, L, G, omega, s_enc, s_dec, partials, s);
    else red_launch<CodecBF16, false>(M, N, E, Mo, No, Eo, L, G, omega, s_enc, s_dec, partials, s);
  } else {
    if (walls) red_launch<CodecFP16, true>(M, N, E, Mo, No, Eo, L, G, omega, s_enc, s_dec, partials, s);
    else red_launch<CodecFP16, false>(M, N, E, Mo, No, Eo, L, G, omega, s_enc, s_dec, partials, s);
  }
  return hipGetLastError();
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_init_bgk_red(const double* rho, const double* u, void* A, const Layout& L,
                               hipStream_t s) {
  k_init_bgk_red<<<nblk(L.nodes()), kBlock, 0, s>>>(rho, u, static_cast<float*>(A),
                                                    const_cast<uint16_t*>(neq_of(A, L, 3)),
                                                    edges_of(A, L), L.nx, L.ny, L.nodes(),
                                                    L.pitch, L.plane);
  return hipGetLastError();
}

hipError_t launch_moments_bgk_red(const void* A, const Layout& L, double* rho, double* u,
                                  hipStream_t s) {
  k_moments_bgk_red<<<nblk(L.nodes()), kBlock, 0, s>>>(static_cast<const float*>(A), L.nx,
                                                       L.nodes(), L.pitch, L.plane, rho, u);
  return hipGetLastError();
}

hipError_t launch_decode_bgk_red(int codec, int i, const void* A, const Layout& L, float s_dec,
                                 double* out, hipStream_t s) {
  const float* M = static_cast<const float*>(A);
  const uint16_t* N = neq_of(A, L, 3);
  if (codec == 0)
    k_decode_bgk_red<CodecBF16><<<nblk(L.nodes()), kBlock, 0, s>>>(i, M, N, L.nx, L.nodes(), L.pitch, L.plane, s_dec, out);
  else
    k_decode_bgk_red<CodecFP16><<<nblk(L.nodes()), kBlock, 0, s>>>(i, M, N, L.nx, L.nodes(), L.pitch, L.plane, s_dec, out);
  return hipGetLastError();
}

}  // namespace lbm
