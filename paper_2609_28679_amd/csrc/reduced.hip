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

// f_i^eq - w_i from drho = rho - 1 and the per-axis deviations
__device__ __forceinline__ float heq_i(int i, float drho, const float (&dx)[3], const float (&dy)[3]) {
  const int a = i % 3, b = i / 3;
  const float pa = wk(a) + dx[a], pb = wk(b) + dy[b];
  return drho * (pa * pb) + (wk(a) * dy[b] + dx[a] * wk(b) + dx[a] * dy[b]);
}

// Stored values of one node: moments (rho - 1, u_x, u_y) and the six codes.
struct RawNode {
  float m[3];
  uint16_t n[kRedF];
};

__device__ __forceinline__ void load_node(const float* __restrict__ M, const uint16_t* __restrict__ N,
                                          int64_t plane, int64_t off, RawNode& v) {
#pragma unroll
  for (int k = 0; k < 3; ++k) v.m[k] = load_nt(M + k * plane + off);
#pragma unroll
  for (int k = 0; k < kRedF; ++k) v.n[k] = load_nt(N + k * plane + off);
}

// Post-collision populations (shifted, h = f~ - w) of a stored node, rebuilt as described above.
template <typename Codec>
__device__ __forceinline__ void rebuild_node(const RawNode& v, float s_dec, float (&h)[9]) {
  const float drho = v.m[0], ux = v.m[1], uy = v.m[2];
  float dx[3], dy[3];
  dpsi3(ux, dx);
  dpsi3(uy, dy);
#pragma unroll
  for (int i = 0; i < 9; ++i)
    if (f_slot(i) >= 0) h[i] = heq_i(i, drho, dx, dy) + Codec::dec(v.n[f_slot(i)], s_dec);
  const float rho = 1.0f + drho;
  h[5] = rho * ux - (h[2] + h[8]) + (h[0] + h[3] + h[6]);
  h[7] = rho * uy - (h[6] + h[8]) + (h[0] + h[1] + h[2]);
  h[4] = drho - (((h[0] + h[1]) + (h[2] + h[3])) + ((h[5] + h[6]) + (h[7] + h[8])));
}

// Wavefront-strip kernel. A wavefront owns 64 consecutive columns (x0 = 64 k) and `rows` rows
// and walks them bottom to top; nothing is shared between wavefronts, so there is no barrier.
// Each lane rebuilds the post-collision populations of its own column once per row and keeps
// the last three rows in registers; a pull from column x - c_x takes the value from the lane
// to the left or right with one wave-wide DPP shift, and the two columns beyond the strip
// (x0 - 1 and x0 + 64, periodic) are rebuilt once per launch for all rows of the strip into a
// small per-wave LDS table (one vectorised pass). The raw stored values of the row after the
// next are loaded while the current row collides. The collision is the plain BGK relaxation
// of Eq. (LBM_f) with f* = f^eq; the new state is written as m = (rho - 1, u) and the six codes
// of (1 - omega)(f - f^eq(m)).
constexpr int kRedHaloRows = 66;  // strip rows + 2 per launch (rows <= 64)

__device__ __forceinline__ float shift_from_left(float v) {  // lane l receives lane l - 1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float shift_from_right(float v) {  // lane l receives lane l + 1
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

template <typename Codec, bool WALLS, bool DIAG>
__global__ void __launch_bounds__(kBlock)
k_bgk_d2q9_red(const float* __restrict__ M, const uint16_t* __restrict__ N, float* __restrict__ Mo,
               uint16_t* __restrict__ No, int nx, int ny, int64_t pitch, int64_t plane,
               float omega, float s_enc, float s_dec, int rows, double* __restrict__ partials) {
  // halo[wave][side][row][k]: side 0 = column x0 - 1 (populations 2, 5, 8 moving +x),
  // side 1 = column x0 + 64 (populations 0, 3, 6 moving -x); row = y - (y0 - 1)
  __shared__ float halo[kBlock / 64][2][kRedHaloRows][3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nbx = (nx + kBlock - 1) / kBlock;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bx = tile % nbx, by = tile / nbx;
  const int x0 = bx * kBlock + wv * 64;  // first column of this wave's strip
  const int x = x0 + lane;
  const bool own = x < nx;
  const int xc = own ? x : nx - 1;       // a valid column for lanes past the edge
  const int y0 = by * rows;
  const int yend = min(y0 + rows, ny);
  const float keep = 1.0f - omega;
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (x0 < nx) {  // strips past the right edge only join the diagnostics reduction
  const int last = min(63, nx - 1 - x0);  // lane holding the strip's last column
  // rows the pulls read: y0 - 1 .. yend (periodic), or only those inside the walls
  auto row_of = [&](int r) { return ((r % ny) + ny) % ny; };
  auto outside = [&](int r) { return WALLS && (r < 0 || r >= ny); };

  // ---- halo columns for all rows of the strip: lane = (side, row) --------------------------
  {
    const int nh = (yend - y0) + 2;
    for (int k = lane; k < 2 * nh; k += 64) {
      const int side = k >= nh, hr = side ? k - nh : k;
      const int r = y0 - 1 + hr;
      if (outside(r)) continue;
      const int xs = side ? (x0 + last + 1 == nx ? 0 : x0 + last + 1) : (x0 == 0 ? nx - 1 : x0 - 1);
      RawNode v;
      const int64_t off = (int64_t)row_of(r) * pitch + xs;
#pragma unroll
      for (int q = 0; q < 3; ++q) v.m[q] = M[q * plane + off];
#pragma unroll
      for (int q = 0; q < kRedF; ++q) v.n[q] = N[q * plane + off];
      float h[9];
      rebuild_node<Codec>(v, s_dec, h);
      float* dst = halo[wv][side][hr];
      if (side == 0) { dst[0] = h[2]; dst[1] = h[5]; dst[2] = h[8]; }
      else { dst[0] = h[0]; dst[1] = h[3]; dst[2] = h[6]; }
    }
  }

  // ---- own column: rows y0 - 1 and y0 rebuilt, y0 + 1 loaded ---------------------------------
  float ring[3][9];  // ring[r mod 3]: rebuilt row r of the own column
  RawNode raw;
  // The loads are unconditional (a row beyond a wall reads the nearest real row, whose values
  // are then not used): a load issued only on some paths would make the compiler wait for every
  // outstanding memory operation, the previous row's stores included, before the next row.
  auto fetch = [&](int r) {
    const int rr = WALLS ? (r < 0 ? 0 : (r > ny - 1 ? ny - 1 : r)) : row_of(r);
    load_node(M, N, plane, (int64_t)rr * pitch + xc, raw);
  };
  auto put = [&](int r, float (&dst)[9]) {
    if (outside(r)) return;
    rebuild_node<Codec>(raw, s_dec, dst);
  };
  fetch(y0 - 1);
  put(y0 - 1, ring[0]);
  fetch(y0);
  put(y0, ring[1]);
  fetch(y0 + 1);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // ring slot of row r: (r - y0 + 1) mod 3, a compile-time constant in the unrolled body; the
  // body always runs all three rows (rows past yend compute on re-read data and store
  // nothing), so the loop has no early exit and no loop-carried register copies, which would
  // make the compiler wait for every outstanding store at the back edge
  for (int yb = y0; yb < yend; yb += 3) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int y = yb + j;
    const bool live = y < yend;
    // rebuild row y + 1 (loaded one iteration ago), load row y + 2
    put(min(y + 1, yend), ring[(j + 2) % 3]);
    fetch(min(y + 2, yend));  // past the last needed row: a harmless re-read
    const float (&rm)[9] = ring[j];            // row y - 1
    const float (&r0)[9] = ring[(j + 1) % 3];  // row y
    const float (&rp)[9] = ring[(j + 2) % 3];  // row y + 1
    const int hr = min(y, yend - 1) - y0 + 1;   // halo row of y (rows past yend: the last)
    // pull: f_i(x) = f~_i(x - c_i); i = (c_x + 1) + 3 (c_y + 1); rows beyond a wall bounce back
    float h[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int ka = i % 3, kb = i / 3;          // c_x = ka - 1, c_y = kb - 1
      const bool bounce = WALLS && ((kb == 2 && y == 0) || (kb == 0 && y == ny - 1));
      if (bounce) {
        h[i] = r0[8 - i];
        continue;
      }
      const float(&src)[9] = kb == 0 ? rp : (kb == 1 ? r0 : rm);  // row y - c_y
      const int hrow = hr - (kb - 1);
      if (ka == 1) {
        h[i] = src[i];
      } else if (ka == 2) {  // from column x - 1
        const float v = shift_from_left(src[i]);
        h[i] = lane == 0 ? halo[wv][0][hrow][i / 3] : v;
      } else {               // from column x + 1
        const float v = shift_from_right(src[i]);
        h[i] = lane == last ? halo[wv][1][hrow][i / 3] : v;
      }
    }
    // moments (sum_i w_i = 1, sum_i c_i w_i = 0) and the relaxation
    const float drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    const float jx = (h[2] + h[5] + h[8]) - (h[0] + h[3] + h[6]);
    const float jy = (h[6] + h[7] + h[8]) - (h[0] + h[1] + h[2]);
    const float rho = 1.0f + drho;
    const float ux = quotient(jx, rho), uy = quotient(jy, rho);
    float dx[3], dy[3];
    dpsi3(ux, dx);
    dpsi3(uy, dy);
    if (own && live) {
      const int64_t self = (int64_t)y * pitch + x;
      store_nt(Mo + self, drho);
      store_nt(Mo + plane + self, ux);
      store_nt(Mo + 2 * plane + self, uy);
#pragma unroll
      for (int i = 0; i < 9; ++i)
        if (f_slot(i) >= 0)
          store_nt(No + f_slot(i) * plane + self,
                   Codec::enc(keep * (h[i] - heq_i(i, drho, dx, dy)), s_enc));
      if (DIAG) {
        const double rho = 1.0 + (double)drho;
        acc[0] += rho;
        acc[1] += (double)jx;
        acc[2] += (double)jy;
        acc[4] += 0.5 * rho * ((double)ux * ux + (double)uy * uy);
      }
    }
  }
  }
  }
  if (DIAG) block_sum_store<kDiagValues>(acc, partials + (int64_t)tile * kDiagValues);
}

// Initial state f = f^eq(rho0, u0): moments stored, non-equilibrium part zero.
__global__ void k_init_bgk_red(const double* __restrict__ rho, const double* __restrict__ u,
                               float* __restrict__ M, uint16_t* __restrict__ N, int nx,
                               int64_t nodes, int64_t pitch, int64_t plane) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  M[off] = (float)(rho[n] - 1.0);
  M[plane + off] = (float)u[n];
  M[2 * plane + off] = (float)u[nodes + n];
  for (int k = 0; k < kRedF; ++k) N[k * plane + off] = 0;  // +0 in both codecs
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
// Tiles of 256 columns (four 64-column wavefront strips) by `rows` rows, launched as a
// one-dimensional grid (tile = bx + nbx by), so tall lattices need no more rows per tile; the
// per-wave halo table holds rows + 2 <= kRedHaloRows rows.
Grid make_grid_red(const Layout& L) {
  Grid G;
  G.bx = kBlock;
  G.nbx = (L.nx + kBlock - 1) / kBlock;
  G.rows = 12;
#ifdef LBM_TUNING_ENV
  if (const char* v = getenv("LBM_RED_ROWS")) G.rows = atoi(v);
#endif
  if (G.rows > kRedHaloRows - 2) G.rows = kRedHaloRows - 2;
  if (G.rows < 1) G.rows = 1;
  G.nby = (L.ny + G.rows - 1) / G.rows;
  return G;
}

template <typename Codec, bool WALLS>
static void red_launch(const float* M, const uint16_t* N, float* Mo, uint16_t* No, const Layout& L,
                       const Grid& G, double omega, float se, float sd, double* partials,
                       hipStream_t s) {
  dim3 grid((unsigned)G.blocks()), block(kBlock);
  const float om = (float)omega;
  if (partials)
    k_bgk_d2q9_red<Codec, WALLS, true><<<grid, block, 0, s>>>(M, N, Mo, No, L.nx, L.ny, L.pitch, L.plane, om, se, sd, G.rows, partials);
  else
    k_bgk_d2q9_red<Codec, WALLS, false><<<grid, block, 0, s>>>(M, N, Mo, No, L.nx, L.ny, L.pitch, L.plane, om, se, sd, G.rows, nullptr);
}

// Buffer layout: 3 float moment planes, then kRedF uint16 planes (plane elements each).
static inline const uint16_t* neq_of(const void* buf, const Layout& L, int nm) {
  return reinterpret_cast<const uint16_t*>(static_cast<const float*>(buf) + nm * L.plane);
}

hipError_t launch_bgk_d2q9_red(int codec, const void* A, void* B, const Layout& L, const Grid& G,
                               double omega, bool walls, float s_enc, float s_dec,
                               double* partials, hipStream_t s) {
  const float* M = static_cast<const float*>(A);
  const uint16_t* N = neq_of(A, L, 3);
  float* Mo = static_cast<float*>(B);
  uint16_t* No = const_cast<uint16_t*>(neq_of(B, L, 3));
  if (codec == 0) {
    if (walls) red_launch<CodecBF16, true>(M, N, Mo, No, L, G, omega, s_enc, s_dec, partials, s);
    else red_launch<CodecBF16, false>(M, N, Mo, No, L, G, omega, s_enc, s_dec, partials, s);
  } else {
    if (walls) red_launch<CodecFP16, true>(M, N, Mo, No, L, G, omega, s_enc, s_dec, partials, s);
    else red_launch<CodecFP16, false>(M, N, Mo, No, L, G, omega, s_enc, s_dec, partials, s);
  }
  return hipGetLastError();
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_init_bgk_red(const double* rho, const double* u, void* A, const Layout& L,
                               hipStream_t s) {
  k_init_bgk_red<<<nblk(L.nodes()), kBlock, 0, s>>>(rho, u, static_cast<float*>(A),
                                                    const_cast<uint16_t*>(neq_of(A, L, 3)), L.nx,
                                                    L.nodes(), L.pitch, L.plane);
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
