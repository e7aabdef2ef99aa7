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

__device__ __forceinline__ double psi_c(int c, double u) {
  const double u2 = u * u;
  return c == 0 ? (2.0 / 3.0) - u2 : (1.0 / 6.0) + 0.5 * (u2 + c * u);
}

// LDS-staged kernel. A workgroup owns 256 columns and `rows` rows and walks them bottom to
// top. Each row that enters the 3-row window is decoded once, node by node, into its nine
// post-collision populations (float32 in LDS, 258 columns with the periodic x halo); the pull
// then reads the nine sources of a node from LDS. Every stored byte is read once per workgroup
// with coalesced loads and every node's equilibrium is rebuilt once.
//
// Arithmetic is in shifted form: h_i = f_i - w_i (w the rest weights), and with
// psi_c = W_c + d_c (W = 2/3, 1/6, 1/6; d_0 = -u^2, d_+- = (u^2 +- u)/2) the equilibrium is
//   f_i^eq - w_i = (rho - 1) psi_a psi_b + (W_a d_b + d_a W_b + d_a d_b).
// The rebuild of the stored rows runs in float64 (held in LDS as float32 h), the collision in
// float32. A float32 rebuild drifts coherently: the float32 values of W repeat the same
// rounding at every node and step, and the velocity rel-L2 against the float64 scheme grew
// linearly to 5e-4 (tau 0.6) and 1.1e-3 (tau 0.51) after 10^4 steps at 256^2, the same for
// bfloat16 and float16 codes. With the float64 rebuild it stays at the storage level:
// bfloat16 1.7e-5 / 8e-5, float16 1.8e-6 / 1.4e-5 after 10^4 steps (tau 0.6 / 0.51), at 52 us
// per 2048^2 step (all float32: 47 us; all float64: 58 us).
constexpr int kRedCols = kBlock + 2;

template <typename T>
__device__ __forceinline__ void dpsi3(T u, T (&d)[3]) {
  const T u2 = u * u;
  d[0] = T(0.5) * (u2 - u);
  d[1] = -u2;
  d[2] = T(0.5) * (u2 + u);
}
template <typename T>
__device__ __forceinline__ T wk(int k) { return k == 1 ? T(2) / T(3) : T(1) / T(6); }

// f_i^eq - w_i for the nine directions from drho = rho - 1 and the per-axis deviations
template <typename T>
__device__ __forceinline__ T heq_i(int i, T drho, const T (&dx)[3], const T (&dy)[3]) {
  const int a = i % 3, b = i / 3;
  const T pa = wk<T>(a) + dx[a], pb = wk<T>(b) + dy[b];
  return drho * (pa * pb) + (wk<T>(a) * dy[b] + dx[a] * wk<T>(b) + dx[a] * dy[b]);
}

template <typename Codec, bool WALLS, bool DIAG>
__global__ void __launch_bounds__(kBlock)
k_bgk_d2q9_red(const float* __restrict__ M, const uint16_t* __restrict__ N, float* __restrict__ Mo,
               uint16_t* __restrict__ No, int nx, int ny, int64_t pitch, int64_t plane,
               double omega_d, float s_enc, float s_dec, int rows, double* __restrict__ partials) {
  __shared__ float ring[3][kRedCols][9];
  const int nbx = gridDim.x;
  const int tile = xcd_tile(blockIdx.x + nbx * blockIdx.y, nbx * gridDim.y);
  const int bx = tile % nbx;
  const int by = tile / nbx;
  const int tid = threadIdx.x;
  const int x0 = bx * kBlock;
  const int x = x0 + tid;
  const int y0 = by * rows;
  const int yend = min(y0 + rows, ny);
  const float keep = (float)(1.0 - omega_d);  // f~ - f^eq = (1 - omega)(f - f^eq)
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};

  // Row staging is software-pipelined: the raw stored values of a row (3 moments + 6 codes per
  // column) are fetched into registers one iteration ahead, so their latency overlaps the
  // collision of the current row; decoding them into LDS slot r mod 3 happens the next
  // iteration. Columns c = 0..257 map to x0 - 1 + c (periodic); thread t owns column t and,
  // for t < 2, column 256 + t.
  struct Raw {
    float m[3];
    uint16_t n[kRedF];
  };
  Raw ra, rb;
  auto fetch = [&](int rr, int c, Raw& v) {
    int xg = x0 - 1 + c;
    xg = ((xg % nx) + nx) % nx;
    const int64_t off = (int64_t)rr * pitch + xg;
#pragma unroll
    for (int k = 0; k < 3; ++k) v.m[k] = M[k * plane + off];
#pragma unroll
    for (int k = 0; k < kRedF; ++k) v.n[k] = N[k * plane + off];
  };
  auto decode = [&](const Raw& v, float (&dst)[9]) {
    double n[9];
#pragma unroll
    for (int i = 0; i < 9; ++i)
      if (f_slot(i) >= 0) n[i] = (double)Codec::dec(v.n[f_slot(i)], s_dec);
    n[5] = n[0] - n[2] + n[3] + n[6] - n[8];
    n[7] = n[0] + n[1] + n[2] - n[6] - n[8];
    n[4] = -(((n[0] + n[1]) + (n[2] + n[3])) + ((n[5] + n[6]) + (n[7] + n[8])));
    double dx[3], dy[3];
    dpsi3((double)v.m[1], dx);
    dpsi3((double)v.m[2], dy);
#pragma unroll
    for (int i = 0; i < 9; ++i) dst[i] = (float)(heq_i(i, (double)v.m[0], dx, dy) + n[i]);
  };
  // rows beyond a wall are never pulled (bounce-back) and are skipped
  auto outside = [&](int r) { return WALLS && (r < 0 || r >= ny); };
  auto fetch_row = [&](int r) {
    if (outside(r)) return;
    const int rr = ((r % ny) + ny) % ny;
    fetch(rr, tid, ra);
    if (tid < kRedCols - kBlock) fetch(rr, kBlock + tid, rb);
  };
  auto put_row = [&](int r) {
    if (outside(r)) return;
    float(*dst)[9] = ring[((r % 3) + 3) % 3];
    decode(ra, dst[tid]);
    if (tid < kRedCols - kBlock) decode(rb, dst[kBlock + tid]);
  };

  fetch_row(y0 - 1);
  put_row(y0 - 1);
  fetch_row(y0);
  put_row(y0);
  fetch_row(y0 + 1);
  for (int y = y0; y < yend; ++y) {
    put_row(y + 1);  // slot (y + 1) mod 3 was last read by row y - 1, before the barrier below
    __syncthreads();
    if (y + 1 < yend) fetch_row(y + 2);  // consumed by the next iteration
    if (x < nx) {
      float h[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int ka = i % 3, kb = i / 3;
        const bool bounce = WALLS && ((kb == 2 && y == 0) || (kb == 0 && y == ny - 1));
        h[i] = bounce ? ring[((y % 3) + 3) % 3][tid + 1][8 - i]
                      : ring[(((y - kb + 1) % 3) + 3) % 3][tid + 1 - (ka - 1)][i];
      }
      // sum_i w_i = 1 and sum_i c_i w_i = 0
      const float drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
      const float jx = (h[2] + h[5] + h[8]) - (h[0] + h[3] + h[6]);
      const float jy = (h[6] + h[7] + h[8]) - (h[0] + h[1] + h[2]);
      const float rho = 1.0f + drho;
      const float ux = jx / rho, uy = jy / rho;
      float dx[3], dy[3];
      dpsi3(ux, dx);
      dpsi3(uy, dy);
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
        acc[0] += 1.0 + (double)drho;
        acc[1] += (double)jx;
        acc[2] += (double)jy;
        acc[4] += 0.5 * (double)rho * ((double)ux * ux + (double)uy * uy);
      }
    }
    __syncthreads();
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
  const double rho = 1.0 + (double)M[off];
  const double feq = rho * psi_c(i % 3 - 1, (double)M[plane + off]) * psi_c(i / 3 - 1, (double)M[2 * plane + off]);
  out[n] = feq + neq_f<Codec>(N, plane, off, i, s_dec);
}

// ---- launchers -----------------------------------------------------------------------------
Grid make_grid_red(const Layout& L) {
  Grid G;
  G.bx = kBlock;
  G.nbx = (L.nx + kBlock - 1) / kBlock;
  G.rows = 16;  // sweep on MI355X at 2048^2: 1 -> 88 us, 4 -> 62, 16 -> 56, 32 -> 77
#ifdef LBM_TUNING_ENV
  if (const char* v = getenv("LBM_RED_ROWS")) G.rows = atoi(v);
#endif
  fit_rows(G, L.ny);  // tall lattices take more rows per workgroup (grid y <= kMaxGridY)
  return G;
}

template <typename Codec, bool WALLS>
static void red_launch(const float* M, const uint16_t* N, float* Mo, uint16_t* No, const Layout& L,
                       const Grid& G, double omega, float se, float sd, double* partials,
                       hipStream_t s) {
  dim3 grid(G.nbx, G.nby), block(kBlock);
  if (partials)
    k_bgk_d2q9_red<Codec, WALLS, true><<<grid, block, 0, s>>>(M, N, Mo, No, L.nx, L.ny, L.pitch, L.plane, omega, se, sd, G.rows, partials);
  else
    k_bgk_d2q9_red<Codec, WALLS, false><<<grid, block, 0, s>>>(M, N, Mo, No, L.nx, L.ny, L.pitch, L.plane, omega, se, sd, G.rows, nullptr);
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
