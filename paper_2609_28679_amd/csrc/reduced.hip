// Isothermal D2Q9 fused pull stream-collide on reduced-precision storage (float32 moments +
// 16-bit non-equilibrium part, see reduced_common.h).
//
// Pull: the pre-collision population i at x is the post-collision population i of the source
// node s = x - c_i, rebuilt from that node's stored moments and non-equilibrium part,
//   f_i(x, t) = f_i^eq(m(s)) + n_i(s)       (f_ibar(x) at a half-way bounce-back wall),
// with the product-form equilibrium of Sec. II C at theta = 1/3. The collision is the plain
// BGK relaxation of Eq. (LBM_f) with f* = f^eq in float64; the new state is written back as
// m(x) = (rho - 1, u) and n(x) = f~(x) - f^eq(m(x)).
#include "reduced_common.h"

namespace lbm {

__device__ __forceinline__ double psi_c(int c, double u) {
  const double u2 = u * u;
  return c == 0 ? (2.0 / 3.0) - u2 : (1.0 / 6.0) + 0.5 * (u2 + c * u);
}

template <typename Codec, bool WALLS, bool DIAG>
__global__ void __launch_bounds__(kBlock)
k_bgk_d2q9_red(const float* __restrict__ M, const uint16_t* __restrict__ N, float* __restrict__ Mo,
               uint16_t* __restrict__ No, int nx, int ny, int64_t pitch, int64_t plane,
               double omega, float s_enc, float s_dec, int rows, double* __restrict__ partials) {
  const int nbx = gridDim.x;
  const int tile = xcd_tile(blockIdx.x + nbx * blockIdx.y, nbx * gridDim.y);
  const int bx = tile % nbx;
  const int by = tile / nbx;
  const int x = bx * blockDim.x + threadIdx.x;
  const int y0 = by * rows;
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};

  if (x < nx) {
    const int xs[3] = {x == nx - 1 ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};  // by c_x + 1
    const int yend = min(y0 + rows, ny);
    for (int y = y0; y < yend; ++y) {
      const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
      const int64_t self = (int64_t)y * pitch + x;
      double f[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int ka = i % 3, kb = i / 3;
        const bool bounce = WALLS && ((kb == 2 && y == 0) || (kb == 0 && y == ny - 1));
        const int ii = bounce ? 8 - i : i;
        const int64_t src = bounce ? self : (int64_t)ys[kb] * pitch + xs[ka];
        const double rho = 1.0 + (double)M[src];
        const double ux = (double)M[plane + src];
        const double uy = (double)M[2 * plane + src];
        const double feq = rho * psi_c(ii % 3 - 1, ux) * psi_c(ii / 3 - 1, uy);
        f[i] = feq + neq_f<Codec>(N, plane, src, ii, s_dec);
      }
      const double rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
      const double jx = (f[2] + f[5] + f[8]) - (f[0] + f[3] + f[6]);
      const double jy = (f[6] + f[7] + f[8]) - (f[0] + f[1] + f[2]);
      const double ux = jx / rho, uy = jy / rho;
      double px[3], py[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        px[k] = psi_c(k - 1, ux);
        py[k] = psi_c(k - 1, uy);
      }
      // post-collision non-equilibrium part: f~ - f^eq = (1 - omega)(f - f^eq)
      double n[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) n[i] = (1.0 - omega) * (f[i] - rho * px[i % 3] * py[i / 3]);
      store_nt(Mo + self, (float)(rho - 1.0));
      store_nt(Mo + plane + self, (float)ux);
      store_nt(Mo + 2 * plane + self, (float)uy);
#pragma unroll
      for (int i = 0; i < 9; ++i)
        if (f_slot(i) >= 0) store_nt(No + f_slot(i) * plane + self, Codec::enc(n[i], s_enc));
      if (DIAG) {
        acc[0] += rho;
        acc[1] += jx;
        acc[2] += jy;
        acc[4] += 0.5 * rho * (ux * ux + uy * uy);
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
  const double rho = 1.0 + (double)M[off];
  const double feq = rho * psi_c(i % 3 - 1, (double)M[plane + off]) * psi_c(i / 3 - 1, (double)M[2 * plane + off]);
  out[n] = feq + neq_f<Codec>(N, plane, off, i, s_dec);
}

// ---- launchers -----------------------------------------------------------------------------
template <typename Codec, bool WALLS>
static void red_launch(const float* M, const uint16_t* N, float* Mo, uint16_t* No, const Layout& L,
                       const Grid& G, double omega, float se, float sd, double* partials,
                       hipStream_t s) {
  dim3 grid(G.nbx, G.nby), block(G.bx);
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
