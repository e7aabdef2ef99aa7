// Double-distribution (f, g) fused pull stream-collide kernel, D2Q9, ideal gas.
//
// One launch advances one time step of Eq. (LBM_f) and Eq. (LBM_g) of Sec. II C in the order
// of Fig. 1 (no body force, no heat source):
//   pull f_i, g_i from x - c_i (periodic in x; periodic or half-way bounce-back walls in y);
//   rho = sum f, rho u = sum c f, rho E = sum g;  T = (E - u^2/2)/c_v, P = rho R T,
//   theta = P/rho (ideal gas, Sec. III A);
//   Galilean correction Phi_aa = -(1/rho) d_a(rho u_a^3 + 3 rho u_a (theta - 1/3)) with a
//   finite-difference derivative of the moments of the neighbouring nodes at the same time
//   level (central, or one-sided on the upwind side of u_a);
//   f^eq, f* = rho prod_a Psi(u_a, theta + u_a^2 + Phi_aa), g^eq = g* (closed form of the
//   operator-generated energy equilibrium; q^c = 0 at Prandtl number 1);
//   beta = 1/(2 tau + 1), tau = mu/P, omega = 2 beta;
//   f~ = f + omega (f^eq - f) + (1 - beta)(f* - f^eq),  g~ = g + omega (g^eq - g).
//
// Tiling. A workgroup of 256 threads owns 256 - 2 HALO columns and `rows` rows; each thread
// holds one column (the HALO columns at either side only supply neighbour moments) and walks
// the rows y0 - HALO .. y0 + rows + HALO - 1 bottom to top. For each row it gathers the
// populations, computes the moments and the correction fluxes phi_a, exchanges phi_x across the
// row through LDS (x derivative) and keeps phi_y of the last 2 HALO + 1 rows of its own column
// in LDS (y derivative). A row is collided HALO rows after it was gathered, when the y
// stencil is complete; its populations wait in a register ring of HALO + 1 slots. Each
// population of the lattice is read once from HBM by its owning workgroup; halo rows and
// columns are re-read by the neighbouring workgroup (L2 hits for the x halo of neighbouring
// tiles on the same XCD).
//
// Storage: float32 or float64 planes holding f_i - w_i and g_i - v_i, where w, v are the
// equilibria at rest at the reference state rho = 1, T = 1 (the part that carries the flow is
// kept with full relative precision). Arithmetic is float64.
#include "ddf_common.h"

namespace lbm {

template <typename S, int HALO, bool WALLS, bool PULL, bool DIAG>
__global__ void __launch_bounds__(kBlock)
k_ddf_d2q9(const S* __restrict__ A, S* __restrict__ B, int nx, int ny, int64_t pitch,
           int64_t plane, DdfParams prm, int rows, double* __restrict__ partials) {
  constexpr int H1 = HALO + 1;
  constexpr int P = 2 * HALO + 1;
  constexpr int TXI = kBlock - 2 * HALO;
  __shared__ double s_phix[2][kBlock];
  __shared__ double s_phiy[P][kBlock];

  const int nbx = gridDim.x;
  const int tile = xcd_tile(blockIdx.x + nbx * blockIdx.y, nbx * gridDim.y);
  const int bx = tile % nbx;
  const int by = tile / nbx;
  const int tid = threadIdx.x;
  const int x0 = bx * TXI;
  const int xu = x0 - HALO + tid;                 // unwrapped column
  const int x = ((xu % nx) + nx) % nx;            // periodic in x
  const bool own = tid >= HALO && tid < kBlock - HALO && xu < nx;
  const int xm = x == 0 ? nx - 1 : x - 1;
  const int xp = x == nx - 1 ? 0 : x + 1;
  const int y0 = by * rows;
  const int yend = min(y0 + rows, ny);
  const int count = (yend - y0) + 2 * HALO;       // window rows

  S ring_f[H1][9], ring_g[H1][9];
  double ring_m[H1][6];  // rho, u_x, u_y, theta, e, Phi_xx
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const S* Ag = A + 9 * plane;
  S* Bf = B;
  S* Bg = B + 9 * plane;

  for (int k = 0; k < count; k += H1) {
#pragma unroll
    for (int j = 0; j < H1; ++j) {
      const int w = k + j;                 // window index (block-uniform)
      const int r = y0 - HALO + w;         // row being gathered
      const bool in_window = w < count;
      const bool row_real = in_window && (WALLS ? (r >= 0 && r < ny) : true);
      const int rr = WALLS ? r : ((r % ny) + ny) % ny;
      double phx = 0.0, phy = 0.0;
      if (row_real) {
        // ---- gather (pull) ----------------------------------------------------------------
        if (PULL) {
          const int ym = rr == 0 ? ny - 1 : rr - 1;
          const int yp = rr == ny - 1 ? 0 : rr + 1;
          const int64_t r0 = (int64_t)rr * pitch, rm = (int64_t)ym * pitch, rp = (int64_t)yp * pitch;
          const bool top = WALLS && rr == ny - 1, bot = WALLS && rr == 0;
          gather9(A, plane, r0, rm, rp, x, xm, xp, top, bot, ring_f[j]);
          gather9(Ag, plane, r0, rm, rp, x, xm, xp, top, bot, ring_g[j]);
        } else {
          const int64_t off = (int64_t)rr * pitch + x;
#pragma unroll
          for (int i = 0; i < 9; ++i) {
            ring_f[j][i] = A[i * plane + off];
            ring_g[j][i] = Ag[i * plane + off];
          }
        }
        // ---- moments and closure ------------------------------------------------------------
        double f[9], g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          f[i] = (double)ring_f[j][i] + prm.wf[i];
          g[i] = (double)ring_g[j][i] + prm.wg[i];
        }
        Moments m;
        moments_closure(f, g, prm, m);
        ring_m[j][0] = m.rho;
        ring_m[j][1] = m.ux;
        ring_m[j][2] = m.uy;
        ring_m[j][3] = m.theta;
        ring_m[j][4] = m.e;
        phx = m.rho * m.ux * (m.ux * m.ux + 3.0 * (m.theta - 1.0 / 3.0));
        phy = m.rho * m.uy * (m.uy * m.uy + 3.0 * (m.theta - 1.0 / 3.0));
      }
      s_phix[w & 1][tid] = phx;
      s_phiy[((r % P) + P) % P][tid] = phy;
      __syncthreads();
      // ---- x derivative of phi_x on the gathered row -----------------------------------------
      if (row_real && own && prm.phi) {
        const double* px = s_phix[w & 1];
        double d;
        if (HALO == 1) {
          d = 0.5 * (px[tid + 1] - px[tid - 1]);
        } else {
          d = upwind_or_central(px[tid - 2], px[tid - 1], px[tid], px[tid + 1], px[tid + 2],
                                ring_m[j][1]);
        }
        ring_m[j][5] = -d / ring_m[j][0];
      }
      // ---- collide the row gathered HALO rows earlier -----------------------------------------
      const int c = r - HALO;
      const int sc = (j + 1) % H1;  // ring slot of row c (a constant once unrolled)
      if (in_window && own && c >= y0 && c < yend) {
        const int cc = WALLS ? c : ((c % ny) + ny) % ny;
        double phyy = 0.0;
        if (prm.phi) {
          double q[5];
#pragma unroll
          for (int o = -HALO; o <= HALO; ++o) {
            int row = c + o;
            if (WALLS) row = row < 0 ? 0 : (row > ny - 1 ? ny - 1 : row);  // zero-order ghosts
            q[o + 2] = s_phiy[((row % P) + P) % P][tid];
          }
          double d;
          if (HALO == 1)
            d = 0.5 * (q[3] - q[1]);
          else
            d = upwind_or_central(q[0], q[1], q[2], q[3], q[4], ring_m[sc][2]);
          phyy = -d / ring_m[sc][0];
        }
        const double phxx = prm.phi ? ring_m[sc][5] : 0.0;
        S of[9], og[9];
        collide_ddf(ring_f[sc], ring_g[sc], ring_m[sc], phxx, phyy, prm, of, og);
        const int64_t off = (int64_t)cc * pitch + x;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          store_nt(Bf + i * plane + off, of[i]);
          store_nt(Bg + i * plane + off, og[i]);
        }
        if (DIAG) {
          const double rho = ring_m[sc][0];
          acc[0] += rho;
          acc[1] += rho * ring_m[sc][1];
          acc[2] += rho * ring_m[sc][2];
          const double u2 = ring_m[sc][1] * ring_m[sc][1] + ring_m[sc][2] * ring_m[sc][2];
          acc[4] += rho * (ring_m[sc][4] + 0.5 * u2);
        }
      }
    }
  }
  if (DIAG) block_sum_store<kDiagValues>(acc, partials + (int64_t)tile * kDiagValues);
}

// f <- f^eq, g <- g^eq of the initial fields (Fig. 1), stored shifted by the rest state.
template <typename S>
__global__ void k_init_ddf(const double* __restrict__ rho, const double* __restrict__ u,
                           const double* __restrict__ T, S* __restrict__ A, int nx, int ny,
                           int64_t pitch, int64_t plane, DdfParams prm) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nodes = (int64_t)nx * ny;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  const double theta = prm.R * T[n];
  double fe[9], ge[9];
  equilibria(rho[n], u[n], u[nodes + n], theta, prm.cv * T[n], fe, ge);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    A[i * plane + off] = (S)(fe[i] - prm.wf[i]);
    A[(9 + i) * plane + off] = (S)(ge[i] - prm.wg[i]);
  }
}

// rho, u, T of the stored state (the collision conserves rho, rho u and rho E).
template <typename S>
__global__ void k_moments_ddf(const S* __restrict__ A, int nx, int ny, int64_t pitch,
                              int64_t plane, DdfParams prm, double* __restrict__ rho,
                              double* __restrict__ u, double* __restrict__ T,
                              double* __restrict__ edens) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nodes = (int64_t)nx * ny;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  double f[9], g[9];
  for (int i = 0; i < 9; ++i) {
    f[i] = (double)A[i * plane + off] + prm.wf[i];
    g[i] = (double)A[(9 + i) * plane + off] + prm.wg[i];
  }
  Moments m;
  moments_closure(f, g, prm, m);
  rho[n] = m.rho;
  u[n] = m.ux;
  u[nodes + n] = m.uy;
  T[n] = m.theta / prm.R;
  edens[n] = m.rho * (m.e + 0.5 * (m.ux * m.ux + m.uy * m.uy));
}

template <typename S>
__global__ void k_decode_ddf(int i, const S* __restrict__ Ai, int nx, int64_t nodes,
                             int64_t pitch, DdfParams prm, double* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  out[n] = (double)Ai[off] + (i < 9 ? prm.wf[i] : prm.wg[i - 9]);
}

__global__ void k_ddf_rest_state(DdfParams prm, double* __restrict__ out) {
  double fe[9], ge[9];
  equilibria(1.0, 0.0, 0.0, prm.R, prm.cv, fe, ge);
  for (int i = 0; i < 9; ++i) {
    out[i] = fe[i];
    out[9 + i] = ge[i];
  }
}

// ---- launchers ------------------------------------------------------------------------------
Grid make_grid_ddf(const Layout& L, int halo) {
  Grid G;
  G.bx = kBlock;
  const int txi = kBlock - 2 * halo;
  G.nbx = (L.nx + txi - 1) / txi;
  G.rows = 32;
  G.nby = (L.ny + G.rows - 1) / G.rows;
  return G;
}

template <typename S, int HALO, bool WALLS, bool PULL>
static void ddf_launch(const void* A, void* B, const Layout& L, const Grid& G,
                       const DdfParams& prm, double* partials, hipStream_t s) {
  dim3 grid(G.nbx, G.nby), block(kBlock);
  auto a = static_cast<const S*>(A);
  auto b = static_cast<S*>(B);
  if (partials)
    k_ddf_d2q9<S, HALO, WALLS, PULL, true><<<grid, block, 0, s>>>(a, b, L.nx, L.ny, L.pitch, L.plane, prm, G.rows, partials);
  else
    k_ddf_d2q9<S, HALO, WALLS, PULL, false><<<grid, block, 0, s>>>(a, b, L.nx, L.ny, L.pitch, L.plane, prm, G.rows, nullptr);
}

template <typename S, int HALO>
static void ddf_launch_w(bool walls, bool pull, const void* A, void* B, const Layout& L,
                         const Grid& G, const DdfParams& prm, double* partials, hipStream_t s) {
  if (walls) {
    if (pull) ddf_launch<S, HALO, true, true>(A, B, L, G, prm, partials, s);
    else ddf_launch<S, HALO, true, false>(A, B, L, G, prm, partials, s);
  } else {
    if (pull) ddf_launch<S, HALO, false, true>(A, B, L, G, prm, partials, s);
    else ddf_launch<S, HALO, false, false>(A, B, L, G, prm, partials, s);
  }
}

hipError_t launch_ddf(int kind, bool walls, bool pull, const void* A, void* B, const Layout& L,
                      const Grid& G, const DdfParams& prm, double* partials, hipStream_t s) {
  const int halo = prm.phi == 2 ? 2 : 1;
  if (kind == 0) {
    if (halo == 1) ddf_launch_w<float, 1>(walls, pull, A, B, L, G, prm, partials, s);
    else ddf_launch_w<float, 2>(walls, pull, A, B, L, G, prm, partials, s);
  } else {
    if (halo == 1) ddf_launch_w<double, 1>(walls, pull, A, B, L, G, prm, partials, s);
    else ddf_launch_w<double, 2>(walls, pull, A, B, L, G, prm, partials, s);
  }
  return hipGetLastError();
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_ddf_rest_state(const DdfParams& prm, double* out, hipStream_t s) {
  k_ddf_rest_state<<<1, 1, 0, s>>>(prm, out);
  return hipGetLastError();
}

hipError_t launch_init_ddf(int kind, const double* rho, const double* u, const double* T,
                           void* A, const Layout& L, const DdfParams& prm, hipStream_t s) {
  if (kind == 0)
    k_init_ddf<float><<<nblk(L.nodes()), kBlock, 0, s>>>(rho, u, T, static_cast<float*>(A), L.nx, L.ny, L.pitch, L.plane, prm);
  else
    k_init_ddf<double><<<nblk(L.nodes()), kBlock, 0, s>>>(rho, u, T, static_cast<double*>(A), L.nx, L.ny, L.pitch, L.plane, prm);
  return hipGetLastError();
}

hipError_t launch_moments_ddf(int kind, const void* A, const Layout& L, const DdfParams& prm,
                              double* rho, double* u, double* T, double* edens, hipStream_t s) {
  if (kind == 0)
    k_moments_ddf<float><<<nblk(L.nodes()), kBlock, 0, s>>>(static_cast<const float*>(A), L.nx, L.ny, L.pitch, L.plane, prm, rho, u, T, edens);
  else
    k_moments_ddf<double><<<nblk(L.nodes()), kBlock, 0, s>>>(static_cast<const double*>(A), L.nx, L.ny, L.pitch, L.plane, prm, rho, u, T, edens);
  return hipGetLastError();
}

hipError_t launch_decode_ddf(int kind, int i, const void* A, const Layout& L,
                             const DdfParams& prm, double* out, hipStream_t s) {
  if (kind == 0)
    k_decode_ddf<float><<<nblk(L.nodes()), kBlock, 0, s>>>(i, static_cast<const float*>(A) + (int64_t)i * L.plane, L.nx, L.nodes(), L.pitch, prm, out);
  else
    k_decode_ddf<double><<<nblk(L.nodes()), kBlock, 0, s>>>(i, static_cast<const double*>(A) + (int64_t)i * L.plane, L.nx, L.nodes(), L.pitch, prm, out);
  return hipGetLastError();
}

}  // namespace lbm
